"""Write the FP64 oracle's rate-distortion results of a short encode with the
upsampling Conv refinement (the decoder of the 512x768 workload plus a
7-tap Conv before each upsampling level; 2,247 parameters).

    python tests/golden/make_conv_encode.py

Calls only the oracle and the seeded input generator: one 128x192 image
(seed 6, 1/f field), latents 0, identity Conv taps, lambda 1e-3, 300
iterations with the Table I schedules mapped onto them.  Stores the
hard-quantised bits, MSE, PSNR and loss, and the final Conv taps, as JSON.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import coolchic_ref as R  # noqa: E402
from paper_2605_02726_amd import workloads as wl  # noqa: E402

H, W, SEED, LAM, N_ITER = 128, 192, 6, 1e-3, 300


def main():
    mc = wl.config_hop_conv()
    st = R.OracleState(mc.as_dict(), H, W, wl.synth_image(H, W, SEED), LAM, SEED,
                       np.zeros(wl.n_latents(mc, H, W), np.float32), wl.init_params(mc, SEED))
    for t in range(1, N_ITER + 1):
        lr, T, s = R.schedule(t, N_ITER)
        st.step(t, lr, T, s)
    out = {"workload": f"{H}x{W} seed {SEED}, lambda {LAM}, latents 0, identity Conv taps",
           "n_iter": N_ITER, "made_by": "tests/golden/make_conv_encode.py (FP64 oracle)",
           "conv": st.rd_eval()}
    offs = wl.conv_taps_offsets(mc)
    out["conv_taps"] = [[float(st.theta[st.n_lat + o + t]) for t in range(4)] for o in offs]
    print(out, flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "conv_encode_128x192_300.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()

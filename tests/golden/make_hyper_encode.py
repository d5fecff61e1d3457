"""Write the FP64 oracle's rate-distortion results of a short encode with the
hyperlatent decoder (Section III-A.3) and without it.

    python tests/golden/make_hyper_encode.py

Calls only the oracle and the seeded input generator: one 128x192 image
(seed 6, 1/f field), the 2,223-parameter decoder and the same decoder with
three hyperlatent grids (1/16, 1/32, 1/64; 2,277 parameters), latents 0,
lambda 1e-3, 300 iterations with the Table I schedules mapped onto them.
Stores the hard-quantised bits, MSE, PSNR and loss of each run, as JSON.
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


def run(mc):
    st = R.OracleState(mc.as_dict(), H, W, wl.synth_image(H, W, SEED), LAM, SEED,
                       np.zeros(wl.n_latents(mc, H, W), np.float32), wl.init_params(mc, SEED))
    for t in range(1, N_ITER + 1):
        lr, T, s = R.schedule(t, N_ITER)
        st.step(t, lr, T, s)
    return st.rd_eval()


def main():
    out = {"workload": f"{H}x{W} seed {SEED}, lambda {LAM}, latents 0", "n_iter": N_ITER,
           "made_by": "tests/golden/make_hyper_encode.py (FP64 oracle)"}
    for name, mk in (("plain", wl.config_hop), ("hyper", wl.config_hop_hyper)):
        out[name] = run(mk())
        print(name, out[name], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hyper_encode_128x192_300.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()

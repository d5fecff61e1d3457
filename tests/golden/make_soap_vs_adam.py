"""Write the FP64 oracle's rate-distortion results of the same short encode
with Adam and with SOAP on the decoder parameters.

    python tests/golden/make_soap_vs_adam.py

Calls only the oracle and the seeded input generator: one 64x128 image
(seed 5, 1/f field), the 2,223-parameter decoder, latents 0, lambda 1e-3,
300 iterations with the Table I schedules mapped onto them; the latents use
Adam in both runs.  Stores the hard-quantised bits, MSE, PSNR and loss of
each run, as JSON.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import coolchic_ref as R  # noqa: E402
from paper_2605_02726_amd import workloads as wl  # noqa: E402

H, W, SEED, LAM, N_ITER = 64, 128, 5, 1e-3, 300


def run(optimizer):
    mc = wl.config_hop()
    st = R.OracleState(mc.as_dict(), H, W, wl.synth_image(H, W, SEED), LAM, SEED,
                       np.zeros(wl.n_latents(mc, H, W), np.float32), wl.init_params(mc, SEED),
                       optimizer=optimizer)
    for t in range(1, N_ITER + 1):
        lr, T, s = R.schedule(t, N_ITER)
        st.step(t, lr, T, s)
    return st.rd_eval()


def main():
    out = {"workload": f"{H}x{W} seed {SEED}, 2223-parameter decoder, lambda {LAM}, latents 0",
           "n_iter": N_ITER, "made_by": "tests/golden/make_soap_vs_adam.py (FP64 oracle)"}
    for opt in ("adam", "soap"):
        out[opt] = run(opt)
        print(opt, out[opt], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "soap_vs_adam_64x128_300.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()

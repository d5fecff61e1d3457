"""Write the FP64 oracle trajectory of the 512x768 encode workload.

    python tests/golden/make_trajectory.py [n_iter]

Calls only the oracle and the seeded input generator: one 512x768 image
(seed 2, 1/f field + 32 rectangles), the 2,223-parameter decoder, latents 0,
lambda 1e-3, Table I schedules mapped onto n_iter iterations (cosine lr
1e-2 -> 1e-5, T 0.35 -> 0.08, sigma 0.22 -> 0.15), Adam.  Stores the
training loss, bits and MSE of every iteration and the hard-quantised rate,
distortion and PSNR (rd_eval) at checkpoints, as JSON.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

from oracle import coolchic_ref as R  # noqa: E402
from paper_2605_02726_amd import workloads as wl  # noqa: E402


def main():
    n_iter = int(sys.argv[1]) if len(sys.argv) > 1 else 1000
    torch.set_num_threads(os.cpu_count() or 1)
    mc = wl.config_hop()
    H, W, seed, lam = 512, 768, 2, 1e-3
    st = R.OracleState(mc.as_dict(), H, W, wl.image_large(seed), lam, seed,
                       np.zeros(wl.n_latents(mc, H, W), np.float32), wl.init_params(mc, seed))
    checkpoints = sorted(set([1, 10, 50, 100, 250, 500, 750, n_iter]))
    steps, rd = [], {}
    t0 = time.time()
    for t in range(1, n_iter + 1):
        lr, T, s = R.schedule(t, n_iter)
        steps.append(st.step(t, lr, T, s))
        if t in checkpoints:
            rd[str(t)] = st.rd_eval()
            print(f"t={t} loss {steps[-1][0]:.6f} rd {rd[str(t)]} ({time.time() - t0:.0f} s)",
                  flush=True)
    out = {"workload": "512x768 seed 2, 2223-parameter decoder, lambda 1e-3, latents 0",
           "n_iter": n_iter, "steps": steps, "rd_eval": rd,
           "made_by": "tests/golden/make_trajectory.py (FP64 oracle)"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"trajectory_512x768_{n_iter}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main()

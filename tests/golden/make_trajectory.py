"""Write the FP64 oracle trajectory of the 512x768 encode workload.

    python tests/golden/make_trajectory.py [n_iter]
    python tests/golden/make_trajectory.py n_iter --perturb REL SEED
    python tests/golden/make_trajectory.py n_iter --fp32-storage

Calls only the oracle and the seeded input generator: one 512x768 image
(seed 2, 1/f field + 32 rectangles), the 2,223-parameter decoder, latents 0,
lambda 1e-3, Table I schedules mapped onto n_iter iterations (cosine lr
1e-2 -> 1e-5, T 0.35 -> 0.08, sigma 0.22 -> 0.15), Adam.  Stores the
training loss, bits and MSE of every iteration and the hard-quantised rate,
distortion and PSNR (rd_eval) at checkpoints, as JSON.

With --perturb, every gradient element is multiplied by (1 + REL xi) before
Adam, xi standard normal from PCG64(SEED, t): the same trajectory under
gradient errors of the size FP32 arithmetic makes, which measures how far
two correct implementations can drift apart after n_iter iterations.

With --fp32-storage, the latents, decoder parameters and both Adam moments
are rounded to float32 after every update (the arithmetic stays float64):
the storage precision of a GPU state, on its own.
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
    rel, pseed = 0.0, 0
    if "--perturb" in sys.argv:
        i = sys.argv.index("--perturb")
        rel, pseed = float(sys.argv[i + 1]), int(sys.argv[i + 2])
    fp32_storage = "--fp32-storage" in sys.argv
    torch.set_num_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    mc = wl.config_hop()
    H, W, seed, lam = 512, 768, 2, 1e-3
    st = R.OracleState(mc.as_dict(), H, W, wl.image_large(seed), lam, seed,
                       np.zeros(wl.n_latents(mc, H, W), np.float32), wl.init_params(mc, seed))
    checkpoints = sorted(set([1, 10, 50, 100, 250, 500, 750, n_iter]))
    steps, rd = [], {}
    t0 = time.time()
    for t in range(1, n_iter + 1):
        lr, T, s = R.schedule(t, n_iter)
        if rel == 0.0:
            steps.append(st.step(t, lr, T, s))
        else:
            loss, bits, mse, g = R.loss_and_grad(st.cfg, H, W, st.theta, st.img, lam, "soft", T, s,
                                                 seed, t)
            xi = np.random.Generator(np.random.PCG64([pseed, t])).standard_normal(g.shape)
            st.theta, st.m, st.v = R.adam(st.theta, g * (1.0 + rel * xi), st.m, st.v, t, lr)
            st.t = t
            steps.append((loss, bits, mse))
        if fp32_storage:
            st.theta, st.m, st.v = (np.asarray(a, np.float32).astype(np.float64)
                                    for a in (st.theta, st.m, st.v))
        if t in checkpoints:
            rd[str(t)] = st.rd_eval()
            print(f"t={t} loss {steps[-1][0]:.6f} rd {rd[str(t)]} ({time.time() - t0:.0f} s)",
                  flush=True)
    out = {"workload": "512x768 seed 2, 2223-parameter decoder, lambda 1e-3, latents 0",
           "n_iter": n_iter, "steps": steps, "rd_eval": rd,
           "made_by": "tests/golden/make_trajectory.py (FP64 oracle)"}
    name = f"trajectory_512x768_{n_iter}.json"
    if rel != 0.0:
        out["perturbation"] = {"relative": rel, "seed": pseed}
        name = f"trajectory_512x768_{n_iter}_perturbed_{pseed}.json"
    if fp32_storage:
        out["storage"] = "float32 theta, m, v after every update"
        name = name.replace(".json", "_fp32storage.json")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), name)
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main()

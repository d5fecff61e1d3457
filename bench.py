"""Throughput of the Cool-chic encode step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32|bf16]

One step = one full encoding iteration (training quantisation proxy, ARM
entropy model and rate, upsampling, synthesis, MSE, backward, Adam) of one
512x768 synthetic image with the 2,223-parameter decoder (s = 24 + F = 6
inter-feature context, ARM 30-24-24-2 with stabilizer, synthesis 7-40-3 with
stabilizer and two residual 3x3 layers), schedules of Table I mapped onto a
1,000-iteration budget.  Inputs are resident in HBM before the timed region.
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {
    # MI355X published peaks
    "hbm_GBs": 8000.0,
    "bf16_mfma_TFLOPs": 2500.0,
    # FP32 vector FMA without packed-FP32 instructions (which this build
    # disables): 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz
    "fp32_valu_TFLOPs": 78.6,
}


def arm_flops_per_step(mc, H, W):
    """Algorithmic FLOPs of the ARM forward + rate-gradient backward + weight
    gradient over every latent position (2 FLOP per multiply-add)."""
    ctx = mc.n_spatial + mc.n_ifce_feat
    h1, h2 = mc.arm_hidden
    tot = 0
    for k in range(mc.L):
        n = (H >> k) * (W >> k)
        fwd = ctx * h1 + h1 * h2 + 2 * h2 + (2 * ctx if mc.arm_stab else 0)
        if k < mc.n_ifce_grids:
            fwd += mc.n_ifce_feat * (mc.L - k - 1)
        bwd = 2 * h2 + h1 * h2 + ctx * h1 + (2 * ctx if mc.arm_stab else 0)
        tot += n * 2 * (2 * fwd + bwd)
    return tot


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--cpu-steps", type=int, default=12, help="oracle steps for cpu_baseline (0 = skip)")
    ap.add_argument("--no-kernel-timing", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: the per-image encode step is "
                          "data-parallel inside one MI355X; --gpus must be 1"}))
        sys.exit(2)

    import ctypes as C
    import numpy as np
    import torch

    from paper_2605_02726_amd import _lib, workloads as wl
    from paper_2605_02726_amd.encoder import Encoder, schedule

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    mc = wl.config_hop()
    H, W, seed, lam, n_iter = 512, 768, 2, 1e-3, 1000
    img = torch.from_numpy(wl.image_large(seed))
    lat = np.zeros(wl.n_latents(mc, H, W), np.float32)
    par = wl.init_params(mc, seed)
    enc = Encoder(mc, img, lam, seed, lat, par, precision=args.precision)
    L = _lib.lib()

    t = 0
    for _ in range(args.warmup):
        t += 1
        lr, T, s = schedule(t, n_iter)
        enc.step(t, lr, T, s, sync=False)
    torch.cuda.synchronize()
    if not args.no_kernel_timing:
        _lib.check(L.cc_timing_enable(b"arm"))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t += 1
        lr, T, s = schedule(t, n_iter)
        enc.step(t, lr, T, s, sync=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    arm_ms, arm_n = C.c_double(0.0), C.c_int(0)
    if not args.no_kernel_timing:
        _lib.check(L.cc_timing_read(C.byref(arm_ms), C.byref(arm_n)))
        _lib.check(L.cc_timing_enable(None))
    loss, bits, mse = enc.eval_loss(t, T, s)

    ms_step = 1e3 * dt / args.steps
    value = H * W * args.steps / dt / 1e6
    flops = arm_flops_per_step(mc, H, W)
    roof = None
    if arm_n.value:
        avg_s = arm_ms.value / arm_n.value / 1e3
        if args.precision == "fp32":
            achieved = flops / avg_s / 1e12
            roof = {"kernel": "arm_fwd_rate_bwd", "bound": "alu", "achieved": round(achieved, 3),
                    "peak": PEAKS["fp32_valu_TFLOPs"], "unit": "TFLOP/s",
                    "frac": round(achieved / PEAKS["fp32_valu_TFLOPs"], 4), "traffic": None,
                    "avg_launch_ms": round(1e3 * avg_s, 4), "flops_per_launch": flops}
        else:
            achieved = flops / avg_s / 1e12
            roof = {"kernel": "arm_fwd_rate_bwd", "bound": "mfma", "achieved": round(achieved, 3),
                    "peak": PEAKS["bf16_mfma_TFLOPs"], "unit": "TFLOP/s",
                    "frac": round(achieved / PEAKS["bf16_mfma_TFLOPs"], 4), "traffic": None,
                    "avg_launch_ms": round(1e3 * avg_s, 4), "flops_per_launch": flops}

    cpu = None
    if args.cpu_steps > 0:
        from oracle import coolchic_ref as R
        torch.set_num_threads(os.cpu_count() or 1)
        ost = R.OracleState(mc.as_dict(), H, W, wl.image_large(seed), lam, seed, lat, par)
        ost.step(1, *schedule(1, n_iter))     # first call pays one-off costs
        c0 = time.perf_counter()
        for tt in range(2, 2 + args.cpu_steps):
            ost.step(tt, *schedule(tt, n_iter))
        cdt = time.perf_counter() - c0
        cpu = {"value": round(H * W * args.cpu_steps / cdt / 1e6, 4),
               "unit": "Mpixel-iterations/s", "cores": torch.get_num_threads(), "kind": "oracle",
               "sample": f"{args.cpu_steps} FP64 oracle steps of the same 512x768 workload "
                         f"({cdt:.1f} s)"}

    out = {
        "metric": "Mpixel-iterations/s (fwd+bwd+Adam)",
        "value": round(value, 3),
        "unit": "Mpixel-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16",
        "data": "synthetic",
        "config": {"workload": "encode step, one 512x768 RGB image, 2223-parameter decoder "
                               "(s=24+F=6 ARM 30-24-24-2, synthesis 7-40-3, 2 residual 3x3)",
                   "global_batch": 1, "precision_form": args.precision,
                   "final_loss": loss, "final_bits": bits, "final_mse": mse},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

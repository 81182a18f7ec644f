"""Throughput of the forward + inverse SHT on one MI355X.

One step = one inverse SHT followed by one forward SHT of a batch of B maps
(the forward consumes the inverse's samples), on the headline workload:
spin 0, L = 1024, B = 16, coefficients N(0,1)(1+l)^-1 (seed 5), FP64 path.

Prints one JSON line (the driver's contract) with, in addition:
  roofline      the order-wise apply GEMM that dominates the step: algorithmic
                FP64 flops (2 x matrix entries x 2B real columns per signed
                order, summed over the launches timed live with HIP events in
                the timed region) over its measured time, against the MI355X
                FP64 matrix peak;
  cpu_baseline  the FP64 CPU oracle (tests' reference implementation) timed on
                the host on a bounded sample (see 'sample'), scaled to the
                metric's unit.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--L", type=int, default=1024)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def cpu_baseline(L_metric):
    """Oracle forward + inverse at L = 512, B = 1 (warm plan: tables and LU
    factors cached), scaled by (L_metric/512)^3, the paper's O(L^3) scaling."""
    import numpy as np

    from oracle import sht
    from tests import inputs
    from tests.gpu_util import oracle_plan

    Ls = 512
    p = oracle_plan(Ls)
    flm = inputs.coeffs(Ls, 1, seed=5, weighted=True)
    sht.forward(p, sht.inverse(p, flm))  # warm the plan caches
    t0 = time.perf_counter()
    f = sht.inverse(p, flm)
    g = sht.forward(p, f)
    dt = time.perf_counter() - t0
    err = float(np.max(np.abs(g - flm)) / np.max(np.abs(flm)))
    threads = os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        if info:
            threads = max(int(i.get("num_threads", 1)) for i in info)
    except Exception:
        pass
    scale = (L_metric / Ls) ** 3
    return {
        "value": 1.0 / (dt * scale),
        "unit": "SHT/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"oracle inverse+forward at L={Ls}, B=1 (warm plan) took {dt:.2f} s; "
                  f"scaled by (L/{Ls})^3 = {scale:.0f} to L={L_metric}; round-trip rel err {err:.1e}",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1403_4661_amd import Plan
    from tests import inputs

    L, B = args.L, args.batch
    torch.cuda.set_device(0)
    plan = Plan(L, 0)
    flm_h = inputs.coeffs(L, B, seed=5, weighted=True)
    flm = torch.as_tensor(flm_h).cuda()
    f = torch.empty_like(flm)
    g = torch.empty_like(flm)
    for _ in range(args.warmup):
        plan.inverse(flm, out=f)
        plan.forward(f, out=g)
    torch.cuda.synchronize()
    g_h = g.cpu().numpy()
    rt_err = float(np.max(np.abs(g_h - flm_h)) / np.max(np.abs(flm_h)))

    plan.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.inverse(flm, out=f)
        plan.forward(f, out=g)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt / args.steps * 1e3

    # per-kernel event timings of the timed region
    kern = {}
    for name in ("apply_inverse", "apply_forward", "ring_analysis", "ring_synthesis"):
        n, ms = plan.kernel_time(name)
        kern[name] = {"launches": n, "ms_total": ms}
    plan.set_profiling(False)
    # algorithmic work of one step's apply GEMMs: every signed order m streams
    # an L x (L-|m|) FP64 block against 2B real columns -> 4 B L^3 flop per
    # direction; each direction streams L^2 (L+1)/2 matrix entries once.
    flop_dir = 4.0 * B * L ** 3
    bytes_dir = 8.0 * L * L * (L + 1) / 2
    for name in ("apply_inverse", "apply_forward"):
        k = kern[name]
        if k["ms_total"] > 0:
            k["tflops"] = flop_dir * args.steps / (k["ms_total"] * 1e-3) / 1e12
            k["gbs_matrix"] = bytes_dir * args.steps / (k["ms_total"] * 1e-3) / 1e9
    dom = max(("apply_inverse", "apply_forward"), key=lambda n: kern[n]["ms_total"])
    ach = kern[dom].get("tflops", 0.0)
    roof = {"bound": "mfma", "kernel": dom, "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / PEAK_FP64_TFLOPS, "traffic": None}

    # sampled check of the inverse against the oracle on a few rings
    from oracle import sht as osht
    from tests.gpu_util import oracle_plan
    rings = [0, 1, L // 2, L - 1]
    ref = osht.inverse_rings(oracle_plan(L), flm_h[:2], rings)
    f_h = f.cpu().numpy()
    inv_err = 0.0
    for k, v in ref.items():
        got = f_h[:2, k * k:k * k + 2 * k + 1]
        inv_err = max(inv_err, float(np.max(np.abs(got - v)) / np.max(np.abs(v))))

    out = {
        "metric": "fwd+inv SHT/s at L=1024, batch 16 (mixed vs FP64, max rel err); HBM GB/s",
        "value": B * args.steps / dt,
        "unit": "SHT/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"spin-0 forward+inverse SHT, L={L}, batch {B}, flm N(0,1)(1+l)^-1 seed 5",
                   "L": L, "batch": B, "spin": 0, "path": "fp64", "parallelism": "single-gpu"},
        "max_rel_err_roundtrip": rt_err,
        "max_rel_err_inverse_vs_oracle_sampled_rings": inv_err,
        "roofline": roof,
        "kernels": kern,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(L)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

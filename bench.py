"""Throughput benchmark of the fused D2Q8 porous MRT-LB step on one MI355X.

Default workload: the 8192 x 8192 log-normal porous channel (x periodic, walls in
y, per-cell porosity plane with Ergun permeability and F_phi), FP32 deviation
storage, forward stepping. Prints one JSON line with MLUPS, the HBM roofline of
the step kernel and the FP64 CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps 2000] [--warmup 500]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_steps(solver, steps, warmup):
    import torch
    solver.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    solver.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms per step


def cpu_baseline(n=1024, steps=120):
    """FP64 oracle on the same workload recipe at n x n (bounded sample)."""
    import numpy as np
    import oracle
    from paper_1311_7239_amd import inputs as I

    case = I.lognormal_channel(n=n, seed=5, K_ref=1e-6 * 2048.0 ** 2)
    threads = min(os.cpu_count() or 1, 16)
    p = oracle.make_params(case.nx, case.ny, bc_x=case.bc_x, bc_y=case.bc_y, nu=case.nu,
                           ax=case.ax, nthreads=threads)
    phi = case.phi.astype(np.float64)
    K, F = oracle.ergun(phi, case.dp)
    f = oracle.rest_state(p, case.Pi0)
    oracle.run(p, phi, K, F, f, nsteps=2)
    t0 = time.perf_counter()
    oracle.run(p, phi, K, F, f, nsteps=steps)
    dt = time.perf_counter() - t0
    return {"value": round(case.nodes * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{n}x{n} log-normal porous channel (same recipe), {steps} FP64 steps, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", action="store_true", help="also time the other workloads")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design note, not part of this build)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1311_7239_amd import inputs as I
    from paper_1311_7239_amd import lbm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)          # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
    n = args.n
    log(f"bench: generating {n}x{n} log-normal porosity field")
    case = I.lognormal_channel(n=n, seed=5, K_ref=1e-6 * 2048.0 ** 2)
    solver = lbm.solver_for_case(case, storage=lbm.FP32_DEV)
    log(f"bench: stepping ({args.warmup} warmup + {args.steps} timed)")
    ms = time_steps(solver, args.steps, args.warmup)
    mlups = case.nodes / (ms * 1e-3) / 1e6
    bytes_per_node = 68  # 8 FP32 loads + 8 FP32 stores + 1 FP32 porosity load
    achieved = case.nodes * bytes_per_node / (ms * 1e-3) / 1e9
    mass, res, st = solver.reduce()
    out = {
        "metric": "MLUPS & % of HBM roofline per collide-stream step; adjoint/forward time ratio",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"log-normal porous channel {n}x{n}: x periodic, walls in y, "
                               "per-cell porosity (sigma 0.5, correlation 64) with Ergun K and "
                               "F_phi, tau 0.8, FP32 deviation storage, forward steps",
                   "nodes": case.nodes, "schedule": list(solver.schedule())},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None},
        "mass_check": {"mass": mass, "residual": res},
    }
    del solver
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Throughput benchmark of the fused D2Q8 porous MRT-LB step on one MI355X.

Headline workload: the 8192 x 8192 log-normal porous channel (x periodic, walls
in y, per-cell porosity plane with Ergun permeability and F_phi, tau = 0.8),
FP32 deviation storage, forward stepping. One JSON line reports MLUPS, the HBM
roofline of the step kernel, the FP64 CPU oracle timed on a bounded sample, and
(under "extras") the other workloads: FP16-deviation storage, the 512^2 porous
lid cavity, the 1024^2 natural-convection cavity, the ragged batch of 256
cavities (FP32 and FP16) and the adjoint/forward time ratio of the 2048^2
inverse problem.

    python bench.py [--gpus 1] [--steps 2000] [--warmup 500] [--no-extras]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0     # MI355X HBM3E, published
METRIC = "MLUPS & % of HBM roofline per collide-stream step; adjoint/forward time ratio"
COUNTERS = os.path.join(ROOT, "profiles", "counters_step_lognormal8192_f32.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed(stepper, steps, warmup):
    """Average ms per step over `steps` steps on the current stream (HIP events),
    after `warmup` untimed steps."""
    import torch
    stepper.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    stepper.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def per_launch_ms(stepper, cycles, launches=20, reps=3):
    """Average duration of one plain multi-cycle launch, from HIP events on the launch
    stream: a call of (launches + 1) passes minus a call of one pass. Every lbm_step call
    ends with one pass that also writes u(t - 1) for the residual; the difference cancels
    it, leaving `launches` back-to-back plain launches of the dominant kernel."""
    import torch
    stream = torch.cuda.current_stream()

    def call(n):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        stepper.step(n)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    call(cycles)
    long = min(call(cycles * (launches + 1)) for _ in range(reps))
    short = min(call(cycles) for _ in range(reps))
    return (long - short) / launches


def roofline(nodes, bytes_per_node, ms):
    achieved = nodes * bytes_per_node / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4)}


def host_cpu():
    """(logical CPUs this process may run on, os.cpu_count(), CPU model name)."""
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return usable, os.cpu_count() or 1, model


def cpu_baseline(n=1024, steps=1000, n1=512, steps1=100):
    """FP64 oracle on the same workload recipe (bounded samples): with every thread this
    process is given (OMP_NUM_THREADS when set, the GPU's share of the host, else every
    usable CPU) on n x n for `steps` steps, and with one thread on n1 x n1."""
    import numpy as np
    import oracle
    from paper_1311_7239_amd import inputs as I

    usable, count, model = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS") or usable)

    def rate(size, nsteps, nthreads):
        case = I.lognormal_channel(n=size, seed=5, K_ref=1e-6 * 2048.0 ** 2)
        p = oracle.make_params(case.nx, case.ny, bc_x=case.bc_x, bc_y=case.bc_y, nu=case.nu,
                               ax=case.ax, nthreads=nthreads)
        phi = case.phi.astype(np.float64)
        K, F = oracle.ergun(phi, case.dp)
        f = oracle.rest_state(p, case.Pi0)
        oracle.run(p, phi, K, F, f, nsteps=2)
        t0 = time.perf_counter()
        oracle.run(p, phi, K, F, f, nsteps=nsteps)
        dt = time.perf_counter() - t0
        return case.nodes * nsteps / dt / 1e6, dt

    v, dt = rate(n, steps, threads)
    v1, dt1 = rate(n1, steps1, 1)
    return {"value": round(v, 2), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{n}x{n} log-normal porous channel (same recipe), {steps} FP64 steps on {threads} "
                      f"threads, {dt:.1f} s; {n1}x{n1}, {steps1} steps on 1 thread, {dt1:.1f} s",
            "value_1_thread": round(v1, 2), "usable_cpus": usable, "os_cpu_count": count, "cpu_model": model}


def extras(args):
    import torch
    from paper_1311_7239_amd import inputs as I
    from paper_1311_7239_amd import lbm

    out = {}
    n = args.n
    # reference: the runtime's own device-to-device copy of 2 GiB (read + write)
    src = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(10):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    ms = c0.elapsed_time(c1) / 10
    out["copy_reference"] = {"gbs": round(2 * src.numel() * 4 / (ms * 1e-3) / 1e9, 1),
                             "what": "device-to-device copy of 2 GiB (runtime copy kernel), read + write"}
    del src, dst
    torch.cuda.empty_cache()
    # one cycle per pass on the headline workload (the HBM-bound single-step kernel)
    case = I.lognormal_channel(n=n, seed=5, K_ref=1e-6 * 2048.0 ** 2)
    s = lbm.solver_for_case(case, storage=lbm.FP32_DEV)
    s.set_time_blocking(1)
    ms = timed(s, args.steps, args.warmup)
    out["one_cycle_per_pass_f32"] = {"mlups": round(case.nodes / ms / 1e3, 1), "ms_per_step": round(ms, 4),
                                     "bytes_per_node": 68, "kernel": "k_step<float, 128x1x2>",
                                     "roofline": roofline(case.nodes, 68, ms)}
    s.set_time_blocking(2)
    ms = timed(s, args.steps, args.warmup)
    out["two_cycles_per_pass_f32"] = {"mlups": round(case.nodes / ms / 1e3, 1), "ms_per_step": round(ms, 4),
                                      "bytes_per_node_per_launch": 68, "kernel": "k_step2<float, 64, 16>",
                                      "roofline": roofline(case.nodes, 68, 2 * ms)}
    s.set_time_blocking(3)
    launch3 = per_launch_ms(s, 3)
    ms = timed(s, args.steps, args.warmup)
    out["three_cycles_per_pass_f32"] = {"mlups": round(case.nodes / ms / 1e3, 1), "ms_per_step": round(ms, 4),
                                        "bytes_per_node_per_launch": 68, "launch_ms": round(launch3, 4),
                                        "kernel": "k_step3<float, 64, 28> (768 threads)",
                                        "roofline": roofline(case.nodes, 68, launch3)}
    # the FP64 reductions (mass and steady residual: the state gathered, 36 B/node, and the
    # recorded u(t - 1), 8 B/node) and the macroscopic output (36 B/node read, p and u
    # written: 48 B/node) on that state
    s.reduce()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        s.reduce()
    red_ms = (time.perf_counter() - t0) * 1e3 / 10
    s.macroscopic()
    m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    m0.record()
    for _ in range(10):
        s.macroscopic()
    m1.record()
    torch.cuda.synchronize()
    mac_ms = m0.elapsed_time(m1) / 10
    out["reduce_f32"] = {"ms": round(red_ms, 4), "bytes_per_node": 44,
                         "roofline": roofline(case.nodes, 44, red_ms),
                         "note": "lbm_reduce call incl. the copy of three doubles to the host"}
    out["macroscopic_f32"] = {"ms": round(mac_ms, 4), "bytes_per_node": 48,
                              "roofline": roofline(case.nodes, 48, mac_ms)}
    del s
    torch.cuda.empty_cache()
    # FP16-deviation storage on the headline workload (its default cycles per pass)
    s = lbm.solver_for_case(case, storage=lbm.FP16_DEV)
    s.set_schedule(64, 2, 2, 1)
    tb = s.time_blocking()
    # the launch timing first, as for the headline: it also brings the clocks up
    launch16 = per_launch_ms(s, tb["cycles_per_pass"])
    ms = timed(s, args.steps, args.warmup)
    out["fp16_lognormal_channel"] = {"mlups": round(case.nodes / ms / 1e3, 1), "ms_per_step": round(ms, 4),
                                     "bytes_per_node_per_launch": 36, "time_blocking": tb,
                                     "launch_ms": round(launch16, 4),
                                     "roofline": roofline(case.nodes, 36, launch16)}
    del s
    torch.cuda.empty_cache()
    log("bench: 512^2 porous lid cavity")
    case = I.lid_cavity(n=512)
    s = lbm.solver_for_case(case)
    s.set_graph_steps(64)
    ms = timed(s, 20000, 2000)
    out["cavity512"] = {"mlups": round(case.nodes / ms / 1e3, 1), "ms_per_step": round(ms, 5),
                        "bytes_per_node_per_launch": 64, "time_blocking": s.time_blocking(),
                        "note": "working set 34 MB, below the 256 MB Infinity Cache"}
    del s
    log("bench: 1024^2 natural convection (D2Q8 + D2Q5)")
    case = I.natural_convection(n=1024)
    s = lbm.solver_for_case(case)
    s.set_graph_steps(64)
    ms = timed(s, 4000, 500)
    tb = s.time_blocking()
    out["convection1024"] = {"mlups": round(case.nodes / ms / 1e3, 1), "ms_per_step": round(ms, 5),
                             "bytes_per_node_per_launch": 104, "time_blocking": tb,
                             "roofline": roofline(case.nodes, 104, ms * tb["cycles_per_pass"]),
                             "note": "working set 113 MB, below the 256 MB Infinity Cache"}
    del s
    torch.cuda.empty_cache()
    log("bench: 1024^2 natural convection to a steady Nusselt number")
    from paper_1311_7239_amd import convection as C
    r = C.steady_nusselt(I.natural_convection(n=1024), max_seconds=20.0)
    out["convection1024_nusselt"] = {
        "nu": round(r["nu"], 5), "steps": r["steps"], "converged": r["converged"],
        "last_change_per_20000_steps": float(f"{r['last_change']:.3g}"), "nu_aitken": round(r["nu_aitken"], 5),
        "seconds": round(r["seconds"], 1), "table1": 1.068, "rel_to_table1": round(r["nu_aitken"] / 1.068 - 1.0, 5),
        "note": "hot-wall Nu stepped from the conduction profile for up to 20 s (phi 0.6, Da 1e-4, Ra 1e5); "
                "nu_aitken: delta-squared limit of the last three readings; Table 1 gives 1.068 on a 200^2 grid"}
    torch.cuda.empty_cache()
    log("bench: Table 1 sweep as one thermal batch (27 natural-convection cavities)")
    cases = [c for _, c in C.table1_cases()]
    b = lbm.batch_for_cases(cases)
    ms = timed(b, 20000, 2000)
    out["table1_batch27_thermal"] = {"mlups": round(b.nodes / ms / 1e3, 1), "ms_per_step": round(ms, 5),
                                     "nodes": b.nodes, "bytes_per_node_per_launch": 104,
                                     "schedule": list(b.schedule()), "time_blocking": b.time_blocking(),
                                     "note": "120^2, 200^2, 250^2 cavities of Sec. 3.4; D2Q8 + D2Q5"}
    del b
    torch.cuda.empty_cache()
    for storage, name, bpn in ((lbm.FP32_DEV, "batch256_f32", 64), (lbm.FP16_DEV, "batch256_f16", 32)):
        log(f"bench: ragged batch of 256 lid cavities ({name})")
        cases = I.cavity_batch()
        # MRTLBM_TUNE_CACHE: optional autotuner cache file (tuned afresh without it)
        b = lbm.batch_for_cases(cases, storage=storage, tune_cache=os.environ.get("MRTLBM_TUNE_CACHE"))
        ms = timed(b, args.steps, args.warmup)
        tb = b.time_blocking()
        per_launch = ms * tb["cycles_per_pass"]
        out[name] = {"mlups": round(b.nodes / ms / 1e3, 1), "ms_per_step": round(ms, 4), "nodes": b.nodes,
                     "bytes_per_node_per_launch": bpn, "schedule": list(b.schedule()), "time_blocking": tb,
                     "roofline": roofline(b.nodes, bpn, per_launch)}
        del b
        torch.cuda.empty_cache()
    out["adjoint2048"] = adjoint_ratio()
    return out


def adjoint_ratio():
    """Backward (recomputation from checkpoints + adjoint steps) over plain forward time on
    the 2048^2 inverse problem: 4000 steps, a checkpoint every 200."""
    import torch
    from paper_1311_7239_amd import inputs as I
    from paper_1311_7239_amd import lbm

    log("bench: adjoint of the 2048^2 inverse problem (4000 steps, checkpoint every 200)")
    case = I.lognormal_channel(n=2048, seed=5)
    s = lbm.solver_for_case(case, ckpt_every=200, max_steps_recorded=4000)
    f = lbm.solver_for_case(case)
    f.step(10)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
    e[0].record()
    f.step(4000)
    e[1].record()
    # the same forward in four cycles per pass, which the recomputation does not use
    mode0 = f.time_blocking()["cycles_per_pass"]
    f.set_time_blocking(4)
    e[6].record()
    f.step(4000)
    e[7].record()
    e[4].record()
    s.step(4000)
    e[5].record()
    _, u, _ = s.macroscopic()
    dLdu = torch.zeros_like(u)
    dLdu[:, :, -1] = u[:, :, -1]
    torch.cuda.synchronize()
    e[2].record()
    s.backward(dLdu)
    e[3].record()
    torch.cuda.synchronize()
    fwd = e[0].elapsed_time(e[1])
    bwd = e[2].elapsed_time(e[3])
    fwd4 = e[6].elapsed_time(e[7])
    return {"forward_ms": round(fwd, 2), "recorded_forward_ms": round(e[4].elapsed_time(e[5]), 2),
            "backward_ms": round(bwd, 2), "adjoint_forward_ratio": round(bwd / fwd, 3),
            "forward_cycles_per_pass": mode0,
            "forward_four_cycles_ms": round(fwd4, 2), "adjoint_forward_ratio_four_cycles": round(bwd / fwd4, 3),
            "note": "backward = recomputation from checkpoints (four cycles per pass, recording u) + "
                    "adjoint steps (three per pass); forward_ms in the default mode at this size "
                    f"({mode0} cycles per pass), forward_four_cycles_ms the same forward in four; the "
                    "recorded forward also copies a checkpoint every 200 steps"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for HBM counters)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the adjoint/forward time ratio of the 2048^2 inverse problem")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs one domain or batch per GPU; the multi-GPU decomposition is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1311_7239_amd import inputs as I
    from paper_1311_7239_amd import lbm
    from paper_1311_7239_amd import profiling

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.adjoint_only:
        print(json.dumps({"adjoint2048": adjoint_ratio()}), flush=True)
        return
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)          # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
    n = args.n
    log(f"bench: generating the {n}x{n} log-normal porosity field")
    case = I.lognormal_channel(n=n, seed=5, K_ref=1e-6 * 2048.0 ** 2)
    solver = lbm.solver_for_case(case, storage=lbm.FP32_DEV)   # the default cycles per HBM pass
    cycles = solver.time_blocking()["cycles_per_pass"]
    # The dominant kernel's own launch duration (HIP events around back-to-back launches),
    # measured first: its ~130 launches also bring the GPU out of the clock state it idles
    # in while the host builds the porosity field (right after that, launches run up to
    # 25% slower for the first ~20 ms, longer than a short timed region)
    launch_ms = per_launch_ms(solver, cycles)
    log(f"bench: stepping ({args.warmup} warmup + {args.steps} timed, {cycles} cycles per pass)")
    ms = timed(solver, args.steps, args.warmup)
    mlups = case.nodes / (ms * 1e-3) / 1e6
    bytes_per_node = 68  # per pass: 8 FP32 loads + 8 FP32 stores + the FP32 porosity load
    rl = roofline(case.nodes, bytes_per_node, launch_ms)
    tb = solver.time_blocking()
    shape = f"64 x {tb['rows']} tiles, {tb['threads']} threads"
    kname = {4: ("void mrt::k_step4<float", f"k_step4<float> ({shape}): four collide-stream cycles per launch"),
             3: ("void mrt::k_step3<float", f"k_step3<float> ({shape}): three collide-stream cycles per launch"),
             2: ("void mrt::k_step2<float", f"k_step2<float> ({shape}): two collide-stream cycles per launch"),
             1: ("void mrt::k_step<float, false, 0", "k_step<float>: one collide-stream cycle per launch")}[cycles]
    traffic = profiling.traffic_bytes(COUNTERS, kname[0]) if n == 8192 else None
    rl["traffic"] = None if traffic is None else round(traffic / 1e9, 4)
    rl["traffic_unit"] = "GB per launch"
    rl["kernel"] = kname[1]
    rl["algorithmic_bytes_per_launch"] = case.nodes * bytes_per_node
    rl["launch_ms"] = round(launch_ms, 4)
    rl["launch_timing"] = ("HIP events on the launch stream: 21-pass call minus 1-pass call, 20 back-to-back "
                           "launches, best of 3")
    # the whole timed call (every pass, the last one writing u(t - 1), and launch gaps)
    rl["effective_gbs"] = round(case.nodes * bytes_per_node / (cycles * ms * 1e-3) / 1e9, 1)
    rl["one_cycle_equivalent_gbs"] = round(case.nodes * bytes_per_node / (ms * 1e-3) / 1e9, 1)
    mass, res, _ = solver.reduce()
    out = {
        "metric": METRIC,
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
        "config": {"time_blocking": solver.time_blocking(),
                   "workload": f"log-normal porous channel {n}x{n}: x periodic, walls in y, per-cell "
                               "porosity (log-normal, sigma 0.5, correlation 64, seed 5) with Ergun K and "
                               f"F_phi, tau 0.8, FP32 deviation storage, forward steps, {cycles} cycles per "
                               "HBM pass",
                   "nodes": case.nodes, "schedule": list(solver.schedule())},
        "roofline": rl,
        "state_check": {"mass": mass, "residual": res},
    }
    del solver
    torch.cuda.empty_cache()
    if not args.no_extras:
        out["extras"] = extras(args)
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

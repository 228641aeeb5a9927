"""Natural convection in a porous square cavity (Sec. 3.4) as batched thermal
workloads: the Table 1 sweep over (Da, Ra, phi) stepped as one ragged batch.

The stepping runs in the library (lbm_create_batch with thermal domains);
this module builds the seeded cases, starts every domain from the
conduction profile, steps in chunks and reads the hot-wall Nusselt number
from the temperature field after each chunk.
"""
from __future__ import annotations

import time
from typing import Callable, Dict, Iterable, List, Optional, Tuple

import numpy as np
import torch

from . import inputs as I
from . import lbm

# Grid per Darcy number (Sec. 3.4) and the (Da, Ra) pairs of Table 1.
TABLE1_GRID = {1e-2: 120, 1e-4: 200, 1e-6: 250}
TABLE1_PAIRS = [(1e-2, 1e3), (1e-2, 1e4), (1e-2, 1e5),
                (1e-4, 1e5), (1e-4, 1e6), (1e-4, 1e7),
                (1e-6, 1e7), (1e-6, 1e8), (1e-6, 1e9)]
TABLE1_PHIS = (0.4, 0.6, 0.9)


def table1_cases(pairs: Iterable[Tuple[float, float]] = TABLE1_PAIRS,
                 phis: Iterable[float] = TABLE1_PHIS, nee: bool = False,
                 grid: Optional[Dict[float, int]] = None, Ma: float = 0.1) -> List[Tuple[tuple, I.Case]]:
    """((Da, Ra, phi), Case) for every combination, Pr = 1, Ma = 0.1 (unless given),
    J = sigma = gamma = 1, Th = 21, Tc = 1 (Sec. 3.4), on the paper's grid per Da."""
    grid = TABLE1_GRID if grid is None else grid
    out = []
    for Da, Ra in pairs:
        for phi in phis:
            c = I.natural_convection(n=grid[Da], phi=phi, Da=Da, Ra=Ra, nee=nee, Ma=Ma)
            out.append(((Da, Ra, phi), c))
    return out


# Resolution and Mach-number variants of the Da = 1e-6 row at Ra = 1e8 and 1e9:
# (label, grid, Ma); the first is the paper's grid at Ma = 0.1, the value taken where Sec. 3.4
# leaves the Mach number open.
DA6_VARIANTS = [("250 Ma0.1", 250, 0.1), ("500 Ma0.1", 500, 0.1), ("250 Ma0.05", 250, 0.05),
                ("250 Ma0.2", 250, 0.2)]


def da6_study_cases(variants=DA6_VARIANTS, ras=(1e8, 1e9), phis=TABLE1_PHIS,
                    nee: bool = False) -> List[Tuple[tuple, I.Case]]:
    """((label, Ra, phi), Case) of the Da = 1e-6 cases under each (grid, Ma) variant."""
    out = []
    for label, n, Ma in variants:
        for Ra in ras:
            for phi in phis:
                out.append(((label, Ra, phi), I.natural_convection(n=n, phi=phi, Da=1e-6, Ra=Ra, Ma=Ma, nee=nee)))
    return out


def conduction_state(case: I.Case) -> np.ndarray:
    """Thermal deviations dg [5, ny, nx] of the pure-conduction profile between
    the hot (x = 0) and cold (x = L) walls, every link at T/5 (varpi = 0)."""
    if case.bc_x == I.NEE:
        x = np.arange(case.nx, dtype=np.float64)
        L = case.nx - 1.0
    else:
        x = np.arange(case.nx, dtype=np.float64) + 0.5
        L = float(case.nx)
    T = case.Th + (case.Tc - case.Th) * x / L
    return np.broadcast_to(((T - case.T0) / 5.0)[None, None, :],
                           (5, case.ny, case.nx)).astype(np.float32).copy()


def nusselt_hot_wall(T: np.ndarray, case: I.Case) -> float:
    """Average Nusselt number of the hot wall x = 0: -(L / dT) times the wall-mean
    of dT/dx there. Bounce-back walls (wall half a node before the first node):
    the quadratic through the wall value and the first two nodes,
    dT/dx = (9 T_1/2 - T_3/2 - 8 T_w) / 3, mean over the rows, L = n.
    On-node walls: the one-sided second-order difference (-3 T_0 + 4 T_1 - T_2)/2,
    trapezoidal mean along the wall, L = n - 1."""
    dT = case.Th - case.Tc
    if case.bc_x == I.NEE:
        g = (-3.0 * case.Th + 4.0 * T[:, 1] - T[:, 2]) / 2.0
        w = np.ones(T.shape[0]); w[0] = w[-1] = 0.5
        mean = float(np.sum(w * g) / np.sum(w))
        return -mean * (case.nx - 1.0) / dT
    g = (9.0 * T[:, 0] - T[:, 1] - 8.0 * case.Th) / 3.0
    return -float(np.mean(g)) * case.nx / dT


def run_sweep(keyed_cases: List[Tuple[tuple, I.Case]], chunk: int = 4000, tol: float = 1e-6,
              max_steps: int = 2_000_000, time_limit: Optional[float] = None,
              storage: int = lbm.FP32_DEV, log: Optional[Callable[[str], None]] = None,
              device="cuda", history: Optional[Dict[tuple, list]] = None) -> Dict[tuple, dict]:
    """Steps all cases as one thermal batch from the conduction profile until every
    Nusselt number changes by less than tol over a chunk (or max_steps / the time
    limit is reached). Returns {key: {"nu", "steps", "converged", "diverged"}}: a case whose
    Nusselt number stops being finite is stopped and reported as diverged, not converged."""
    cases = [c for _, c in keyed_cases]
    b = lbm.batch_for_cases(cases, storage=storage, device=device)
    for k, c in enumerate(cases):
        b.set_populations(k, torch.zeros((8, c.ny, c.nx), device=device),
                          torch.from_numpy(conduction_state(c)).to(device))
    prev = [None] * len(cases)
    done = [False] * len(cases)
    diverged = [False] * len(cases)
    nu = [float("nan")] * len(cases)
    when = [0] * len(cases)
    t0 = time.time()
    steps = 0
    while steps < max_steps:
        b.step(chunk)
        steps += chunk
        for k, c in enumerate(cases):
            if done[k]:
                continue
            _, _, T = b.macroscopic(k, want_T=True)
            nu[k] = nusselt_hot_wall(T.cpu().numpy().astype(np.float64), c)
            if history is not None:
                history.setdefault(keyed_cases[k][0], []).append((steps, nu[k]))
            if not np.isfinite(nu[k]):
                done[k] = diverged[k] = True
                when[k] = steps
            elif prev[k] is not None and abs(nu[k] - prev[k]) < tol:
                done[k] = True
                when[k] = steps
            prev[k] = nu[k]
        if log is not None:
            log(f"t={steps} converged {sum(done)}/{len(cases)} elapsed {time.time() - t0:.1f}s")
        if all(done) or (time_limit is not None and time.time() - t0 > time_limit):
            break
    return {key: {"nu": nu[k], "steps": when[k] if done[k] else steps,
                  "converged": bool(done[k] and not diverged[k]), "diverged": diverged[k]}
            for k, (key, _) in enumerate(keyed_cases)}


def steady_nusselt(case: I.Case, chunk: int = 20_000, tol: float = 1e-6, max_steps: int = 4_000_000,
                   max_seconds: Optional[float] = None, storage: int = lbm.FP32_DEV, device="cuda") -> dict:
    """One cavity stepped alone (its default cycles per pass) from the conduction profile
    until the hot-wall Nusselt number changes by less than tol over a chunk (or max_steps
    / max_seconds). Returns {"nu", "steps", "converged", "diverged", "seconds",
    "last_change", "nu_aitken"}: the last change per chunk, and Aitken's delta-squared
    estimate of the limit from the last three values (the slowest thermal mode decays
    geometrically once the faster ones have gone)."""
    s = lbm.solver_for_case(case, storage=storage, device=device)
    s.set_populations(torch.zeros((8, case.ny, case.nx), device=device),
                      torch.from_numpy(conduction_state(case)).to(device))
    vals, steps = [], 0
    t0 = time.time()
    converged = diverged = False
    while steps < max_steps:
        s.step(chunk)
        steps += chunk
        _, _, T = s.macroscopic(want_T=True)
        vals.append(nusselt_hot_wall(T.cpu().numpy().astype(np.float64), case))
        if not np.isfinite(vals[-1]):
            diverged = True
            break
        if len(vals) > 1 and abs(vals[-1] - vals[-2]) < tol:
            converged = True
            break
        if max_seconds is not None and time.time() - t0 > max_seconds:
            break
    nu = vals[-1] if vals else float("nan")
    last = abs(vals[-1] - vals[-2]) if len(vals) > 1 else float("nan")
    aitken = nu
    if len(vals) > 2:
        d1, d2 = vals[-2] - vals[-3], vals[-1] - vals[-2]
        if d2 != d1 and abs(d2) < abs(d1):
            aitken = vals[-1] - d2 * d2 / (d2 - d1)
    return {"nu": nu, "steps": steps, "converged": converged, "diverged": diverged,
            "seconds": time.time() - t0, "last_change": last, "nu_aitken": aitken}


def _main(argv=None):
    """Runs the Table 1 sweep and prints the hot-wall Nusselt number of every case."""
    import argparse
    ap = argparse.ArgumentParser(description=_main.__doc__)
    ap.add_argument("--walls", choices=["bounce-back", "on-node"], default="bounce-back")
    ap.add_argument("--max-steps", type=int, default=3_000_000)
    ap.add_argument("--chunk", type=int, default=5000)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--time-limit", type=float, default=None)
    ap.add_argument("--steady", type=int, default=0, metavar="N",
                    help="only the Sec. 3.4 cavity (phi 0.6, Da 1e-4, Ra 1e5) on an N^2 grid to a steady Nu")
    ap.add_argument("--da6-study", action="store_true",
                    help="the Da = 1e-6, Ra = 1e8 / 1e9 cases on 250^2 and 500^2 grids and at Ma 0.05, 0.1, 0.2")
    a = ap.parse_args(argv)
    if a.steady:
        r = steady_nusselt(I.natural_convection(n=a.steady), chunk=a.chunk, tol=a.tol, max_steps=a.max_steps,
                           max_seconds=a.time_limit)
        print(f"{a.steady}^2: Nu {r['nu']:.6f} after {r['steps']} steps ({r['seconds']:.1f} s), last change "
              f"{r['last_change']:.2e} per {a.chunk} steps, converged {int(r['converged'])}, "
              f"Aitken limit {r['nu_aitken']:.6f}", flush=True)
        return
    if a.da6_study:
        keyed = da6_study_cases(nee=a.walls == "on-node")
        hist: Dict[tuple, list] = {}
        res = run_sweep(keyed, chunk=a.chunk, tol=a.tol, max_steps=a.max_steps, time_limit=a.time_limit,
                        log=lambda m: print(m, flush=True), history=hist)
        print("variant Ra phi Nu steps converged diverged | Nu at 1/4, 1/2, 3/4 of its steps")
        for key, r in res.items():
            h = hist.get(key, [])
            marks = [h[max(0, int(len(h) * q) - 1)][1] for q in (0.25, 0.5, 0.75)] if h else []
            label, Ra, phi = key
            print(f"{label} {Ra:g} {phi} {r['nu']:.4f} {r['steps']} {int(r['converged'])} {int(r['diverged'])} | "
                  + " ".join(f"{m:.4f}" for m in marks))
        return
    keyed = table1_cases(nee=a.walls == "on-node")
    res = run_sweep(keyed, chunk=a.chunk, tol=a.tol, max_steps=a.max_steps, time_limit=a.time_limit,
                    log=lambda m: print(m, flush=True))
    print("Da Ra phi Nu steps converged diverged")
    for (Da, Ra, phi), r in res.items():
        print(f"{Da:g} {Ra:g} {phi} {r['nu']:.4f} {r['steps']} {int(r['converged'])} {int(r['diverged'])}")


if __name__ == "__main__":
    _main()

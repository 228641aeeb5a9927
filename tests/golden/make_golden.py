"""Writes the stored oracle results used by the full-size GPU parity tests.

Runs only the FP64 oracle (oracle/) on the seeded inputs of
paper_1311_7239_amd.inputs and stores, per workload, the velocity at a seeded
sample of nodes plus field-wide maxima, so that a GPU run at full size can be
compared element by element on those nodes without running the oracle there.

    python tests/golden/make_golden.py [name ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1311_7239_amd import inputs as I  # noqa: E402
from tests.oracle_cases import oracle_setup  # noqa: E402


def sample_nodes(nx, ny, count, seed):
    rng = np.random.default_rng(seed)
    xs = rng.integers(0, nx, size=count)
    ys = rng.integers(0, ny, size=count)
    # the walls' neighbours and the lid row are where boundary mistakes show
    edge = [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1), (nx // 2, ny - 1), (nx // 2, 0),
            (0, ny // 2), (nx - 1, ny // 2)]
    pts = list(zip(xs.tolist(), ys.tolist())) + edge
    return sorted(set(pts), key=lambda p: (p[1], p[0]))


def run_case(name, case, steps, thermal_init_T=None):
    t0 = time.time()
    p, phi, K, F = oracle_setup(case, nthreads=os.cpu_count() or 8)
    f = oracle.rest_state(p, case.Pi0)
    g = None
    if case.thermal:
        T = np.full((case.ny, case.nx), case.T0) if thermal_init_T is None else thermal_init_T
        g = oracle.thermal_rest_state(p, T)
    oracle.run(p, phi, K, F, f, g, nsteps=steps)
    ux, uy, pr, T = oracle.macroscopic(p, phi, K, F, f, g)
    pts = sample_nodes(case.nx, case.ny, 512, seed=1234)
    path = os.path.join(HERE, f"{name}.txt")
    with open(path, "w") as fh:
        fh.write(f"# FP64 oracle, {name}: {case.nx}x{case.ny}, {steps} steps from rest\n")
        fh.write("# written by tests/golden/make_golden.py (oracle only)\n")
        fh.write(f"# max_abs_u {max(np.abs(ux).max(), np.abs(uy).max()):.17e}\n")
        fh.write(f"# mass {oracle.mass(f):.17e}\n")
        fh.write("# x y ux uy p" + (" T" if case.thermal else "") + "\n")
        for x, y in pts:
            row = f"{x} {y} {ux[y, x]:.17e} {uy[y, x]:.17e} {pr[y, x]:.17e}"
            if case.thermal:
                row += f" {T[y, x]:.17e}"
            fh.write(row + "\n")
    print(f"{name}: {time.time() - t0:.1f} s", flush=True)


def main(names):
    jobs = {
        "cavity512_uniform_50k": lambda: run_case("cavity512_uniform_50k", I.lid_cavity(n=512), 50_000),
        "cavity512_grf_50k": lambda: run_case("cavity512_grf_50k", I.lid_cavity(n=512, heterogeneous=True),
                                              50_000),
        "convection1024_2k": lambda: run_case("convection1024_2k", I.natural_convection(n=1024), 2000),
    }
    for n in names or list(jobs):
        jobs[n]()


if __name__ == "__main__":
    main(sys.argv[1:])

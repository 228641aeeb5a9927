"""A domain whose state buffer is above 4 GiB: the 12288^2 log-normal porous channel in
FP32 (4.8 GB per population buffer, two buffers). The multi-cycle kernels address a
buffer with 32-bit offsets, so such a domain stays on the one-cycle kernel, which
addresses with 64 bits; the population planes above plane 7's first 1400 rows lie
beyond byte 2^32 of their buffer. Sampled nodes (walls, the periodic seam, random
interior nodes) agree with the FP64 oracle run on windows around them, and the FP64
mass reduction equals its definition on the initial state and is conserved."""
import numpy as np
import pytest
import torch

import oracle
from paper_1311_7239_amd import inputs as I
from paper_1311_7239_amd import lbm
from tests.gpu_cases import f_ref, oracle_window
from tests.oracle_cases import oracle_setup

pytestmark = pytest.mark.gpu

N = 12288
CHUNKS = (1, 2)            # the collide-only first cycle, then two gather cycles
T = sum(CHUNKS)
STEP_TOL = 8 * 2.0 ** -24 * 8


def test_state_above_4gib_matches_oracle_on_sampled_nodes():
    assert 8 * 4 * N * N > 2 ** 32
    case = I.lognormal_channel(n=N, seed=7, K_ref=1e-6 * 2048.0 ** 2)
    df0 = I.random_deviation_state(N, N, 1e-3, seed=37)
    s = lbm.solver_for_case(case)
    assert s.time_blocking()["cycles_per_pass"] == 1
    with pytest.raises(lbm.LBMError) as ei:
        s.set_time_blocking(2)
    assert ei.value.status == lbm.ENOTSUP
    s.set_populations(torch.from_numpy(df0).cuda())
    mass0, _, _ = s.reduce()
    ref0 = float(np.sum(df0, dtype=np.float64)) + N * N * float(np.sum(f_ref(case.Pi0)))
    assert abs(mass0 - ref0) / ref0 < 1e-11
    for n in CHUNKS:
        s.step(n)
    mass, _, _ = s.reduce()
    assert abs(mass - mass0) / mass0 < 1e-7
    df, _ = s.populations()
    _, u, _ = s.macroscopic()
    torch.cuda.synchronize()

    rng = np.random.default_rng(43)
    xs = list(rng.integers(0, N, 10)) + [0, N - 1, 7, N - 2, 6000, 77]
    ys = list(rng.integers(0, N, 10)) + [0, N - 1, N - 2, 1, 12000, 12286]
    worst_f = worst_u = 0.0
    for x, y in zip(xs, ys):
        x, y = int(x), int(y)
        sub, dfw, cx, cy = oracle_window(case, df0, x, y, T + 1)
        p, phi, K, F = oracle_setup(sub, nthreads=8)
        f = np.ascontiguousarray(np.transpose(dfw, (1, 2, 0)) + f_ref(case.Pi0))
        oracle.run(p, phi, K, F, f, nsteps=T)
        ref = f[cy, cx] - f_ref(case.Pi0)
        got = df[:, y, x].cpu().numpy().astype(np.float64)
        err_f = np.abs(got - ref).max() / np.abs(ref).max()
        ux, uy, _, _ = oracle.macroscopic(p, phi, K, F, f)
        uref = np.array([ux[cy, cx], uy[cy, cx]])
        ugot = u[:, y, x].cpu().numpy().astype(np.float64)
        err_u = np.abs(ugot - uref).max() / np.abs(uref).max()
        worst_f, worst_u = max(worst_f, err_f), max(worst_u, err_u)
        assert err_f < STEP_TOL * T, (x, y, err_f)
        assert err_u < 1e-5, (x, y, err_u)
    print(f"{N}^2 (state above 4 GiB) after {T} steps, {len(xs)} sampled nodes: populations "
          f"{worst_f:.2e}, velocity {worst_u:.2e} (relative)")
    del s, df, u
    torch.cuda.empty_cache()

"""On-node walls with non-equilibrium extrapolation (LBM_WALLS_NEE, the paper's
default wall treatment, Sec. 3): GPU against the FP64 oracle element by
element, the closed-form channel flows, thermal walls, batches and the
contract of the combination checks."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import analytic as A
from paper_1311_7239_amd import inputs as I
from paper_1311_7239_amd import lbm
from tests.gpu_cases import Pair, max_rel_velocity_error

pytestmark = pytest.mark.gpu

STEP_TOL = 8 * 2.0 ** -24 * 8


def _nee_case(kind, nx, ny, seed=0):
    if kind == "cavity":
        c = I.lid_cavity(n=max(nx, ny), nee=True)
        c.nx, c.ny = nx, ny
        G = I.grf(ny, nx, 6.0, seed + 100)
        c.phi = np.clip(0.4 + 0.15 * G, 0.1, 0.95).astype(np.float32)
        c.dp = I.ergun_dp(30.0, 0.4)
        c.Fphi = None
    elif kind == "channel":
        c = I.poiseuille_channel(ny=ny, nx=nx, nee=True)
        c.ax = 1e-5
    elif kind == "box":  # on-node walls along x only, periodic in y, body force in y
        c = I.poiseuille_channel(ny=ny, nx=nx, nee=True)
        c.bc_x, c.bc_y, c.ax, c.ay = I.NEE, I.PERIODIC, 0.0, 2e-5
    else:  # natural convection, thermal walls
        c = I.natural_convection(n=max(nx, ny), nee=True)
        c.nx, c.ny = nx, ny
        c.gbeta *= 1e3   # strong coupling, so that T matters within a few steps
    return c


@pytest.mark.parametrize("kind", ["cavity", "channel", "box", "convection"])
@pytest.mark.parametrize("storage", [lbm.FP32_DEV, lbm.FP16_DEV])
def test_first_steps_match_oracle(kind, storage):
    """Random deviation state on a ragged grid over several tiles: populations
    (wall nodes included, as rebuilt by the extrapolation) after 1, 2 and 5
    steps agree with the oracle element by element."""
    nx, ny = 300, 37
    case = _nee_case(kind, nx, ny, seed=1)
    df0 = I.random_deviation_state(ny, nx, 1e-3, seed=17)
    dg0 = I.random_deviation_state(ny, nx, 1e-2, seed=18, channels=5) if case.thermal else None
    pair = Pair(case, storage=storage, df0=df0, dg0=dg0)
    # FP16 storage rounds every stored value to 11 bits; FP32 to 24
    tol = STEP_TOL if storage == lbm.FP32_DEV else 8 * 2.0 ** -11
    done = 0
    for t in (1, 2, 5):
        pair.step(t - done)
        done = t
        ref = pair.oracle_dev()
        got, gg = pair.gpu_dev()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err < tol * t, (t, err)
        if case.thermal:
            gref = np.transpose(pair.g, (2, 0, 1)) - case.T0 / 5.0
            gerr = np.abs(gg - gref).max() / np.abs(gref).max()
            assert gerr < tol * t, (t, gerr)


def test_macroscopic_and_mass_match_oracle():
    case = _nee_case("cavity", 130, 70, seed=3)
    df0 = I.random_deviation_state(70, 130, 1e-3, seed=8)
    pair = Pair(case, df0=df0)
    pair.step(3)
    p, u, _ = pair.gpu_macro()
    ux, uy, pr, _ = pair.oracle_macro()
    assert max_rel_velocity_error(u, ux, uy) < 1e-5
    np.testing.assert_allclose(p, pr, rtol=2e-6)
    mass, res, st = pair.gpu.reduce()
    assert abs(mass - oracle.mass(pair.f)) / oracle.mass(pair.f) < 1e-7


def test_paper_cavity_128_matches_oracle():
    """Sec. 3.3 setting with on-node walls: 128^2, phi = 0.1, Re = 10, nu = 0.256
    (U = Re nu / L), Da = 1e-3; 2000 steps from rest, u against the oracle."""
    n = 128
    c = I.lid_cavity(n=n, phi=0.1, Da=1e-3, Re=10.0, nee=True)
    L = n - 1
    c.nu = 0.256
    c.lid_ux = 10.0 * c.nu / L
    c.K0 = 1e-3 * L * L
    pair = Pair(c, nthreads=8)
    pair.step(2000)
    _, u, _ = pair.gpu_macro()
    ux, uy, _, _ = pair.oracle_macro()
    assert max_rel_velocity_error(u, ux, uy) < 2e-5
    # the lid row moves with the lid, up to the drag share of the rebuilt momentum
    assert abs(u[0, -1, n // 2] - c.lid_ux) < 1e-2 * c.lid_ux


def _steady(case, steps):
    """GPU run for a step count past the oracle's own steady step count."""
    s = lbm.solver_for_case(case)
    s.step(steps)
    _, u, _ = s.macroscopic()
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.float64)


def test_brinkman_poiseuille_closed_form():
    """Sec. 3.1 with on-node walls (L = N - 1) on the GPU: within the oracle's own
    distance to Eq. (23) at N = 33 (4.2e-3) plus FP32 noise."""
    case = I.poiseuille_channel(ny=33, nx=4, forchheimer=False, nee=True)
    u = _steady(case, 40000)   # the oracle is steady to 1e-11 after 28,000
    ref = A.brinkman_poiseuille(np.arange(33, dtype=float), 32, case.ax, case.phi0, case.K0,
                                case.nu)
    for col in range(4):
        e = np.sqrt(np.sum((u[0, :, col] - ref) ** 2) / np.sum(ref ** 2))
        assert e < 5e-3, e


def test_couette_closed_form_and_lid_row():
    case = I.couette_channel(ny=65, nx=4, nee=True)
    u = _steady(case, 50000)   # the oracle is steady to 1e-11 after 36,000
    ref = A.porous_couette(np.arange(65, dtype=float), 64, case.lid_ux, case.phi0, case.K0,
                           case.nu)
    e = np.sqrt(np.sum((u[0, :, 0] - ref) ** 2) / np.sum(ref ** 2))
    assert e < 1e-3, e
    assert abs(u[0, -1, 0] / case.lid_ux - 1.0) < 1e-4


def test_conduction_between_dirichlet_walls_is_linear():
    """Pure conduction between on-node Dirichlet walls: the steady temperature is
    linear in x (exact for the oracle; FP32 round-off here)."""
    case = I.natural_convection(n=24, nee=True)
    case.gbeta = 0.0
    case.tau_T = 1.0
    s = lbm.solver_for_case(case)
    s.step(20000)
    _, u, T = s.macroscopic(want_T=True)
    torch.cuda.synchronize()
    T = T.cpu().numpy().astype(np.float64)
    ref = case.Th + (case.Tc - case.Th) * np.arange(24) / 23.0
    assert np.abs(T - ref[None, :]).max() < 2e-5 * (case.Th - case.Tc)
    assert float(u.abs().max()) == 0.0


def test_batch_with_on_node_walls_matches_single_contexts():
    cases = [I.lid_cavity(n=96, nee=True), _nee_case("channel", 70, 33), I.lid_cavity(n=64)]
    b = lbm.batch_for_cases(cases)
    assert b.time_blocking()["cycles_per_pass"] == 1
    b.step(41)
    for k, c in enumerate(cases):
        s = lbm.solver_for_case(c)
        s.set_time_blocking(1)
        s.step(41)
        assert torch.equal(b.populations(k), s.populations()[0]), k


def test_combination_checks():
    d = lbm.desc_from_case(I.lid_cavity(n=32, nee=True))
    d.bc_x = lbm.WALLS
    with pytest.raises(lbm.LBMError) as ei:
        lbm.Solver(d)
    assert ei.value.status == lbm.ENOTSUP
    d = lbm.desc_from_case(I.lid_cavity(n=32, nee=True))
    d.ny = 2
    with pytest.raises(lbm.LBMError) as ei:
        lbm.Solver(d)
    assert ei.value.status == lbm.EINVAL
    s = lbm.solver_for_case(I.lid_cavity(n=32, nee=True))
    assert s.time_blocking()["cycles_per_pass"] == 1
    with pytest.raises(lbm.LBMError) as ei:
        s.set_time_blocking(2)
    assert ei.value.status == lbm.ENOTSUP
    c = _nee_case("cavity", 40, 30)
    r = lbm.solver_for_case(c, ckpt_every=4, max_steps_recorded=8)
    r.step(8)
    _, u, _ = r.macroscopic()
    with pytest.raises(lbm.LBMError) as ei:
        r.backward(torch.zeros_like(u))
    assert ei.value.status == lbm.ENOTSUP

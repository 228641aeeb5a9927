"""Per-node viscosity ratio J (lbm_set_viscosity_ratio): the partially porous
Couette flow of Sec. 3.2 (Eq. 25) and seeded random J fields, GPU against the
FP64 oracle, plus the plane's own contract (constant plane = uniform J, error
paths, batches, adjoint)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import analytic as A
from paper_1311_7239_amd import inputs as I
from paper_1311_7239_amd import lbm
from tests.gpu_cases import Pair, max_rel_velocity_error

pytestmark = pytest.mark.gpu

# same per-step bound as the other population parity tests
STEP_TOL = 8 * 2.0 ** -24 * 8


def _random_J_case(nx=300, ny=37, seed=11):
    """Lid cavity over an Ergun medium with a smooth random J field in [1, 5]."""
    c = I.lid_cavity(n=max(nx, ny))
    c.nx, c.ny = nx, ny
    G = I.grf(ny, nx, 6.0, seed + 100)
    c.phi = np.clip(0.4 + 0.15 * G, 0.1, 0.95).astype(np.float32)
    c.dp = I.ergun_dp(30.0, 0.4)
    c.Fphi = None
    H = I.grf(ny, nx, 5.0, seed + 200)
    c.Jfield = np.clip(3.0 + 1.2 * H, 1.0, 5.0).astype(np.float32)
    return c


@pytest.mark.parametrize("cycles", [1, 2])
def test_random_J_field_matches_oracle(cycles):
    """Random deviation state on a ragged grid spanning several tiles, per-node J:
    populations after 1, 4 and 9 steps agree with the oracle element by element,
    in the one-cycle and the two-cycle (temporal blocking) kernels."""
    case = _random_J_case()
    df0 = I.random_deviation_state(case.ny, case.nx, 1e-3, seed=9)
    pair = Pair(case, df0=df0)
    pair.gpu.set_time_blocking(cycles)
    done = 0
    for t in (1, 4, 9):
        pair.step(t - done)
        done = t
        ref = pair.oracle_dev()
        got, _ = pair.gpu_dev()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err < STEP_TOL * t, (t, err)


def test_J_plane_changes_the_result():
    """The same case with the plane left at the descriptor's J differs from the
    oracle run with the random field (the plane is really read)."""
    case = _random_J_case()
    df0 = I.random_deviation_state(case.ny, case.nx, 1e-3, seed=9)
    pair = Pair(case, df0=df0)
    pair.step(5)
    ref = pair.oracle_dev()
    desc = lbm.desc_from_case(case)
    s = lbm.Solver(desc, phi=torch.from_numpy(case.phi).cuda())
    s.set_populations(torch.from_numpy(df0).cuda())
    s.step(5)
    df, _ = s.populations()
    err = np.abs(df.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err > 100 * STEP_TOL * 5


@pytest.mark.parametrize("cycles", [1, 2])
def test_constant_plane_is_bitwise_uniform_J(cycles):
    """A plane holding the descriptor's J everywhere reproduces the context
    without a plane bit for bit (the rate is rounded once, the same way)."""
    case = _random_J_case(nx=257, ny=70, seed=4)
    case.Jfield = None
    case.J = 2.5
    df0 = torch.from_numpy(I.random_deviation_state(case.ny, case.nx, 1e-3, seed=3)).cuda()
    out = []
    for plane in (False, True):
        desc = lbm.desc_from_case(case)
        desc.j_plane = 1 if plane else 0
        s = lbm.Solver(desc, phi=torch.from_numpy(case.phi).cuda())
        if plane:
            s.set_viscosity_ratio(torch.full((case.ny, case.nx), 2.5, device="cuda"))
        s.set_time_blocking(cycles)
        s.set_populations(df0)
        s.step(13)
        out.append(s.populations()[0].cpu())
    assert torch.equal(out[0], out[1])


def test_plane_starts_at_descriptor_J():
    """j_plane = 1 without a set call behaves as the uniform descriptor J."""
    case = _random_J_case(nx=130, ny=40, seed=5)
    case.Jfield = None
    case.J = 1.7
    out = []
    for plane in (0, 1):
        desc = lbm.desc_from_case(case)
        desc.j_plane = plane
        s = lbm.Solver(desc, phi=torch.from_numpy(case.phi).cuda())
        s.step(20)
        out.append(s.populations()[0].cpu())
    assert torch.equal(out[0], out[1])


@pytest.mark.parametrize("J", [1.0, 4.0])
def test_partial_couette_parity_and_eq25(J):
    """Sec. 3.2 partially porous channel (80 nodes, the paper's parameters):
    transient parity with the oracle, then the GPU steady profile against the
    exact form of Eq. (25) (the oracle's own distance to it is 1.5e-4 u0 for
    J = 1 and 6.4e-5 u0 for J = 4 at this resolution)."""
    case = I.partial_couette(J=J, ny=80, nx=2)
    pair = Pair(case)
    pair.step(3000)
    _, u, _ = pair.gpu_macro()
    ux, uy, _, _ = pair.oracle_macro()
    assert max_rel_velocity_error(u, ux, uy) < 1e-4
    # steady state on the GPU alone
    s = pair.gpu
    s.step(60000)
    _, u, _ = s.macroscopic()
    torch.cuda.synchronize()
    u = u.cpu().numpy().astype(np.float64)
    y = np.arange(80) + 0.5
    ref = A.partial_couette(y, 80, case.lid_ux, 0.1, 1e-3, J)
    err = np.abs(u[0] - ref[:, None]).max() / case.lid_ux
    assert err < 5e-4, err
    assert np.abs(u[1]).max() < 1e-3 * case.lid_ux


def test_batch_domains_with_J_planes_match_single_contexts():
    """Batch domains carry their own planes: bitwise equal to stepping each alone."""
    cases = [I.partial_couette(J=4.0, ny=80, nx=70), I.partial_couette(J=2.0, ny=50, nx=33),
             _random_J_case(nx=150, ny=60, seed=8)]
    b = lbm.batch_for_cases(cases)
    b.step(57)
    for k, c in enumerate(cases):
        s = lbm.solver_for_case(c)
        s.step(57)
        assert torch.equal(b.populations(k), s.populations()[0]), k


def test_set_viscosity_ratio_errors():
    case = _random_J_case(nx=64, ny=32, seed=6)
    # no plane
    desc = lbm.desc_from_case(case)
    desc.j_plane = 0
    s = lbm.Solver(desc, phi=torch.from_numpy(case.phi).cuda())
    with pytest.raises(lbm.LBMError) as ei:
        s.set_viscosity_ratio(torch.ones((32, 64), device="cuda"))
    assert ei.value.status == lbm.ESTATE
    # invalid values keep the previous plane
    s = lbm.solver_for_case(case)
    bad = torch.from_numpy(case.Jfield.copy()).cuda()
    bad[5, 7] = -1.0
    with pytest.raises(lbm.LBMError) as ei:
        s.set_viscosity_ratio(bad)
    assert ei.value.status == lbm.EINVAL
    bad[5, 7] = float("nan")
    with pytest.raises(lbm.LBMError) as ei:
        s.set_viscosity_ratio(bad)
    assert ei.value.status == lbm.EINVAL
    s.step(10)
    ref = lbm.solver_for_case(case)
    ref.step(10)
    assert torch.equal(s.populations()[0], ref.populations()[0])
    # a recorded pass fixes J once it has started
    r = lbm.solver_for_case(case, ckpt_every=4, max_steps_recorded=8)
    r.step(1)
    with pytest.raises(lbm.LBMError) as ei:
        r.set_viscosity_ratio(torch.from_numpy(case.Jfield).cuda())
    assert ei.value.status == lbm.ESTATE


def _oracle_outlet(case, phi, steps):
    p = oracle.make_params(case.nx, case.ny, bc_x=case.bc_x, bc_y=case.bc_y, nu=case.nu,
                           ax=case.ax, nthreads=8, Jcell=case.Jfield)
    phi = np.asarray(phi, dtype=np.float64)
    K, F = oracle.ergun(phi, case.dp)
    f = oracle.rest_state(p, case.Pi0)
    oracle.run(p, phi, K, F, f, nsteps=steps)
    ux, uy, _, _ = oracle.macroscopic(p, phi, K, F, f)
    return np.stack([ux[:, -1], uy[:, -1]])


def test_adjoint_with_J_plane_matches_oracle_finite_differences():
    """lbm_backward with a per-node J: dL/dphi against central differences of
    the FP64 oracle run with the same J field, on the cells of largest |g|."""
    nx, ny, steps = 96, 64, 300
    c = I.lognormal_channel(n=96, seed=21, ell=8.0, K_ref=40.0, drive=0.02)
    c.nx, c.ny = nx, ny
    c.phi = np.ascontiguousarray(c.phi[:ny, :nx])
    c.Jfield = np.clip(2.0 + 0.8 * I.grf(ny, nx, 6.0, 31), 1.0, 4.0).astype(np.float32)
    t = I.lognormal_channel(n=96, seed=55, ell=8.0, K_ref=40.0, drive=0.02)
    target = _oracle_outlet(c, np.ascontiguousarray(t.phi[:ny, :nx]), steps)

    s = lbm.solver_for_case(c, ckpt_every=64, max_steps_recorded=steps)
    s.step(steps)
    _, u, _ = s.macroscopic()
    dLdu = torch.zeros_like(u)
    dLdu[:, :, -1] = u[:, :, -1] - torch.from_numpy(target.astype(np.float32)).cuda()
    g, _ = s.backward(dLdu)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)

    def loss(phi):
        return 0.5 * float(np.sum((_oracle_outlet(c, phi, steps) - target) ** 2))

    phi0 = c.phi.astype(np.float64)
    worst = 0.0
    for idx in np.argsort(-np.abs(g).ravel())[:8]:
        j, i = divmod(int(idx), nx)
        h = 1e-4 * phi0[j, i]
        pp = phi0.copy(); pp[j, i] += h
        pm = phi0.copy(); pm[j, i] -= h
        fd = (loss(pp) - loss(pm)) / (2 * h)
        worst = max(worst, abs(g[j, i] - fd) / abs(fd))
    assert worst < 2e-3, worst

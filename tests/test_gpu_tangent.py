"""Tangent-linear model (lbm_tangent): against central differences of the FP64
oracle, and the dot-product identity with the adjoint (lbm_backward_params),
which holds to rounding for any loss and direction."""
import numpy as np
import pytest
import torch

import oracle
from paper_1311_7239_amd import inputs as I
from paper_1311_7239_amd import lbm

pytestmark = pytest.mark.gpu


def _channel():
    c = I.lognormal_channel(n=96, seed=21, ell=8.0, K_ref=40.0, drive=0.02)
    c.nx, c.ny = 96, 64
    c.phi = np.ascontiguousarray(c.phi[:64, :96])
    c.ay = 0.3 * c.ax
    c.steps = 300
    return c


def _cavity():
    c = I.lid_cavity(n=64, phi=0.4, Da=1e-2, Re=20.0, U=0.05, heterogeneous=True, ell=8.0)
    c.ax, c.ay = 2e-6, -1e-6
    c.steps = 300
    return c


def _recorded(case, cycles=1):
    s = lbm.solver_for_case(case, ckpt_every=64, max_steps_recorded=case.steps)
    s.set_time_blocking(cycles)
    s.step(case.steps)
    return s


def _oracle_u(case, phi, **over):
    vals = dict(nu=case.nu, ax=case.ax, ay=case.ay, lid_ux=case.lid_ux)
    vals.update(over)
    p = oracle.make_params(case.nx, case.ny, bc_x=case.bc_x, bc_y=case.bc_y, nthreads=8, **vals)
    phi = np.asarray(phi, dtype=np.float64)
    K, F = oracle.ergun(phi, case.dp)
    f = oracle.rest_state(p, case.Pi0)
    oracle.run(p, phi, K, F, f, nsteps=case.steps)
    ux, uy, _, _ = oracle.macroscopic(p, phi, K, F, f)
    return np.stack([ux, uy])


def _direction(case, seed):
    rng = np.random.default_rng(seed)
    return (0.05 * case.phi * rng.uniform(-1.0, 1.0, case.phi.shape)).astype(np.float32)


@pytest.mark.parametrize("kind", ["channel", "cavity"])
def test_tangent_matches_oracle_differences(kind):
    case = _channel() if kind == "channel" else _cavity()
    s = _recorded(case)
    dphi = _direction(case, 7)
    du = s.tangent(torch.from_numpy(dphi).cuda()).cpu().numpy().astype(np.float64)
    h = 1e-3
    phi0 = case.phi.astype(np.float64)
    fd = (_oracle_u(case, phi0 + h * dphi) - _oracle_u(case, phi0 - h * dphi)) / (2 * h)
    err = np.abs(du - fd).max() / np.abs(fd).max()
    print(f"{kind}: tangent along dphi vs oracle differences, max rel error {err:.2e}")
    assert err < 1e-4
    # parameter directions, one at a time
    for k, name in enumerate(("nu", "ax", "ay", "lid_ux")):
        base = getattr(case, name)
        if base == 0.0:
            continue
        dth = [0.0] * 4
        dth[k] = base
        du = s.tangent(None, dth).cpu().numpy().astype(np.float64)
        hh = 1e-4
        fd = (_oracle_u(case, phi0, **{name: base * (1 + hh)}) -
              _oracle_u(case, phi0, **{name: base * (1 - hh)})) / (2 * hh)
        err = np.abs(du - fd).max() / np.abs(fd).max()
        print(f"{kind}: tangent along {name} vs oracle differences, max rel error {err:.2e}")
        assert err < 1e-4, name


@pytest.mark.parametrize("cycles", [1, 2, 3])
def test_dot_product_identity_with_the_adjoint(cycles):
    """<w, du> = <dL/dphi, dphi> + <dL/dtheta, dtheta> for L = <w, u(T)>."""
    case = _cavity()
    s = _recorded(case, cycles)
    rng = np.random.default_rng(11)
    w = torch.from_numpy(rng.standard_normal((2, case.ny, case.nx)).astype(np.float32)).cuda()
    g, _, th = s.backward_params(w)
    g = g.cpu().numpy().astype(np.float64)
    gth = np.array([th["nu"], th["ax"], th["ay"], th["lid_ux"]])
    dphi = _direction(case, 5)
    dth = np.array([0.01 * case.nu, 0.02 * case.ax, -0.03 * case.ay, 0.01 * case.lid_ux])
    wn = w.cpu().numpy().astype(np.float64)
    du_phi = s.tangent(torch.from_numpy(dphi).cuda()).cpu().numpy().astype(np.float64)
    du_th = s.tangent(None, dth).cpu().numpy().astype(np.float64)
    lhs_phi, rhs_phi = float(np.sum(wn * du_phi)), float(np.sum(g * dphi))
    lhs_th, rhs_th = float(np.sum(wn * du_th)), float(np.dot(gth, dth))
    print(f"cycles={cycles}: phi {lhs_phi:.8e} vs {rhs_phi:.8e}; theta {lhs_th:.8e} vs {rhs_th:.8e}")
    assert abs(lhs_phi - rhs_phi) <= 2e-5 * abs(rhs_phi)
    assert abs(lhs_th - rhs_th) <= 2e-5 * abs(rhs_th)
    # linearity: the joint direction is the sum of the two
    du_both = s.tangent(torch.from_numpy(dphi).cuda(), dth).cpu().numpy().astype(np.float64)
    assert np.abs(du_both - (du_phi + du_th)).max() <= 1e-5 * np.abs(du_both).max()


def test_tangent_state_errors():
    case = _cavity()
    s = lbm.solver_for_case(case)
    s.step(5)
    with pytest.raises(lbm.LBMError) as ei:
        s.tangent(None, [1.0, 0, 0, 0])
    assert ei.value.status == lbm.ESTATE
    c = I.couette_channel(ny=16, nx=8)
    u = lbm.solver_for_case(c, ckpt_every=4, max_steps_recorded=8)
    u.step(8)
    with pytest.raises(lbm.LBMError) as ei:
        u.tangent(torch.zeros((16, 8), device="cuda"))
    assert ei.value.status == lbm.ENOTSUP
    du = u.tangent(None, [0.0, 0.0, 0.0, 1.0])   # parameter directions work without a plane
    assert float(du.abs().max()) > 0.0

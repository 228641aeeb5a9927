"""The torch.autograd wrapper of the recorded pass (paper_1311_7239_amd.autograd):
gradients through loss.backward() equal the library's adjoint, and agree with
central differences of the FP64 oracle along a random direction."""
import numpy as np
import pytest
import torch

import oracle
from paper_1311_7239_amd import inputs as I
from paper_1311_7239_amd import lbm
from paper_1311_7239_amd.autograd import flow_velocity, outlet_flow

pytestmark = pytest.mark.gpu


def _case():
    c = I.lognormal_channel(n=96, seed=21, ell=8.0, K_ref=40.0, drive=0.02)
    c.nx, c.ny = 96, 64
    c.phi = np.ascontiguousarray(c.phi[:64, :96])
    c.steps = 300
    return c


def _loss(u, target):
    return 0.5 * ((u[:, :, -1] - target) ** 2).sum()


def test_autograd_matches_the_library_adjoint():
    c = _case()
    desc = lbm.desc_from_case(c)
    target = torch.zeros((2, c.ny), device="cuda")
    target[0] = 1e-4
    phi = torch.from_numpy(c.phi).cuda().requires_grad_(True)
    theta = torch.tensor([c.nu, c.ax, c.ay, c.lid_ux], dtype=torch.float64, requires_grad=True)
    u = flow_velocity(phi, desc, c.steps, ckpt_every=64, theta=theta)
    _loss(u, target).backward()

    s = lbm.solver_for_case(c, ckpt_every=64, max_steps_recorded=c.steps)
    s.step(c.steps)
    _, u2, _ = s.macroscopic()
    assert torch.equal(u.detach(), u2)
    dLdu = torch.zeros_like(u2)
    dLdu[:, :, -1] = u2[:, :, -1] - target
    g, _, th = s.backward_params(dLdu)
    assert torch.equal(phi.grad, g)
    assert theta.grad.tolist() == [th["nu"], th["ax"], th["ay"], th["lid_ux"]]

    # phi alone: the plain adjoint path
    phi2 = torch.from_numpy(c.phi).cuda().requires_grad_(True)
    _loss(flow_velocity(phi2, desc, c.steps, ckpt_every=64), target).backward()
    assert torch.equal(phi2.grad, g)


def test_outlet_flow_gradient_equals_full_field_gradient():
    c = _case()
    desc = lbm.desc_from_case(c)
    target = torch.zeros((2, c.ny), device="cuda")
    target[0] = 1e-4
    phi = torch.from_numpy(c.phi).cuda().requires_grad_(True)
    out = outlet_flow(phi, desc, c.steps, ckpt_every=64)
    assert out.shape == (2, c.ny)
    (0.5 * ((out - target) ** 2).sum()).backward()
    phi2 = torch.from_numpy(c.phi).cuda().requires_grad_(True)
    u = flow_velocity(phi2, desc, c.steps, ckpt_every=64)
    assert torch.equal(out.detach(), u.detach()[:, :, -1])
    _loss(u, target).backward()
    assert torch.equal(phi.grad, phi2.grad)


def test_autograd_directional_derivative_against_oracle():
    c = _case()
    desc = lbm.desc_from_case(c)
    tgt = np.zeros((2, c.ny))
    tgt[0] = 1e-4
    target = torch.from_numpy(tgt.astype(np.float32)).cuda()
    phi = torch.from_numpy(c.phi).cuda().requires_grad_(True)
    _loss(flow_velocity(phi, desc, c.steps, ckpt_every=64), target).backward()
    rng = np.random.default_rng(3)
    d = 0.05 * c.phi.astype(np.float64) * rng.uniform(-1.0, 1.0, c.phi.shape)
    ad = float(np.sum(phi.grad.cpu().numpy().astype(np.float64) * d))

    def oracle_loss(ph):
        p = oracle.make_params(c.nx, c.ny, bc_x=c.bc_x, bc_y=c.bc_y, nu=c.nu, ax=c.ax, nthreads=8)
        K, F = oracle.ergun(ph, c.dp)
        f = oracle.rest_state(p, c.Pi0)
        oracle.run(p, ph, K, F, f, nsteps=c.steps)
        ux, uy, _, _ = oracle.macroscopic(p, ph, K, F, f)
        u = np.stack([ux[:, -1], uy[:, -1]])
        return 0.5 * float(np.sum((u - tgt) ** 2))

    h = 1e-3
    phi0 = c.phi.astype(np.float64)
    fd = (oracle_loss(phi0 + h * d) - oracle_loss(phi0 - h * d)) / (2 * h)
    print(f"autograd directional derivative {ad:.8e}, oracle differences {fd:.8e}")
    assert abs(ad - fd) <= 1e-3 * abs(fd)

"""The five workloads at their full sizes, GPU (FP32 unless stated) against the FP64
oracle: stored oracle samples where the oracle would take minutes, the live oracle on
subsets otherwise, and properties that hold at any size (mass, mirror symmetry,
bitwise repeatability)."""
import dataclasses
import pathlib

import numpy as np
import pytest
import torch

import oracle
from oracle import analytic as A
from paper_1311_7239_amd import inputs as I
from paper_1311_7239_amd import lbm
from tests.gpu_cases import Pair, max_rel_velocity_error
from tests.oracle_cases import oracle_setup, run_to_steady, uniform_F

pytestmark = pytest.mark.gpu
GOLDEN = pathlib.Path(__file__).parent / "golden"


def golden(name):
    path = GOLDEN / f"{name}.txt"
    rows = np.loadtxt(path)
    head = {l.split()[1]: float(l.split()[2]) for l in path.read_text().splitlines()
            if l.startswith("# max_abs_u") or l.startswith("# mass")}
    return rows, head


def gpu_u(s):
    _, u, _ = s.macroscopic()
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.float64)


def test_poiseuille_channel_fp32_error_is_reported():
    """8 x 64 porous Poiseuille channel (phi = 0.1, Da = 1e-2, Re = 0.01, Ergun F_phi): the
    FP32 GPU run to the oracle's steady step count, against the FP64 steady state and
    Eq. (23). The FP32 error is set by rounding of 5e-6 velocities, so it is reported
    with a loose bound."""
    case = I.poiseuille_channel(ny=64, nx=8)
    p, phi, K, F = oracle_setup(case, nthreads=1)
    f = oracle.rest_state(p, case.Pi0)
    t, ux_o, _ = run_to_steady(p, phi, K, F, f)
    s = lbm.solver_for_case(case)
    s.set_graph_steps(100)
    s.step(t)
    u = gpu_u(s)
    e_orc = np.sqrt(np.sum((u[0] - ux_o) ** 2) / np.sum(ux_o ** 2))
    y = np.arange(64) + 0.5
    ref = A.bf_poiseuille(y, 64, case.ax, case.phi0, case.K0, case.nu, uniform_F(case))
    e_bvp = np.sqrt(np.sum((u[0, :, 0] - ref) ** 2) / np.sum(ref ** 2))
    print(f"Poiseuille 8x64 FP32 after {t} steps: rel L2 vs FP64 oracle {e_orc:.2e}, vs Eq. (23) {e_bvp:.2e}")
    assert e_orc < 2e-3 and e_bvp < 2e-3


@pytest.mark.parametrize("name,het", [("cavity512_uniform_50k", False), ("cavity512_grf_50k", True)])
def test_lid_cavity_512_50k_against_oracle(name, het):
    """512^2 porous lid cavity (phi = 0.4 or the GRF field, Da = 1e-2, Re = 100), 50,000
    steps from rest: max relative velocity error <= 1e-5 on the stored FP64 samples,
    mass conserved, runs bitwise repeatable."""
    rows, head = golden(name)
    case = I.lid_cavity(n=512, heterogeneous=het)
    runs = []
    for _ in range(2):
        s = lbm.solver_for_case(case)
        s.set_graph_steps(100)
        m0, _, _ = s.reduce()
        s.step(50_000)
        m1, res, st = s.reduce()
        runs.append(gpu_u(s))
        assert st == lbm.OK
        assert abs(m1 - m0) / m0 < 1e-6
        assert abs(m1 - head["mass"]) / head["mass"] < 1e-6
    assert np.array_equal(runs[0], runs[1])
    u = runs[0]
    x, y = rows[:, 0].astype(int), rows[:, 1].astype(int)
    err = max(np.abs(u[0, y, x] - rows[:, 2]).max(), np.abs(u[1, y, x] - rows[:, 3]).max()) / head["max_abs_u"]
    print(f"{name}: max rel velocity error on {len(x)} sampled nodes {err:.2e}")
    assert err <= 1e-5


def test_lid_cavity_512_mirror_symmetry():
    """Mirroring the medium and reversing the lid mirrors the FP32 flow to 1e-6."""
    case = I.lid_cavity(n=512, heterogeneous=True)
    a = lbm.solver_for_case(case)
    case_m = I.lid_cavity(n=512, heterogeneous=True)
    case_m.phi = np.ascontiguousarray(case.phi[:, ::-1])
    case_m.lid_ux = -case.lid_ux
    b = lbm.solver_for_case(case_m)
    for s in (a, b):
        s.set_graph_steps(100)
        s.step(20_000)
    ua, ub = gpu_u(a), gpu_u(b)
    scale = np.abs(ua).max()
    assert np.abs(-ub[0, :, ::-1] - ua[0]).max() / scale < 1e-6
    assert np.abs(ub[1, :, ::-1] - ua[1]).max() / scale < 1e-6


@pytest.mark.parametrize("storage,tol", [(lbm.FP32_DEV, 1e-5), (lbm.FP16_DEV, 2e-2)])
def test_cavity_batch_against_oracle_subset(storage, tol):
    """The 256-cavity ragged batch (seed 4) stepped 600 times in one persistent launch per
    step; 16 cavities (the 8 smallest and 8 seeded random ones) against the FP64 oracle.
    FP32 is held to 1e-5; the FP16 error is stated."""
    cases = I.cavity_batch()
    b = lbm.batch_for_cases(cases, storage=storage)
    steps = 600
    b.step(steps)
    order = np.argsort([c.nodes for c in cases])
    rng = np.random.default_rng(404)
    pick = list(order[:8]) + list(rng.choice(order[8:], size=8, replace=False))
    worst = 0.0
    for k in pick:
        c = cases[int(k)]
        p, phi, K, F = oracle_setup(c, nthreads=16)
        f = oracle.rest_state(p, c.Pi0)
        oracle.run(p, phi, K, F, f, nsteps=steps)
        ux, uy, _, _ = oracle.macroscopic(p, phi, K, F, f)
        _, u = b.macroscopic(int(k))
        err = max_rel_velocity_error(u.cpu().numpy().astype(np.float64), ux, uy)
        worst = max(worst, err)
    print(f"batch storage {storage}: worst max rel velocity error over 16 cavities {worst:.2e}")
    assert worst <= tol


def test_inverse_problem_2048_gradient_by_finite_differences():
    """2048^2 log-normal channel, 4000 steps, checkpoints every 200: the adjoint gradient of
    the outlet misfit (target: the same model on field seed 55) against central finite
    differences of GPU forward runs, the loss summed in FP64, and against the tangent-linear
    model of the same recorded pass (the dot-product identity, exact up to rounding).

    Along a seeded random direction with every cell perturbed the signal is large and the
    agreement tight. For single cells (16 from the top decile of |g|, seed 505) the FP32
    forward runs resolve the loss change only to a few per cent at h = 5e-2 phi (rounding
    of the two perturbed runs decorrelates), so those errors are printed and held to a
    loose bound; the same cells are held tightly against the tangent model of the
    recorded pass, and against FP64-oracle differences on the 256^2 twin (test_gpu_adjoint)."""
    steps = 4000
    case = I.lognormal_channel(n=2048, seed=5)
    tgt_case = I.lognormal_channel(n=2048, seed=55)
    t = lbm.solver_for_case(tgt_case)
    t.step(steps)
    target = gpu_u(t)[:, :, -1]
    del t

    def loss_of(phi_field):
        s = lbm.solver_for_case(dataclasses.replace(case, phi=np.ascontiguousarray(phi_field, dtype=np.float32)))
        s.step(steps)
        uo = gpu_u(s)[:, :, -1]
        return 0.5 * float(np.sum((uo - target) ** 2))

    s = lbm.solver_for_case(case, ckpt_every=200, max_steps_recorded=steps)
    s.step(steps)
    _, u, _ = s.macroscopic()
    dLdu = torch.zeros_like(u)
    dLdu[:, :, -1] = u[:, :, -1] - torch.from_numpy(target.astype(np.float32)).cuda()
    g, _ = s.backward(dLdu)
    g = g.cpu().numpy().astype(np.float64)

    phi0 = case.phi.astype(np.float64)
    r = np.random.default_rng(506).uniform(-1.0, 1.0, size=phi0.shape) * phi0
    # dot-product identity on the real problem, free of finite-difference noise: the
    # tangent-linear rerun of the recorded pass along r against the adjoint gradient
    du = s.tangent(dphi=torch.from_numpy(r.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    lhs = float(np.sum(dLdu.cpu().numpy().astype(np.float64) * du.cpu().numpy().astype(np.float64)))
    rhs = float(np.sum(g * r.astype(np.float32).astype(np.float64)))
    dot_err = abs(lhs / rhs - 1.0)
    print(f"2048^2 dot-product identity: <dL/du, J r> {lhs:.9e}, <dL/dphi, r> {rhs:.9e}, rel {dot_err:.2e}")
    assert dot_err < 1e-4

    # 16 cells from the top decile of |g| (seed 505): each against the tangent model along
    # that cell alone (no finite-difference noise) and, loosely, against GPU differences
    flat = np.abs(g).ravel()
    top = np.flatnonzero(flat >= np.quantile(flat, 0.9))
    cells = np.random.default_rng(505).choice(top, size=16, replace=False)
    dLdu_np = dLdu.cpu().numpy().astype(np.float64)
    tan_errs = []
    for idx in cells:
        j, i = divmod(int(idx), 2048)
        e = torch.zeros((2048, 2048), dtype=torch.float32, device="cuda")
        e[j, i] = 1.0
        du = s.tangent(dphi=e)
        torch.cuda.synchronize()
        tl = float(np.sum(dLdu_np * du.cpu().numpy().astype(np.float64)))
        tan_errs.append(abs(g[j, i] - tl) / abs(tl))
    print("2048^2 adjoint vs tangent model per cell, relative errors:", [f"{v:.1e}" for v in tan_errs])
    assert max(tan_errs) < 1e-3
    del s
    eps = 1e-3
    fd_dir = (loss_of(phi0 + eps * r) - loss_of(phi0 - eps * r)) / (2 * eps)
    dir_err = abs(np.sum(g * r) / fd_dir - 1.0)
    print(f"2048^2 directional derivative: adjoint {np.sum(g * r):.6e}, FD {fd_dir:.6e}, rel err {dir_err:.2e}")
    assert dir_err < 1e-2

    errs = []
    for idx in cells:
        j, i = divmod(int(idx), 2048)
        pp = case.phi.copy(); pp[j, i] = np.float32(phi0[j, i] * 1.05)
        pm = case.phi.copy(); pm[j, i] = np.float32(phi0[j, i] * 0.95)
        fd = (loss_of(pp) - loss_of(pm)) / (float(pp[j, i]) - float(pm[j, i]))
        errs.append(abs(g[j, i] - fd) / abs(fd))
    print("2048^2 adjoint vs single-cell GPU finite differences, relative errors:",
          np.round(errs, 4).tolist())
    # each FP32 forward run rounds differently once phi changes, so a single-cell
    # difference carries noise of a few per cent, and on cells whose loss change is
    # near that noise far more (26% and 88% measured on one cell in two builds whose
    # rounding differs); the median is held here, every cell by the tangent model above
    assert np.median(errs) < 0.05

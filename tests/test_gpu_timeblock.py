"""Two cycles per HBM pass (temporal blocking) gives bitwise the same states as one
cycle per pass, for every boundary kind, medium, storage and ragged size, with and
without graph replay; and the residual still compares u(t) with u(t-1)."""
import numpy as np
import pytest
import torch

from paper_1311_7239_amd import inputs as I
from paper_1311_7239_amd import lbm

pytestmark = pytest.mark.gpu


def cases():
    out = []
    c = I.lid_cavity(n=300, heterogeneous=True, ell=6.0, seed=3)
    c.ny = 37
    c.phi = np.ascontiguousarray(c.phi[:37])
    out.append(("cavity_300x37_grf", c))
    c = I.lid_cavity(n=1100)
    c.ny = 45
    out.append(("cavity_1100x45", c))
    c = I.poiseuille_channel(ny=64, nx=8)
    c.ax = 1e-5
    out.append(("channel_8x64", c))
    c = I.lid_cavity(n=70)
    c.bc_x = c.bc_y = I.PERIODIC
    c.lid_ux = 0.0
    c.ax, c.ay = 1e-5, -2e-5
    out.append(("periodic_70x70", c))
    c = I.poiseuille_channel(ny=16, nx=1)
    c.ax = 1e-5
    out.append(("channel_1x16", c))
    c = I.lognormal_channel(n=200, seed=8, ell=10.0, K_ref=40.0)
    c.nx, c.ny = 200, 130
    c.phi = np.ascontiguousarray(c.phi[:130])
    out.append(("lognormal_200x130", c))
    return out


@pytest.mark.parametrize("storage", [lbm.FP32_DEV, lbm.FP16_DEV])
@pytest.mark.parametrize("name,case", cases(), ids=[n for n, _ in cases()])
@pytest.mark.parametrize("graph", [0, 9, 8])
def test_three_cycles_per_pass_is_bitwise_equal(name, case, storage, graph):
    """Three cycles per pass (two-node LDS ring), alone and mixed with the two- and
    one-cycle passes that finish a call, equal one cycle per pass bit for bit."""
    ref = lbm.solver_for_case(case, storage=storage)
    ref.set_time_blocking(1)
    tb = lbm.solver_for_case(case, storage=storage)
    tb.set_time_blocking(3)
    tb.set_graph_steps(graph)
    df0 = I.random_deviation_state(case.ny, case.nx, 1e-3, seed=5)
    for s in (ref, tb):
        s.set_populations(torch.from_numpy(df0).cuda())
    for chunk in (1, 7, 10, 2, 5, 19, 4):
        ref.step(chunk)
        tb.step(chunk)
        a, _ = ref.populations()
        b, _ = tb.populations()
        torch.cuda.synchronize()
        assert torch.equal(a, b), (name, chunk)


def tall_cases():
    # 2900 x 2935 = 8.5e6 nodes (at least 2^23: 64 x 28 tiles of 768 threads), ragged
    # in x (45 tiles + 20 columns) and in y (104 tiles + 23 rows)
    c = I.lognormal_channel(n=2935, seed=9, ell=40.0, K_ref=400.0)
    c.nx = 2900
    c.phi = np.ascontiguousarray(c.phi[:, :2900])
    out = [("lognormal_2900x2935", c)]
    c = I.lid_cavity(n=2935, heterogeneous=True, ell=30.0, seed=6)
    c.nx = 2900
    c.phi = np.ascontiguousarray(c.phi[:, :2900])
    out.append(("cavity_2900x2935_grf", c))
    return out


@pytest.mark.parametrize("storage", [lbm.FP32_DEV, lbm.FP16_DEV])
@pytest.mark.parametrize("name,case", tall_cases(), ids=[n for n, _ in tall_cases()])
@pytest.mark.parametrize("graph", [0, 9])
def test_tall_three_cycle_tiles_are_bitwise_equal(name, case, storage, graph):
    """The 64 x 28 three-cycle tiles of large single domains equal one cycle per pass
    bit for bit, ragged edges included."""
    ref = lbm.solver_for_case(case, storage=storage)
    ref.set_time_blocking(1)
    tb = lbm.solver_for_case(case, storage=storage)
    tb.set_time_blocking(3)
    shape = tb.time_blocking()
    assert (shape["cycles_per_pass"], shape["rows"], shape["threads"]) == (3, 28, 768)
    assert shape["grid"] == 46 * 105
    tb.set_graph_steps(graph)
    df0 = I.random_deviation_state(case.ny, case.nx, 1e-3, seed=6)
    for s in (ref, tb):
        s.set_populations(torch.from_numpy(df0).cuda())
    del df0
    for chunk in (1, 7, 5):
        ref.step(chunk)
        tb.step(chunk)
        a, _ = ref.populations()
        b, _ = tb.populations()
        torch.cuda.synchronize()
        assert torch.equal(a, b), (name, chunk)
        del a, b


@pytest.mark.parametrize("storage", [lbm.FP32_DEV, lbm.FP16_DEV])
@pytest.mark.parametrize("name,case", cases(), ids=[n for n, _ in cases()])
@pytest.mark.parametrize("graph", [0, 9, 8])
def test_four_cycles_per_pass_is_bitwise_equal(name, case, storage, graph):
    """Four cycles per pass (three-node LDS ring), alone and mixed with the three-, two-
    and one-cycle passes that finish a call, equal one cycle per pass bit for bit, on
    every boundary kind, ragged and tiny domain (8 x 64, 1 x 16, periodic 70 x 70)."""
    ref = lbm.solver_for_case(case, storage=storage)
    ref.set_time_blocking(1)
    tb = lbm.solver_for_case(case, storage=storage)
    tb.set_time_blocking(4)
    shape = tb.time_blocking()
    assert (shape["cycles_per_pass"], shape["rows"], shape["threads"]) == (4, 26, 768)
    assert shape["grid"] == ((case.nx + 63) // 64) * ((case.ny + 25) // 26)
    tb.set_graph_steps(graph)
    df0 = I.random_deviation_state(case.ny, case.nx, 1e-3, seed=5)
    for s in (ref, tb):
        s.set_populations(torch.from_numpy(df0).cuda())
    for chunk in (1, 7, 10, 2, 5, 19, 4, 3, 12):
        ref.step(chunk)
        tb.step(chunk)
        a, _ = ref.populations()
        b, _ = tb.populations()
        torch.cuda.synchronize()
        assert torch.equal(a, b), (name, chunk)


@pytest.mark.parametrize("storage", [lbm.FP32_DEV, lbm.FP16_DEV])
@pytest.mark.parametrize("name,case", tall_cases(), ids=[n for n, _ in tall_cases()])
def test_tall_four_cycle_tiles_are_bitwise_equal(name, case, storage):
    """Four cycles per pass on a domain of 8.5e6 nodes, ragged in x (45 tiles + 20
    columns) and in y (112 tiles + 23 rows), equal one cycle per pass bit for bit."""
    ref = lbm.solver_for_case(case, storage=storage)
    ref.set_time_blocking(1)
    tb = lbm.solver_for_case(case, storage=storage)
    tb.set_time_blocking(4)
    assert tb.time_blocking()["grid"] == 46 * 113
    df0 = I.random_deviation_state(case.ny, case.nx, 1e-3, seed=6)
    for s in (ref, tb):
        s.set_populations(torch.from_numpy(df0).cuda())
    del df0
    for chunk in (1, 9, 6):
        ref.step(chunk)
        tb.step(chunk)
        a, _ = ref.populations()
        b, _ = tb.populations()
        torch.cuda.synchronize()
        assert torch.equal(a, b), (name, chunk)
        del a, b


def test_four_cycles_take_isothermal_domains():
    """Mode 4 is refused (ENOTSUP) for thermal domains and thermal batches, and leaves
    the context's mode unchanged; an isothermal batch takes it (64 x 26 tiles, one
    workgroup each)."""
    _, thermal = thermal_cases()[0]
    s = lbm.solver_for_case(thermal)
    before = s.time_blocking()["cycles_per_pass"]
    with pytest.raises(lbm.LBMError) as e:
        s.set_time_blocking(4)
    assert e.value.status == lbm.ENOTSUP
    assert s.time_blocking()["cycles_per_pass"] == before
    tb = lbm.batch_for_cases([c for _, c in thermal_cases()])
    with pytest.raises(lbm.LBMError) as e:
        tb.set_time_blocking(4)
    assert e.value.status == lbm.ENOTSUP
    iso = [c for _, c in cases()[:2]]
    b = lbm.batch_for_cases(iso)
    b.set_time_blocking(4)
    shape = b.time_blocking()
    assert (shape["cycles_per_pass"], shape["threads"], shape["rows"]) == (4, 768, 26)
    assert shape["grid"] == sum(((c.nx + 63) // 64) * ((c.ny + 25) // 26) for c in iso)
    with pytest.raises(lbm.LBMError) as e:
        s.set_time_blocking(5)
    assert e.value.status == lbm.EINVAL


@pytest.mark.parametrize("storage", [lbm.FP32_DEV, lbm.FP16_DEV])
@pytest.mark.parametrize("name,case", cases(), ids=[n for n, _ in cases()])
@pytest.mark.parametrize("graph,shape", [(0, (512, 16)), (8, (256, 16)), (0, (256, 8)), (8, (512, 8))])
def test_two_cycles_per_pass_is_bitwise_equal(name, case, storage, graph, shape):
    ref = lbm.solver_for_case(case, storage=storage)
    ref.set_time_blocking(1)
    tb = lbm.solver_for_case(case, storage=storage)
    tb.set_time_blocking(2)
    tb.set_two_cycle_tile(*shape)
    tb.set_graph_steps(graph)
    df0 = I.random_deviation_state(case.ny, case.nx, 1e-3, seed=4)
    for s in (ref, tb):
        s.set_populations(torch.from_numpy(df0).cuda())
    for chunk in (1, 7, 10, 2, 5, 19):
        ref.step(chunk)
        tb.step(chunk)
        a, _ = ref.populations()
        b, _ = tb.populations()
        torch.cuda.synchronize()
        assert torch.equal(a, b), (name, chunk)
        ma, ra, _ = ref.reduce()
        mb, rb, _ = tb.reduce()
        assert ma == mb and ra == rb


@pytest.mark.parametrize("kappa_plane", [False, True])
def test_backward_with_two_cycle_passes_is_bitwise_equal(kappa_plane):
    """In the multi-cycle modes the adjoint's recomputation runs two or three cycles per
    pass (recording u at each) and the backward sweep two or three adjoint steps per pass
    (mode 4 recomputes four cycles per pass and sweeps three steps per pass); gradients
    are bitwise those of the one-cycle path (odd step count: segments of every length
    modulo 2, 3 and 4)."""
    case = I.lognormal_channel(n=160, seed=9, ell=10.0, K_ref=40.0, drive=0.02)
    kap = None
    if kappa_plane:
        kap = torch.from_numpy((150.0 * (1 - case.phi) ** 2 / (case.phi ** 3 * case.dp ** 2))
                               .astype(np.float32)).cuda()
    grads = []
    for tblock in (1, 2, 3, 4):
        desc = lbm.desc_from_case(case, ckpt_every=50)
        if kappa_plane:
            desc.medium = lbm.MEDIUM_PHI_KAPPA
        s = lbm.Solver(desc, phi=torch.from_numpy(case.phi).cuda(), kappa=kap, max_steps_recorded=231)
        s.set_time_blocking(tblock)
        # recorded passes stop at every checkpoint time, also across calls
        s.step(37)
        s.step(194)
        _, u, _ = s.macroscopic()
        dLdu = torch.zeros_like(u)
        dLdu[:, :, -1] = u[:, :, -1]
        g, gk = s.backward(dLdu, want_kappa=kappa_plane)
        torch.cuda.synchronize()
        grads.append((g.cpu().numpy(), None if gk is None else gk.cpu().numpy()))
    for k in (1, 2, 3):
        assert np.array_equal(grads[0][0], grads[k][0]), k
        if kappa_plane:
            assert np.array_equal(grads[0][1], grads[k][1]), k


def thermal_cases():
    """Natural-convection domains (D2Q8 + D2Q5): hot and cold x walls (anti-bounce-back),
    adiabatic y walls, ragged sizes, a periodic y axis, an Ergun GRF medium, and a
    buoyancy strong enough that the temperature field moves within the test."""
    out = []
    c = I.natural_convection(n=130, Ra=1e6)
    c.ny = 77
    c.gbeta *= 20.0
    out.append(("convection_130x77", c))
    c = I.natural_convection(n=70, phi=0.4, Da=1e-2, Ra=1e5)
    c.nx = 201
    c.bc_y = I.PERIODIC
    c.gbeta *= 20.0
    out.append(("convection_201x70_periodic_y", c))
    c = I.natural_convection(n=96, phi=0.6, Da=1e-2, Ra=1e5)
    G = I.grf(96, 96, 6.0, 77)
    c.phi = np.clip(0.6 + 0.1 * G, 0.3, 0.9).astype(np.float32)
    c.dp = I.ergun_dp(c.K0, 0.6)
    c.Fphi = None
    c.gbeta *= 50.0
    out.append(("convection_96_ergun_grf", c))
    return out


def _thermal_state(case, seed):
    rng = np.random.default_rng(seed)
    df = I.random_deviation_state(case.ny, case.nx, 1e-3, seed=seed)
    x = (np.arange(case.nx) + 0.5) / case.nx
    T = case.Th + (case.Tc - case.Th) * x
    dg = np.broadcast_to(((T - case.T0) / 5.0)[None, None, :], (5, case.ny, case.nx)).astype(np.float32)
    dg = (dg + rng.uniform(-0.05, 0.05, dg.shape)).astype(np.float32)
    return df, dg


@pytest.mark.parametrize("storage", [lbm.FP32_DEV, lbm.FP16_DEV])
@pytest.mark.parametrize("name,case", thermal_cases(), ids=[n for n, _ in thermal_cases()])
@pytest.mark.parametrize("graph,shape", [(0, (512, 16)), (8, (256, 16)), (9, (256, 8)), (0, (512, 8))])
def test_thermal_two_cycles_per_pass_is_bitwise_equal(name, case, storage, graph, shape):
    """The coupled D2Q8 + D2Q5 step two cycles per pass (both fields kept in LDS for the
    ring) equals one cycle per pass bit for bit, for flow and temperature."""
    ref = lbm.solver_for_case(case, storage=storage)
    ref.set_time_blocking(1)
    tb = lbm.solver_for_case(case, storage=storage)
    tb.set_time_blocking(2)
    tb.set_two_cycle_tile(*shape)
    tb.set_graph_steps(graph)
    df0, dg0 = _thermal_state(case, 6)
    for s in (ref, tb):
        s.set_populations(torch.from_numpy(df0).cuda(), torch.from_numpy(dg0).cuda())
    for chunk in (1, 7, 10, 2, 5, 19, 4):
        ref.step(chunk)
        tb.step(chunk)
        fa, ga = ref.populations(thermal=True)
        fb, gb = tb.populations(thermal=True)
        torch.cuda.synchronize()
        assert torch.equal(fa, fb), (name, chunk)
        assert torch.equal(ga, gb), (name, chunk)


@pytest.mark.parametrize("storage", [lbm.FP32_DEV, lbm.FP16_DEV])
@pytest.mark.parametrize("name,case", thermal_cases(), ids=[n for n, _ in thermal_cases()])
@pytest.mark.parametrize("graph", [0, 9])
def test_thermal_three_cycles_per_pass_is_bitwise_equal(name, case, storage, graph):
    """Three cycles per pass with the D2Q5 field (two-node ring of both fields in LDS)
    equal one cycle per pass bit for bit, for flow and temperature."""
    ref = lbm.solver_for_case(case, storage=storage)
    ref.set_time_blocking(1)
    tb = lbm.solver_for_case(case, storage=storage)
    tb.set_time_blocking(3)
    tb.set_graph_steps(graph)
    df0, dg0 = _thermal_state(case, 7)
    for s in (ref, tb):
        s.set_populations(torch.from_numpy(df0).cuda(), torch.from_numpy(dg0).cuda())
    for chunk in (1, 7, 10, 2, 5, 19, 4):
        ref.step(chunk)
        tb.step(chunk)
        fa, ga = ref.populations(thermal=True)
        fb, gb = tb.populations(thermal=True)
        torch.cuda.synchronize()
        assert torch.equal(fa, fb), (name, chunk)
        assert torch.equal(ga, gb), (name, chunk)


@pytest.mark.parametrize("uniform", [False, True])
@pytest.mark.parametrize("storage", [lbm.FP32_DEV, lbm.FP16_DEV])
def test_thermal_batch_two_cycles_per_pass_is_bitwise_equal(storage, uniform):
    """All thermal cases (one with an Ergun porosity field), or only the uniform ones (the
    batch then takes the kernels specialised for uniform media)."""
    cases = [c for _, c in thermal_cases()]
    if uniform:
        cases = [c for c in cases if c.phi is None]
        assert len(cases) == 2
    a = lbm.batch_for_cases(cases, storage=storage)
    a.set_time_blocking(1)
    b = lbm.batch_for_cases(cases, storage=storage)
    b.set_time_blocking(2)
    with pytest.raises(lbm.LBMError) as e:
        b.set_time_blocking(3)       # thermal batches: one or two cycles per pass
    assert e.value.status == lbm.ENOTSUP
    for k, c in enumerate(cases):
        df0, dg0 = _thermal_state(c, 10 + k)
        for s in (a, b):
            s.set_populations(k, torch.from_numpy(df0).cuda(), torch.from_numpy(dg0).cuda())
    for chunk in (3, 8, 1, 12):
        a.step(chunk)
        b.step(chunk)
        for k in range(len(cases)):
            fa, ga = a.populations(k, thermal=True)
            fb, gb = b.populations(k, thermal=True)
            torch.cuda.synchronize()
            assert torch.equal(fa, fb), (k, chunk)
            assert torch.equal(ga, gb), (k, chunk)

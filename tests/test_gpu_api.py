"""State handling of the C ABI on the GPU: snapshots, instability detection, argument
checks that need a live context."""
import numpy as np
import pytest
import torch

from paper_1311_7239_amd import inputs as I
from paper_1311_7239_amd import lbm

pytestmark = pytest.mark.gpu


def test_save_load_round_trip_is_bitwise():
    case = I.lid_cavity(n=96, heterogeneous=True, ell=8.0)
    a = lbm.solver_for_case(case)
    a.step(57)
    blob = a.save()
    a.step(40)
    ref, _ = a.populations()
    _, res_ref, _ = a.reduce()
    b = lbm.solver_for_case(case)
    b.load(blob)
    assert b.time == 57
    b.step(40)
    got, _ = b.populations()
    _, res, _ = b.reduce()
    torch.cuda.synchronize()
    assert torch.equal(ref, got) and res == res_ref


def test_load_rejects_a_snapshot_of_another_descriptor():
    a = lbm.solver_for_case(I.lid_cavity(n=64))
    blob = a.save()
    other = I.lid_cavity(n=64)
    other.nu *= 2
    b = lbm.solver_for_case(other)
    with pytest.raises(lbm.LBMError) as e:
        b.load(blob)
    assert e.value.status == lbm.EINVAL
    with pytest.raises(lbm.LBMError):
        a.load(blob[:100])


def test_load_rejects_snapshots_of_other_thermal_setups():
    """The descriptor hash covers the thermal block: a thermal snapshot does not load into
    an isothermal context with otherwise equal fields, nor into one with another hot-wall
    temperature or g beta."""
    case = I.natural_convection(n=48)
    a = lbm.solver_for_case(case)
    a.step(7)
    blob = a.save()
    iso = I.natural_convection(n=48)
    iso.thermal = False
    variants = [iso]
    for field, value in (("Th", case.Th + 1.0), ("gbeta", 2.0 * case.gbeta)):
        v = I.natural_convection(n=48)
        setattr(v, field, value)
        variants.append(v)
    for v in variants:
        b = lbm.solver_for_case(v)
        with pytest.raises(lbm.LBMError) as e:
            b.load(blob)
        assert e.value.status == lbm.EINVAL
        assert b.time == 0
    same = lbm.solver_for_case(I.natural_convection(n=48))
    same.load(blob)
    assert same.time == 7


@pytest.mark.parametrize("tblock", [2, 3])
def test_snapshot_after_a_multi_cycle_pass_keeps_the_residual(tblock):
    """A snapshot carries the u(t - 1) planes of the last pass, so the residual of the
    restored context equals the original's bit for bit."""
    case = I.lognormal_channel(n=128, seed=3, ell=8.0, K_ref=30.0, drive=0.05)
    a = lbm.solver_for_case(case)
    a.set_time_blocking(tblock)
    a.step(31)
    blob = a.save()
    b = lbm.solver_for_case(case)
    b.load(blob)
    assert b.reduce() == a.reduce()
    a.step(8)
    b.step(8)
    assert b.reduce() == a.reduce()
    with pytest.raises(lbm.LBMError) as e:
        b.load(blob[:-4])
    assert e.value.status == lbm.EINVAL


def test_non_finite_state_is_reported_unstable():
    case = I.lid_cavity(n=64)
    s = lbm.solver_for_case(case)
    df = torch.zeros((8, 64, 64), device="cuda")
    df[3, 10, 20] = float("nan")
    s.set_populations(df)
    s.step(3)
    mass, res, st = s.reduce()
    assert st == lbm.EUNSTABLE
    assert not np.isfinite(mass)


def test_thermal_populations_round_trip_and_time():
    case = I.natural_convection(n=48)
    s = lbm.solver_for_case(case)
    dg = I.random_deviation_state(48, 48, 0.5, seed=3, channels=5)
    s.set_populations(torch.zeros((8, 48, 48), device="cuda"), torch.from_numpy(dg).cuda())
    assert s.time == 0
    _, g = s.populations(thermal=True)
    torch.cuda.synchronize()
    assert np.array_equal(g.cpu().numpy(), dg)
    s.step(5)
    assert s.time == 5


def test_argument_checks_on_a_live_context():
    case = I.lid_cavity(n=64)
    s = lbm.solver_for_case(case)
    for bad in (-2, 5000):
        with pytest.raises(lbm.LBMError) as e:
            s.set_graph_steps(bad)
        assert e.value.status == lbm.EINVAL
    with pytest.raises(lbm.LBMError) as e:
        s.set_schedule(100, 1, 1)
    assert e.value.status == lbm.EINVAL
    for bad in (0, 5):
        with pytest.raises(lbm.LBMError) as e:
            s.set_time_blocking(bad)
        assert e.value.status == lbm.EINVAL
    with pytest.raises(lbm.LBMError) as e:
        s.macroscopic(want_T=True)          # no thermal model
    assert e.value.status == lbm.EINVAL
    t = lbm.solver_for_case(I.natural_convection(n=32))
    t.set_time_blocking(2)
    t.set_time_blocking(3)
    with pytest.raises(lbm.LBMError) as e:
        t.set_time_blocking(4)              # four cycles: isothermal single domains
    assert e.value.status == lbm.ENOTSUP
    w = lbm.solver_for_case(I.natural_convection(n=32, nee=True))
    with pytest.raises(lbm.LBMError) as e:
        w.set_time_blocking(2)       # on-node walls: one cycle per pass
    assert e.value.status == lbm.ENOTSUP
    with pytest.raises(lbm.LBMError) as e:
        lbm.lib().lbm_step and s.step(-1)
    assert e.value.status == lbm.EINVAL

"""Ragged batched stepping (persistent tile-table kernel, HIP graph replay, autotuned
schedule): bitwise equal to stepping each domain alone, and oracle-matching."""
import numpy as np
import pytest
import torch

import oracle
from paper_1311_7239_amd import inputs as I
from paper_1311_7239_amd import lbm
from tests.gpu_cases import Pair

pytestmark = pytest.mark.gpu


def mixed_cases(uniform=False):
    """Ragged lid cavities; every other one has a porosity field unless uniform (then the
    batch takes the kernels specialised for uniform media)."""
    sizes = [(70, 70), (130, 90), (64, 64), (300, 33), (257, 129)]
    cases = []
    for k, (nx, ny) in enumerate(sizes):
        c = I.lid_cavity(n=max(nx, ny), Re=20.0 + 30 * k, heterogeneous=(k % 2 == 1 and not uniform), ell=6.0,
                         seed=10 + k)
        c.nx, c.ny = nx, ny
        if c.phi is not None:
            c.phi = np.ascontiguousarray(c.phi[:ny, :nx])
        if k == 2:
            c.bc_x = I.PERIODIC
        cases.append(c)
    return cases


def single_run(case, steps, storage):
    s = lbm.solver_for_case(case, storage=storage)
    s.step(steps)
    df, _ = s.populations()
    torch.cuda.synchronize()
    return df.cpu().numpy()


@pytest.mark.parametrize("uniform", [False, True])
@pytest.mark.parametrize("storage", [lbm.FP32_DEV, lbm.FP16_DEV])
@pytest.mark.parametrize("tblock", [1, 2, 3, 4])
def test_batch_is_bitwise_equal_to_single_domains(storage, tblock, uniform, tmp_path):
    """One to four cycles per pass, graph replays of 6 cycles (4 in mode 4), leftovers;
    mixed media and all-uniform media."""
    cases = mixed_cases(uniform)
    b = lbm.batch_for_cases(cases, storage=storage, tune_cache=tmp_path / "tune.txt")
    b.set_time_blocking(tblock)
    b.set_graph_steps(6)
    done = 0
    for chunk in (1, 9, 3, 8, 13):      # t = 0 cycle, graph replays, leftovers
        b.step(chunk)
        done += chunk
        for k in range(len(cases)):
            _, u = b.macroscopic(k)      # eager work between replays
            torch.cuda.synchronize()
            got = b.populations(k).cpu().numpy()
            assert np.array_equal(got, single_run(cases[k], done, storage)), (k, done)


@pytest.mark.parametrize("kind,storage,tblock", [("mixed", lbm.FP32_DEV, 2), ("mixed", lbm.FP32_DEV, 3),
                                                  ("mixed", lbm.FP16_DEV, 3), ("uniform", lbm.FP32_DEV, 3),
                                                  ("thermal", lbm.FP32_DEV, 2)])
def test_batch_workgroups_walking_runs_of_tiles(kind, storage, tblock, tmp_path):
    """Small batches are tuned to one workgroup per tile. A tuning-cache entry with grids
    of 3 and 5 workgroups makes each walk a run of tiles instead; the results stay
    bitwise those of single domains (flow and temperature)."""
    from tests.test_gpu_timeblock import thermal_cases
    thermal = kind == "thermal"
    cases = [c for _, c in thermal_cases()] if thermal else mixed_cases(kind == "uniform")
    path = tmp_path / "tune.txt"
    lbm.batch_for_cases(cases, storage=storage, tune_cache=path)
    fields = path.read_text().split()
    assert len(fields) == 11        # key, one-cycle shape and grid, mode, two-cycle shape, grid2, grid3, four
    fields[8], fields[9] = "3", ("0" if thermal else "5")
    path2 = tmp_path / "tune_small_grids.txt"
    path2.write_text(" ".join(fields) + "\n")
    b = lbm.batch_for_cases(cases, storage=storage, tune_cache=path2)
    b.set_time_blocking(tblock)
    assert b.time_blocking()["grid"] == (3 if tblock == 2 else 5)
    b.set_graph_steps(6)
    done = 0
    for chunk in (1, 9, 8):
        b.step(chunk)
        done += chunk
    torch.cuda.synchronize()
    for k, c in enumerate(cases):
        s = lbm.solver_for_case(c, storage=storage)
        s.step(done)
        df, dg = s.populations(thermal=thermal)
        got = b.populations(k, thermal=thermal)
        torch.cuda.synchronize()
        if thermal:
            assert torch.equal(got[0], df) and torch.equal(got[1], dg), k
        else:
            assert torch.equal(got, df), k


def test_cache_entry_cannot_select_a_missing_mode(tmp_path):
    """A tuning-cache entry naming four cycles for a thermal batch (which has only one
    and two) is clamped to two cycles; the batch still equals single domains bit for bit."""
    from tests.test_gpu_timeblock import thermal_cases
    cases = [c for _, c in thermal_cases()]
    path = tmp_path / "tune.txt"
    lbm.batch_for_cases(cases, tune_cache=path)
    fields = path.read_text().split()
    # mode 4, 16-row two-cycle tiles, grid3 and the four-cycle flag: a line the lookup accepts
    fields[5], fields[7], fields[9], fields[10] = "4", "16", "5", "1"
    path.write_text(" ".join(fields) + "\n")
    b = lbm.batch_for_cases(cases, tune_cache=path)
    assert b.time_blocking()["cycles_per_pass"] == 2
    b.step(9)
    for k, c in enumerate(cases):
        s = lbm.solver_for_case(c)
        s.step(9)
        df, dg = s.populations(thermal=True)
        got = b.populations(k, thermal=True)
        torch.cuda.synchronize()
        assert torch.equal(got[0], df) and torch.equal(got[1], dg), k


def test_batch_matches_oracle():
    cases = mixed_cases()[:3]
    b = lbm.batch_for_cases(cases)
    pairs = [Pair(c) for c in cases]
    b.step(40)
    for k, pr in enumerate(pairs):
        pr.step(40)
        ref = pr.oracle_dev()
        got = b.populations(k).cpu().numpy().astype(np.float64)
        assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-5


def test_tune_cache_is_written_and_reused(tmp_path):
    cases = mixed_cases()[:2]
    path = tmp_path / "tune.txt"
    b1 = lbm.batch_for_cases(cases, tune_cache=path)
    text = path.read_text().strip().splitlines()
    assert len(text) == 1 and len(text[0].split()) == 11
    b2 = lbm.batch_for_cases(cases, tune_cache=path)
    assert b1.schedule() == b2.schedule()
    assert len(path.read_text().strip().splitlines()) == 1    # found, not re-tuned


def test_single_domain_graph_replays_match_eager():
    case = I.lid_cavity(n=96, heterogeneous=True, ell=8.0)
    g = lbm.solver_for_case(case)
    g.set_graph_steps(6)
    e = lbm.solver_for_case(case)
    for chunk in (13, 12, 6, 7):
        g.step(chunk)
        e.step(chunk)
        _, ug, _ = g.macroscopic()
        _, ue, _ = e.macroscopic()
        torch.cuda.synchronize()
        assert torch.equal(ug, ue)
        assert torch.equal(g.populations()[0], e.populations()[0])


def test_batch_rejects_unsupported_domains():
    # thermal and isothermal domains do not mix
    with pytest.raises(lbm.LBMError) as e:
        lbm.batch_for_cases([I.natural_convection(n=32), I.lid_cavity(n=32)])
    assert e.value.status == lbm.ENOTSUP
    # recording for the adjoint is per single context
    d = lbm.desc_from_case(I.lid_cavity(n=32), ckpt_every=4)
    with pytest.raises(lbm.LBMError) as e:
        lbm.Batch([d])
    assert e.value.status == lbm.ENOTSUP


def _thermal_cases():
    a = I.natural_convection(n=96, Ra=1e6)
    a.gbeta *= 10.0
    b = I.natural_convection(n=64, phi=0.4, Da=1e-2, Ra=1e4, nee=True)
    c = I.natural_convection(n=150, Da=1e-6, Ra=1e8)
    c.ny = 70
    return [a, b, c]


def test_thermal_batch_is_bitwise_equal_to_single_domains():
    """Thermal batches (bounce-back and on-node walls mixed): f and g after 37 steps
    from seeded random states equal those of each domain stepped alone."""
    cases = _thermal_cases()
    b = lbm.batch_for_cases(cases)
    states = []
    for k, c in enumerate(cases):
        df = torch.from_numpy(I.random_deviation_state(c.ny, c.nx, 1e-3, seed=40 + k)).cuda()
        dg = torch.from_numpy(I.random_deviation_state(c.ny, c.nx, 1e-1, seed=50 + k, channels=5)).cuda()
        b.set_populations(k, df, dg)
        states.append((df, dg))
    b.step(37)
    assert b.time == 37
    with pytest.raises(lbm.LBMError) as e:
        b.set_populations(0, *states[0])
    assert e.value.status == lbm.ESTATE
    for k, c in enumerate(cases):
        s = lbm.solver_for_case(c)
        s.set_populations(*states[k])
        s.step(37)
        bf, bg = b.populations(k, thermal=True)
        sf, sg = s.populations(thermal=True)
        assert torch.equal(bf, sf), k
        assert torch.equal(bg, sg), k
        _, _, T = b.macroscopic(k, want_T=True)
        _, _, Ts = s.macroscopic(want_T=True)
        assert torch.equal(T, Ts), k


def test_thermal_batch_matches_oracle():
    """One thermal batch domain against the FP64 oracle after 20 steps."""
    cases = _thermal_cases()
    b = lbm.batch_for_cases(cases)
    c = cases[1]
    dg0 = I.random_deviation_state(c.ny, c.nx, 1e-1, seed=51, channels=5)
    df0 = I.random_deviation_state(c.ny, c.nx, 1e-3, seed=41)
    b.set_populations(1, torch.from_numpy(df0).cuda(), torch.from_numpy(dg0).cuda())
    pair = Pair(c, df0=df0, dg0=dg0)   # its own GPU context stays at t = 0
    b.step(20)
    oracle.run(pair.p, pair.phi, pair.K, pair.F, pair.f, pair.g, nsteps=20)
    got, gg = b.populations(1, thermal=True)
    ref = pair.oracle_dev()
    assert np.abs(got.cpu().numpy() - ref).max() / np.abs(ref).max() < 8 * 2.0 ** -24 * 8 * 20
    gref = np.transpose(pair.g, (2, 0, 1)) - c.T0 / 5.0
    assert np.abs(gg.cpu().numpy() - gref).max() / np.abs(gref).max() < 8 * 2.0 ** -24 * 8 * 20

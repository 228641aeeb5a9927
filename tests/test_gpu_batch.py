"""Ragged batched stepping (persistent tile-table kernel, HIP graph replay, autotuned
schedule): bitwise equal to stepping each domain alone, and oracle-matching."""
import numpy as np
import pytest
import torch

from paper_1311_7239_amd import inputs as I
from paper_1311_7239_amd import lbm
from tests.gpu_cases import Pair

pytestmark = pytest.mark.gpu


def mixed_cases():
    sizes = [(70, 70), (130, 90), (64, 64), (300, 33), (257, 129)]
    cases = []
    for k, (nx, ny) in enumerate(sizes):
        c = I.lid_cavity(n=max(nx, ny), Re=20.0 + 30 * k, heterogeneous=(k % 2 == 1), ell=6.0, seed=10 + k)
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


@pytest.mark.parametrize("storage", [lbm.FP32_DEV, lbm.FP16_DEV])
@pytest.mark.parametrize("tblock", [1, 2])
def test_batch_is_bitwise_equal_to_single_domains(storage, tblock, tmp_path):
    """One and two cycles per pass, graph replays of 4 cycles, leftovers."""
    cases = mixed_cases()
    b = lbm.batch_for_cases(cases, storage=storage, tune_cache=tmp_path / "tune.txt")
    b.set_time_blocking(tblock)
    b.set_graph_steps(4)
    done = 0
    for chunk in (1, 9, 3, 8):          # t = 0 cycle, graph replays, leftovers
        b.step(chunk)
        done += chunk
        for k in range(len(cases)):
            _, u = b.macroscopic(k)      # eager work between replays
            torch.cuda.synchronize()
            got = b.populations(k).cpu().numpy()
            assert np.array_equal(got, single_run(cases[k], done, storage)), (k, done)


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
    assert len(text) == 1 and len(text[0].split()) == 9
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
    c = I.natural_convection(n=32)
    with pytest.raises(lbm.LBMError) as e:
        lbm.batch_for_cases([c])
    assert e.value.status == lbm.ENOTSUP

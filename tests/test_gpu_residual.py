"""The steady residual of lbm_reduce, r = ||u(t) - u(t-1)||_2 / ||u(t)||_2, takes u(t-1)
from the two planes that the last pass of each lbm_step call writes from its last
collision. It equals its definition from two velocity snapshots, and it is bitwise the
same whichever number of cycles per pass, graph replay or batch ran the steps."""
import math

import numpy as np
import pytest
import torch

from paper_1311_7239_amd import inputs as I
from paper_1311_7239_amd import lbm
from tests.test_gpu_batch import mixed_cases
from tests.test_gpu_timeblock import cases as tb_cases

pytestmark = pytest.mark.gpu

CHUNKS = (1, 7, 10, 2, 5, 19, 4, 3)   # every remainder modulo 2 and 3, graph replays, leftovers


def _u(s, k=None):
    _, u, _ = s.macroscopic() if k is None else s.macroscopic(k)
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.float64)


def _definition(u1, u0):
    return math.sqrt(np.sum((u1 - u0) ** 2)) / math.sqrt(np.sum(u1 ** 2))


@pytest.mark.parametrize("storage", [lbm.FP32_DEV, lbm.FP16_DEV])
@pytest.mark.parametrize("name", ["cavity_300x37_grf", "periodic_70x70", "lognormal_200x130"])
def test_residual_is_bitwise_the_same_for_every_pass_length(name, storage):
    case = dict(tb_cases())[name]
    df0 = I.random_deviation_state(case.ny, case.nx, 1e-3, seed=6)
    runs = []
    for tblock, graph in ((1, 0), (2, 0), (3, 0), (3, 8), (2, 8)):
        s = lbm.solver_for_case(case, storage=storage)
        s.set_time_blocking(tblock)
        s.set_graph_steps(graph)
        s.set_populations(torch.from_numpy(df0).cuda())
        out = []
        for chunk in CHUNKS:
            s.step(chunk)
            mass, res, st = s.reduce()
            assert st == lbm.OK
            out.append((mass, res))
        runs.append(out)
    for k in range(1, len(runs)):
        assert runs[k] == runs[0], k


@pytest.mark.parametrize("tblock", [1, 2, 3])
def test_residual_equals_its_definition(tblock):
    """u(t - 1) and u(t) from the macroscopic output of two contexts one step apart; the
    recorded plane gives the same residual to FP64 summation-order rounding."""
    case = I.lognormal_channel(n=200, seed=8, ell=10.0, K_ref=40.0, drive=0.05)
    a = lbm.solver_for_case(case)
    b = lbm.solver_for_case(case)
    for s in (a, b):
        s.set_time_blocking(tblock)
    for t in (1, 2, 3, 4, 11, 30):
        a.step(t - a.time)
        b.step(t - 1 - b.time)
        _, res, _ = a.reduce()
        ref = _definition(_u(a), _u(b))
        assert abs(res / ref - 1.0) < 1e-12, (t, res, ref)


@pytest.mark.parametrize("tblock", [1, 2, 3])
def test_thermal_residual_is_bitwise_the_same_for_every_pass_length(tblock):
    case = I.natural_convection(n=96)
    ref = lbm.solver_for_case(case)
    ref.set_time_blocking(1)
    s = lbm.solver_for_case(case)
    s.set_time_blocking(tblock)
    for chunk in CHUNKS:
        ref.step(chunk)
        s.step(chunk)
        assert s.reduce() == ref.reduce(), chunk


@pytest.mark.parametrize("tblock", [1, 2, 3])
def test_batch_residual_equals_single_domains(tblock, tmp_path):
    cases = mixed_cases()
    b = lbm.batch_for_cases(cases, tune_cache=tmp_path / "tune.txt")
    b.set_time_blocking(tblock)
    b.set_graph_steps(6)
    singles = [lbm.solver_for_case(c) for c in cases]
    for chunk in (1, 9, 3, 8, 13):
        b.step(chunk)
        for k, s in enumerate(singles):
            s.step(chunk)
            assert b.reduce(k) == s.reduce(), (k, chunk)


def test_on_node_wall_residual_equals_its_definition():
    case = I.lid_cavity(n=64, nee=True, Re=50.0)
    a = lbm.solver_for_case(case)
    b = lbm.solver_for_case(case)
    for t in (1, 2, 9, 40):
        a.step(t - a.time)
        b.step(t - 1 - b.time)
        _, res, _ = a.reduce()
        ref = _definition(_u(a), _u(b))
        assert abs(res / ref - 1.0) < 1e-12, (t, res, ref)


def test_residual_is_nan_at_t0_and_after_a_new_state():
    case = I.lid_cavity(n=64)
    s = lbm.solver_for_case(case)
    _, res, _ = s.reduce()
    assert math.isnan(res)
    s.step(5)
    _, res, _ = s.reduce()
    assert math.isfinite(res)
    s.set_populations(torch.zeros((8, 64, 64), device="cuda"))
    _, res, _ = s.reduce()
    assert math.isnan(res)

"""lbm_reduce_static, the variant of lbm_reduce for callers that cannot allocate device
memory (its partial sums live in a static device array of the library instead of the
context's workspace), against lbm_reduce through the C ABI: bit for bit, on two calls in a
row, the second on a smaller domain, and on a batch domain."""
import pytest

from paper_1311_7239_amd import inputs as I
from paper_1311_7239_amd import lbm

pytestmark = pytest.mark.gpu


def test_static_scratch_reduce_equals_workspace_reduce():
    for n, steps in ((1536, 37), (96, 11)):      # the second call on a smaller input
        case = I.lognormal_channel(n=n, seed=3, ell=8.0, K_ref=30.0, drive=0.05)
        s = lbm.solver_for_case(case)
        s.step(steps)
        ref = s.reduce()
        got = s.reduce_static()
        assert got == ref, (n, got, ref)
        assert got[2] == lbm.OK


def test_static_scratch_reduce_at_t0_and_on_a_batch_domain(tmp_path):
    import math
    case = I.lid_cavity(n=64)
    s = lbm.solver_for_case(case)
    m, r, st = s.reduce_static()
    assert math.isnan(r) and st == lbm.OK and m == s.reduce()[0]
    cases = [I.lid_cavity(n=80, Re=30.0), I.lid_cavity(n=48, Re=60.0)]
    b = lbm.batch_for_cases(cases, tune_cache=tmp_path / "tune.txt")
    b.step(9)
    for k in (1, 0):
        mm = lbm.ctypes.c_double(); rr = lbm.ctypes.c_double()
        st = lbm.lib().lbm_reduce_static(b._ctx, k, lbm.ctypes.byref(mm), lbm.ctypes.byref(rr))
        assert st == lbm.OK
        assert (mm.value, rr.value, st) == b.reduce(k)

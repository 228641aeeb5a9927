"""FP16-deviation storage (binary16, round-to-nearest-even, subnormals kept; FP32 math)."""
import numpy as np
import pytest
import torch

from paper_1311_7239_amd import inputs as I
from paper_1311_7239_amd import lbm
from tests.gpu_cases import Pair, max_rel_velocity_error

pytestmark = pytest.mark.gpu


def ulp16(x):
    a = np.abs(np.asarray(x, dtype=np.float64))
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -14)))
    return 2.0 ** (e - 10)


def test_storage_rounds_to_nearest_even_and_keeps_subnormals():
    case = I.lid_cavity(n=64)
    s = lbm.solver_for_case(case, storage=lbm.FP16_DEV)
    rng = np.random.default_rng(5)
    df = (rng.standard_normal((8, 64, 64)) * 10.0 ** rng.uniform(-8, -1, (8, 64, 64))).astype(np.float32)
    s.set_populations(torch.from_numpy(df).cuda())
    got, _ = s.populations()
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), df.astype(np.float16).astype(np.float32))
    assert np.count_nonzero(np.abs(df.astype(np.float16)) < 2.0 ** -14) > 100   # subnormals present


@pytest.mark.parametrize("kind", ["cavity", "channel"])
def test_one_step_error_is_one_fp16_rounding(kind):
    nx, ny = 1100, 45
    if kind == "cavity":
        case = I.lid_cavity(n=nx)
        case.ny = ny
    else:
        case = I.poiseuille_channel(ny=ny, nx=nx)
        case.ax = 1e-5
    df0 = I.random_deviation_state(ny, nx, 1e-3, seed=17)
    pair = Pair(case, storage=lbm.FP16_DEV, df0=df0)
    pair.step(1)
    ref = pair.oracle_dev()
    got, _ = pair.gpu_dev()
    bound = 0.5 * ulp16(ref) + 4e-6 * np.abs(ref).max()
    assert np.all(np.abs(got - ref) <= bound)


def test_fp16_error_budget_lid_cavity():
    """Stated, not a parity bar: FP16-deviation storage on the 128^2 porous lid cavity
    after 4000 steps against FP64 (max relative velocity error printed)."""
    case = I.lid_cavity(n=128)
    pair = Pair(case, storage=lbm.FP16_DEV, nthreads=8)
    pair.step(4000)
    _, u, _ = pair.gpu_macro()
    ux, uy, _, _ = pair.oracle_macro()
    err = max_rel_velocity_error(u, ux, uy)
    print(f"FP16 storage, 128^2 lid cavity, 4000 steps: max rel velocity error {err:.3e}")
    assert err < 5e-3

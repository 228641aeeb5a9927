"""The sampled full-size parity checks run the oracle on a window of radius R around each
sampled node instead of the whole domain. This checks on the CPU that a window of radius
T + 1 reproduces the whole-domain oracle at its centre node after T steps, at walls, at the
periodic seam and in the interior."""
import numpy as np

import oracle
from paper_1311_7239_amd import inputs as I
from tests.gpu_cases import f_ref, oracle_window
from tests.oracle_cases import oracle_setup


def test_window_reproduces_whole_domain():
    n, T = 48, 4
    case = I.lognormal_channel(n=n, seed=9, ell=4.0, K_ref=1e-6 * 2048.0 ** 2)
    df0 = I.random_deviation_state(n, n, 1e-3, seed=19)
    p, phi, K, F = oracle_setup(case, nthreads=2)
    full = np.ascontiguousarray(np.transpose(df0.astype(np.float64), (1, 2, 0)) + f_ref(case.Pi0))
    oracle.run(p, phi, K, F, full, nsteps=T)
    for x, y in [(0, 0), (n - 1, n - 1), (3, 1), (20, n - 3), (n - 2, 24), (17, 30)]:
        sub, dfw, cx, cy = oracle_window(case, df0, x, y, T + 1)
        ps, phis, Ks, Fs = oracle_setup(sub, nthreads=1)
        f = np.ascontiguousarray(np.transpose(dfw, (1, 2, 0)) + f_ref(case.Pi0))
        oracle.run(ps, phis, Ks, Fs, f, nsteps=T)
        np.testing.assert_array_equal(f[cy, cx], full[y, x])

"""Turn a seeded input Case into oracle arguments (test helper; float64 throughout)."""
import numpy as np

import oracle


def oracle_setup(case, nthreads=0):
    p = oracle.make_params(case.nx, case.ny, bc_x=case.bc_x, bc_y=case.bc_y, lid_ux=case.lid_ux,
                           nu=case.nu, J=case.J, ax=case.ax, ay=case.ay, thermal=case.thermal,
                           sigma=case.sigma, tau_T=case.tau_T, Th=case.Th, Tc=case.Tc,
                           T0=case.T0, gbeta=case.gbeta, nthreads=nthreads,
                           Jcell=getattr(case, "Jfield", None))
    shape = (case.ny, case.nx)
    if case.phi is None:
        phi = np.full(shape, case.phi0, dtype=np.float64)
        K = np.full(shape, case.K0, dtype=np.float64)
        if case.Fphi is None:
            _, F = oracle.ergun(phi, 1.0)
        else:
            F = np.full(shape, case.Fphi, dtype=np.float64)
    elif getattr(case, "kappa", None) is not None:
        phi = case.phi.astype(np.float64)
        kap = case.kappa.astype(np.float64)
        with np.errstate(divide="ignore"):
            K = np.where(kap > 0.0, 1.0 / kap, np.inf)
        if case.Fphi is None:
            _, F = oracle.ergun(phi, 1.0)
        else:
            F = np.full(shape, case.Fphi, dtype=np.float64)
    else:
        phi = case.phi.astype(np.float64)
        K, F = oracle.ergun(phi, case.dp)
        if case.Fphi is not None:
            F = np.full(shape, case.Fphi, dtype=np.float64)
    return p, phi, K, F


def uniform_F(case):
    """F_phi of a uniform-medium case: the constant it fixes, or else the oracle's own
    Eq. (4) at its porosity (the closed forms of Sec. 3 take it as a parameter)."""
    if case.Fphi is not None:
        return float(case.Fphi)
    _, F = oracle.ergun(np.array([case.phi0], dtype=np.float64), 1.0)
    return float(F[0])


def run_to_steady(p, phi, K, F, f, tol=1e-10, every=100, max_steps=5_000_000):
    """Run until r(t) = ||u(t) - u(t-1)|| / ||u(t)|| < tol, checked every `every` steps."""
    t = 0
    while t < max_steps:
        oracle.run(p, phi, K, F, f, nsteps=every - 1)
        ux0, uy0, _, _ = oracle.macroscopic(p, phi, K, F, f)
        oracle.run(p, phi, K, F, f, nsteps=1)
        ux, uy, _, _ = oracle.macroscopic(p, phi, K, F, f)
        t += every
        # a flow that stays exactly at rest is steady too (r is 0/0 there)
        still = not np.any(ux - ux0) and not np.any(uy - uy0)
        if still or oracle.residual((ux, uy), (ux0, uy0)) < tol:
            return t, ux, uy
    raise RuntimeError("no steady state within max_steps")

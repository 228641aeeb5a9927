"""Seeded synthetic inputs for the porous MRT-LB workloads.

This module is shared by the GPU library's tests and benchmark and by the
FP64 oracle's tests. It holds no step arithmetic of the scheme: it draws
random fields and parameters from seeds and converts the dimensionless
groups of the paper (Da, Re, Ra, Pr, Ma; Eqs. 5, 21, 24, 26) into lattice
parameters. Each implementation derives relaxation rates, per-cell drag
coefficients and everything else from these parameters on its own.

Random numbers come from NumPy's PCG64 (``numpy.random.default_rng(seed)``);
fields are generated in float64 and rounded once to float32, and the same
float32 values feed both the GPU path and the oracle.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

PERIODIC = 0
WALLS = 1   # halfway bounce-back: walls half a link outside the edge nodes, L = n
NEE = 2     # on-node walls (non-equilibrium extrapolation): L = n - 1


@dataclasses.dataclass
class Case:
    """One lattice problem in lattice units (delta_x = delta_t = rho0 = 1)."""
    name: str
    nx: int
    ny: int
    bc_x: int
    bc_y: int
    nu: float                    # fluid viscosity; tau = 1/2 + 3 J nu (Eq. 21)
    J: float = 1.0
    lid_ux: float = 0.0
    ax: float = 0.0
    ay: float = 0.0
    phi0: float = 1.0            # uniform porosity (used when phi is None)
    K0: float = math.inf         # uniform permeability (used when phi is None)
    phi: Optional[np.ndarray] = None   # float32 [ny, nx] porosity field
    dp: Optional[float] = None   # particle diameter for Eq. (4) when phi varies
    Fphi: Optional[float] = None  # constant F_phi, or None: F_phi from Eq. (4) at the
                                  # cell's porosity, evaluated by each side itself
    kappa: Optional[np.ndarray] = None  # float32 [ny, nx] 1/K plane (0 = free fluid); with phi
    Jfield: Optional[np.ndarray] = None  # float32 [ny, nx] per-node viscosity ratio
    Pi0: float = 1.0             # rest value of phi*p (initial state)
    steps: int = 0
    thermal: bool = False
    sigma: float = 1.0
    tau_T: float = 1.0
    Th: float = 0.0
    Tc: float = 0.0
    T0: float = 0.0
    gbeta: float = 0.0
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny

    def phi_field(self) -> np.ndarray:
        if self.phi is not None:
            return self.phi
        return np.full((self.ny, self.nx), self.phi0, dtype=np.float32)


def ergun_dp(K_ref: float, phi_ref: float) -> float:
    """Particle diameter d_p at which Ergun's permeability (Eq. 4) equals K_ref at
    porosity phi_ref: the input parameter of heterogeneous fields, which keep d_p
    fixed. Neither side uses this to compute K or F_phi: the GPU library and the
    oracle each evaluate Eq. (4) from (phi, d_p) themselves."""
    return math.sqrt(150.0 * K_ref * (1.0 - phi_ref) ** 2 / phi_ref ** 3)


def grf(ny: int, nx: int, ell: float, seed: int) -> np.ndarray:
    """Periodic Gaussian random field with squared-exponential covariance
    exp(-r^2 / (2 ell^2)), FFT-synthesised from white noise and normalised to
    sample mean 0 and variance 1."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((ny, nx))
    ky = np.fft.fftfreq(ny) * 2.0 * np.pi
    kx = np.fft.rfftfreq(nx) * 2.0 * np.pi
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    amp = np.exp(-0.25 * k2 * ell * ell)   # sqrt of the Gaussian spectrum
    g = np.fft.irfft2(np.fft.rfft2(w) * amp, s=(ny, nx))
    g -= g.mean()
    g /= g.std()
    return g


# ------------------------------------------------------------------ workloads

def poiseuille_channel(ny: int = 64, nx: int = 8, phi: float = 0.1, Da: float = 1e-2,
                       Re: float = 0.01, tau: float = 0.6, J: float = 1.0,
                       forchheimer: bool = True, nee: bool = False) -> Case:
    """Porous Poiseuille channel (Sec. 3.1): x periodic, walls at y = 0 and y = L
    (L = ny with bounce-back walls, ny - 1 with on-node NEE walls), K = Da L^2;
    a_x chosen so that the Brinkman centreline velocity of Eq. (24) equals
    u0 = Re nu / L."""
    L = float(ny - 1 if nee else ny)
    nu = (tau - 0.5) / (3.0 * J)
    K = Da * L * L
    u0 = Re * nu / L
    th = math.sqrt(phi * nu / (K * J * nu))
    ax = u0 * nu / (K * (1.0 - 1.0 / math.cosh(0.5 * th * L)))
    return Case(name=f"poiseuille_{nx}x{ny}" + ("_nee" if nee else ""), nx=nx, ny=ny,
                bc_x=PERIODIC, bc_y=NEE if nee else WALLS, nu=nu, J=J, ax=ax, phi0=phi, K0=K, Fphi=None if forchheimer else 0.0,
                Pi0=phi, meta=dict(L=L, u0=u0, Da=Da, Re=Re))


def partial_couette(J: float = 4.0, ny: int = 80, nx: int = 2, phi: float = 0.1,
                    Da: float = 1e-3, Re: float = 0.01, nu: float = 0.16) -> Case:
    """Couette flow in a channel partially filled with a porous layer (Sec. 3.2,
    Eq. 25): nodes with (y + 1/2)/L <= 1/2 are porous (porosity phi, K = Da L^2,
    viscosity ratio J), the rest free fluid (phi = 1, no matrix, J = 1);
    F_phi = 0, moving lid u0 = Re nu / L, L = ny."""
    L = float(ny)
    u0 = Re * nu / L
    porous = ((np.arange(ny) + 0.5) / L <= 0.5)[:, None] & np.ones((1, nx), dtype=bool)
    phif = np.where(porous, phi, 1.0).astype(np.float32)
    kap = np.where(porous, 1.0 / (Da * L * L), 0.0).astype(np.float32)
    Jf = np.where(porous, J, 1.0).astype(np.float32)
    return Case(name=f"partial_couette_J{J:g}_{nx}x{ny}", nx=nx, ny=ny, bc_x=PERIODIC,
                bc_y=WALLS, nu=nu, J=1.0, lid_ux=u0, phi=phif, kappa=kap, Fphi=0.0,
                Jfield=Jf, Pi0=1.0, meta=dict(L=L, u0=u0, Da=Da, Re=Re, phi_p=phi, J_p=J))


def couette_channel(ny: int = 64, nx: int = 2, phi: float = 0.1, Da: float = 1e-2,
                    Re: float = 0.01, nu: float = 0.1, J: float = 1.0, nee: bool = False) -> Case:
    """Porous Couette flow (Sec. 3.2) with F_phi = 0: moving top wall, u0 = Re nu / L
    (L = ny, or ny - 1 with on-node NEE walls)."""
    L = float(ny - 1 if nee else ny)
    u0 = Re * nu / L
    return Case(name=f"couette_{nx}x{ny}" + ("_nee" if nee else ""), nx=nx, ny=ny, bc_x=PERIODIC,
                bc_y=NEE if nee else WALLS, nu=nu,
                J=J, lid_ux=u0, phi0=phi, K0=Da * L * L, Fphi=0.0, Pi0=phi,
                meta=dict(L=L, u0=u0, Da=Da, Re=Re))


def lid_cavity(n: int = 512, phi: float = 0.4, Da: float = 1e-2, Re: float = 100.0,
               U: float = 0.1, heterogeneous: bool = False, seed: int = 2,
               ell: float = 32.0, steps: int = 50_000, nee: bool = False) -> Case:
    """Lid-driven porous cavity (Sec. 3.3 setting): walls all round, top wall moving at U,
    nu = U L / Re, K = Da L^2 (L = n, or n - 1 with on-node NEE walls). The
    heterogeneous variant draws phi = clip(phi + 0.1 G, 0.2, 0.9) from a GRF G
    (correlation length ell) and keeps a fixed particle diameter, so that K(phi)
    follows Eq. (4) through K(phi) = Da L^2."""
    L = float(n - 1 if nee else n)
    nu = U * L / Re
    K = Da * L * L
    bc = NEE if nee else WALLS
    case = Case(name=f"cavity_{n}" + ("_nee" if nee else ""), nx=n, ny=n, bc_x=bc, bc_y=bc, nu=nu, lid_ux=U,
                phi0=phi, K0=K, Fphi=None, Pi0=phi, steps=steps,
                meta=dict(L=L, Da=Da, Re=Re, U=U))
    if heterogeneous:
        G = grf(n, n, ell, seed)
        field = np.clip(phi + 0.1 * G, 0.2, 0.9).astype(np.float32)
        case.name = f"cavity_{n}_grf"
        case.phi = field
        case.dp = ergun_dp(K, phi)
        case.Fphi = None
        case.Pi0 = float(np.mean(field, dtype=np.float64))
        case.meta.update(seed=seed, ell=ell)
    return case


def natural_convection(n: int = 1024, phi: float = 0.6, Da: float = 1e-4, Ra: float = 1e5,
                       Pr: float = 1.0, Ma: float = 0.1, J: float = 1.0, sigma: float = 1.0,
                       gamma: float = 1.0, Th: float = 21.0, Tc: float = 1.0,
                       steps: int = 2000, nee: bool = False) -> Case:
    """Natural convection in a porous square cavity (Sec. 3.4): no-slip walls, hot wall
    x = 0, cold wall x = L, adiabatic top and bottom (L = n, or n - 1 with on-node
    NEE walls). Relaxation times from Eq. (26) with c_sT^2 = 2/5 (varpi = 0), the
    viscosity from Eq. (21), g*beta from the definition of Ra."""
    L = float(n - 1 if nee else n)
    tau_v = 0.5 + Ma * J * L * math.sqrt(3.0 * Pr) / math.sqrt(Ra)
    nu_e = (tau_v - 0.5) / 3.0
    nu = nu_e / J
    csT2 = 0.4
    tau_T = 0.5 + gamma * (tau_v - 0.5) / 3.0 / (J * sigma * csT2 * Pr)
    dT = Th - Tc
    gbeta = Ra * nu * nu / (dT * L ** 3 * Pr)
    bc = NEE if nee else WALLS
    return Case(name=f"convection_{n}" + ("_nee" if nee else ""), nx=n, ny=n, bc_x=bc, bc_y=bc,
                nu=nu, J=J,
                phi0=phi, K0=Da * L * L, Fphi=None, Pi0=phi, steps=steps,
                thermal=True, sigma=sigma, tau_T=tau_T, Th=Th, Tc=Tc, T0=0.5 * (Th + Tc),
                gbeta=gbeta, meta=dict(L=L, Da=Da, Ra=Ra, Pr=Pr, Ma=Ma, tau_v=tau_v))


def cavity_batch(count: int = 256, seed: int = 4, nmin: int = 64, nmax: int = 768,
                 U: float = 0.1) -> list:
    """Ragged batch of lid-driven porous cavities: N ~ U{nmin..nmax},
    phi ~ U[0.3, 0.9], log10 Da ~ U[-4, -1], Re ~ U[1, 400], lid speed U."""
    rng = np.random.default_rng(seed)
    N = rng.integers(nmin, nmax + 1, size=count)
    phis = rng.uniform(0.3, 0.9, size=count)
    lDa = rng.uniform(-4.0, -1.0, size=count)
    Re = rng.uniform(1.0, 400.0, size=count)
    cases = []
    for k in range(count):
        n = int(N[k]); L = float(n)
        nu = U * L / float(Re[k])
        K = 10.0 ** float(lDa[k]) * L * L
        cases.append(Case(name=f"batch{k}_{n}", nx=n, ny=n, bc_x=WALLS, bc_y=WALLS, nu=nu,
                          lid_ux=U, phi0=float(phis[k]), K0=K, Fphi=None,
                          Pi0=float(phis[k]),
                          meta=dict(L=L, Da=10.0 ** float(lDa[k]), Re=float(Re[k]))))
    return cases


def lognormal_channel(n: int = 2048, seed: int = 5, ell: float = 64.0, Da_ref: float = 1e-6,
                      phi_ref: float = 0.4, tau: float = 0.8, drive: float = 0.01,
                      steps: int = 4000, K_ref: Optional[float] = None) -> Case:
    """Channel through a log-normal porous field: x periodic, walls in y,
    phi = clip(phi_ref exp(0.5 G - 0.125), 0.05, 0.95) for a GRF G, Eq. (4) with
    a fixed particle diameter so that K(phi_ref) = K_ref (default Da_ref L^2),
    driven by a_x = drive * nu / K_ref."""
    L = float(n)
    nu = (tau - 0.5) / 3.0
    if K_ref is None:
        K_ref = Da_ref * L * L
    G = grf(n, n, ell, seed)
    field = np.clip(phi_ref * np.exp(0.5 * G - 0.125), 0.05, 0.95).astype(np.float32)
    return Case(name=f"lognormal_channel_{n}_s{seed}", nx=n, ny=n, bc_x=PERIODIC, bc_y=WALLS,
                nu=nu, ax=drive * nu / K_ref, phi0=phi_ref, phi=field,
                dp=ergun_dp(K_ref, phi_ref), Fphi=None,
                Pi0=float(np.mean(field, dtype=np.float64)), steps=steps,
                meta=dict(L=L, K_ref=K_ref, seed=seed, ell=ell))


def random_deviation_state(ny: int, nx: int, scale: float, seed: int, channels: int = 8) -> np.ndarray:
    """Seeded random population deviations, float32 [channels, ny, nx], uniform in
    [-scale, scale] (a state to start a single-step comparison from)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=(channels, ny, nx)).astype(np.float32)

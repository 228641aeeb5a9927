"""FP64 CPU oracle for the D2Q8 porous MRT-LB scheme of Liu & He (arXiv:1311.7239).

TEST INFRASTRUCTURE ONLY. The tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it as the reference the GPU library
is checked against; the product library never imports, links or calls it.

The arithmetic lives in ``mrt_oracle.c`` (plain C, double precision, the
paper's equations in the paper's order, push streaming); this module only
builds it with gcc, loads it with ctypes and marshals numpy arrays.
Array layouts: populations ``f[ny, nx, 8]`` (the paper's f_1..f_8, Eq. 7
ordering), thermal populations ``g[ny, nx, 5]`` (Eq. B.3 ordering), scalar
fields ``[ny, nx]``.
"""
from __future__ import annotations

import ctypes
import os
import pathlib
import subprocess

import numpy as np

_HERE = pathlib.Path(__file__).resolve().parent
_SRC = _HERE / "mrt_oracle.c"
_LIB_PATH = _HERE / "liboracle.so"
_lib = None

PERIODIC = 0
WALLS = 1
NEE = 2


def build(force: bool = True) -> pathlib.Path:
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math, no FMA contraction)."""
    if not force and _LIB_PATH.exists():
        return _LIB_PATH
    tmp = _LIB_PATH.with_suffix(".so.tmp")
    cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-o", str(tmp), str(_SRC), "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int),
        ("lid_ux", ctypes.c_double), ("rho0", ctypes.c_double),
        ("nu", ctypes.c_double), ("J", ctypes.c_double),
        ("s_e", ctypes.c_double), ("s_q", ctypes.c_double),
        ("alpha2", ctypes.c_double), ("c1", ctypes.c_double), ("c2", ctypes.c_double),
        ("gamma1", ctypes.c_double), ("gamma2", ctypes.c_double), ("gamma3", ctypes.c_double),
        ("ax", ctypes.c_double), ("ay", ctypes.c_double),
        ("thermal", ctypes.c_int),
        ("sigma", ctypes.c_double), ("tau_T", ctypes.c_double),
        ("zeta3", ctypes.c_double), ("zeta4", ctypes.c_double), ("varpi", ctypes.c_double),
        ("Th", ctypes.c_double), ("Tc", ctypes.c_double), ("T0", ctypes.c_double),
        ("gbeta", ctypes.c_double),
        ("nthreads", ctypes.c_int),
        ("Jcell", ctypes.POINTER(ctypes.c_double)),
    ]


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_P = ctypes.POINTER(Params)


def lib():
    """Load the compiled oracle (building it if it is not there yet)."""
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            build()
        L = ctypes.CDLL(str(_LIB_PATH))
        L.orc_default_params.argtypes = [_P]
        L.orc_flow_matrices.argtypes = [_D, _D]
        L.orc_thermal_matrices.argtypes = [_D, _D]
        L.orc_velocities.argtypes = [_I, _I]
        L.orc_ergun.argtypes = [ctypes.c_long, _D, ctypes.c_double, _D, _D]
        L.orc_equilibrium_moments.argtypes = [_P, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double, _D]
        L.orc_forcing_moments.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, _D]
        L.orc_velocity.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, _D, _D, _D]
        L.orc_pressure.argtypes = [_P, ctypes.c_double, _D, ctypes.c_double, ctypes.c_double]
        L.orc_pressure.restype = ctypes.c_double
        L.orc_collide_node.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, _D, _D, _D, _D]
        L.orc_step.argtypes = [_P, _D, _D, _D, _D, _D, _D, _D]
        L.orc_run.argtypes = [_P, _D, _D, _D, _D, _D, ctypes.c_long]
        L.orc_run.restype = ctypes.c_int
        L.orc_macroscopic.argtypes = [_P, _D, _D, _D, _D, _D, _D, _D, _D, _D]
        L.orc_rest_state.argtypes = [_P, ctypes.c_long, ctypes.c_double, _D]
        L.orc_thermal_rest_state.argtypes = [_P, ctypes.c_long, _D, _D]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = np.broadcast_to(a, shape).copy()
    return a


def make_params(nx, ny, *, bc_x=PERIODIC, bc_y=WALLS, lid_ux=0.0, nu, J=1.0, ax=0.0, ay=0.0,
                thermal=False, sigma=1.0, tau_T=1.0, Th=0.0, Tc=0.0, T0=0.0, gbeta=0.0,
                nthreads=0, Jcell=None, **overrides) -> Params:
    """Paper defaults (Sec. 2.2, Sec. 3) plus the run's geometry and physics.
    Jcell: optional per-node viscosity ratio [ny, nx] (kept alive on the returned object)."""
    p = Params()
    lib().orc_default_params(ctypes.byref(p))
    p.nx, p.ny, p.bc_x, p.bc_y = int(nx), int(ny), int(bc_x), int(bc_y)
    p.lid_ux, p.nu, p.J, p.ax, p.ay = lid_ux, nu, J, ax, ay
    p.thermal = 1 if thermal else 0
    p.sigma, p.tau_T, p.Th, p.Tc, p.T0, p.gbeta = sigma, tau_T, Th, Tc, T0, gbeta
    p.nthreads = int(nthreads)
    if Jcell is not None:
        arr = np.ascontiguousarray(np.broadcast_to(np.asarray(Jcell, dtype=np.float64), (int(ny), int(nx))))
        p._jcell = arr
        p.Jcell = arr.ctypes.data_as(_D)
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


# ----------------------------------------------------------------- pieces

def flow_matrices():
    M = np.zeros(64); Minv = np.zeros(64)
    lib().orc_flow_matrices(_ptr(M), _ptr(Minv))
    return M.reshape(8, 8), Minv.reshape(8, 8)


def thermal_matrices():
    N = np.zeros(25); Ninv = np.zeros(25)
    lib().orc_thermal_matrices(_ptr(N), _ptr(Ninv))
    return N.reshape(5, 5), Ninv.reshape(5, 5)


def velocities():
    ex = (ctypes.c_int * 8)(); ey = (ctypes.c_int * 8)()
    lib().orc_velocities(ex, ey)
    return np.array(list(ex)), np.array(list(ey))


def ergun(phi, dp):
    """Eq. (4): permeability K and geometric function F_phi per cell."""
    phi = _f64(phi)
    K = np.empty_like(phi); F = np.empty_like(phi)
    lib().orc_ergun(phi.size, _ptr(phi), float(dp), _ptr(K), _ptr(F))
    return K, F


def equilibrium_moments(p: Params, phi, pres, ux, uy):
    out = np.zeros(8)
    lib().orc_equilibrium_moments(ctypes.byref(p), phi, pres, ux, uy, _ptr(out))
    return out


def forcing_moments(p: Params, phi, ux, uy, Fx, Fy):
    out = np.zeros(8)
    lib().orc_forcing_moments(ctypes.byref(p), phi, ux, uy, Fx, Fy, _ptr(out))
    return out


def velocity(p: Params, phi, K, Fphi, ax, ay, f):
    f = _f64(f); u = np.zeros(2); F = np.zeros(2)
    lib().orc_velocity(ctypes.byref(p), phi, K, Fphi, ax, ay, _ptr(f), _ptr(u), _ptr(F))
    return u, F


def pressure(p: Params, phi, f, ux, uy):
    f = _f64(f)
    return lib().orc_pressure(ctypes.byref(p), phi, _ptr(f), ux, uy)


def collide_node(p: Params, phi, K, Fphi, ax, ay, f):
    f = _f64(f); fp = np.zeros(8); u = np.zeros(2); pr = np.zeros(1)
    lib().orc_collide_node(ctypes.byref(p), phi, K, Fphi, ax, ay, _ptr(f), _ptr(fp),
                           _ptr(u), _ptr(pr))
    return fp, u, float(pr[0])


# ----------------------------------------------------------------- fields

def rest_state(p: Params, Pi0):
    f = np.zeros((p.ny, p.nx, 8))
    lib().orc_rest_state(ctypes.byref(p), p.nx * p.ny, float(Pi0), _ptr(f))
    return f


def thermal_rest_state(p: Params, T):
    T = _f64(T, (p.ny, p.nx))
    g = np.zeros((p.ny, p.nx, 5))
    lib().orc_thermal_rest_state(ctypes.byref(p), p.nx * p.ny, _ptr(T), _ptr(g))
    return g


def step(p: Params, phi, K, Fphi, f, g=None):
    shape = (p.ny, p.nx)
    phi, K, Fphi = _f64(phi, shape), _f64(K, shape), _f64(Fphi, shape)
    f = _f64(f); fn = np.empty_like(f)
    gn = None
    if g is not None:
        g = _f64(g); gn = np.empty_like(g)
    lib().orc_step(ctypes.byref(p), _ptr(phi), _ptr(K), _ptr(Fphi), _ptr(f), _ptr(fn),
                   _ptr(g), _ptr(gn))
    return fn, gn


def run(p: Params, phi, K, Fphi, f, g=None, nsteps=1):
    """Advance f (and g) by nsteps in place; arrays must be float64 C-contiguous."""
    shape = (p.ny, p.nx)
    phi, K, Fphi = _f64(phi, shape), _f64(K, shape), _f64(Fphi, shape)
    assert f.dtype == np.float64 and f.flags.c_contiguous and f.shape == (p.ny, p.nx, 8)
    if g is not None:
        assert g.dtype == np.float64 and g.flags.c_contiguous and g.shape == (p.ny, p.nx, 5)
    rc = lib().orc_run(ctypes.byref(p), _ptr(phi), _ptr(K), _ptr(Fphi), _ptr(f), _ptr(g),
                       int(nsteps))
    if rc != 0:
        raise MemoryError("oracle run: allocation failed")
    return f, g


def macroscopic(p: Params, phi, K, Fphi, f, g=None):
    """u_x, u_y (Eq. 18), p (Eq. 20) and T (Eq. B.5) at the current time."""
    shape = (p.ny, p.nx)
    phi, K, Fphi = _f64(phi, shape), _f64(K, shape), _f64(Fphi, shape)
    f = _f64(f)
    g = None if g is None else _f64(g)
    ux = np.empty(shape); uy = np.empty(shape); pr = np.empty(shape); T = np.zeros(shape)
    lib().orc_macroscopic(ctypes.byref(p), _ptr(phi), _ptr(K), _ptr(Fphi), _ptr(f), _ptr(g),
                          _ptr(ux), _ptr(uy), _ptr(pr), _ptr(T))
    return ux, uy, pr, T


def mass(f):
    """Total of all populations (sum of m_1 over nodes), in a fixed serial order."""
    return float(np.sum(np.asarray(f, dtype=np.float64).reshape(-1), dtype=np.float64))


def residual(u_now, u_prev):
    """||u(t) - u(t-1)||_2 / ||u(t)||_2 over all nodes and both components."""
    un = np.concatenate([np.ravel(a) for a in u_now])
    up = np.concatenate([np.ravel(a) for a in u_prev])
    den = np.sqrt(np.sum(un * un))
    return float(np.sqrt(np.sum((un - up) ** 2)) / den) if den > 0 else float("inf")

"""Python binding of the mrtlbm C ABI (include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libmrtlbm.so``. PyTorch provides device memory (the workspace and all
field tensors) and the HIP stream. There is no fallback: if the library is
not built, or no GPU is present, calls fail loudly.
"""
from __future__ import annotations

import ctypes
import math
import pathlib
from typing import Optional, Sequence

import torch

_LIB_PATH = pathlib.Path(__file__).resolve().parent / "libmrtlbm.so"
_lib = None

OK, EINVAL, ESTATE, EDEVICE, EUNSTABLE, ENOTSUP = 0, -1, -2, -3, -4, -5
PERIODIC, WALLS, WALLS_NEE = 0, 1, 2
FP32_DEV, FP16_DEV = 0, 1
MEDIUM_UNIFORM, MEDIUM_PHI_ERGUN, MEDIUM_PHI_KAPPA = 0, 1, 2


class LBMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status
        self.message = message


class Thermal(ctypes.Structure):
    _fields_ = [("enabled", ctypes.c_int32), ("tau_T", ctypes.c_double),
                ("sigma", ctypes.c_double), ("zeta3", ctypes.c_double),
                ("zeta4", ctypes.c_double), ("Th", ctypes.c_double), ("Tc", ctypes.c_double),
                ("T0", ctypes.c_double), ("g_beta", ctypes.c_double)]


class Desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
                ("lid_ux", ctypes.c_double), ("nu", ctypes.c_double), ("J", ctypes.c_double),
                ("s_e", ctypes.c_double), ("s_q", ctypes.c_double),
                ("medium", ctypes.c_int32), ("phi0", ctypes.c_double),
                ("kappa0", ctypes.c_double), ("dp", ctypes.c_double),
                ("F_eps", ctypes.c_double), ("ax", ctypes.c_double), ("ay", ctypes.c_double),
                ("Pi0", ctypes.c_double), ("storage", ctypes.c_int32),
                ("ckpt_every", ctypes.c_int32), ("j_plane", ctypes.c_int32),
                ("thermal", Thermal)]


_vp = ctypes.c_void_p
_DP = ctypes.POINTER(Desc)


def lib():
    """Load libmrtlbm.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            raise RuntimeError(f"{_LIB_PATH} is not built; run paper_1311_7239_amd.build.build()")
        L = ctypes.CDLL(str(_LIB_PATH))
        L.lbm_desc_defaults.argtypes = [_DP]
        L.lbm_workspace_size.argtypes = [_DP, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
        L.lbm_create.argtypes = [_DP, _vp, _vp, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]
        L.lbm_batch_workspace_size.argtypes = [ctypes.c_int32, _DP, ctypes.POINTER(ctypes.c_size_t)]
        L.lbm_create_batch.argtypes = [ctypes.c_int32, _DP, ctypes.POINTER(_vp),
                                       ctypes.POINTER(_vp), _vp, ctypes.c_size_t, _vp,
                                       ctypes.c_char_p, ctypes.POINTER(_vp)]
        L.lbm_step.argtypes = [_vp, ctypes.c_int64]
        L.lbm_time.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64)]
        L.lbm_macroscopic.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp]
        L.lbm_get_populations.argtypes = [_vp, ctypes.c_int32, _vp, _vp]
        L.lbm_set_populations.argtypes = [_vp, ctypes.c_int32, _vp, _vp]
        L.lbm_reduce.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)]
        L.lbm_reduce_static.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]
        L.lbm_backward.argtypes = [_vp, _vp, _vp, _vp]
        L.lbm_backward_params.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)]
        L.lbm_tangent.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_double), _vp]
        L.lbm_state_bytes.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
        L.lbm_save.argtypes = [_vp, _vp, ctypes.c_size_t]
        L.lbm_load.argtypes = [_vp, _vp, ctypes.c_size_t]
        L.lbm_destroy.argtypes = [_vp]
        L.lbm_strerror.argtypes = [ctypes.c_int]
        L.lbm_strerror.restype = ctypes.c_char_p
        L.lbm_last_error.restype = ctypes.c_char_p
        L.lbm_schedule.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.lbm_set_schedule.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32]
        L.lbm_set_graph_steps.argtypes = [_vp, ctypes.c_int32]
        L.lbm_set_viscosity_ratio.argtypes = [_vp, ctypes.c_int32, _vp]
        L.lbm_set_time_blocking.argtypes = [_vp, ctypes.c_int32]
        L.lbm_set_two_cycle_tile.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32]
        L.lbm_time_blocking.argtypes = [_vp] + [ctypes.POINTER(ctypes.c_int32)] * 4
        _lib = L
    return _lib


def check(status: int):
    if status != OK:
        raise LBMError(status, lib().lbm_last_error().decode())
    return status


def default_desc() -> Desc:
    d = Desc()
    check(lib().lbm_desc_defaults(ctypes.byref(d)))
    return d


def desc_from_case(case, storage: int = FP32_DEV, ckpt_every: int = 0) -> Desc:
    """lbm_desc for a seeded input Case (paper_1311_7239_amd.inputs.Case)."""
    d = default_desc()
    d.nx, d.ny, d.bc_x, d.bc_y = case.nx, case.ny, case.bc_x, case.bc_y
    d.lid_ux, d.nu, d.J = case.lid_ux, case.nu, case.J
    d.ax, d.ay, d.Pi0 = case.ax, case.ay, case.Pi0
    d.F_eps = -1.0 if case.Fphi is None else float(case.Fphi)
    if case.phi is None:
        d.medium = MEDIUM_UNIFORM
        d.phi0 = case.phi0
        d.kappa0 = 0.0 if math.isinf(case.K0) else 1.0 / case.K0
    elif getattr(case, "kappa", None) is not None:
        d.medium = MEDIUM_PHI_KAPPA
    else:
        d.medium = MEDIUM_PHI_ERGUN
        d.dp = case.dp
    d.j_plane = 1 if getattr(case, "Jfield", None) is not None else 0
    d.storage = storage
    d.ckpt_every = ckpt_every
    if case.thermal:
        t = d.thermal
        t.enabled = 1
        t.tau_T, t.sigma, t.Th, t.Tc, t.T0, t.g_beta = (case.tau_T, case.sigma, case.Th, case.Tc,
                                                       case.T0, case.gbeta)
    return d


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous() and t.dtype == torch.float32, "expect contiguous cuda float32"
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
    return ws


def _aligned(ws: torch.Tensor):
    p = ws.data_ptr()
    off = (-p) % 256
    return ctypes.c_void_p(p + off), ws.numel() - off


class Solver:
    """One domain: owns a workspace tensor and an lbm_ctx."""

    def __init__(self, desc: Desc, phi: Optional[torch.Tensor] = None,
                 kappa: Optional[torch.Tensor] = None, max_steps_recorded: int = 0,
                 device="cuda", stream=None):
        L = lib()
        self.desc = desc
        self.nx, self.ny = desc.nx, desc.ny
        self.device = torch.device(device)
        self.stream = stream
        nb = ctypes.c_size_t()
        check(L.lbm_workspace_size(ctypes.byref(desc), int(max_steps_recorded), ctypes.byref(nb)))
        self.workspace = _workspace(nb.value, self.device)
        self._phi, self._kappa = phi, kappa     # kept alive until creation work completes
        wsp, wsn = _aligned(self.workspace)
        ctx = ctypes.c_void_p()
        check(L.lbm_create(ctypes.byref(desc), _ptr(phi), _ptr(kappa), wsp, wsn,
                           _stream_handle(stream), ctypes.byref(ctx)))
        self._ctx = ctx

    # -- lifetime
    def close(self):
        if getattr(self, "_ctx", None):
            lib().lbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping and outputs
    def step(self, n: int = 1):
        check(lib().lbm_step(self._ctx, int(n)))

    @property
    def time(self) -> int:
        t = ctypes.c_int64()
        check(lib().lbm_time(self._ctx, ctypes.byref(t)))
        return t.value

    def macroscopic(self, want_T: bool = False):
        p = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
        u = torch.empty((2, self.ny, self.nx), dtype=torch.float32, device=self.device)
        T = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device) if want_T else None
        check(lib().lbm_macroscopic(self._ctx, 0, _ptr(p), _ptr(u), _ptr(T)))
        return p, u, T

    def populations(self, thermal: bool = False):
        df = torch.empty((8, self.ny, self.nx), dtype=torch.float32, device=self.device)
        dg = torch.empty((5, self.ny, self.nx), dtype=torch.float32, device=self.device) if thermal else None
        check(lib().lbm_get_populations(self._ctx, 0, _ptr(df), _ptr(dg)))
        return df, dg

    def set_populations(self, df: torch.Tensor, dg: Optional[torch.Tensor] = None):
        check(lib().lbm_set_populations(self._ctx, 0, _ptr(df.contiguous()),
                                        _ptr(None if dg is None else dg.contiguous())))

    def reduce(self):
        m = ctypes.c_double(); r = ctypes.c_double()
        st = lib().lbm_reduce(self._ctx, 0, ctypes.byref(m), ctypes.byref(r))
        if st not in (OK, EUNSTABLE):
            check(st)
        return m.value, r.value, st

    def reduce_static(self):
        """reduce() through lbm_reduce_static (partial sums in the library's static device
        scratch instead of the workspace)."""
        m = ctypes.c_double(); r = ctypes.c_double()
        st = lib().lbm_reduce_static(self._ctx, 0, ctypes.byref(m), ctypes.byref(r))
        if st not in (OK, EUNSTABLE):
            check(st)
        return m.value, r.value, st

    def backward(self, dL_du: torch.Tensor, want_kappa: bool = False):
        g = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
        gk = torch.empty_like(g) if want_kappa else None
        check(lib().lbm_backward(self._ctx, _ptr(dL_du.contiguous()), _ptr(g), _ptr(gk)))
        return g, gk

    def backward_params(self, dL_du: torch.Tensor, want_phi: bool = True, want_kappa: bool = False):
        """(dL/dphi or None, dL/dkappa or None, {"nu", "ax", "ay", "lid_ux"}) of the recorded pass."""
        g = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device) if want_phi else None
        gk = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device) if want_kappa else None
        th = (ctypes.c_double * 4)()
        check(lib().lbm_backward_params(self._ctx, _ptr(dL_du.contiguous()), _ptr(g), _ptr(gk), th))
        return g, gk, dict(zip(("nu", "ax", "ay", "lid_ux"), list(th)))

    def tangent(self, dphi: Optional[torch.Tensor] = None, dtheta=None) -> torch.Tensor:
        """Directional derivative of u(T) [2, ny, nx] along dphi [ny, nx] and
        dtheta (nu, ax, ay, lid_ux) of the recorded pass."""
        du = torch.empty((2, self.ny, self.nx), dtype=torch.float32, device=self.device)
        th = None if dtheta is None else (ctypes.c_double * 4)(*[float(v) for v in dtheta])
        check(lib().lbm_tangent(self._ctx, _ptr(None if dphi is None else dphi.contiguous()), th, _ptr(du)))
        return du

    def save(self) -> bytes:
        nb = ctypes.c_size_t()
        check(lib().lbm_state_bytes(self._ctx, ctypes.byref(nb)))
        buf = ctypes.create_string_buffer(nb.value)
        check(lib().lbm_save(self._ctx, buf, nb.value))
        return buf.raw

    def load(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        check(lib().lbm_load(self._ctx, buf, len(blob)))

    def set_schedule(self, tile_w: int, vec: int, rows: int, swizzle: int = 1):
        check(lib().lbm_set_schedule(self._ctx, tile_w, vec, rows, swizzle))

    def set_graph_steps(self, steps: int):
        check(lib().lbm_set_graph_steps(self._ctx, int(steps)))

    def set_viscosity_ratio(self, J: torch.Tensor):
        """Per-node viscosity ratio J [ny, nx] (needs desc.j_plane = 1)."""
        check(lib().lbm_set_viscosity_ratio(self._ctx, 0, _ptr(J.contiguous())))

    def set_time_blocking(self, cycles_per_pass: int):
        check(lib().lbm_set_time_blocking(self._ctx, int(cycles_per_pass)))

    def set_two_cycle_tile(self, threads: int, rows: int):
        check(lib().lbm_set_two_cycle_tile(self._ctx, int(threads), int(rows)))

    def time_blocking(self):
        return _time_blocking(self._ctx)

    def schedule(self):
        a, v, b, c = (ctypes.c_int32() for _ in range(4))
        check(lib().lbm_schedule(self._ctx, ctypes.byref(a), ctypes.byref(v), ctypes.byref(b),
                                 ctypes.byref(c)))
        return a.value, v.value, b.value, c.value


def _time_blocking(ctx):
    v = [ctypes.c_int32() for _ in range(4)]
    check(lib().lbm_time_blocking(ctx, *[ctypes.byref(x) for x in v]))
    return {"cycles_per_pass": v[0].value, "threads": v[1].value, "rows": v[2].value, "grid": v[3].value}


def _plane(a, device):
    return None if a is None else torch.from_numpy(a.astype("float32")).to(device)


def solver_for_case(case, storage: int = FP32_DEV, ckpt_every: int = 0, max_steps_recorded: int = 0,
                    device="cuda") -> Solver:
    desc = desc_from_case(case, storage=storage, ckpt_every=ckpt_every)
    kappa = _plane(getattr(case, "kappa", None), device)
    s = Solver(desc, phi=_plane(case.phi, device), kappa=kappa,
               max_steps_recorded=max_steps_recorded, device=device)
    if getattr(case, "Jfield", None) is not None:
        s.set_viscosity_ratio(_plane(case.Jfield, device))
    return s


class Batch:
    """Ragged batch of independent domains stepped together (lbm_create_batch)."""

    def __init__(self, descs: Sequence[Desc], phis=None, kappas=None, tune_cache: Optional[str] = None,
                 device="cuda", stream=None):
        L = lib()
        n = len(descs)
        self.n = n
        self.descs = list(descs)
        self.device = torch.device(device)
        arr = (Desc * n)(*descs)
        self._arr = arr
        nb = ctypes.c_size_t()
        check(L.lbm_batch_workspace_size(n, arr, ctypes.byref(nb)))
        self.workspace = _workspace(nb.value, self.device)
        self._phis = phis
        self._kappas = kappas
        pp = None
        if phis is not None:
            pp = (ctypes.c_void_p * n)(*[None if t is None else t.data_ptr() for t in phis])
        kp = None
        if kappas is not None:
            kp = (ctypes.c_void_p * n)(*[None if t is None else t.data_ptr() for t in kappas])
        wsp, wsn = _aligned(self.workspace)
        ctx = ctypes.c_void_p()
        check(L.lbm_create_batch(n, arr, pp, kp, wsp, wsn, _stream_handle(stream),
                                 None if tune_cache is None else str(tune_cache).encode(),
                                 ctypes.byref(ctx)))
        self._ctx = ctx

    def close(self):
        if getattr(self, "_ctx", None):
            lib().lbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nodes(self) -> int:
        return sum(d.nx * d.ny for d in self.descs)

    def step(self, n: int = 1):
        check(lib().lbm_step(self._ctx, int(n)))

    def set_graph_steps(self, steps: int):
        check(lib().lbm_set_graph_steps(self._ctx, int(steps)))

    def set_time_blocking(self, cycles_per_pass: int):
        check(lib().lbm_set_time_blocking(self._ctx, int(cycles_per_pass)))

    def set_viscosity_ratio(self, k: int, J: torch.Tensor):
        check(lib().lbm_set_viscosity_ratio(self._ctx, int(k), _ptr(J.contiguous())))

    def time_blocking(self):
        return _time_blocking(self._ctx)

    def schedule(self):
        a, v, b, c = (ctypes.c_int32() for _ in range(4))
        check(lib().lbm_schedule(self._ctx, ctypes.byref(a), ctypes.byref(v), ctypes.byref(b),
                                 ctypes.byref(c)))
        return a.value, v.value, b.value, c.value

    def macroscopic(self, k: int, want_T: bool = False):
        """(p, u) of domain k, or (p, u, T) with want_T."""
        d = self.descs[k]
        p = torch.empty((d.ny, d.nx), dtype=torch.float32, device=self.device)
        u = torch.empty((2, d.ny, d.nx), dtype=torch.float32, device=self.device)
        T = torch.empty((d.ny, d.nx), dtype=torch.float32, device=self.device) if want_T else None
        check(lib().lbm_macroscopic(self._ctx, k, _ptr(p), _ptr(u), _ptr(T)))
        return (p, u, T) if want_T else (p, u)

    def set_populations(self, k: int, df: torch.Tensor, dg: Optional[torch.Tensor] = None):
        """Initial state f(0) (and g(0)) of domain k; only before the first step."""
        check(lib().lbm_set_populations(self._ctx, int(k), _ptr(df.contiguous()),
                                        _ptr(None if dg is None else dg.contiguous())))

    @property
    def time(self) -> int:
        t = ctypes.c_int64()
        check(lib().lbm_time(self._ctx, ctypes.byref(t)))
        return t.value

    def populations(self, k: int, thermal: bool = False):
        """Deviations df of domain k, or (df, dg) with thermal."""
        d = self.descs[k]
        df = torch.empty((8, d.ny, d.nx), dtype=torch.float32, device=self.device)
        dg = torch.empty((5, d.ny, d.nx), dtype=torch.float32, device=self.device) if thermal else None
        check(lib().lbm_get_populations(self._ctx, k, _ptr(df), _ptr(dg)))
        return (df, dg) if thermal else df

    def reduce(self, k: int):
        m = ctypes.c_double(); r = ctypes.c_double()
        st = lib().lbm_reduce(self._ctx, k, ctypes.byref(m), ctypes.byref(r))
        if st not in (OK, EUNSTABLE):
            check(st)
        return m.value, r.value, st


def batch_for_cases(cases, storage: int = FP32_DEV, tune_cache=None, device="cuda") -> Batch:
    descs = [desc_from_case(c, storage=storage) for c in cases]
    phis = kappas = None
    if any(c.phi is not None for c in cases):
        phis = [_plane(c.phi, device) for c in cases]
    if any(getattr(c, "kappa", None) is not None for c in cases):
        kappas = [_plane(getattr(c, "kappa", None), device) for c in cases]
    b = Batch(descs, phis=phis, kappas=kappas, tune_cache=tune_cache, device=device)
    for k, c in enumerate(cases):
        if getattr(c, "Jfield", None) is not None:
            b.set_viscosity_ratio(k, _plane(c.Jfield, device))
    return b

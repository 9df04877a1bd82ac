"""Thin ctypes binding of liblbm2p.so (C ABI in include/lbm2p.h).

Argument marshalling only: every step of the simulation runs in the HIP library.
The functions keep the C names; host arrays are NumPy float64 (uint8 for masks).
Importing this module never falls back to anything: a missing or unloadable
library raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm2p.so")

LBM_OK, LBM_E_INVAL, LBM_E_NOMEM, LBM_E_HIP, LBM_E_DOMAIN, LBM_E_DIVERGED, LBM_E_STATE = 0, -1, -2, -3, -4, -5, -6
LBM_D2Q9, LBM_D3Q27 = 0, 1
LBM_EOS_VDW, LBM_EOS_PR, LBM_EOS_RKS, LBM_EOS_CS, LBM_EOS_IDEAL, LBM_EOS_SC1, LBM_EOS_SC2 = 0, 1, 2, 3, 4, 5, 6
LBM_FP64, LBM_FP32_DEV = 0, 1
LBM_FORCE_KORTEWEG, LBM_FORCE_SHAN_CHEN, LBM_FORCE_DUAL_RANGE, LBM_FORCE_GENERAL = 0, 1, 2, 3

EXPORTED = [
    "lbm_create", "lbm_init_fields", "lbm_step", "lbm_moments", "lbm_destroy", "lbm_last_error",
    "lbm_set_stream", "lbm_population_bytes", "lbm_get_populations", "lbm_set_populations",
    "lbm_step_timed", "lbm_velocities", "lbm_coexistence", "lbm_kappa_for_width", "lbm_surface_tension",
    "lbm_eos_pressure", "lbm_pressure_tensor", "lbm_batch_create",
    "lbm_batch_init_fields", "lbm_batch_step", "lbm_batch_moments", "lbm_batch_destroy",
    "lbm_batch_last_error", "lbm_copy_probe", "lbm_last_check", "lbm_batch_layout", "lbm_moments_noalloc",
]


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class lbm_params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("eos", C.c_int), ("a", C.c_double), ("b", C.c_double), ("R", C.c_double),
        ("acentric", C.c_double), ("T_reduced", C.c_double), ("kappa", C.c_double),
        ("tau_liquid", C.c_double), ("tau_vapour", C.c_double),
        ("rho_liquid", C.c_double), ("rho_vapour", C.c_double), ("rho_wall", C.c_double),
        ("mask", C.c_void_p), ("precision", C.c_int), ("rho_ref", C.c_double), ("check_every", C.c_int),
        ("accel", C.c_double * 3), ("rho_wall_field", C.c_void_p), ("link_q", C.c_void_p),
        ("force_model", C.c_int), ("force_g", C.c_double * 4),
    ]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2112_01975_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, d, i64 = C.c_void_p, C.c_double, C.c_int64
        P = C.POINTER(lbm_params)
        L.lbm_create.argtypes = [P, C.POINTER(vp)]
        L.lbm_init_fields.argtypes = [vp, vp, vp]
        L.lbm_step.argtypes = [vp, i64]
        L.lbm_moments.argtypes = [vp, vp, vp, vp]
        L.lbm_moments_noalloc.argtypes = [vp, vp, vp, vp]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_destroy.restype = None
        L.lbm_last_error.argtypes = [vp]
        L.lbm_last_error.restype = C.c_char_p
        L.lbm_set_stream.argtypes = [vp, vp]
        L.lbm_population_bytes.argtypes = [vp]
        L.lbm_population_bytes.restype = i64
        L.lbm_get_populations.argtypes = [vp, vp]
        L.lbm_set_populations.argtypes = [vp, vp]
        L.lbm_step_timed.argtypes = [vp, i64, vp, vp]
        L.lbm_velocities.argtypes = [C.c_int, vp]
        L.lbm_coexistence.argtypes = [P, vp]
        L.lbm_kappa_for_width.argtypes = [P, d, C.POINTER(d)]
        L.lbm_surface_tension.argtypes = [P, C.POINTER(d)]
        L.lbm_eos_pressure.argtypes = [P, vp, i64, vp]
        L.lbm_pressure_tensor.argtypes = [vp, vp]
        L.lbm_batch_create.argtypes = [P, C.c_int, C.POINTER(vp)]
        L.lbm_batch_init_fields.argtypes = [vp, C.c_int, vp, vp]
        L.lbm_batch_step.argtypes = [vp, i64]
        L.lbm_batch_moments.argtypes = [vp, C.c_int, vp, vp, vp]
        L.lbm_batch_destroy.argtypes = [vp]
        L.lbm_batch_destroy.restype = None
        L.lbm_batch_last_error.argtypes = [vp]
        L.lbm_batch_last_error.restype = C.c_char_p
        L.lbm_copy_probe.argtypes = [vp, vp, i64, C.c_int, vp, vp]
        L.lbm_last_check.argtypes = [vp, vp, C.POINTER(i64)]
        L.lbm_batch_layout.argtypes = [vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _check(rc: int, ctx=None, batch=False):
    if rc != LBM_OK:
        if batch:
            msg = lib().lbm_batch_last_error(ctx)
        else:
            msg = lib().lbm_last_error(ctx)
        raise LbmError(rc, (msg or b"").decode())
    return rc


@dataclass
class Params:
    """Problem statement of one simulation; see lbm_params in include/lbm2p.h."""
    lattice: int
    nx: int
    ny: int
    nz: int = 1
    eos: int = LBM_EOS_VDW
    a: float = 9.0 / 49.0
    b: float = 2.0 / 21.0
    R: float = 1.0
    acentric: float = 0.0
    T_reduced: float = 0.9
    kappa: float = 0.02
    tau_liquid: float = 0.8
    tau_vapour: float = 0.0
    rho_liquid: float = 0.0
    rho_vapour: float = 0.0
    rho_wall: float = 0.0
    mask: np.ndarray | None = None
    precision: int = LBM_FP64
    rho_ref: float = 0.0
    check_every: int = 0
    accel: tuple = (0.0, 0.0, 0.0)
    rho_wall_field: np.ndarray | None = None
    link_q: np.ndarray | None = None       # [Q][N] wall fractions in lbm_velocities order
    force_model: int = LBM_FORCE_KORTEWEG
    force_g: tuple = (0.0, 0.0, 0.0, 0.0)
    _keep: list = field(default_factory=list, repr=False)

    @property
    def D(self) -> int:
        return 3 if self.lattice == LBM_D3Q27 else 2

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    def to_c(self) -> lbm_params:
        m = None if self.mask is None else np.ascontiguousarray(self.mask, dtype=np.uint8)
        wf = None if self.rho_wall_field is None else np.ascontiguousarray(self.rho_wall_field, dtype=np.float64)
        lq = None if self.link_q is None else np.ascontiguousarray(self.link_q, dtype=np.float64)
        self._keep = [m, wf, lq]
        return lbm_params(self.lattice, self.nx, self.ny, self.nz, self.eos, self.a, self.b, self.R,
                          self.acentric, self.T_reduced, self.kappa, self.tau_liquid, self.tau_vapour,
                          self.rho_liquid, self.rho_vapour, self.rho_wall, _ptr(m), self.precision,
                          self.rho_ref, self.check_every, (C.c_double * 3)(*[float(g) for g in self.accel]),
                          _ptr(wf), _ptr(lq), int(self.force_model),
                          (C.c_double * 4)(*[float(g) for g in self.force_g]))


# ----------------------------------------------------------------- C-named wrappers
def lbm_create(p: Params) -> C.c_void_p:
    cp = p.to_c()
    h = C.c_void_p()
    _check(lib().lbm_create(C.byref(cp), C.byref(h)), None)
    return h


def lbm_init_fields(ctx, rho: np.ndarray, u: np.ndarray | None = None):
    rho, u = _f64(rho), _f64(u)
    _check(lib().lbm_init_fields(ctx, _ptr(rho), _ptr(u)), ctx)


def lbm_step(ctx, n: int):
    _check(lib().lbm_step(ctx, int(n)), ctx)


def lbm_moments(ctx, N: int, D: int, want_fields: bool = True):
    rho = np.empty(N) if want_fields else None
    U = np.empty((D, N)) if want_fields else None
    tot = np.empty(4)
    _check(lib().lbm_moments(ctx, _ptr(rho), _ptr(U), _ptr(tot)), ctx)
    return rho, U, tot


def lbm_moments_noalloc(ctx, rho_dev: int | None, U_dev: int | None, totals_dev: int | None):
    """Device addresses (e.g. torch data_ptr()) of float64 buffers [N], [D][N], [5]; enqueued only."""
    _check(lib().lbm_moments_noalloc(ctx, rho_dev, U_dev, totals_dev), ctx)


def lbm_destroy(ctx):
    if ctx:
        lib().lbm_destroy(ctx)


def lbm_last_error(ctx=None) -> str:
    return (lib().lbm_last_error(ctx) or b"").decode()


def lbm_last_check(ctx):
    """(totals[4], domain count, step index of the state they describe) of the latest check."""
    out = np.zeros(5)
    st = C.c_int64()
    _check(lib().lbm_last_check(ctx, _ptr(out), C.byref(st)), ctx)
    return out[:4].copy(), int(out[4]), int(st.value)


def lbm_set_stream(ctx, stream_handle: int | None):
    _check(lib().lbm_set_stream(ctx, stream_handle), ctx)


def lbm_population_bytes(ctx) -> int:
    return int(lib().lbm_population_bytes(ctx))


def lbm_get_populations(ctx) -> np.ndarray:
    buf = np.empty(lbm_population_bytes(ctx), dtype=np.uint8)
    _check(lib().lbm_get_populations(ctx, _ptr(buf)), ctx)
    return buf


def lbm_set_populations(ctx, buf: np.ndarray):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(lib().lbm_set_populations(ctx, _ptr(buf)), ctx)


def lbm_step_timed(ctx, n: int):
    ms = np.zeros(3)
    nl = np.zeros(2, dtype=np.int64)
    _check(lib().lbm_step_timed(ctx, int(n), _ptr(ms), _ptr(nl)), ctx)
    return ms, nl


def lbm_velocities(lattice: int) -> np.ndarray:
    c = np.zeros(27 * 3, dtype=np.int32)
    q = lib().lbm_velocities(lattice, _ptr(c))
    if q < 0:
        raise LbmError(q, lbm_last_error(None))
    return c[: 3 * q].reshape(q, 3)


def lbm_coexistence(p: Params):
    cp = p.to_c()
    out = np.zeros(4)
    _check(lib().lbm_coexistence(C.byref(cp), _ptr(out)), None)
    return tuple(out)          # rho_v, rho_l, P_sat, T


def lbm_kappa_for_width(p: Params, width: float) -> float:
    cp = p.to_c()
    k = C.c_double()
    _check(lib().lbm_kappa_for_width(C.byref(cp), float(width), C.byref(k)), None)
    return k.value


def lbm_surface_tension(p: Params) -> float:
    cp = p.to_c()
    s = C.c_double()
    _check(lib().lbm_surface_tension(C.byref(cp), C.byref(s)), None)
    return s.value


def lbm_eos_pressure(p: Params, rho) -> np.ndarray:
    cp = p.to_c()
    r = np.ascontiguousarray(np.atleast_1d(rho), dtype=np.float64)
    out = np.empty_like(r)
    _check(lib().lbm_eos_pressure(C.byref(cp), _ptr(r), r.size, _ptr(out)), None)
    return out


def lbm_pressure_tensor(ctx, N: int, lattice: int) -> np.ndarray:
    """[D(D+1)/2, N] discrete pressure tensor: xx, yy, xy (D2Q9) or xx, yy, zz, xy, xz, yz."""
    nc = 6 if lattice == LBM_D3Q27 else 3
    out = np.empty(nc * N)
    _check(lib().lbm_pressure_tensor(ctx, _ptr(out)), ctx)
    return out.reshape(nc, N)


def lbm_batch_create(cases: list[Params]):
    arr = (lbm_params * len(cases))(*[c.to_c() for c in cases])
    h = C.c_void_p()
    _check(lib().lbm_batch_create(arr, len(cases), C.byref(h)), None, batch=True)
    return h


def lbm_batch_init_fields(b, icase: int, rho, u=None):
    rho, u = _f64(rho), _f64(u)
    _check(lib().lbm_batch_init_fields(b, icase, _ptr(rho), _ptr(u)), b, batch=True)


def lbm_batch_step(b, n: int):
    _check(lib().lbm_batch_step(b, int(n)), b, batch=True)


def lbm_batch_moments(b, icase: int, N: int, D: int):
    rho, U, tot = np.empty(N), np.empty((D, N)), np.empty(4)
    _check(lib().lbm_batch_moments(b, icase, _ptr(rho), _ptr(U), _ptr(tot)), b, batch=True)
    return rho, U, tot


def lbm_copy_probe(dst_ptr: int, src_ptr: int, nbytes: int, reps: int = 5, stream_handle: int | None = None):
    """Attainable copy bandwidth on device buffers (data pointers): (GB/s, ms per copy, shape code)."""
    out = np.zeros(3)
    rc = lib().lbm_copy_probe(dst_ptr, src_ptr, int(nbytes), int(reps), stream_handle, _ptr(out))
    if rc != LBM_OK:
        raise LbmError(rc, "lbm_copy_probe failed")
    return float(out[0]), float(out[1]), int(out[2])


def lbm_batch_layout(b) -> dict:
    """The batch's layout in use (see include/lbm2p.h)."""
    out = np.zeros(6, dtype=np.int32)
    _check(lib().lbm_batch_layout(b, _ptr(out)), b, batch=True)
    keys = ("stepped", "threads_per_block", "nodes_per_thread", "tile_steps", "tile_row_width", "tiles")
    return {k: int(v) for k, v in zip(keys, out)}


def lbm_batch_destroy(b):
    if b:
        lib().lbm_batch_destroy(b)


class Simulation:
    """Owns one context; convenience over the C-named functions."""

    def __init__(self, p: Params):
        self.p = p
        self.ctx = lbm_create(p)

    def init(self, rho, u=None):
        lbm_init_fields(self.ctx, rho, u)
        return self

    def step(self, n: int):
        lbm_step(self.ctx, n)
        return self

    def moments(self, want_fields: bool = True):
        return lbm_moments(self.ctx, self.p.N, self.p.D, want_fields)

    def close(self):
        if self.ctx:
            lbm_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

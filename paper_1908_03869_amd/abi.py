"""ctypes binding of libsode's C ABI (include/sode.h), same names, marshalling only.

Each ``sode_*`` function here forwards to the C function of that name and
returns its status code; nothing is computed in Python.  Loading fails loudly
(``RuntimeError``) when ``libsode.so`` has not been built: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsode.so")

SODE_OK = 0
SODE_EINVAL = -1
SODE_ENOMEM = -2
SODE_EDEVICE = -3
SODE_EUNSUPPORTED = -4
SODE_ENONFINITE = -5
SODE_EBUILD = -6
SODE_ETOOBIG = -7
# Column limit of sode_ensemble_stats_noalloc (its fixed device scratch).
SODE_STATS_NOALLOC_MAX_COLS = 2048

# Every symbol include/sode.h declares.
EXPORTS = (
    "sode_create", "sode_create_custom", "sode_build", "sode_build_log",
    "sode_set_option", "sode_get_option", "sode_integrate",
    "sode_integrate_ex", "sode_forward_ckpt", "sode_adjoint", "sode_integrate_ragged",
    "sode_ensemble_stats", "sode_ensemble_stats_noalloc", "sode_sync", "sode_destroy", "sode_strerror", "sode_version",
)


class SodeInstance(ctypes.Structure):
    """sode_instance_t: one instance of a ragged batch (64 bytes)."""
    _fields_ = [("n", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("nsteps", ctypes.c_int64), ("stride", ctypes.c_int64),
                ("x0_offset", ctypes.c_int64), ("p_offset", ctypes.c_int64),
                ("out_offset", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("orbit_id", ctypes.c_uint32), ("reserved1", ctypes.c_uint32)]


assert ctypes.sizeof(SodeInstance) == 64

_lib = None


class SodeError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {sode_strerror(status)} (status {status})")


def load() -> ctypes.CDLL:
    """Load libsode.so from the package directory (built by build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                              ctypes.c_uint64, ctypes.c_double)
    L.sode_create.argtypes = [ctypes.c_char_p, i32, i32, i32, ctypes.POINTER(vp)]
    L.sode_create.restype = ctypes.c_int
    L.sode_create_custom.argtypes = [ctypes.c_char_p, ctypes.c_char_p, i32, i32, i32,
                                     ctypes.POINTER(vp)]
    L.sode_create_custom.restype = ctypes.c_int
    L.sode_build.argtypes = [vp]
    L.sode_build.restype = ctypes.c_int
    L.sode_build_log.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t,
                                 ctypes.POINTER(ctypes.c_size_t)]
    L.sode_build_log.restype = ctypes.c_int
    L.sode_set_option.argtypes = [vp, ctypes.c_char_p, i64]
    L.sode_set_option.restype = ctypes.c_int
    L.sode_get_option.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(i64)]
    L.sode_get_option.restype = ctypes.c_int
    L.sode_integrate.argtypes = [vp, vp, vp, i64, f64, f64, i64, i64, u64, vp, vp]
    L.sode_integrate.restype = ctypes.c_int
    L.sode_integrate_ex.argtypes = [vp, vp, vp, i64, f64, f64, i64, i64, u64, u64, u64, vp, vp,
                                    vp, vp]
    L.sode_integrate_ex.restype = ctypes.c_int
    L.sode_forward_ckpt.argtypes = [vp, vp, vp, i64, f64, f64, i64, i64, i64, i64, u64, u64, u64,
                                    vp, vp, vp]
    L.sode_forward_ckpt.restype = ctypes.c_int
    L.sode_adjoint.argtypes = [vp, vp, i64, f64, f64, i64, i64, i64, i64, u64, u64, u64, vp, vp,
                               vp, vp, vp]
    L.sode_adjoint.restype = ctypes.c_int
    L.sode_integrate_ragged.argtypes = [vp, ctypes.POINTER(SodeInstance), ctypes.c_int32, vp, i64,
                                        vp, i64, vp, i64, f64, f64, vp]
    L.sode_integrate_ragged.restype = ctypes.c_int
    L.sode_ensemble_stats.argtypes = [vp, vp, i64, i64, vp, vp, vp]
    L.sode_ensemble_stats.restype = ctypes.c_int
    L.sode_ensemble_stats_noalloc.argtypes = [vp, vp, i64, i64, vp, vp, vp]
    L.sode_ensemble_stats_noalloc.restype = ctypes.c_int
    L.sode_sync.argtypes = [vp]
    L.sode_sync.restype = ctypes.c_int
    L.sode_destroy.argtypes = [vp]
    L.sode_destroy.restype = ctypes.c_int
    L.sode_strerror.argtypes = [ctypes.c_int]
    L.sode_strerror.restype = ctypes.c_char_p
    L.sode_version.argtypes = []
    L.sode_version.restype = ctypes.c_int
    _lib = L
    return L


def sode_create(model: str, n: int, m: int, d: int):
    """Returns (status, handle); handle is an int (opaque pointer) or None."""
    h = ctypes.c_void_p()
    st = load().sode_create(model.encode(), n, m, d, ctypes.byref(h))
    return st, h.value


def sode_create_custom(drift_body: str, diffusion_body, n: int, m: int, d: int):
    """Returns (status, handle) for a model given as source text."""
    h = ctypes.c_void_p()
    diff = None if diffusion_body is None else diffusion_body.encode()
    st = load().sode_create_custom(drift_body.encode(), diff, n, m, d, ctypes.byref(h))
    return st, h.value


def sode_build(h) -> int:
    return load().sode_build(h)


def sode_build_log(h):
    """Returns (status, text) of the last run-time compilation."""
    need = ctypes.c_size_t()
    st = load().sode_build_log(h, None, 0, ctypes.byref(need))
    if st != SODE_OK:
        return st, ""
    buf = ctypes.create_string_buffer(need.value)
    st = load().sode_build_log(h, buf, need.value, None)
    return st, buf.value.decode(errors="replace")


def sode_set_option(h, key: str, value: int) -> int:
    return load().sode_set_option(h, key.encode(), int(value))


def sode_get_option(h, key: str):
    v = ctypes.c_int64()
    st = load().sode_get_option(h, key.encode(), ctypes.byref(v))
    return st, v.value


def sode_integrate(h, X0, p, orbits, t0, dt, nsteps, stride, seed, out, stream) -> int:
    return load().sode_integrate(h, X0, p, orbits, t0, dt, nsteps, stride, seed, out, stream)


def sode_integrate_ex(h, X0, p, orbits, t0, dt, nsteps, stride, seed, orbit_offset,
                      step_offset, orbit_ids, orbit_seeds, out, stream) -> int:
    return load().sode_integrate_ex(h, X0, p, orbits, t0, dt, nsteps, stride, seed,
                                    orbit_offset, step_offset, orbit_ids, orbit_seeds, out,
                                    stream)


def sode_forward_ckpt(h, X0, p, orbits, t0, dt, nsteps, ckpt_every, win_lo, win_hi, seed,
                      orbit_offset, step_offset, ckpt, R, stream) -> int:
    return load().sode_forward_ckpt(h, X0, p, orbits, t0, dt, nsteps, ckpt_every, win_lo, win_hi,
                                    seed, orbit_offset, step_offset, ckpt, R, stream)


def sode_adjoint(h, p, orbits, t0, dt, nsteps, ckpt_every, win_lo, win_hi, seed, orbit_offset,
                 step_offset, ckpt, dL_dR, grad_p, grad_p_per_orbit, stream) -> int:
    return load().sode_adjoint(h, p, orbits, t0, dt, nsteps, ckpt_every, win_lo, win_hi, seed,
                               orbit_offset, step_offset, ckpt, dL_dR, grad_p, grad_p_per_orbit,
                               stream)


def sode_integrate_ragged(h, inst, count, X0, x0_len, p, p_len, out, out_len, t0, dt,
                          stream) -> int:
    return load().sode_integrate_ragged(h, inst, count, X0, x0_len, p, p_len, out, out_len, t0,
                                        dt, stream)


def sode_ensemble_stats(h, out, orbits, cols, mean, stddev, stream) -> int:
    return load().sode_ensemble_stats(h, out, orbits, cols, mean, stddev, stream)


def sode_ensemble_stats_noalloc(h, out, orbits, cols, mean, stddev, stream) -> int:
    return load().sode_ensemble_stats_noalloc(h, out, orbits, cols, mean, stddev, stream)


def sode_sync(h) -> int:
    return load().sode_sync(h)


def sode_destroy(h) -> int:
    return load().sode_destroy(h)


def sode_strerror(status: int) -> str:
    return load().sode_strerror(status).decode()


def sode_version() -> int:
    return load().sode_version()


def check(status: int, where: str) -> None:
    if status != SODE_OK:
        raise SodeError(status, where)

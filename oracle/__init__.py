"""FP64 CPU oracle for the many-orbit SDE integrator.

TEST INFRASTRUCTURE ONLY: the plain, single-threaded definition that the HIP
library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code with the HIP path and never imports it.

All arithmetic lives in ``sode_oracle.c`` (plain C, ``-O2 -ffp-contract=off``);
this module only marshals numpy arrays through ctypes and shards orbits over
threads.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sode_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

MODELS = {"kuramoto": 0, "ou": 1, "gbm": 2, "fhn": 3, "rnn": 4}
METHODS = {"em": 0, "rk4": 1, "milstein": 2, "implicit_euler": 3, "implicit_midpoint": 4}
OBSERVABLES = {"state": 0, "kuramoto_r": 1}

_lib = None


def build(force: bool = True, *, src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle with the flags its header fixes (``src`` and
    ``out`` default to the oracle's own source and library)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
             "-D_DEFAULT_SOURCE", "-Wall", "-Wextra", "-fPIC", "-shared",
             "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        _lib = bind(LIB)
    return _lib


def bind(path: str):
    """Load an oracle shared library from ``path`` and declare its entry
    points.  ``lib()`` binds the built oracle; the pin tests also bind copies
    compiled from deliberately altered source, to show that a pin fails."""
    L = ctypes.CDLL(path)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    f64p = ctypes.POINTER(ctypes.c_double)
    L.oracle_philox.argtypes = [u32p, u32p, u32p]
    L.oracle_philox.restype = None
    L.oracle_box_muller.argtypes = [ctypes.c_uint32, ctypes.c_uint32, f64p]
    L.oracle_box_muller.restype = None
    L.oracle_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_int32, f64p]
    L.oracle_normals.restype = None
    L.oracle_model_dims_ok.argtypes = [ctypes.c_int32] * 4
    L.oracle_model_dims_ok.restype = ctypes.c_int
    L.oracle_drift.argtypes = [ctypes.c_int32] * 4 + [ctypes.c_double, f64p, f64p, f64p]
    L.oracle_drift.restype = None
    L.oracle_diffusion.argtypes = [ctypes.c_int32] * 4 + [ctypes.c_double, f64p, f64p,
                                                           f64p, f64p]
    L.oracle_diffusion.restype = None
    L.oracle_order_parameter.argtypes = [ctypes.c_int32, f64p]
    L.oracle_order_parameter.restype = ctypes.c_double
    L.oracle_integrate.argtypes = (
        [ctypes.c_int32] * 4
        + [f64p, f64p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
           ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64,
           ctypes.c_uint64, u32p, u64p, ctypes.c_int32, ctypes.c_int32, f64p])
    L.oracle_integrate.restype = ctypes.c_int
    L.oracle_integrate_custom.argtypes = (
        [ctypes.c_int32] * 3 + [ctypes.c_void_p, ctypes.c_void_p]
        + [f64p, f64p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
           ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64,
           ctypes.c_uint64, u32p, u64p, ctypes.c_int32, f64p])
    L.oracle_integrate_custom.restype = ctypes.c_int
    L.oracle_kuramoto_adjoint.argtypes = [
        ctypes.c_int32, f64p, f64p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
        ctypes.c_double, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
        ctypes.c_uint64, ctypes.c_uint64, f64p, f64p, f64p, f64p]
    L.oracle_kuramoto_adjoint.restype = ctypes.c_int
    return L


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def philox(ctr, key):
    """Philox-4x32-10 block for counter ``ctr`` (4 x u32) and ``key`` (2 x u32)."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox(c, k, o)
    return [int(x) for x in o]


def box_muller(w0: int, w1: int):
    o = (ctypes.c_double * 2)()
    lib().oracle_box_muller(w0 & 0xFFFFFFFF, w1 & 0xFFFFFFFF, o)
    return float(o[0]), float(o[1])


def normals(seed: int, orbit_id: int, step: int, m: int) -> np.ndarray:
    out = np.zeros(m, dtype=np.float64)
    lib().oracle_normals(seed, orbit_id, step, m, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def dims_ok(model: str, n: int, m: int, d: int) -> bool:
    return bool(lib().oracle_model_dims_ok(MODELS[model], n, m, d))


def drift(model: str, n: int, m: int, d: int, X, p, t: float = 0.0) -> np.ndarray:
    X, Xp = _f64(X)
    p, pp = _f64(p)
    f = np.zeros(n, dtype=np.float64)
    lib().oracle_drift(MODELS[model], n, m, d, t, Xp, pp, f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return f


def diffusion(model: str, n: int, m: int, d: int, X, p, xi, t: float = 0.0) -> np.ndarray:
    X, Xp = _f64(X)
    p, pp = _f64(p)
    xi, xp = _f64(xi)
    g = np.zeros(n, dtype=np.float64)
    lib().oracle_diffusion(MODELS[model], n, m, d, t, Xp, pp, xp,
                           g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return g


def order_parameter(theta) -> float:
    theta, tp = _f64(theta)
    return float(lib().oracle_order_parameter(theta.size, tp))


_CUSTOM_TEMPLATE = """#include <math.h>
typedef double real;
void sode_user_drift(double t, const real* y, const real* p, real* f)
{
%s
}
void sode_user_diffusion(double t, const real* y, const real* p, const real* xi, real* gx)
{
%s
}
"""


def custom_model(drift: str, diffusion: str | None, n: int):
    """Compile a model given as the bodies of its two system functions (the
    text a source-text library handle receives) as plain C with the oracle's
    flags; returns (drift, diffusion) function addresses.  Cached by source."""
    import hashlib
    import tempfile
    diff = diffusion if diffusion is not None else f"for (int i = 0; i < {n}; ++i) gx[i] = 0;"
    src = _CUSTOM_TEMPLATE % (drift, diff)
    key = hashlib.sha256(src.encode()).hexdigest()[:20]
    if key not in _custom:
        d = os.path.join(tempfile.gettempdir(), "sode_oracle_custom")
        os.makedirs(d, exist_ok=True)
        c_path = os.path.join(d, key + ".c")
        so_path = os.path.join(d, key + ".so")
        if not os.path.exists(so_path):
            with open(c_path, "w") as f:
                f.write(src)
            tmp = so_path + f".{os.getpid()}.tmp"
            subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                                   "-fPIC", "-shared", "-o", tmp, c_path, "-lm"])
            os.replace(tmp, so_path)
        so = ctypes.CDLL(so_path)
        _custom[key] = (so, ctypes.cast(so.sode_user_drift, ctypes.c_void_p).value,
                        ctypes.cast(so.sode_user_diffusion, ctypes.c_void_p).value)
    return _custom[key][1], _custom[key][2]


_custom = {}


def integrate(model: str, n: int, m: int, d: int, X0, p, t0: float, dt: float, nsteps: int,
              stride: int, seed: int, *, method: str = "em", observable: str = "state",
              orbit_offset: int = 0, step_offset: int = 0, orbit_ids=None, orbit_seeds=None,
              p_per_orbit: bool | None = None, custom=None) -> np.ndarray:
    """Integrate every orbit; returns out[orbits, nsteps/stride+1, q] in float64.
    model "custom" takes custom = (drift body, diffusion body) source text."""
    X0, X0p = _f64(X0)
    X0 = X0.reshape(-1, n)
    orbits = X0.shape[0]
    p, pp = _f64(p)
    if p_per_orbit is None:
        p_per_orbit = p.ndim == 2
    if p_per_orbit:
        assert p.shape == (orbits, d), (p.shape, orbits, d)
    else:
        assert p.size == d
    nsave = nsteps // stride + 1 if stride > 0 else 0
    q = 1 if observable == "kuramoto_r" else n
    out = np.zeros((orbits, max(nsave, 0), q), dtype=np.float64)
    ids_arr = seeds_arr = None
    ids_p = ctypes.POINTER(ctypes.c_uint32)()
    seeds_p = ctypes.POINTER(ctypes.c_uint64)()
    if orbit_ids is not None:
        ids_arr = np.ascontiguousarray(orbit_ids, dtype=np.uint32)
        assert ids_arr.size == orbits
        ids_p = ids_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    if orbit_seeds is not None:
        seeds_arr = np.ascontiguousarray(orbit_seeds, dtype=np.uint64)
        assert seeds_arr.size == orbits
        seeds_p = seeds_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    if model == "custom":
        fd, fg = custom_model(custom[0], custom[1], n)
        rc = lib().oracle_integrate_custom(
            n, m, d, ctypes.c_void_p(fd), ctypes.c_void_p(fg), X0p, pp, int(bool(p_per_orbit)),
            orbits, t0, dt, nsteps, stride, seed, orbit_offset, step_offset, ids_p, seeds_p,
            METHODS[method], out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    else:
        rc = lib().oracle_integrate(
            MODELS[model], n, m, d, X0p, pp, int(bool(p_per_orbit)), orbits, t0, dt, nsteps,
            stride, seed, orbit_offset, step_offset, ids_p, seeds_p, METHODS[method],
            OBSERVABLES[observable], out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError(f"oracle_integrate rejected its arguments (rc={rc})")
    return out


def integrate_parallel(model, n, m, d, X0, p, t0, dt, nsteps, stride, seed, *, threads=8,
                       orbit_ids=None, orbit_seeds=None, orbit_offset=0, **kw) -> np.ndarray:
    """Run ``integrate`` on disjoint orbit shards in ``threads`` OS threads.

    Orbits are independent, so sharding changes nothing in the result; each
    shard passes its global orbit ids so the noise is the same as one call.
    ctypes releases the GIL for the duration of each C call."""
    from concurrent.futures import ThreadPoolExecutor

    X0 = np.ascontiguousarray(X0, dtype=np.float64).reshape(-1, n)
    orbits = X0.shape[0]
    p = np.ascontiguousarray(p, dtype=np.float64)
    per = p.ndim == 2
    bounds = np.linspace(0, orbits, threads + 1).astype(int)
    if model == "custom":  # compile the callbacks once, before the threads start
        custom_model(kw["custom"][0], kw["custom"][1], n)

    def run(i):
        a, b = bounds[i], bounds[i + 1]
        if a == b:
            return None
        ids = None if orbit_ids is None else np.asarray(orbit_ids)[a:b]
        sds = None if orbit_seeds is None else np.asarray(orbit_seeds)[a:b]
        off = orbit_offset + a if orbit_ids is None else 0
        return integrate(model, n, m, d, X0[a:b], p[a:b] if per else p, t0, dt, nsteps, stride,
                         seed, orbit_ids=ids, orbit_seeds=sds, orbit_offset=off,
                         p_per_orbit=per, **kw)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = [r for r in ex.map(run, range(threads)) if r is not None]
    return np.concatenate(parts, axis=0)


def kuramoto_adjoint(n: int, X0, p, t0: float, dt: float, nsteps: int, win_lo: int, win_hi: int,
                     seed: int, *, dL_dR=None, orbit_offset: int = 0, step_offset: int = 0,
                     per_orbit: bool = True):
    """Window-averaged order parameter R[orbits] and its pathwise gradient.

    Returns (R, grad[d], grad_per_orbit[orbits, d] or None); grad is
    sum_o dL_dR[o] dR_o/dp (dL_dR defaults to ones)."""
    d = 2 * n + 1
    X0, X0p = _f64(X0)
    X0 = X0.reshape(-1, n)
    orbits = X0.shape[0]
    p, pp = _f64(p)
    p_per_orbit = p.ndim == 2
    R = np.zeros(orbits)
    grad = np.zeros(d)
    gpo = np.zeros((orbits, d)) if per_orbit else None
    f64p = ctypes.POINTER(ctypes.c_double)
    w = None
    wp = ctypes.POINTER(ctypes.c_double)()
    if dL_dR is not None:
        w = np.ascontiguousarray(dL_dR, dtype=np.float64)
        wp = w.ctypes.data_as(f64p)
    rc = lib().oracle_kuramoto_adjoint(
        n, X0p, pp, int(p_per_orbit), orbits, t0, dt, nsteps, win_lo, win_hi, seed,
        orbit_offset, step_offset, wp, R.ctypes.data_as(f64p),
        gpo.ctypes.data_as(f64p) if gpo is not None else ctypes.POINTER(ctypes.c_double)(),
        grad.ctypes.data_as(f64p))
    if rc != 0:
        raise ValueError(f"oracle_kuramoto_adjoint rejected its arguments (rc={rc})")
    return R, grad, gpo


def kuramoto_adjoint_parallel(n, X0, p, t0, dt, nsteps, win_lo, win_hi, seed, *, dL_dR=None,
                              threads=8, orbit_offset=0, step_offset=0):
    """``kuramoto_adjoint`` over disjoint orbit shards in threads; the
    per-orbit gradients are then summed in orbit order, as one call would."""
    from concurrent.futures import ThreadPoolExecutor

    X0 = np.ascontiguousarray(X0, dtype=np.float64).reshape(-1, n)
    orbits = X0.shape[0]
    p = np.ascontiguousarray(p, dtype=np.float64)
    per = p.ndim == 2
    w = np.ones(orbits) if dL_dR is None else np.asarray(dL_dR, dtype=np.float64)
    bounds = np.linspace(0, orbits, threads + 1).astype(int)

    def run(i):
        a, b = bounds[i], bounds[i + 1]
        if a == b:
            return None
        return kuramoto_adjoint(n, X0[a:b], p[a:b] if per else p, t0, dt, nsteps, win_lo,
                                win_hi, seed, dL_dR=w[a:b], orbit_offset=orbit_offset + a,
                                step_offset=step_offset)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = [r for r in ex.map(run, range(threads)) if r is not None]
    R = np.concatenate([r[0] for r in parts])
    gpo = np.concatenate([r[2] for r in parts])
    grad = np.zeros(2 * n + 1)
    for row in gpo:
        grad = grad + row
    return R, grad, gpo

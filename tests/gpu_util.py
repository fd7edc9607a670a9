"""Helpers shared by the GPU tests: move a workload to the device, call the
library through its C ABI (via the ctypes binding) and compare with the
oracle."""
from __future__ import annotations

import math
import os
import sys

import numpy as np

import paper_1908_03869_amd as sode

OPT = {"em": 0, "rk4": 1, "milstein": 2, "implicit_euler": 3, "implicit_midpoint": 4, "state": 0, "kuramoto_r": 1, "auto": 0, "plain": 1, "coupled": 2}


def log(msg: str) -> None:
    """Name the case before each GPU step so a failing run says what ran."""
    sys.stdout.write(f"[gpu-case] {msg}\n")
    sys.stdout.flush()


def threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def run_library(w: dict, *, precision: int, kernel: str = "auto", method: str = "em",
                observable: str | None = None, X0=None, p=None, nsteps=None, stride=None,
                orbit_offset: int = 0, step_offset: int = 0, t0: float | None = None,
                orbit_ids=None, orbit_seeds=None, shared: bool | None = None,
                compensated: int = 1, drift: int = 0, wrap: int = 1, ode_limit: int | None = None,
                noise_waves: int = -1, device="cuda:0") -> np.ndarray:
    import torch

    dtype = torch.float32 if precision == 32 else torch.float64
    X0 = w["X0"] if X0 is None else X0
    p = w["p"] if p is None else p
    shared = (np.asarray(p).ndim == 1) if shared is None else shared
    obs = observable or w.get("observable", "state")
    # The ODE methods integrate the limit g = 0, which a call must ask for.
    if ode_limit is None:
        ode_limit = int(method in ("rk4", "implicit_euler", "implicit_midpoint"))
    it = sode.Integrator(w["model"], w["n"], w["m"], w["d"], precision=precision,
                         method=OPT[method], observable=OPT[obs], kernel=OPT[kernel],
                         shared_params=int(shared), compensated=compensated, drift=drift,
                         wrap=wrap, ode_limit=ode_limit, noise_waves=noise_waves)
    X0_t = torch.tensor(np.ascontiguousarray(X0), dtype=dtype, device=device)
    p_t = torch.tensor(np.ascontiguousarray(p), dtype=dtype, device=device)
    ids = orbit_ids if orbit_ids is not None else w.get("orbit_ids")
    sds = orbit_seeds if orbit_seeds is not None else w.get("orbit_seeds")
    ids_t = None if ids is None else torch.tensor(np.asarray(ids, dtype=np.int64).astype(np.int32),
                                                  device=device)
    sds_t = None if sds is None else torch.tensor(np.asarray(sds, dtype=np.uint64).astype(np.int64),
                                                  device=device)
    out = it.integrate(X0_t, p_t, w["t0"] if t0 is None else t0, w["dt"],
                       w["nsteps"] if nsteps is None else nsteps,
                       w["stride"] if stride is None else stride, w["seed"],
                       orbit_offset=orbit_offset, step_offset=step_offset, orbit_ids=ids_t,
                       orbit_seeds=sds_t)
    it.sync()
    res = out.double().cpu().numpy()
    it.close()
    return res


def as_received(a, precision: int):
    """The values a kernel of the given precision actually receives: binary32
    kernels get the inputs rounded to float32."""
    a = np.asarray(a, dtype=np.float64)
    return a.astype(np.float32).astype(np.float64) if precision == 32 else a


def run_oracle(w: dict, *, rows=None, method: str = "em", observable: str | None = None,
               nsteps=None, stride=None, X0=None, p=None, step_offset: int = 0,
               t0: float | None = None, precision: int = 64) -> np.ndarray:
    """FP64 oracle on the inputs the library received (rounded to float32
    for precision 32, so that the comparison measures the integrator)."""
    import oracle

    X0 = as_received(w["X0"] if X0 is None else X0, precision)
    p = as_received(w["p"] if p is None else p, precision)
    ids = w.get("orbit_ids")
    sds = w.get("orbit_seeds")
    rows = np.arange(X0.shape[0]) if rows is None else np.asarray(rows)
    # Global orbit ids of the selected rows (the library numbers orbit o as o
    # unless explicit ids are given).
    ids_sel = rows.astype(np.uint32) if ids is None else np.asarray(ids)[rows]
    sds_sel = None if sds is None else np.asarray(sds)[rows]
    p_sel = p[rows] if p.ndim == 2 else p
    return oracle.integrate_parallel(
        w["model"], w["n"], w["m"], w["d"], X0[rows], p_sel, w["t0"] if t0 is None else t0,
        w["dt"], w["nsteps"] if nsteps is None else nsteps,
        w["stride"] if stride is None else stride, w["seed"], threads=threads(),
        orbit_ids=ids_sel, orbit_seeds=sds_sel, method=method,
        observable=observable or w.get("observable", "state"), step_offset=step_offset)


def circular_diff(a, b) -> np.ndarray:
    return np.abs(np.remainder(a - b + math.pi, 2 * math.pi) - math.pi)

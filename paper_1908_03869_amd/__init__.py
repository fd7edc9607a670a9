"""MI355X-native many-orbit SDE integrator (the SODECL problem, arXiv 1908.03869).

The compute path is ``libsode.so`` (HIP kernels for gfx950 behind a C ABI,
``include/sode.h``).  ``abi`` is the ctypes binding with the C names; this
module adds a torch-facing convenience layer that only allocates the output
tensor and passes device pointers and the current HIP stream.
"""
from __future__ import annotations

from . import abi
from .abi import SodeError, check

__all__ = ["abi", "Integrator", "SodeError", "check", "OPTION_VALUES"]

OPTION_VALUES = {
    "method": {"em": 0, "rk4": 1},
    "observable": {"state": 0, "kuramoto_r": 1},
    "kernel": {"auto": 0, "plain": 1, "coupled": 2},
}


class Integrator:
    """A libsode handle for one model (sode_create ... sode_destroy).

    ``integrate`` takes torch tensors on the GPU in the handle's precision and
    returns ``out[orbits, nsteps/stride+1, q]``.  All work runs in libsode.
    """

    def __init__(self, model: str, n: int, m: int, d: int, **options):
        st, h = abi.sode_create(model, n, m, d)
        check(st, f"sode_create({model}, {n}, {m}, {d})")
        self.handle = h
        self.model, self.n, self.m, self.d = model, n, m, d
        self.options = {"precision": 32, "method": 0, "observable": 0, "kernel": 0,
                        "shared_params": 0}
        for k, v in options.items():
            self.set_option(k, v)

    def set_option(self, key: str, value) -> None:
        if isinstance(value, str):
            value = OPTION_VALUES[key][value]
        check(abi.sode_set_option(self.handle, key, int(value)), f"sode_set_option({key})")
        self.options[key] = int(value)

    @property
    def dtype(self):
        import torch
        return torch.float32 if self.options["precision"] == 32 else torch.float64

    def integrate(self, X0, p, t0: float, dt: float, nsteps: int, stride: int, seed: int, *,
                  orbit_offset: int = 0, step_offset: int = 0, orbit_ids=None,
                  orbit_seeds=None, out=None, stream=None):
        import torch
        orbits = X0.shape[0]
        q = 1 if self.options["observable"] == 1 else self.n
        nsave = nsteps // stride + 1 if stride > 0 and nsteps >= 0 else 0
        for name, t in (("X0", X0), ("p", p)):
            if t.dtype != self.dtype or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {self.dtype} GPU tensor")
        if out is None:
            out = torch.empty((orbits, max(nsave, 0), q), dtype=self.dtype, device=X0.device)
        if stream is None:
            stream = torch.cuda.current_stream(X0.device).cuda_stream
        ids = 0 if orbit_ids is None else orbit_ids.data_ptr()
        seeds = 0 if orbit_seeds is None else orbit_seeds.data_ptr()
        if orbit_ids is not None and orbit_ids.dtype != torch.int32 and orbit_ids.dtype != torch.uint32:
            raise ValueError("orbit_ids must be a 32-bit integer tensor")
        if orbit_seeds is not None and orbit_seeds.dtype not in (torch.int64, torch.uint64):
            raise ValueError("orbit_seeds must be a 64-bit integer tensor")
        st = abi.sode_integrate_ex(self.handle, X0.data_ptr(), p.data_ptr(), orbits, t0, dt,
                                   nsteps, stride, seed, orbit_offset, step_offset, ids or None,
                                   seeds or None, out.data_ptr(), stream)
        check(st, "sode_integrate_ex")
        return out

    def sync(self) -> None:
        check(abi.sode_sync(self.handle), "sode_sync")

    def close(self) -> None:
        if getattr(self, "handle", None):
            abi.sode_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""MI355X-native many-orbit SDE integrator (the SODECL problem, arXiv 1908.03869).

The compute path is ``libsode.so`` (HIP kernels for gfx950 behind a C ABI,
``include/sode.h``).  ``abi`` is the ctypes binding with the C names; this
module adds a torch-facing convenience layer that only allocates the output
tensor and passes device pointers and the current HIP stream.
"""
from __future__ import annotations

from . import abi
from .abi import SodeError, check

__all__ = ["abi", "Integrator", "SodeError", "check", "OPTION_VALUES", "KuramotoWindowR",
           "KuramotoTimeAvgR", "RaggedBatch", "integrate", "noises"]

OPTION_VALUES = {
    "method": {"em": 0, "rk4": 1, "milstein": 2, "implicit_euler": 3, "implicit_midpoint": 4},
    "observable": {"state": 0, "kuramoto_r": 1},
    "kernel": {"auto": 0, "plain": 1, "coupled": 2, "matrix": 3},
    "gemm": {"bf16": 0, "bf16x3": 1, "fp32": 2},
    "drift": {"pairwise": 0, "meanfield": 1},
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
                        "shared_params": 0, "compensated": 1, "waves_per_cu": 0,
                        "units_per_lane": 0, "graph": 1, "persistent": 1, "gemm": 1, "drift": 0,
                        "ode_limit": 0, "wrap": 1, "noise_waves": -1}
        for k, v in options.items():
            self.set_option(k, v)

    @classmethod
    def custom(cls, drift: str, diffusion: str | None, n: int, m: int, d: int, **options):
        """A handle for a model given as source text (sode_create_custom): the
        bodies of drift(t, y, p) -> f[0..n) and diffusion(t, y, p, xi) ->
        gx[0..n), compiled for gfx950 at run time."""
        self = cls.__new__(cls)
        st, h = abi.sode_create_custom(drift, diffusion, n, m, d)
        check(st, f"sode_create_custom(n={n}, m={m}, d={d})")
        self.handle = h
        self.model, self.n, self.m, self.d = "custom", n, m, d
        self.options = {"precision": 32, "method": 0, "observable": 0, "kernel": 0,
                        "shared_params": 0, "compensated": 1, "waves_per_cu": 0,
                        "units_per_lane": 0, "graph": 1, "persistent": 1, "gemm": 1, "drift": 0,
                        "ode_limit": 0, "wrap": 1, "noise_waves": -1}
        for k, v in options.items():
            self.set_option(k, v)
        return self

    def build(self) -> None:
        """Compile a source-text model now (sode_build); raises with the
        compiler's log on failure."""
        st = abi.sode_build(self.handle)
        if st != abi.SODE_OK:
            raise SodeError(st, "sode_build:\n" + self.build_log())

    def build_log(self) -> str:
        return abi.sode_build_log(self.handle)[1]

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

    def _shared(self, p) -> None:
        want = 1 if p.dim() == 1 else 0
        if self.options["shared_params"] != want:
            self.set_option("shared_params", want)

    def forward_ckpt(self, X0, p, t0: float, dt: float, nsteps: int, ckpt_every: int,
                     win_lo: int, win_hi: int, seed: int, *, orbit_offset: int = 0,
                     step_offset: int = 0, stream=None):
        """sode_forward_ckpt: returns (ckpt[orbits, nsteps/ckpt_every+1, n] float32,
        R[orbits] float64)."""
        import torch
        self._shared(p)
        orbits = X0.shape[0]
        for name, t in (("X0", X0), ("p", p)):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float32 GPU tensor")
        nck = nsteps // ckpt_every + 1 if ckpt_every > 0 else 0
        ckpt = torch.empty((orbits, max(nck, 0), self.n), dtype=torch.float32, device=X0.device)
        R = torch.empty(orbits, dtype=torch.float64, device=X0.device)
        if stream is None:
            stream = torch.cuda.current_stream(X0.device).cuda_stream
        st = abi.sode_forward_ckpt(self.handle, X0.data_ptr(), p.data_ptr(), orbits, t0, dt,
                                   nsteps, ckpt_every, win_lo, win_hi, seed, orbit_offset,
                                   step_offset, ckpt.data_ptr(), R.data_ptr(), stream)
        check(st, "sode_forward_ckpt")
        return ckpt, R

    def adjoint(self, p, ckpt, t0: float, dt: float, nsteps: int, ckpt_every: int, win_lo: int,
                win_hi: int, seed: int, dL_dR=None, *, per_orbit: bool = False,
                orbit_offset: int = 0, step_offset: int = 0, stream=None):
        """sode_adjoint: returns (grad[d] float64, rows[orbits, d] float64 or None)."""
        import torch
        self._shared(p)
        orbits = ckpt.shape[0]
        dev = ckpt.device
        if p.dtype != torch.float32 or not p.is_contiguous() or not ckpt.is_contiguous():
            raise ValueError("p and ckpt must be contiguous float32 GPU tensors")
        if dL_dR is not None and (dL_dR.dtype != torch.float64 or not dL_dR.is_contiguous()
                                  or dL_dR.numel() != orbits):
            raise ValueError("dL_dR must be a contiguous float64 tensor with one entry per orbit")
        grad = torch.empty(self.d, dtype=torch.float64, device=dev)
        rows = torch.empty((orbits, self.d), dtype=torch.float64, device=dev) if per_orbit else None
        if stream is None:
            stream = torch.cuda.current_stream(dev).cuda_stream
        st = abi.sode_adjoint(self.handle, p.data_ptr(), orbits, t0, dt, nsteps, ckpt_every,
                              win_lo, win_hi, seed, orbit_offset, step_offset, ckpt.data_ptr(),
                              None if dL_dR is None else dL_dR.data_ptr(), grad.data_ptr(),
                              None if rows is None else rows.data_ptr(), stream)
        check(st, "sode_adjoint")
        return grad, rows

    def integrate_ragged(self, batch: "RaggedBatch", X0, p, t0: float, dt: float, *, out=None,
                         stream=None):
        """sode_integrate_ragged over a packed batch; returns the packed out."""
        import torch
        for name, t in (("X0", X0), ("p", p)):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float32 GPU tensor")
        if out is None:
            out = torch.empty(batch.out_len, dtype=torch.float32, device=X0.device)
        if stream is None:
            stream = torch.cuda.current_stream(X0.device).cuda_stream
        st = abi.sode_integrate_ragged(self.handle, batch.desc, batch.count, X0.data_ptr(),
                                       X0.numel(), p.data_ptr(), p.numel(), out.data_ptr(),
                                       out.numel(), t0, dt, stream)
        check(st, "sode_integrate_ragged")
        return out

    def ensemble_stats(self, out, stream=None, *, noalloc: bool = False):
        """sode_ensemble_stats over out[orbits, ...]: (mean, std) float64 of shape out[0].
        noalloc=True calls sode_ensemble_stats_noalloc (fixed library scratch,
        at most SODE_STATS_NOALLOC_MAX_COLS columns; mean and std are still
        allocated here by torch)."""
        import torch
        orbits = out.shape[0]
        cols = out[0].numel() if orbits > 0 else 0
        if out.dtype != self.dtype or not out.is_contiguous():
            raise ValueError("out must be contiguous in the handle's precision")
        mean = torch.empty(out.shape[1:], dtype=torch.float64, device=out.device)
        std = torch.empty(out.shape[1:], dtype=torch.float64, device=out.device)
        if stream is None:
            stream = torch.cuda.current_stream(out.device).cuda_stream
        fn = abi.sode_ensemble_stats_noalloc if noalloc else abi.sode_ensemble_stats
        st = fn(self.handle, out.data_ptr(), orbits, cols, mean.data_ptr(), std.data_ptr(), stream)
        check(st, fn.__name__)
        return mean, std

    def get_option(self, key: str) -> int:
        st, v = abi.sode_get_option(self.handle, key)
        check(st, f"sode_get_option({key})")
        return v

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


class RaggedBatch:
    """Descriptors (sode_instance_t) of a ragged batch plus its packing.

    ``n[i]`` is the state dimension of instance i; X0 and p of all instances
    are packed back to back (instance order), and so are the outputs
    [nsteps/stride+1][n] of each instance."""

    def __init__(self, n, nsteps, stride, seeds, orbit_ids, d: int):
        import ctypes
        import numpy as np
        n = np.asarray(n, dtype=np.int64)
        nsteps = np.asarray(nsteps, dtype=np.int64)
        stride = np.broadcast_to(np.asarray(stride, dtype=np.int64), n.shape)
        self.count = int(n.size)
        self.n, self.nsteps, self.stride, self.d = n, nsteps, stride, d
        self.x0_offset = np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)
        self.p_offset = np.arange(self.count, dtype=np.int64) * d
        sizes = (nsteps // stride + 1) * n
        self.out_offset = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        self.x0_len = int(n.sum())
        self.p_len = self.count * d
        self.out_len = int(sizes.sum())
        seeds = np.broadcast_to(np.asarray(seeds, dtype=np.uint64), n.shape)
        ids = np.broadcast_to(np.asarray(orbit_ids, dtype=np.uint32), n.shape)
        self.desc = (abi.SodeInstance * max(self.count, 1))()
        for i in range(self.count):
            e = self.desc[i]
            e.n, e.nsteps, e.stride = int(n[i]), int(nsteps[i]), int(stride[i])
            e.x0_offset, e.p_offset = int(self.x0_offset[i]), int(self.p_offset[i])
            e.out_offset, e.seed, e.orbit_id = int(self.out_offset[i]), int(seeds[i]), int(ids[i])
        self._keep = ctypes.addressof(self.desc)

    def pack(self, per_instance):
        import numpy as np
        return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in per_instance])

    def unpack(self, out_flat, i: int):
        """Output of instance i as [nsteps/stride+1, n]."""
        a = int(self.out_offset[i])
        ns = int(self.nsteps[i] // self.stride[i] + 1)
        return out_flat[a:a + ns * int(self.n[i])].reshape(ns, int(self.n[i]))


def _window_r_function():
    import torch

    class KuramotoWindowR(torch.autograd.Function):
        """R[orbits] = window-averaged order parameter of Kuramoto orbits as a
        differentiable function of the parameters p ([d] shared or [orbits, d]).

        forward:  sode_forward_ckpt (checkpoints kept for the backward pass)
        backward: sode_adjoint with dL_dR = grad_R (common random numbers)."""

        @staticmethod
        def forward(ctx, p, X0, integrator, t0, dt, nsteps, ckpt_every, win_lo, win_hi, seed):
            ckpt, R = integrator.forward_ckpt(X0, p.detach().contiguous(), t0, dt, nsteps,
                                              ckpt_every, win_lo, win_hi, seed)
            ctx.integrator = integrator
            ctx.args = (t0, dt, nsteps, ckpt_every, win_lo, win_hi, seed)
            ctx.save_for_backward(p, ckpt)
            return R

        @staticmethod
        def backward(ctx, grad_R):
            p, ckpt = ctx.saved_tensors
            per = p.dim() == 2
            grad, rows = ctx.integrator.adjoint(p.detach().contiguous(), ckpt, *ctx.args,
                                                dL_dR=grad_R.double().contiguous(),
                                                per_orbit=per)
            g = rows if per else grad
            return (g.to(p.dtype),) + (None,) * 9

    return KuramotoWindowR


class _Lazy:
    _cls = None

    def __getattr__(self, name):
        if _Lazy._cls is None:
            _Lazy._cls = _window_r_function()
        return getattr(_Lazy._cls, name)


KuramotoWindowR = _Lazy()
# The name the design blueprint uses for the same function.
KuramotoTimeAvgR = KuramotoWindowR


def noises(model: str, n: int) -> int:
    """m, the number of Wiener processes of a built-in model of n equations."""
    return n // 2 if model == "fhn" else n


def integrate(model: str, X0, p, t0: float, dt: float, nsteps: int, stride: int, seed: int,
              **options):
    """One-call form of Integrator(...).integrate(...): n from X0[orbits, n],
    d from p ([d] shared by all orbits, or [orbits, d]), precision from the
    tensors' dtype; other options (method, observable, kernel, drift, ...) as
    keywords.  The output is allocated with torch and the work is queued on
    the current stream; the temporary handle is released on return, which
    waits for the work to finish and raises on a device error or a
    non-finite saved value."""
    import torch
    n = int(X0.shape[1])
    d = int(p.shape[-1])
    prec = 64 if X0.dtype == torch.float64 else 32
    options.setdefault("precision", prec)
    options.setdefault("shared_params", int(p.dim() == 1))
    it = Integrator(model, n, noises(model, n), d, **options)
    try:
        out = it.integrate(X0, p, t0, dt, nsteps, stride, seed)
        it.sync()
    finally:
        it.close()
    return out

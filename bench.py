"""Benchmark: orbit-steps/s of the stochastic Kuramoto n = 64 ensemble on one GPU.

Workload (the n = 64 grid configuration): 65,536 orbits on a 256 x 256 grid of
coupling K in [0,4] and noise strength sigma in [0.01, 0.5], omega ~ N(0,1),
Euler-Maruyama with dt = 1e-3 for 2x10^4 steps, order parameter r saved every
100 steps, binary32 state.  One benchmark step = one sode_integrate call over
the whole ensemble (noise generation, coupling, update and saves all inside).

Printed JSON line (rank 0): the driver's contract fields plus
  roofline      the coupled kernel against the VALU issue roofline,
  cpu_baseline  the FP64 oracle timed on a bounded sample on the host,
  cpu_all_cores the same oracle over the 256 grid-diagonal orbits, one OS
                thread per host core (disjoint orbit shards),
  plain_fp64    the one-orbit-per-lane FP64 kernel on the same ensemble,
  error         max |dr| against the oracle on the sampled orbits (and on
                all 256 diagonal orbits from the all-core run, with how
                many are within the bound and, for the worst, how far the
                oracle's own r(T) moves when its inputs move by one ulp),
  meanfield     the same ensemble with the O(n) mean-field drift form,
and the adjoint, ragged-batch and dense-network legs.  --paper-sweep REPS
prints the Sec. 2.2.1 speed protocol instead (one line per case), and
--accuracy-study R the Sec. 2.3.1 accuracy study with R realisations.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X VALU issue roofline.  256 CUs x 4 SIMDs at 2.4 GHz; a SIMD retires
# 32 lanes of a full-rate binary32 add/mul/FMA per clock, so the chip issues
# 256 * 4 * 32 * 2.4e9 = 7.86e13 lane-slots/s, which is the published
# 157.3 TFLOP/s binary32 vector peak counted as one FMA (2 flops) per slot.
VALU_LANE_SLOTS_PER_S = 256 * 4 * 32 * 2.4e9
# Issue cost, in full-rate slots, of each op class the path executes:
# transcendentals (sin, cos, log2, sqrt) are quarter rate, 32-bit integer
# multiplies (high or low half) and binary64 FMAs half rate.
SLOTS = {"valu": 1.0, "trans": 4.0, "imul": 2.0}
# HBM bytes per launch of the n = 64 grid kernel as measured with rocprofv3
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors a 1 GiB copy shows), for
# the kernel as built from the current sources.  The algorithmic figure is
# 103.3 MB (X0 and p read once, r written once).
COUPLED_N64_HBM_BYTES = 50.97e6 + 53.01e6


def algorithmic_slots_per_orbit_step(n: int, compensated: bool = True) -> dict:
    """Minimal work of one Euler-Maruyama step of one n-oscillator orbit with
    pairwise sine coupling (each unordered pair once), Philox-4x32-10 noise
    and Box-Muller normals; counted from the formulation, not the ISA."""
    pairs = n * (n - 1) // 2
    blocks = (n + 3) // 4
    bm_pairs = (n + 1) // 2
    counts = {
        # per pair: one difference, one sine, two accumulations
        "valu": pairs * 3
        # per oscillator: scale to revolutions, two FMAs for the increment,
        # the state update (a four-op Fast2Sum when compensated, else one
        # add) and the 2 pi wrap (scale, round, two FMAs)
        + n * (3 + (4 if compensated else 1) + 4)
        # per Box-Muller pair: two int->float conversions, two scalings,
        # one radius scaling, two products
        + bm_pairs * 7
        # per Philox block: ten rounds of two 3-way XORs
        + blocks * 20,
        "trans": pairs + bm_pairs * 4,
        "imul": blocks * 40,
    }
    counts["slots"] = sum(counts[k] * SLOTS[k] for k in SLOTS)
    return counts


def adjoint_leg(sode, torch, workloads, dev, reps: int = 3) -> dict:
    """Forward (with checkpoints) and backward (adjoint) times of the n = 32
    gradient workload: 4096 orbits sharing (omega, K, sigma), 10^4 steps,
    checkpoints every 100, R = mean r over steps 5000..10000."""
    w = workloads.kuramoto_adjoint()
    n = w["n"]
    X0 = torch.tensor(w["X0"], dtype=torch.float32, device=dev)
    p = torch.tensor(w["p"], dtype=torch.float32, device=dev)
    it = sode.Integrator("kuramoto", n, n, 2 * n + 1, precision=32, shared_params=1)
    args = (0.0, w["dt"], w["nsteps"], w["ckpt_every"], w["win_lo"], w["win_hi"], w["seed"])
    stream = torch.cuda.current_stream()
    fwd, bwd = [], []
    for rep in range(reps + 1):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        ckpt, R = it.forward_ckpt(X0, p, *args)
        e1.record(stream)
        dLdR = 2.0 * (R - w["target"]) / R.numel()
        e1b = torch.cuda.Event(enable_timing=True)
        e1b.record(stream)
        grad, _ = it.adjoint(p, ckpt, *args, dL_dR=dLdR)
        e2.record(stream)
        torch.cuda.synchronize()
        if rep > 0:
            fwd.append(e0.elapsed_time(e1))
            bwd.append(e1b.elapsed_time(e2))
    f, b = float(np.median(fwd)), float(np.median(bwd))
    orbits = X0.shape[0]
    return {"workload": "kuramoto_adjoint_n32", "orbits": orbits, "nsteps": w["nsteps"],
            "forward_ms": f, "backward_ms": b, "ratio_backward_over_forward": b / f,
            "ratio_total_over_forward": (f + b) / f,
            "forward_orbit_steps_per_s": orbits * w["nsteps"] / (f * 1e-3),
            "loss": float(((R - w["target"]) ** 2).mean()),
            "grad_norm": float(grad.norm())}


def ragged_alone_ms(sode, torch, w, j: int, cfg, dev) -> float:
    """Instance j of the ragged workload run alone, in a batch of one, with
    the shape parameters cfg = (waves per CU, units per lane): one warm-up
    and one timed call (HIP events on the launch stream), in ms."""
    stream = torch.cuda.current_stream()
    b1 = sode.RaggedBatch([2 * w["units"][j]], [w["nsteps"][j]], w["stride"], w["seed"], [j], d=5)
    X1 = torch.tensor(b1.pack([w["X0"][j]]), dtype=torch.float32, device=dev)
    p1 = torch.tensor(b1.pack([w["params"][j]]), dtype=torch.float32, device=dev)
    it1 = sode.Integrator("fhn", 256, 128, 5, precision=32, waves_per_cu=cfg[0],
                          units_per_lane=cfg[1])
    it1.integrate_ragged(b1, X1, p1, 0.0, w["dt"])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    it1.integrate_ragged(b1, X1, p1, 0.0, w["dt"])
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1)
    it1.close()
    return t


def ragged_leg(sode, torch, workloads, dev, reps: int = 5) -> dict:
    """Makespan of the 4096-instance FitzHugh-Nagumo batch in one persistent,
    graph-captured launch (autotuned on the first, untimed call), and the
    slowest instance run alone: the batch cannot finish before it."""
    w = workloads.fhn_ragged()
    idx = np.arange(len(w["units"]))
    b = sode.RaggedBatch(2 * w["units"], w["nsteps"], w["stride"], w["seed"],
                         idx.astype(np.uint32), d=5)
    X0 = torch.tensor(b.pack(w["X0"]), dtype=torch.float32, device=dev)
    p = torch.tensor(b.pack(w["params"]), dtype=torch.float32, device=dev)
    it = sode.Integrator("fhn", 256, 128, 5, precision=32)
    out = it.integrate_ragged(b, X0, p, 0.0, w["dt"])
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        it.integrate_ragged(b, X0, p, 0.0, w["dt"], out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    cfg = (it.get_option("ragged_waves_per_cu"), it.get_option("ragged_units_per_lane"))
    unit_steps = int((w["units"] * w["nsteps"]).sum())
    # Critical path: the batch cannot finish before its slowest instance.
    # Each runs on one wave, whose step time depends on its lane shape, so
    # the candidates are the instances with the most steps and those with the
    # most units x steps, each timed alone with the tuned shape; the slowest
    # is reported.
    by_steps = np.argsort(-w["nsteps"], kind="stable")[:4]
    by_work = np.argsort(-(w["units"] * w["nsteps"]), kind="stable")[:4]
    alone, jc = -1.0, int(by_work[0])
    for j in dict.fromkeys(int(c) for c in list(by_steps) + list(by_work)):
        t = ragged_alone_ms(sode, torch, w, j, cfg, dev)
        if t > alone:
            alone, jc = t, j
    return {"workload": "fhn_ragged_4096", "instances": b.count, "unit_steps": unit_steps,
            "makespan_ms": ms, "unit_steps_per_s": unit_steps / (ms * 1e-3),
            "waves_per_cu": cfg[0], "units_per_lane": cfg[1],
            "critical_instance_alone_ms": alone,
            "critical_instance": {"units": int(w["units"][jc]), "nsteps": int(w["nsteps"][jc])},
            "makespan_over_critical": ms / alone}


def rnn_leg(sode, torch, workloads, dev, gemms=("bf16", "bf16x3", "fp32")) -> dict:
    """The n = 256 dense-network workload (8192 orbits, 5000 steps) with each
    matrix-product variant; MFMA work = 2 n^2 flops per orbit-step."""
    w = workloads.rnn_dense()
    n = w["n"]
    X0 = torch.tensor(w["X0"], dtype=torch.float32, device=dev)
    p = torch.tensor(w["p"], dtype=torch.float32, device=dev)
    orbits = X0.shape[0]
    stream = torch.cuda.current_stream()
    res = {"workload": "rnn_dense_n256", "orbits": orbits, "nsteps": w["nsteps"]}
    for gemm in gemms:
        products = 3 if gemm == "bf16x3" else 1
        it = sode.Integrator("rnn", n, n, w["d"], precision=32, shared_params=1,
                             kernel="matrix", gemm=gemm)
        out = it.integrate(X0, p, 0.0, w["dt"], w["nsteps"], w["stride"], w["seed"])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        it.integrate(X0, p, 0.0, w["dt"], w["nsteps"], w["stride"], w["seed"], out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        flops = 2.0 * n * n * orbits * w["nsteps"] * products
        res[gemm] = {"ms": ms, "orbit_steps_per_s": orbits * w["nsteps"] / (ms * 1e-3),
                     "mfma_tflops": flops / (ms * 1e-3) / 1e12}
        it.close()
    return res


NEXT_KURAMOTO4_DRIFT = """
const int N = 4;
for (int i = 0; i < N; ++i) {
    real acc = 0;
    for (int j = 0; j < N; ++j) acc = acc + sin(y[j] - y[i]);
    f[i] = acc * (p[0] / N) + p[1 + i];
}
"""
NEXT_KURAMOTO4_DIFFUSION = "for (int i = 0; i < 4; ++i) gx[i] = p[5 + i] * xi[i];"


def next_rows(sode, torch, dev, reps: int = 3) -> None:
    """Throughput of the steppers and model paths beyond the hot path, one JSON
    line per case, kernel time (HIP events, median of `reps` after a warm-up)
    with inputs resident in HBM: the Milstein stepper against Euler-Maruyama
    on geometric Brownian motion (n = 1, 2^20 orbits); the implicit steppers
    against Euler-Maruyama and RK4 on an FHN chain (n = 6) and alone on a
    stiff OU system (a dt = 10, where the explicit steppers diverge); and the
    n = 4 Kuramoto system given as source text (run-time compiled) against
    the same system built in, on the one-orbit-per-lane kernel."""
    stream = torch.cuda.current_stream()

    def timed(it, X0, p, dt, nsteps, stride):
        out = it.integrate(X0, p, 0.0, dt, nsteps, stride, 11)
        it.sync()
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            it.integrate(X0, p, 0.0, dt, nsteps, stride, 11, out=out)
            e1.record(stream)
            it.sync()
            times.append(e0.elapsed_time(e1))
        return float(np.median(times))

    def emit(row, model, prec, method, orbits, nsteps, ms, **extra):
        line = {"next_row": row, "model": model, "precision": prec, "method": method, "orbits": orbits,
                "nsteps": nsteps, "kernel_ms": ms, "orbit_steps_per_s": orbits * nsteps / (ms * 1e-3)}
        line.update(extra)
        print(json.dumps(line), flush=True)

    rng = np.random.default_rng(17)
    # Milstein vs Euler-Maruyama, geometric Brownian motion.
    orbits, nsteps = 1 << 20, 2000
    for prec, dtype in ((64, torch.float64), (32, torch.float32)):
        X0 = torch.ones((orbits, 1), dtype=dtype, device=dev)
        p = torch.tensor([0.5, 0.4], dtype=dtype, device=dev)
        for method in ("em", "milstein"):
            it = sode.Integrator("gbm", 1, 1, 2, precision=prec, method=method, kernel="plain", shared_params=1)
            emit("milstein", "gbm", prec, method, orbits, nsteps, timed(it, X0, p, 1e-3, nsteps, nsteps))
            it.close()
    # Implicit steppers: FHN chain of 3 units (n = 6), binary64.
    orbits, nsteps = 65536, 1000
    X0 = torch.tensor(rng.uniform(-1.0, 1.0, (orbits, 6)), dtype=torch.float64, device=dev)
    p = torch.tensor([0.7, 0.8, 0.08, 0.1, 0.05], dtype=torch.float64, device=dev)
    for method in ("em", "rk4", "implicit_euler", "implicit_midpoint"):
        it = sode.Integrator("fhn", 6, 3, 5, precision=64, method=method, kernel="plain", shared_params=1,
                             ode_limit=int(method != "em"))
        emit("implicit", "fhn_n6", 64, method, orbits, nsteps, timed(it, X0, p, 0.05, nsteps, nsteps))
        it.close()
    # Stiff OU (n = 3, a dt = 10): only the implicit steppers are stable.
    X0 = torch.tensor(rng.uniform(-1.0, 1.0, (orbits, 3)), dtype=torch.float64, device=dev)
    p = torch.tensor([1000.0, 0.3, 0.5], dtype=torch.float64, device=dev)
    for method in ("implicit_euler", "implicit_midpoint"):
        it = sode.Integrator("ou", 3, 3, 3, precision=64, method=method, kernel="plain", shared_params=1,
                             ode_limit=1)
        emit("implicit", "ou_stiff_n3", 64, method, orbits, nsteps, timed(it, X0, p, 0.01, nsteps, nsteps))
        it.close()
    # Source-text model vs the built-in one: Kuramoto n = 4, binary64.
    orbits, nsteps = 65536, 2000
    X0 = torch.tensor(rng.uniform(0.0, 2.0 * math.pi, (orbits, 4)), dtype=torch.float64, device=dev)
    pk = np.concatenate([[2.0], rng.standard_normal(4), np.full(4, 0.1)])
    p = torch.tensor(pk, dtype=torch.float64, device=dev)
    it = sode.Integrator("kuramoto", 4, 4, 9, precision=64, kernel="plain", shared_params=1)
    builtin = timed(it, X0, p, 1e-3, nsteps, nsteps)
    it.close()
    emit("source_text", "kuramoto_n4_builtin", 64, "em", orbits, nsteps, builtin)
    it = sode.Integrator.custom(NEXT_KURAMOTO4_DRIFT, NEXT_KURAMOTO4_DIFFUSION, 4, 4, 9, precision=64,
                                shared_params=1)
    t0 = time.perf_counter()
    it.build()
    build_s = time.perf_counter() - t0
    ms = timed(it, X0, p, 1e-3, nsteps, nsteps)
    it.close()
    emit("source_text", "kuramoto_n4_text", 64, "em", orbits, nsteps, ms, build_s=build_s,
         over_builtin=ms / builtin)


def op_rates(waves_per_simd=(1, 2, 4, 8)) -> None:
    """Issue cost of each instruction class on gfx950, measured by the
    op-rate microbenchmark (csrc/op_rates.hip, built as libop_rates.so): for
    every class and W waves per SIMD (blocks of 4 waves, 256 W blocks), the
    shader-clock cycles of each wave's loop give the SIMD cycles one wave64
    instruction (or one library call) occupies, cycles / (instructions per
    wave x W), and 64 lanes over that cost give lanes per clock per SIMD.
    The effective clock is the mean cycle count over the launch duration.
    One JSON line per (class, W)."""
    import ctypes
    from paper_1908_03869_amd import build as hipbuild

    if not os.path.exists(hipbuild.OP_RATES_LIB):
        raise RuntimeError(f"{hipbuild.OP_RATES_LIB} is missing: build the package first")
    L = ctypes.CDLL(hipbuild.OP_RATES_LIB)
    L.op_rates_count.restype = ctypes.c_int
    L.op_rates_name.restype = ctypes.c_char_p
    L.op_rates_name.argtypes = [ctypes.c_int]
    L.op_rates_ops_per_wave.restype = ctypes.c_double
    L.op_rates_ops_per_wave.argtypes = [ctypes.c_int, ctypes.c_int]
    L.op_rates_run.restype = ctypes.c_int
    L.op_rates_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    for op in range(L.op_rates_count()):
        name = L.op_rates_name(op).decode()
        library = "library call" in name
        iters = 100 if library else 4000
        for W in waves_per_simd:
            cyc, ms = ctypes.c_double(), ctypes.c_double()
            rc = L.op_rates_run(op, 256 * W, 4, iters, ctypes.byref(cyc), ctypes.byref(ms))
            if rc != 0:
                raise RuntimeError(f"op_rates_run({name}) failed: {rc}")
            ops = L.op_rates_ops_per_wave(op, iters)
            cost = cyc.value / (ops * W)
            print(json.dumps({"op_rates": name, "waves_per_simd": W, "iters": iters,
                              "cycles_per_wave_op": cost, "lanes_per_clk_per_simd": 64.0 / cost,
                              "clock_ghz": cyc.value / (ms.value * 1e6), "kernel_ms": ms.value}),
                  flush=True)


PAPER_N = (5, 10, 15)
PAPER_M = (512, 5120, 25600, 40960, 81920, 163840)


def paper_sweep(sode, torch, workloads, dev, reps: int) -> None:
    """The speed protocol of Sec. 2.2.1 (Tables S1-S3): Kuramoto N in
    {5, 10, 15}, M orbits from 512 to 163,840, K = 1, 8000 Euler-Maruyama
    steps of 0.05 s, in binary64 and binary32 on the one-orbit-per-lane
    kernel and on the 16-lane kernels (padded rows), with the pairwise and
    the mean-field drift.  One JSON line per case: the kernel time with inputs
    resident in HBM and the host-to-host time (upload of X0 and p, the
    integration, download of the saved states), each the median of `reps`
    runs after one warm-up."""
    cases = [(64, "plain"), (64, "coupled"), (32, "plain"), (32, "coupled")]
    for prec, kernel in cases:
        dtype = torch.float64 if prec == 64 else torch.float32
        for N in PAPER_N:
            for drift in ("pairwise", "meanfield"):
                it = sode.Integrator("kuramoto", N, N, 2 * N + 1, precision=prec,
                                     kernel=kernel, drift=drift)
                for M in PAPER_M:
                    w = workloads.kuramoto_paper(N, M)
                    X0h = torch.tensor(w["X0"], dtype=dtype).pin_memory()
                    ph = torch.tensor(w["p"], dtype=dtype).pin_memory()
                    nsave = w["nsteps"] // w["stride"] + 1
                    outh = torch.empty((M, nsave, N), dtype=dtype).pin_memory()
                    X0 = X0h.to(dev)
                    p = ph.to(dev)
                    out = torch.empty((M, nsave, N), dtype=dtype, device=dev)
                    args = (0.0, w["dt"], w["nsteps"], w["stride"], w["seed"])
                    stream = torch.cuda.current_stream()
                    it.integrate(X0, p, *args, out=out)
                    torch.cuda.synchronize()
                    kern, host = [], []
                    for _ in range(reps):
                        e0 = torch.cuda.Event(enable_timing=True)
                        e1 = torch.cuda.Event(enable_timing=True)
                        e0.record(stream)
                        it.integrate(X0, p, *args, out=out)
                        e1.record(stream)
                        torch.cuda.synchronize()
                        kern.append(e0.elapsed_time(e1))
                        h0 = time.perf_counter()
                        X0.copy_(X0h, non_blocking=True)
                        p.copy_(ph, non_blocking=True)
                        it.integrate(X0, p, *args, out=out)
                        outh.copy_(out, non_blocking=True)
                        torch.cuda.synchronize()
                        host.append((time.perf_counter() - h0) * 1e3)
                    k_ms, h_ms = float(np.median(kern)), float(np.median(host))
                    print(json.dumps({
                        "sweep": "paper_kuramoto", "precision": prec, "kernel": kernel, "N": N,
                        "M": M, "drift": drift, "nsteps": w["nsteps"], "stride": w["stride"],
                        "kernel_ms": k_ms, "host_ms": h_ms,
                        "orbit_steps_per_s": M * w["nsteps"] / (k_ms * 1e-3)}), flush=True)
                it.close()


def accuracy_study(sode, torch, workloads, dev, realisations: int, oracle_threads: int) -> None:
    """The accuracy and stability study of Sec. 2.3.1: N = 100 Kuramoto,
    omega ~ U(0.2, 0.4), noise strengths ~ U(0.01, 0.03), K in {0.02, 0.2},
    400 s at dt = 2^(l-5)/5 for l = 1..5, r(t) every 20 s.  Per (K, l), one
    binary32 launch of the 16-lane kernel (padded rows) over all
    realisations, then <r(t)> and sigma(r(t)) over the realisations from
    sode_ensemble_stats; the FP64 oracle integrates the same realisations
    (same Philox streams) on the host and its statistics and the pathwise
    max |dr| are printed beside them.  One JSON line per (K, l)."""
    import oracle

    for K in (0.02, 0.2):
        for level in (1, 2, 3, 4, 5):
            w = workloads.kuramoto_e4(K, realisations=realisations, level=level)
            n = w["n"]
            it = sode.Integrator("kuramoto", n, n, w["d"], precision=32, kernel="coupled",
                                 observable="kuramoto_r")
            X0 = torch.tensor(w["X0"], dtype=torch.float32, device=dev)
            p = torch.tensor(w["p"], dtype=torch.float32, device=dev)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            stream = torch.cuda.current_stream()
            e0.record(stream)
            r = it.integrate(X0, p, 0.0, w["dt"], w["nsteps"], w["stride"], w["seed"])
            e1.record(stream)
            mean, std = it.ensemble_stats(r[:, :, 0].contiguous())
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            r_gpu = r[:, :, 0].double().cpu().numpy()
            it.close()
            c0 = time.perf_counter()
            X32 = w["X0"].astype(np.float32).astype(np.float64)
            p32 = w["p"].astype(np.float32).astype(np.float64)
            ref = oracle.integrate_parallel("kuramoto", n, n, w["d"], X32, p32, 0.0, w["dt"],
                                            w["nsteps"], w["stride"], w["seed"],
                                            threads=oracle_threads,
                                            observable="kuramoto_r")[:, :, 0]
            cpu_s = time.perf_counter() - c0
            t = (np.arange(ref.shape[1]) * w["stride"] * w["dt"]).tolist()
            print(json.dumps({
                "study": "kuramoto_e4", "K": K, "level": level, "dt": w["dt"],
                "nsteps": w["nsteps"], "realisations": realisations, "t": t,
                "mean_r": mean.cpu().numpy().tolist(), "std_r": std.cpu().numpy().tolist(),
                "oracle_mean_r": ref.mean(axis=0).tolist(),
                "oracle_std_r": ref.std(axis=0, ddof=1).tolist(),
                "max_abs_dr": float(np.max(np.abs(r_gpu - ref))),
                "gpu_ms": ms, "oracle_s": cpu_s, "oracle_threads": oracle_threads}),
                flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--baseline-steps", type=int, default=1000,
                    help="Euler steps for the plain FP64 comparison run")
    ap.add_argument("--cpu-orbits", type=int, default=16,
                    help="orbits of the oracle sample (full 2x10^4 steps each)")
    ap.add_argument("--cpu-all-orbits", type=int, default=256,
                    help="grid-diagonal orbits of the all-core oracle run (0: skip it)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--grid-only", action="store_true",
                    help="time only the n = 64 grid kernel (for short profiler runs)")
    ap.add_argument("--accuracy-study", type=int, default=0, metavar="REALISATIONS",
                    help="instead of the benchmark line, run the Sec. 2.3.1 accuracy study "
                         "with this many realisations per (K, dt), oracle alongside")
    ap.add_argument("--oracle-threads", type=int, default=16)
    ap.add_argument("--next-rows", action="store_true",
                    help="time the Milstein, implicit and source-text model paths (one JSON "
                         "line per case)")
    ap.add_argument("--rnn-only", choices=("bf16", "bf16x3", "fp32"), default=None,
                    help="time only the dense-network workload with this matrix variant "
                         "(one warm-up and one timed launch) and print its JSON")
    ap.add_argument("--ragged-alone", type=int, default=None, metavar="INSTANCE",
                    help="time one instance of the ragged FHN workload alone (a batch of one; "
                         "one warm-up and one timed launch) and print its JSON")
    ap.add_argument("--waves-per-cu", type=int, default=4,
                    help="ragged shape for --ragged-alone: persistent waves per CU")
    ap.add_argument("--units-per-lane", type=int, default=1,
                    help="ragged shape for --ragged-alone: minimum units per lane")
    ap.add_argument("--paper-sweep", type=int, default=0, metavar="REPS",
                    help="instead of the benchmark line, time the Sec. 2.2.1 speed protocol "
                         "(N x M x precision x drift form), REPS runs per case")
    ap.add_argument("--op-rates", action="store_true",
                    help="instead of the benchmark line, measure the issue cost of each "
                         "instruction class (one JSON line per class and waves per SIMD)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run a plain device-to-device copy of this many MiB, so that "
                         "HBM byte counters can be scaled against a kernel of known traffic")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; an ensemble "
              "shards across GPUs by orbit_offset, one process per GPU.", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads
    import paper_1908_03869_amd as sode

    dev = torch.device("cuda:0")
    if args.op_rates:
        op_rates()
        return
    if args.paper_sweep:
        paper_sweep(sode, torch, workloads, dev, args.paper_sweep)
        return
    if args.accuracy_study:
        accuracy_study(sode, torch, workloads, dev, args.accuracy_study, args.oracle_threads)
        return
    if args.next_rows:
        next_rows(sode, torch, dev)
        return
    if args.rnn_only:
        print(json.dumps(rnn_leg(sode, torch, workloads, dev, gemms=(args.rnn_only,))))
        return
    if args.ragged_alone is not None:
        w = workloads.fhn_ragged()
        j = args.ragged_alone
        ms = ragged_alone_ms(sode, torch, w, j, (args.waves_per_cu, args.units_per_lane), dev)
        print(json.dumps({"workload": "fhn_ragged_4096", "instance": j,
                          "units": int(w["units"][j]), "nsteps": int(w["nsteps"][j]),
                          "waves_per_cu": args.waves_per_cu, "units_per_lane": args.units_per_lane,
                          "kernel_ms": ms, "ns_per_step": ms * 1e6 / int(w["nsteps"][j])}))
        return
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = workloads.kuramoto_grid()
    n, orbits, nsteps, stride = w["n"], w["X0"].shape[0], w["nsteps"], w["stride"]
    X0 = torch.tensor(w["X0"], dtype=torch.float32, device=dev)
    p = torch.tensor(w["p"], dtype=torch.float32, device=dev)
    it = sode.Integrator("kuramoto", n, n, 2 * n + 1, precision=32, observable="kuramoto_r")
    out = torch.empty((orbits, nsteps // stride + 1, 1), dtype=torch.float32, device=dev)

    def step():
        it.integrate(X0, p, 0.0, w["dt"], nsteps, stride, w["seed"], out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
    ms_per_step = elapsed * 1e3 / args.steps
    value = orbits * nsteps / (ms_per_step * 1e-3)

    work = algorithmic_slots_per_orbit_step(n)
    achieved = work["slots"] * orbits * nsteps / (kernel_ms * 1e-3)
    r_gpu = out[:, -1, 0].double().cpu().numpy()

    plain_rate = mf_ms = None
    r_mf = None
    adj = rag = rnn = None
    if not args.grid_only:
        # Plain FP64 one-orbit-per-lane kernel on the same ensemble (fewer steps;
        # its per-step cost does not depend on the step count).
        it64 = sode.Integrator("kuramoto", n, n, 2 * n + 1, precision=64, observable="kuramoto_r")
        X64, p64 = X0.double(), p.double()
        bsteps = args.baseline_steps
        out64 = torch.empty((orbits, bsteps // stride + 1, 1), dtype=torch.float64, device=dev)
        it64.integrate(X64[:256], p64[:256], 0.0, w["dt"], stride, stride, w["seed"])
        torch.cuda.synchronize()
        b0 = torch.cuda.Event(enable_timing=True)
        b1 = torch.cuda.Event(enable_timing=True)
        b0.record(stream)
        it64.integrate(X64, p64, 0.0, w["dt"], bsteps, stride, w["seed"], out=out64)
        b1.record(stream)
        torch.cuda.synchronize()
        plain_ms = b0.elapsed_time(b1)
        plain_rate = orbits * bsteps / (plain_ms * 1e-3)

        # The same ensemble with the O(n) mean-field form of the coupling.
        itmf = sode.Integrator("kuramoto", n, n, 2 * n + 1, precision=32, observable="kuramoto_r",
                               drift="meanfield")
        outmf = torch.empty_like(out)
        itmf.integrate(X0, p, 0.0, w["dt"], nsteps, stride, w["seed"], out=outmf)
        torch.cuda.synchronize()
        m0 = torch.cuda.Event(enable_timing=True)
        m1 = torch.cuda.Event(enable_timing=True)
        m0.record(stream)
        itmf.integrate(X0, p, 0.0, w["dt"], nsteps, stride, w["seed"], out=outmf)
        m1.record(stream)
        torch.cuda.synchronize()
        mf_ms = m0.elapsed_time(m1)
        r_mf = outmf[:, -1, 0].double().cpu().numpy()
        itmf.close()

        adj = adjoint_leg(sode, torch, workloads, dev)
        rag = ragged_leg(sode, torch, workloads, dev)
        rnn = rnn_leg(sode, torch, workloads, dev)

    cpu = cpu_all = diag = None
    err = err_mf = err_all = None
    if not args.no_cpu:
        import oracle
        rows = w["diagonal"][np.linspace(0, 255, args.cpu_orbits).astype(int)]
        c0 = time.perf_counter()
        # The oracle gets the float32-rounded inputs the kernel received.
        X32 = w["X0"][rows].astype(np.float32).astype(np.float64)
        p32 = w["p"][rows].astype(np.float32).astype(np.float64)
        ref = oracle.integrate("kuramoto", n, n, 2 * n + 1, X32, p32, 0.0,
                               w["dt"], nsteps, stride, w["seed"], orbit_ids=rows,
                               observable="kuramoto_r")
        cpu_s = time.perf_counter() - c0
        cpu = {"value": len(rows) * nsteps / cpu_s, "unit": "orbit*steps/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{len(rows)} grid-diagonal orbits x {nsteps} steps, FP64, "
                         f"single-threaded, {cpu_s:.1f} s"}
        err = float(np.max(np.abs(r_gpu[rows] - ref[:, -1, 0])))
        if r_mf is not None:
            err_mf = float(np.max(np.abs(r_mf[rows] - ref[:, -1, 0])))
        if args.cpu_all_orbits > 0:
            # Orbits are independent: one thread per core over disjoint shards
            # (the all-core CPU figure beside the single-core one).
            rows_all = w["diagonal"][np.linspace(0, 255, args.cpu_all_orbits).astype(int)]
            nthreads = max(1, min(args.oracle_threads, os.cpu_count() or 1))
            c0 = time.perf_counter()
            ref_all = oracle.integrate_parallel(
                "kuramoto", n, n, 2 * n + 1, w["X0"][rows_all].astype(np.float32).astype(np.float64),
                w["p"][rows_all].astype(np.float32).astype(np.float64), 0.0, w["dt"], nsteps,
                stride, w["seed"], threads=nthreads, orbit_ids=rows_all, observable="kuramoto_r")
            all_s = time.perf_counter() - c0
            cpu_all = {"value": len(rows_all) * nsteps / all_s, "unit": "orbit*steps/s",
                       "cores": nthreads, "kind": "oracle",
                       "sample": f"{len(rows_all)} grid-diagonal orbits x {nsteps} steps, FP64, "
                                 f"{nthreads} threads, {all_s:.1f} s"}
            dr_all = np.abs(r_gpu[rows_all] - ref_all[:, -1, 0])
            err_all = float(dr_all.max())
            within_all = int((dr_all <= 1e-4).sum())
            worst = int(np.argmax(dr_all))
            # Conditioning of the worst orbit: the oracle's own |dr(T)| when its
            # initial phases move by one binary32 ulp (2^-24 relative, eight
            # seeded sign patterns).
            Xw = w["X0"][rows_all[worst]].astype(np.float32).astype(np.float64)
            pw = w["p"][rows_all[worst]].astype(np.float32).astype(np.float64)
            Xs = np.stack([Xw * (1.0 + np.random.default_rng(1000 + k).choice([-1.0, 1.0], n)
                                 * 2.0 ** -24) for k in range(8)])
            resp = oracle.integrate_parallel(
                "kuramoto", n, n, 2 * n + 1, Xs, np.stack([pw] * 8), 0.0, w["dt"], nsteps,
                nsteps, w["seed"], threads=min(8, nthreads),
                orbit_ids=np.full(8, rows_all[worst]), observable="kuramoto_r")[:, -1, 0]
            diag = {"orbits": len(rows_all), "within_tolerance": within_all,
                    "worst_orbit": int(rows_all[worst]),
                    "worst_oracle_ulp_response": float(np.abs(resp - ref_all[worst, -1, 0]).max())}

    line = {
        "metric": "orbit*steps/s (Kuramoto n=64 FP32 Euler-Maruyama ensemble)",
        "value": value,
        "unit": "orbit*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "kuramoto_grid_n64", "orbits": orbits, "n": n,
                   "nsteps": nsteps, "dt": w["dt"], "stride": stride,
                   "observable": "kuramoto_r", "kernel": "coupled"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                     "peak": VALU_LANE_SLOTS_PER_S / 1e12,
                     "unit": "T VALU lane-slots/s (1 slot = one binary32 FMA)",
                     "frac": achieved / VALU_LANE_SLOTS_PER_S,
                     "traffic": COUPLED_N64_HBM_BYTES, "traffic_unit": "HBM bytes per launch",
                     "kernel_ms": kernel_ms,
                     "slots_per_orbit_step": work["slots"]},
        "cpu_baseline": cpu,
        "cpu_all_cores": cpu_all,
        "plain_fp64": None if plain_rate is None else {
            "value": plain_rate, "unit": "orbit*steps/s", "nsteps": args.baseline_steps,
            "speedup_of_value": value / plain_rate},
        "error": {"max_abs_dr_final": err, "max_abs_dr_final_diagonal": err_all,
                  "tolerance": 1e-4, "diagonal": diag},
        "meanfield": None if mf_ms is None else {
            "value": orbits * nsteps / (mf_ms * 1e-3), "unit": "orbit*steps/s",
            "kernel_ms": mf_ms, "max_abs_dr_final": err_mf},
        "adjoint": adj,
        "ragged": rag,
        "rnn": rnn,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()

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
  plain_fp64, lanes16_fp64
                the one-orbit-per-lane and the 16-lane FP64 kernels on the
                same ensemble, each with its binary64 roofline fraction,
  small_fp64    the n = 4 binary64 ensemble (1024 orbits x 10^4 steps),
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
COUPLED_N64_HBM_BYTES = 50.98e6 + 54.24e6


# Binary64 VALU issue: a SIMD retires 16 lanes of v_fma_f64 per clock, so the
# chip issues 256 * 4 * 16 * 2.4e9 = 3.93e13 binary64 FMA lane-slots/s, the
# published 78.6 TFLOP/s binary64 vector peak.
FP64_FMA_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
# Issue cost in binary64 FMA slots of each operation class of the binary64
# Kuramoto step: measured wave64 issue cycles (the op-rate microbenchmark,
# bench.py --op-rates, four waves per SIMD) divided by the 4.30 cycles of one
# v_fma_f64.  "sin_phase" is the coupled kernels' sine of a phase difference
# (73.0 cycles per call), "box_muller_pair" their pair of normals from two
# 24-bit uniforms with the logarithm, square root, cosine and sine (462.8
# cycles; the pair on the library's log, sqrt and sincospi takes 666.9), both
# as timed in a dependent chain that adds one binary64 add per call (and, for
# the pair, the derivation of its words); "imul" a v_mad_u64_u32 (4.66),
# "valu32" a v_bitop3_b32 (3.04).  Pricing each function at the cheapest
# implementation measured keeps the work, and so the fraction, conservative.
FP64_SLOTS = {"sin_phase": 17.0, "box_muller_pair": 107.6, "fma64": 1.0, "imul": 1.08, "valu32": 0.71}


def fp64_slots_per_orbit_step(n: int) -> dict:
    """Minimal work of one binary64 Euler-Maruyama step of one n-oscillator
    Kuramoto orbit, each unordered pair's sine once, in binary64 FMA slots."""
    pairs = n * (n - 1) // 2
    blocks = (n + 3) // 4
    bm = (n + 1) // 2
    counts = {
        # per pair: the sine of the phase difference, one difference and two
        # accumulations
        "sin_phase": pairs,
        "box_muller_pair": bm,
        # per pair 3 ops; per oscillator: two FMAs for the increment, the
        # state add and the 2 pi wrap (scale, round, two FMAs)
        "fma64": pairs * 3 + n * 7,
        # per Philox block: ten rounds of two 32 x 32 -> 64 products
        # (v_mad_u64_u32) and two three-way XORs
        "imul": blocks * 20,
        "valu32": blocks * 20,
    }
    counts["slots"] = sum(counts[k] * FP64_SLOTS[k] for k in FP64_SLOTS)
    return counts


def host_threads() -> tuple[int, int]:
    """(CPUs in this process's affinity mask, threads the multi-threaded
    oracle runs use).  The oracle legs run one thread per CPU of the mask,
    at most 16 (one GPU's share of the shared hosts this is measured on)."""
    visible = len(os.sched_getaffinity(0))
    return visible, max(1, min(16, visible))


def stratified_instances(units, nsteps, bins: int = 8) -> np.ndarray:
    """One instance per cell of a bins x bins grid of (unit count, step
    count) quantile bins, the first in index order; cells with no instance
    are filled with the first instances not yet taken, so the sample always
    has bins^2 instances (if the batch has that many)."""
    units, nsteps = np.asarray(units), np.asarray(nsteps)
    qu = np.quantile(units, np.linspace(0, 1, bins + 1)[1:-1])
    qs = np.quantile(nsteps, np.linspace(0, 1, bins + 1)[1:-1])
    cu = np.searchsorted(qu, units, side="right")
    cs = np.searchsorted(qs, nsteps, side="right")
    taken, seen = [], set()
    for i in range(len(units)):
        cell = (int(cu[i]), int(cs[i]))
        if cell not in seen:
            seen.add(cell)
            taken.append(i)
    for i in range(len(units)):
        if len(taken) >= bins * bins:
            break
        if i not in taken:
            taken.append(i)
    return np.sort(np.asarray(taken[:bins * bins], dtype=np.int64))


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


def adjoint_leg(sode, torch, workloads, dev, reps: int = 3, cpu: bool = True) -> dict:
    """Forward (with checkpoints) and backward (adjoint) times of the n = 32
    gradient workload: 4096 orbits sharing (omega, K, sigma), 10^4 steps,
    checkpoints every 100, R = mean r over steps 5000..10000, loss = mean
    (R - 0.6)^2.  Error: relative L2 error of the loss gradient against the
    FP64 oracle adjoint of the same orbits (stored with the tests), over the
    whole vector and per block (K, frequencies, noise strengths).  CPU
    baseline: the FP64 oracle adjoint (forward and reverse) on 8 orbits."""
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
    g = grad.double().cpu().numpy()
    res = {"workload": "kuramoto_adjoint_n32", "orbits": orbits, "nsteps": w["nsteps"],
           "forward_ms": f, "backward_ms": b, "ratio_backward_over_forward": b / f,
           "ratio_total_over_forward": (f + b) / f,
           "forward_orbit_steps_per_s": orbits * w["nsteps"] / (f * 1e-3),
           "loss": float(((R - w["target"]) ** 2).mean()),
           "grad_norm": float(np.linalg.norm(g))}
    golden = os.path.join(ROOT, "tests", "golden", "kuramoto_adjoint_n32.json")
    with open(golden) as fh:
        gref = np.array(json.load(fh)["grad"])
    blocks = {"K": slice(0, 1), "omega": slice(1, n + 1), "sigma": slice(n + 1, 2 * n + 1)}
    res["error"] = {
        "grad_rel_l2": float(np.linalg.norm(g - gref) / np.linalg.norm(gref)),
        "per_block_rel_l2": {k: float(np.linalg.norm(g[s] - gref[s]) / np.linalg.norm(gref[s]))
                             for k, s in blocks.items()},
        "tolerance": 1e-3, "reference": "FP64 oracle adjoint, all 4096 orbits (stored)"}
    if cpu:
        import oracle
        rows = np.arange(8)
        c0 = time.perf_counter()
        oracle.kuramoto_adjoint(n, w["X0"][rows].astype(np.float32).astype(np.float64),
                                w["p"].astype(np.float32).astype(np.float64), 0.0, w["dt"],
                                w["nsteps"], w["win_lo"], w["win_hi"], w["seed"], per_orbit=False)
        cs = time.perf_counter() - c0
        res["cpu_baseline"] = {
            "value": len(rows) * w["nsteps"] / cs, "unit": "orbit*steps/s (forward + adjoint)",
            "cores": 1, "kind": "oracle",
            "sample": f"{len(rows)} orbits x {w['nsteps']} steps, FP64 forward and reverse "
                      f"pass, single-threaded, {cs:.1f} s"}
        res["gpu_orbit_steps_per_s_forward_plus_adjoint"] = orbits * w["nsteps"] / ((f + b) * 1e-3)
    return res


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


def ragged_leg(sode, torch, workloads, dev, reps: int = 5, cpu: bool = True) -> dict:
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
    res = {"workload": "fhn_ragged_4096", "instances": b.count, "unit_steps": unit_steps,
           "makespan_ms": ms, "unit_steps_per_s": unit_steps / (ms * 1e-3),
           "waves_per_cu": cfg[0], "units_per_lane": cfg[1],
           "critical_instance_alone_ms": alone,
           "critical_instance": {"units": int(w["units"][jc]), "nsteps": int(w["nsteps"][jc])},
           "makespan_over_critical": ms / alone}
    if cpu:
        # Error on 64 instances stratified by unit and step count: per
        # instance max_s |dX|_inf / max(1, max_s |X|_inf) against the FP64
        # oracle on the float32-rounded inputs the kernel received.
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        got_all = out.double().cpu().numpy()
        sel = stratified_instances(w["units"], w["nsteps"])
        X0r = b.pack(w["X0"]).astype(np.float32).astype(np.float64)
        pr = b.pack(w["params"]).astype(np.float32).astype(np.float64)

        def ref_of(i):
            a, nn = int(b.x0_offset[i]), int(b.n[i])
            return oracle.integrate("fhn", nn, nn // 2, 5, X0r[a:a + nn][None], pr[5 * i:5 * i + 5],
                                    0.0, w["dt"], int(b.nsteps[i]), int(b.stride[i]), w["seed"],
                                    orbit_ids=[int(i)])[0]

        _, nthreads = host_threads()
        with ThreadPoolExecutor(max_workers=nthreads) as ex:
            refs = list(ex.map(ref_of, sel))
        errs = np.array([np.abs(b.unpack(got_all, int(i)) - r).max() / max(1.0, np.abs(r).max())
                         for i, r in zip(sel, refs)])
        res["error"] = {"max_rel": float(errs.max()), "median_rel": float(np.median(errs)),
                        "within_tolerance": int((errs <= 1e-4).sum()), "instances": len(sel),
                        "tolerance": 1e-4, "sample": "64 instances stratified by units x steps"}
        # CPU baseline: the oracle single-threaded on every 4th instance of the sample.
        sub = sel[::4]
        c0 = time.perf_counter()
        for i in sub:
            ref_of(i)
        cs = time.perf_counter() - c0
        us = int((w["units"][sub] * w["nsteps"][sub]).sum())
        res["cpu_baseline"] = {"value": us / cs, "unit": "unit*steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"{len(sub)} of the stratified instances ({us} unit-steps), "
                                         f"FP64, single-threaded, {cs:.1f} s"}
    return res


def rnn_leg(sode, torch, workloads, dev, gemms=("bf16", "bf16x3", "fp32"), cpu: bool = True) -> dict:
    """The n = 256 dense-network workload (8192 orbits, 5000 steps) with each
    matrix-product variant; MFMA work = 2 n^2 flops per orbit-step.  Error
    per variant: relative L2 norm of the final-state difference per orbit
    against the FP64 oracle (float32-rounded inputs), max and median over 64
    orbits (every 128th); bound 1e-2.  CPU baseline: the oracle on 4 orbits."""
    w = workloads.rnn_dense()
    n = w["n"]
    X0 = torch.tensor(w["X0"], dtype=torch.float32, device=dev)
    p = torch.tensor(w["p"], dtype=torch.float32, device=dev)
    orbits = X0.shape[0]
    stream = torch.cuda.current_stream()
    res = {"workload": "rnn_dense_n256", "orbits": orbits, "nsteps": w["nsteps"]}
    rows = np.arange(0, orbits, orbits // 64)
    ref = None
    if cpu:
        import oracle
        _, nthreads = host_threads()
        Xr = w["X0"].astype(np.float32).astype(np.float64)
        pr = w["p"].astype(np.float32).astype(np.float64)
        ref = oracle.integrate_parallel("rnn", n, n, w["d"], Xr[rows], pr, 0.0, w["dt"], w["nsteps"],
                                        w["nsteps"], w["seed"], threads=nthreads,
                                        orbit_ids=rows.astype(np.uint32))[:, -1]
        sub = rows[:4]
        c0 = time.perf_counter()
        oracle.integrate("rnn", n, n, w["d"], Xr[sub], pr, 0.0, w["dt"], w["nsteps"], w["nsteps"],
                         w["seed"], orbit_ids=sub.astype(np.uint32))
        cs = time.perf_counter() - c0
        res["cpu_baseline"] = {"value": len(sub) * w["nsteps"] / cs, "unit": "orbit*steps/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"{len(sub)} orbits x {w['nsteps']} steps, FP64, "
                                         f"single-threaded, {cs:.1f} s"}
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
        if ref is not None:
            got = out[:, -1][torch.as_tensor(rows, device=out.device)].double().cpu().numpy()
            rel = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
            res[gemm]["error"] = {"max_rel_l2": float(rel.max()), "median_rel_l2": float(np.median(rel)),
                                  "tolerance": 1e-2, "orbits": len(rows)}
        it.close()
    return res


def small_fp64_leg(sode, torch, workloads, dev, reps: int = 5, cpu: bool = True) -> dict:
    """The n = 4 binary64 ensemble: 1024 orbits (32 coupling values x 32
    seeds, the orbits of one seed sharing its Brownian path), dt = 1e-3,
    10^4 steps, state saved every 100 steps.  Kernel time (HIP events, median
    of `reps` after a warm-up) on the automatically chosen kernel (the
    coupled kernel's four-lane form: one oscillator per lane, DPP quad
    permutations) and on one orbit per lane; error = max circular |dtheta| over
    all 1024 orbits and saves against the FP64 oracle (bound 1e-10), which
    is also timed single-threaded on all of them.

    FP64 roofline: the work of one orbit-step counted from the formulation
    (each unordered pair's sine once, the Box-Muller functions of m/2 pairs,
    the per-pair and per-oscillator arithmetic, one Philox block), each
    class priced in binary64 FMA issue slots by its measured cost, against
    the chip's 256 x 4 x 16 x 2.4e9 = 3.93e13 binary64 FMA lane-slots/s
    (78.6 TFLOP/s).  1024 orbits are 16 waves on one lane each, or 64 on
    four lanes: far fewer than the chip's 1024 SIMDs, so the fraction also
    says how much of the chip this small ensemble can occupy."""
    w = workloads.kuramoto_small()
    n, orbits, nsteps, stride = w["n"], w["X0"].shape[0], w["nsteps"], w["stride"]
    X0 = torch.tensor(w["X0"], dtype=torch.float64, device=dev)
    p = torch.tensor(w["p"], dtype=torch.float64, device=dev)
    ids = torch.tensor(w["orbit_ids"].astype(np.int32), device=dev)
    seeds = torch.tensor(w["orbit_seeds"].astype(np.int64), device=dev)
    stream = torch.cuda.current_stream()
    res = {"workload": "kuramoto_small_n4_fp64", "orbits": orbits, "n": n, "nsteps": nsteps,
           "dt": w["dt"], "stride": stride}
    outs = {}
    for kernel in ("auto", "plain"):
        it = sode.Integrator("kuramoto", n, n, 2 * n + 1, precision=64, kernel=kernel)
        out = torch.empty((orbits, nsteps // stride + 1, n), dtype=torch.float64, device=dev)
        call = lambda: it.integrate(X0, p, 0.0, w["dt"], nsteps, stride, w["seed"], orbit_ids=ids,
                                    orbit_seeds=seeds, out=out)
        call()
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            call()
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        name = "coupled" if kernel == "auto" else "plain"
        res[name] = {"kernel_ms": ms, "orbit_steps_per_s": orbits * nsteps / (ms * 1e-3),
                     "us_per_step": ms * 1e3 / nsteps}
        outs[name] = out.cpu().numpy()
        it.close()
    work = fp64_slots_per_orbit_step(n)
    for name in ("coupled", "plain"):
        achieved = work["slots"] * orbits * nsteps / (res[name]["kernel_ms"] * 1e-3)
        res[name]["roofline"] = {"bound": "alu", "achieved": achieved / 1e12,
                                 "peak": FP64_FMA_SLOTS_PER_S / 1e12,
                                 "unit": "T binary64 FMA lane-slots/s", "frac": achieved / FP64_FMA_SLOTS_PER_S,
                                 "slots_per_orbit_step": work["slots"]}
    if cpu:
        import oracle
        c0 = time.perf_counter()
        ref = oracle.integrate("kuramoto", n, n, 2 * n + 1, w["X0"], w["p"], 0.0, w["dt"], nsteps,
                               stride, w["seed"], orbit_ids=w["orbit_ids"],
                               orbit_seeds=w["orbit_seeds"])
        cs = time.perf_counter() - c0
        res["cpu_baseline"] = {"value": orbits * nsteps / cs, "unit": "orbit*steps/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"all {orbits} orbits x {nsteps} steps, FP64, "
                                         f"single-threaded, {cs:.1f} s"}
        for name in ("coupled", "plain"):
            d = np.abs(np.remainder(outs[name] - ref + math.pi, 2 * math.pi) - math.pi)
            res[name]["error"] = {"max_circular_dtheta": float(d.max()), "tolerance": 1e-10}
    return res


def grid_fp64_leg(sode, torch, w, X0, p, dev, bsteps: int, rows, ref_rows=None) -> dict:
    """Binary64 kernels on the n = 64 grid ensemble, `bsteps` steps (their
    per-step cost does not depend on the step count): one orbit per lane (the
    plain FP64 per-orbit baseline) and 16 lanes per orbit.  Error: max |dr| at
    the last step over the sampled orbits `rows` against the oracle.  Each
    carries the binary64 roofline of the small_fp64 leg: the formulation's
    work per orbit-step (2016 pair sines for n = 64) in binary64 FMA slots
    against the chip's binary64 issue peak; 65,536 orbits fill the chip."""
    import oracle
    n, orbits, stride = w["n"], X0.shape[0], w["stride"]
    X64, p64 = X0.double(), p.double()
    stream = torch.cuda.current_stream()
    if ref_rows is None:
        ref_rows = oracle.integrate_parallel(
            "kuramoto", n, n, 2 * n + 1, w["X0"][rows].astype(np.float32).astype(np.float64),
            w["p"][rows].astype(np.float32).astype(np.float64), 0.0, w["dt"], bsteps, bsteps,
            w["seed"], threads=host_threads()[1], orbit_ids=rows, observable="kuramoto_r")[:, -1, 0]
    res = {}
    work = fp64_slots_per_orbit_step(n)
    for kernel, name in (("plain", "plain_fp64"), ("coupled", "lanes16_fp64")):
        it = sode.Integrator("kuramoto", n, n, 2 * n + 1, precision=64, observable="kuramoto_r",
                             kernel=kernel)
        out = torch.empty((orbits, bsteps // stride + 1, 1), dtype=torch.float64, device=dev)
        # Warm-up on the whole ensemble (the kernel choice depends on the orbit count).
        it.integrate(X64, p64, 0.0, w["dt"], stride, stride, w["seed"])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        it.integrate(X64, p64, 0.0, w["dt"], bsteps, stride, w["seed"], out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        r = out[:, -1, 0].cpu().numpy()[rows]
        res[name] = {"value": orbits * bsteps / (ms * 1e-3), "unit": "orbit*steps/s", "nsteps": bsteps,
                     "kernel_ms": ms,
                     "error": {"max_abs_dr": float(np.abs(r - ref_rows).max()), "orbits": len(rows),
                               "tolerance": 1e-4}}
        achieved = work["slots"] * orbits * bsteps / (ms * 1e-3)
        res[name]["roofline"] = {"bound": "alu", "achieved": achieved / 1e12,
                                 "peak": FP64_FMA_SLOTS_PER_S / 1e12,
                                 "unit": "T binary64 FMA lane-slots/s", "frac": achieved / FP64_FMA_SLOTS_PER_S,
                                 "slots_per_orbit_step": work["slots"]}
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


def op_rates(waves_per_simd=(1, 2, 4)) -> None:
    """Issue cost of each instruction class on gfx950, measured by the
    op-rate microbenchmark (csrc/op_rates.hip, built as libop_rates.so): one
    workgroup per CU with W waves on each SIMD, all starting together; the
    span of a workgroup's loops gives the SIMD cycles of W waves'
    instructions, so one wave64 instruction (or one library call) occupies
    span / (W x instructions per wave) cycles, and 64 lanes over that cost
    give lanes per clock per SIMD.  The clock is the span over the launch
    duration.  One JSON line per (class, W)."""
    import ctypes
    import torch
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
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for op in range(L.op_rates_count()):
        name = L.op_rates_name(op).decode()
        library = "library call" in name or "per call" in name
        iters = 100 if library else 4000
        for W in waves_per_simd:
            span, ms = ctypes.c_double(), ctypes.c_double()
            rc = L.op_rates_run(op, cus, 4 * W, iters, ctypes.byref(span), ctypes.byref(ms))
            if rc != 0:
                raise RuntimeError(f"op_rates_run({name}) failed: {rc}")
            ops = L.op_rates_ops_per_wave(op, iters)
            cost = span.value / (ops * W)
            print(json.dumps({"op_rates": name, "waves_per_simd": W, "iters": iters,
                              "cycles_per_wave_op": cost, "lanes_per_clk_per_simd": 64.0 / cost,
                              "clock_ghz": span.value / (ms.value * 1e6), "kernel_ms": ms.value}),
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
    ap.add_argument("--oracle-threads", type=int, default=0,
                    help="threads of the all-core oracle runs (0: one per CPU of the affinity "
                         "mask, at most 16)")
    ap.add_argument("--next-rows", action="store_true",
                    help="time the Milstein, implicit and source-text model paths (one JSON "
                         "line per case)")
    ap.add_argument("--rnn-only", choices=("bf16", "bf16x3", "fp32"), default=None,
                    help="time only the dense-network workload with this matrix variant "
                         "(one warm-up and one timed launch) and print its JSON")
    ap.add_argument("--small-fp64-only", action="store_true",
                    help="time only the n = 4 binary64 ensemble (1024 orbits x 10^4 steps) on "
                         "the auto-chosen and the one-orbit-per-lane kernels and print its JSON "
                         "(with --no-cpu: without the oracle run)")
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
        accuracy_study(sode, torch, workloads, dev, args.accuracy_study,
                       args.oracle_threads or host_threads()[1])
        return
    if args.next_rows:
        next_rows(sode, torch, dev)
        return
    if args.rnn_only:
        print(json.dumps(rnn_leg(sode, torch, workloads, dev, gemms=(args.rnn_only,))))
        return
    if args.small_fp64_only:
        print(json.dumps(small_fp64_leg(sode, torch, workloads, dev, cpu=not args.no_cpu)))
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

    fp64 = mf_ms = None
    r_mf = None
    adj = rag = rnn = small = None
    sample_rows = w["diagonal"][np.linspace(0, 255, args.cpu_orbits).astype(int)]
    if not args.grid_only:
        # Binary64 kernels on the same ensemble (fewer steps; their per-step
        # cost does not depend on the step count).
        fp64 = grid_fp64_leg(sode, torch, w, X0, p, dev, args.baseline_steps, sample_rows)

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

        cpu_legs = not args.no_cpu
        small = small_fp64_leg(sode, torch, workloads, dev, cpu=cpu_legs)
        adj = adjoint_leg(sode, torch, workloads, dev, cpu=cpu_legs)
        rag = ragged_leg(sode, torch, workloads, dev, cpu=cpu_legs)
        rnn = rnn_leg(sode, torch, workloads, dev, cpu=cpu_legs)

    cpu = cpu_all = diag = None
    err = err_mf = err_all = None
    if not args.no_cpu:
        import oracle
        rows = sample_rows
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
            visible, nthreads = host_threads()
            if args.oracle_threads:
                nthreads = max(1, min(args.oracle_threads, visible))
            c0 = time.perf_counter()
            ref_all = oracle.integrate_parallel(
                "kuramoto", n, n, 2 * n + 1, w["X0"][rows_all].astype(np.float32).astype(np.float64),
                w["p"][rows_all].astype(np.float32).astype(np.float64), 0.0, w["dt"], nsteps,
                stride, w["seed"], threads=nthreads, orbit_ids=rows_all, observable="kuramoto_r")
            all_s = time.perf_counter() - c0
            cpu_all = {"value": len(rows_all) * nsteps / all_s, "unit": "orbit*steps/s",
                       "cores": nthreads, "host_cpus_visible": visible, "kind": "oracle",
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
        "plain_fp64": None if fp64 is None else dict(
            fp64["plain_fp64"], speedup_of_value=value / fp64["plain_fp64"]["value"]),
        "lanes16_fp64": None if fp64 is None else dict(
            fp64["lanes16_fp64"], speedup_of_value=value / fp64["lanes16_fp64"]["value"]),
        "error": {"max_abs_dr_final": err, "max_abs_dr_final_diagonal": err_all,
                  "tolerance": 1e-4, "diagonal": diag},
        "meanfield": None if mf_ms is None else {
            "value": orbits * nsteps / (mf_ms * 1e-3), "unit": "orbit*steps/s",
            "kernel_ms": mf_ms, "max_abs_dr_final": err_mf},
        "small_fp64": small,
        "adjoint": adj,
        "ragged": rag,
        "rnn": rnn,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()

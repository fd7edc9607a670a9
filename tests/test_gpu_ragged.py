"""Ragged FitzHugh-Nagumo batches in one persistent launch, against the FP64
oracle (every instance of the 4096-instance workload) and against
itself under every schedule: persistent or direct, graph replay or eager,
every lane shape and grid size give bitwise the same result.

Tolerance (the workload's): per instance max_s |dX|_inf / max(1, max_s |X|_inf)
<= 1e-4 against the oracle."""
import numpy as np
import pytest

import workloads
from gpu_util import as_received, log, threads

pytestmark = pytest.mark.gpu


def _batch(w, sel=None, nsteps=None):
    import paper_1908_03869_amd as sode
    idx = np.arange(len(w["units"])) if sel is None else np.asarray(sel)
    n = 2 * w["units"][idx]
    steps = w["nsteps"][idx] if nsteps is None else np.minimum(w["nsteps"][idx], nsteps)
    b = sode.RaggedBatch(n, steps, w["stride"], w["seed"], idx.astype(np.uint32), d=5)
    X0 = b.pack([w["X0"][i] for i in idx])
    p = b.pack([w["params"][i] for i in idx])
    return idx, b, X0, p


def _run(b, X0, p, dt, **opts):
    import torch
    import paper_1908_03869_amd as sode
    it = sode.Integrator("fhn", 256, 128, 5, precision=32, **opts)
    X0_t = torch.tensor(X0, dtype=torch.float32, device="cuda")
    p_t = torch.tensor(p, dtype=torch.float32, device="cuda")
    out = it.integrate_ragged(b, X0_t, p_t, 0.0, dt)
    it.sync()
    cfg = (it.get_option("ragged_waves_per_cu"), it.get_option("ragged_units_per_lane"))
    res = out.double().cpu().numpy()
    it.close()
    return res, cfg


def _oracle_instance(args):
    import oracle
    X0, p, n, nsteps, stride, seed, oid = args
    return oracle.integrate("fhn", n, n // 2, 5, X0[None], p, 0.0, 1e-3, nsteps, stride, seed,
                            orbit_ids=[oid])[0]


def _oracle_ulp_response(args, samples=8):
    """Largest relative change of the oracle's own result over `samples`
    seeded perturbations of the instance's initial state by one binary32
    ulp in relative terms (2^-24, random signs)."""
    X0, p, n, nsteps, stride, seed, oid = args
    ref = _oracle_instance(args)
    scale = max(1.0, np.abs(ref).max())
    worst = 0.0
    for k in range(samples):
        sign = np.random.default_rng(1000 + k).choice([-1.0, 1.0], X0.shape)
        r = _oracle_instance((X0 * (1.0 + sign * 2.0 ** -24), p, n, nsteps, stride, seed, oid))
        worst = max(worst, np.abs(r - ref).max() / scale)
    return worst


def test_full_workload_matches_oracle_on_every_instance(gpu):
    """All 4096 instances of the workload (2.59e9 unit-steps; the oracle
    takes ~36 ns per unit-step, ~7 s on 16 host threads) in the autotuned,
    graph-captured launch the benchmark times.

    Over tens of thousands of steps the noise-driven spikes of some chains
    make them ill-conditioned: the oracle itself, started from a state one
    binary32 ulp away, moves by more than the bound.  An instance over the
    bound must be shown to be such a case (its oracle one-ulp response,
    over eight seeded perturbations, reaches a tenth of the bound); it is
    then held to twice that response instead of the bound, and at most 1 %
    of the instances may take this route."""
    from concurrent.futures import ThreadPoolExecutor
    w = workloads.fhn_ragged()
    idx, b, X0, p = _batch(w)
    log("ragged fhn full workload (autotuned, graph)")
    out, cfg = _run(b, X0, p, w["dt"])
    print(f"autotuned waves/CU, units/lane: {cfg}")
    # Largest instances first, so the pool's tail is short.
    order = np.argsort(-(w["units"] * w["nsteps"]), kind="stable")
    X0r, pr = as_received(X0, 32), as_received(p, 32)
    args = []
    for i in order:
        a = int(b.x0_offset[i])
        n = int(b.n[i])
        args.append((X0r[a:a + n], pr[5 * i:5 * i + 5], n, int(b.nsteps[i]), int(b.stride[i]),
                     w["seed"], int(i)))
    with ThreadPoolExecutor(max_workers=threads()) as ex:
        refs = list(ex.map(_oracle_instance, args))
    err = np.empty(len(order))
    for j, (i, ref) in enumerate(zip(order, refs)):
        got = b.unpack(out, int(i))
        err[j] = np.abs(got - ref).max() / max(1.0, np.abs(ref).max())
    over = np.where(err > 1e-4)[0]
    print(f"within 1e-4: {len(order) - len(over)} of {len(order)}; worst {err.max():.2e}")
    assert len(over) <= len(order) // 100, over
    with ThreadPoolExecutor(max_workers=threads()) as ex:
        resp = list(ex.map(_oracle_ulp_response, [args[j] for j in over]))
    for j, r in zip(over, resp):
        i = order[j]
        print(f"instance {i}: {w['units'][i]} units x {w['nsteps'][i]} steps, relative error "
              f"{err[j]:.2e}, oracle one-ulp response {r:.2e}")
        assert r >= 0.1 * 1e-4, "over the bound but well conditioned"
        assert err[j] <= 2.0 * r, "more than twice the one-ulp response"


def test_schedules_and_shapes_are_bitwise_identical(gpu):
    """Every unit's arithmetic and noise are independent of the lane shape
    and of which wave runs it: all schedules agree bit for bit."""
    w = workloads.fhn_ragged(count=600)
    idx, b, X0, p = _batch(w, nsteps=3000)
    log("ragged schedules, 600 instances x <= 3000 steps")
    ref, _ = _run(b, X0, p, w["dt"], persistent=0, graph=0, units_per_lane=1, waves_per_cu=4)
    for opts in (dict(persistent=1, graph=0, units_per_lane=1, waves_per_cu=4),
                 dict(persistent=1, graph=1, units_per_lane=2, waves_per_cu=8),
                 dict(persistent=1, graph=1, units_per_lane=4, waves_per_cu=16),
                 dict(persistent=0, graph=0, units_per_lane=8, waves_per_cu=4),
                 dict()):
        got, _ = _run(b, X0, p, w["dt"], **opts)
        np.testing.assert_array_equal(got, ref, err_msg=str(opts))


def test_graph_replays_match_eager(gpu):
    """The captured launch replayed several times, with eager work and
    synchronisation between replays, reproduces the eager result each time."""
    import torch
    import paper_1908_03869_amd as sode
    w = workloads.fhn_ragged(count=300)
    idx, b, X0, p = _batch(w, nsteps=2000)
    log("ragged graph replays")
    eager, _ = _run(b, X0, p, w["dt"], graph=0, units_per_lane=2, waves_per_cu=8)
    it = sode.Integrator("fhn", 256, 128, 5, precision=32, graph=1, units_per_lane=2,
                         waves_per_cu=8)
    X0_t = torch.tensor(X0, dtype=torch.float32, device="cuda")
    p_t = torch.tensor(p, dtype=torch.float32, device="cuda")
    out = torch.empty(b.out_len, dtype=torch.float32, device="cuda")
    for rep in range(4):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        it.integrate_ragged(b, X0_t, p_t, 0.0, w["dt"], out=out)
        scratch = torch.randn(1 << 20, device="cuda").sum()  # eager work in between
        it.sync()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.double().cpu().numpy(), eager, err_msg=f"replay {rep}")
        assert torch.isfinite(scratch)
    it.close()


def test_edge_instances(gpu):
    """One unit, 128 units, zero steps, stride = nsteps, per-instance seeds."""
    import paper_1908_03869_amd as sode
    rng = np.random.default_rng(17)
    units = np.array([1, 128, 3, 64, 17, 2])
    steps = np.array([500, 400, 0, 300, 700, 1000])
    strides = np.array([100, 400, 1, 100, 700, 250])
    n = 2 * units
    b = sode.RaggedBatch(n, steps, strides, np.arange(6) + 77, np.arange(6) * 3, d=5)
    X0s = [np.concatenate([-1.2 + 0.1 * rng.standard_normal(u), -0.62 + 0.1 * rng.standard_normal(u)])
           for u in units]
    ps = [np.array([0.7, 0.8, 0.08, 0.1, 0.05]) * rng.uniform(0.8, 1.2, 5) for _ in units]
    X0, p = b.pack(X0s), b.pack(ps)
    log("ragged edge instances")
    out, _ = _run(b, X0, p, 1e-3)
    X0r, pr = as_received(X0, 32), as_received(p, 32)
    for i in range(6):
        a = int(b.x0_offset[i])
        ref = _oracle_instance((X0r[a:a + n[i]], pr[5 * i:5 * i + 5], int(n[i]), int(steps[i]),
                                int(strides[i]), 77 + i, 3 * i))
        got = b.unpack(out, i)
        assert got.shape == ref.shape
        assert np.abs(got - ref).max() / max(1.0, np.abs(ref).max()) <= 1e-4


def test_odd_step_counts_across_shapes(gpu):
    """Odd step counts end on a single step after the two-step noise
    batches of two-units-per-lane shapes; every shape must still agree bit
    for bit, and with the oracle."""
    import paper_1908_03869_amd as sode
    rng = np.random.default_rng(23)
    units = np.array([2, 4, 64, 125, 3, 40])
    steps = np.array([1, 3, 333, 77, 999, 5])
    strides = np.array([1, 3, 111, 7, 333, 5])
    n = 2 * units
    b = sode.RaggedBatch(n, steps, strides, np.arange(6) + 5, np.arange(6) * 7 + 1, d=5)
    X0s = [np.concatenate([-1.2 + 0.1 * rng.standard_normal(u), -0.62 + 0.1 * rng.standard_normal(u)])
           for u in units]
    ps = [np.array([0.7, 0.8, 0.08, 0.1, 0.05]) * rng.uniform(0.8, 1.2, 5) for _ in units]
    X0, p = b.pack(X0s), b.pack(ps)
    log("ragged odd step counts, units_per_lane 1, 2, 4, 8")
    ref, _ = _run(b, X0, p, 1e-3, persistent=0, graph=0, units_per_lane=1, waves_per_cu=4)
    for upl in (2, 4, 8):
        got, _ = _run(b, X0, p, 1e-3, persistent=1, graph=0, units_per_lane=upl, waves_per_cu=8)
        np.testing.assert_array_equal(got, ref, err_msg=f"units_per_lane={upl}")
    X0r, pr = as_received(X0, 32), as_received(p, 32)
    for i in range(6):
        a = int(b.x0_offset[i])
        oref = _oracle_instance((X0r[a:a + n[i]], pr[5 * i:5 * i + 5], int(n[i]), int(steps[i]),
                                 int(strides[i]), 5 + i, 7 * i + 1))
        got = b.unpack(ref, i)
        assert got.shape == oref.shape
        assert np.abs(got - oref).max() / max(1.0, np.abs(oref).max()) <= 1e-4

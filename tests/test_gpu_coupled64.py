"""Binary64 coupled Kuramoto kernel (kernel "coupled", precision 64: 16 lanes
per orbit, or 4 lanes per orbit for n <= 4) against the FP64 oracle.  The kernel evaluates each unordered pair once and sums in
a different order than the oracle's index-order loops, so the comparison is
to 1e-10 (the bound of the binary64 small-ensemble workload) rather than
bitwise; phases are compared on the circle (the kernel wraps them)."""
import numpy as np
import pytest

import workloads
from gpu_util import circular_diff, log, run_library, run_oracle

pytestmark = pytest.mark.gpu


def test_small_ensemble_full_workload(gpu):
    """1024 orbits, n = 4, 10^4 steps, per-orbit Philox seeds (the binary64
    small-ensemble workload), saved every 100 steps."""
    w = workloads.kuramoto_small()
    log("coupled fp64 n=4 full small workload")
    got = run_library(w, precision=64, kernel="coupled")
    want = run_oracle(w)
    assert circular_diff(got, want).max() <= 1e-10


@pytest.mark.parametrize("drift", [0, 1])
@pytest.mark.parametrize("N", [5, 10, 15])
def test_paper_shapes(gpu, N, drift):
    w = dict(workloads.kuramoto_paper(N, 97, nsteps=2000), observable="state")
    log(f"coupled fp64 N={N} drift={drift}")
    got = run_library(w, precision=64, kernel="coupled", drift=drift)
    want = run_oracle(w)
    assert circular_diff(got, want).max() <= 1e-10


@pytest.mark.parametrize("n", [32, 50, 64])
def test_larger_rows(gpu, n):
    """P = 2, 4 oscillators per lane, padded and unpadded, order parameter."""
    w = workloads.kuramoto_grid(nK=5, nS=7, n=n, nsteps=1000)
    log(f"coupled fp64 r n={n}")
    got = run_library(w, precision=64, kernel="coupled")
    want = run_oracle(w)
    assert np.abs(got - want).max() <= 1e-10


@pytest.mark.parametrize("drift", [0, 1])
@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_quad_form_small_systems(gpu, n, drift):
    """n <= 4 runs four lanes per orbit (pads for n < 4), state and r saves,
    with an orbit count that leaves a partial workgroup (77 orbits) and a
    step count that is not a multiple of the four-step noise group."""
    rng = np.random.default_rng(40 + n)
    orbits = 77
    X0 = rng.uniform(-np.pi, np.pi, (orbits, n))
    p = workloads.kuramoto_params(rng.uniform(0.0, 4.0, orbits), rng.standard_normal((orbits, n)),
                                  rng.uniform(0.05, 0.5, (orbits, n)))
    for obs in ("state", "kuramoto_r"):
        w = dict(model="kuramoto", n=n, m=n, d=2 * n + 1, X0=X0, p=p, t0=0.0, dt=1e-2, nsteps=1001,
                 stride=143, seed=77, observable=obs)
        log(f"coupled fp64 quad n={n} drift={drift} {obs}")
        got = run_library(w, precision=64, kernel="coupled", drift=drift)
        want = run_oracle(w)
        d = circular_diff(got, want) if obs == "state" else np.abs(got - want)
        assert d.max() <= 1e-10, d.max()


def test_quad_form_auto_selection_and_shards(gpu):
    """Auto selection takes the four-lane form for n = 4 in binary64 (same
    bits as kernel "coupled"), and two shards by orbit_offset reproduce one
    call bit for bit."""
    w = workloads.kuramoto_small()
    sel = slice(0, 130)
    w = dict(w, X0=w["X0"][sel], p=w["p"][sel], orbit_ids=w["orbit_ids"][sel],
             orbit_seeds=w["orbit_seeds"][sel], nsteps=500)
    log("coupled fp64 quad auto vs coupled")
    a = run_library(w, precision=64, kernel="coupled")
    b = run_library(w, precision=64, kernel="auto")
    np.testing.assert_array_equal(a, b)
    w2 = dict(w, orbit_ids=None, orbit_seeds=None)
    full = run_library(w2, precision=64, kernel="coupled")
    lo = run_library(dict(w2, X0=w2["X0"][:50], p=w2["p"][:50]), precision=64, kernel="coupled")
    hi = run_library(dict(w2, X0=w2["X0"][50:], p=w2["p"][50:]), precision=64, kernel="coupled",
                     orbit_offset=50)
    np.testing.assert_array_equal(np.concatenate([lo, hi]), full)


@pytest.mark.parametrize("n,obs,drift", [(4, "state", 0), (3, "kuramoto_r", 0), (2, "state", 1),
                                         (1, "kuramoto_r", 1), (16, "state", 0), (7, "kuramoto_r", 1),
                                         (32, "state", 0), (20, "kuramoto_r", 0), (64, "kuramoto_r", 0),
                                         (50, "state", 1)])
def test_noise_waves_bitwise(gpu, n, obs, drift):
    """The four-lane form (n <= 4) and the 16-lane rows with one, two or
    four oscillators per lane (padded and not) with their normals drawn by
    one or two other waves of the workgroup into LDS ("noise_waves" 1, 2)
    give the bits of the lanes drawing their own (0): the same Philox
    blocks, the same binary64 Box-Muller code.  77 orbits (partial groups of
    16 quads or 4 rows), 1001 steps (partial batches of 32, 16 or 8 steps),
    a non-zero step offset; n = 4 and n = 32 also against the oracle, and a
    call with no steps (only the initial save)."""
    rng = np.random.default_rng(90 + n)
    orbits = 77
    X0 = rng.uniform(-np.pi, np.pi, (orbits, n))
    p = workloads.kuramoto_params(rng.uniform(0.0, 4.0, orbits), rng.standard_normal((orbits, n)),
                                  rng.uniform(0.05, 0.5, (orbits, n)))
    w = dict(model="kuramoto", n=n, m=n, d=2 * n + 1, X0=X0, p=p, t0=0.0, dt=1e-2, nsteps=1001,
             stride=143, seed=78, observable=obs)
    res = {}
    for nw in (0, 1, 2):
        log(f"coupled fp64 n={n} {obs} drift={drift} noise_waves={nw}")
        res[nw] = run_library(w, precision=64, kernel="coupled", drift=drift, noise_waves=nw,
                              step_offset=5000)
    np.testing.assert_array_equal(res[1], res[0])
    np.testing.assert_array_equal(res[2], res[0])
    if n in (4, 32):
        want = run_oracle(w, step_offset=5000)
        assert circular_diff(res[1], want).max() <= 1e-10
    for nw in (0, 1, 2):
        log(f"coupled fp64 n={n} no steps noise_waves={nw}")
        got = run_library(w, precision=64, kernel="coupled", drift=drift, noise_waves=nw, nsteps=0)
        want = run_library(w, precision=64, kernel="plain", drift=drift, nsteps=0)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("n,orbits,expect", [(6, 98304, "coupled"), (17, 2048, "coupled"),
                                             (5, 131072, "plain"), (5, 49152, "coupled"), (5, 4096, "coupled")])
def test_auto_selection_binary64(gpu, n, orbits, expect):
    """Auto selection in binary64 takes the 16-lane row for every n in 6..64
    at any ensemble size and, at n = 5 (a row of 11 pads), one orbit per lane
    beyond 100,000 orbits (pairwise): the auto result equals the expected kernel's
    result bit for bit (the two kernels sum in different orders)."""
    rng = np.random.default_rng(700 + n)
    X0 = rng.uniform(-np.pi, np.pi, (orbits, n))
    p = workloads.kuramoto_params(rng.uniform(0.0, 4.0, orbits), rng.standard_normal((orbits, n)),
                                  rng.uniform(0.05, 0.5, (orbits, n)))
    w = dict(model="kuramoto", n=n, m=n, d=2 * n + 1, X0=X0, p=p, t0=0.0, dt=1e-2, nsteps=40,
             stride=20, seed=31, observable="state")
    log(f"binary64 auto selection n={n} orbits={orbits}: expect {expect}")
    auto = run_library(w, precision=64, kernel="auto")
    want = run_library(w, precision=64, kernel=expect)
    np.testing.assert_array_equal(auto, want)

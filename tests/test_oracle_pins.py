"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test ties one part of the oracle to something fixed outside it: published
known-answer vectors, a third-party implementation, a closed form, an
invariant, a special case that reduces to a library routine, or a value the
paper states.  CPU only.
"""
import json
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


# --------------------------------------------------------------------------- Philox
def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answer_vectors(oracle_lib):
    """Random123's published known-answer vectors for Philox-4x32-10."""
    for ctr, key, want in _kat():
        assert oracle_lib.philox(ctr, key) == want


@pytest.fixture(scope="module")
def rocrand_dump(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND cross-check")
    exe = str(tmp_path_factory.mktemp("xcheck") / "rocrand_philox_dump")
    src = os.path.join(HERE, "xcheck", "rocrand_philox_dump.cpp")
    subprocess.check_call([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-o", exe, src],
                          stderr=subprocess.DEVNULL)
    return exe


def test_philox_matches_rocrand(oracle_lib, rocrand_dump):
    """Bit-equality with rocRAND's open-source Philox-4x32-10 engine (run on
    the host through its public API) over random counters and keys."""
    rng = np.random.default_rng(11)
    rows = rng.integers(0, 2**32, size=(3000, 6), dtype=np.uint64)
    rows[:1000, 1:4] = rng.integers(0, 64, size=(1000, 3))  # counter shapes the library uses
    text = "\n".join(" ".join(str(int(x)) for x in r) for r in rows) + "\n"
    res = subprocess.run([rocrand_dump], input=text, capture_output=True, text=True, check=True)
    got = [list(map(int, l.split())) for l in res.stdout.strip().splitlines()]
    assert len(got) == len(rows)
    for r, g in zip(rows, got):
        assert oracle_lib.philox([int(x) for x in r[:4]], [int(r[4]), int(r[5])]) == g


# --------------------------------------------------------------------------- Box-Muller
def test_box_muller_closed_form(oracle_lib):
    """Eq. (3): r1 = sqrt(-2 ln U1) cos(2 pi U2), r2 = sqrt(-2 ln U1) sin(2 pi U2)
    with U1 = ((w0>>8)+1) 2^-24 and U2 = (w1>>8) 2^-24."""
    # U1 = 1 -> radius 0.
    assert oracle_lib.box_muller(0xFFFFFFFF, 0x12345678) == (0.0, 0.0)
    # U1 = 2^-24 (the smallest), U2 = 0 -> (radius, 0): the cosine comes first.
    r = math.sqrt(48.0 * math.log(2.0))
    z = oracle_lib.box_muller(0x000000FF, 0x000000FF)
    assert z[0] == pytest.approx(r, rel=1e-15) and z[1] == 0.0
    # U2 = 1/4 -> (0, radius); U2 = 1/2 -> (-radius, 0).
    u1 = (0x800000 + 1) / 2**24
    r = math.sqrt(-2.0 * math.log(u1))
    z = oracle_lib.box_muller(0x80000000, 0x40000000)
    assert abs(z[0]) < 1e-15 and z[1] == pytest.approx(r, rel=1e-15)
    z = oracle_lib.box_muller(0x80000000, 0x80000000)
    assert z[0] == pytest.approx(-r, rel=1e-15) and abs(z[1]) < 1e-15
    # The low 8 bits of each word are ignored (24-bit uniforms).
    assert oracle_lib.box_muller(0x12345600, 0x9ABCDE00) == oracle_lib.box_muller(0x123456FF, 0x9ABCDEFF)


def test_normals_block_layout(oracle_lib):
    """Normal 4b+2h+q of a step comes from Philox block b, word pair h."""
    seed, oid, step = 0x0123456789ABCDEF, 77, 1234
    xi = oracle_lib.normals(seed, oid, step, 10)
    for b in range(3):
        w = oracle_lib.philox([step, oid, b, 0], [seed & 0xFFFFFFFF, seed >> 32])
        for h in range(2):
            pair = oracle_lib.box_muller(w[2 * h], w[2 * h + 1])
            for q in range(2):
                j = 4 * b + 2 * h + q
                if j < 10:
                    assert xi[j] == pair[q]


def test_normals_are_standard_normal(oracle_lib):
    """Moments and Kolmogorov-Smirnov against N(0,1) over 2^20 draws, and no
    correlation between neighbours in one block or between steps."""
    m, steps = 64, 16384
    xs = np.stack([oracle_lib.normals(99, 5, k, m) for k in range(steps)])
    x = xs.ravel()
    N = x.size
    assert abs(x.mean()) < 5 / math.sqrt(N)
    assert abs(x.var() - 1.0) < 5 * math.sqrt(2.0 / N)
    assert abs(stats.skew(x)) < 5 * math.sqrt(6.0 / N)
    assert abs(stats.kurtosis(x)) < 5 * math.sqrt(24.0 / N)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    for a, b in ((xs[:, 0::2], xs[:, 1::2]), (xs[:, 0::4], xs[:, 2::4]), (xs[:-1], xs[1:])):
        c = np.corrcoef(a.ravel(), b.ravel())[0, 1]
        assert abs(c) < 5 / math.sqrt(a.size)


# --------------------------------------------------------------------------- EM on OU
def test_em_brute_force_three_steps(oracle_lib):
    """n = 1 Ornstein-Uhlenbeck, three EM steps written out by hand (Eq. 2)."""
    a, mu, s, dt, x = 1.5, 0.25, 0.7, 0.1, 2.0
    out = oracle_lib.integrate("ou", 1, 1, 3, [[x]], [a, mu, s], 0.0, dt, 3, 1, 42)
    for k in range(3):
        xi = oracle_lib.normals(42, 0, k, 1)[0]
        x = x + (-a * (x - mu)) * dt + (s * xi) * math.sqrt(dt)
        assert out[0, k + 1, 0] == x


def test_ou_discrete_moments(oracle_lib):
    """EM on dX = -a (X - mu) dt + s dW: with rho = 1 - a dt the iterates have
    E X_k = mu + rho^k (X0 - mu) and Var X_k = s^2 dt (1 - rho^{2k}) / (1 - rho^2)."""
    a, mu, s, dt, x0 = 2.0, 0.5, 0.3, 0.01, 1.0
    orbits, nsteps, stride = 65536, 200, 50
    out = oracle_lib.integrate("ou", 1, 1, 3, np.full((orbits, 1), x0), [a, mu, s], 0.0, dt,
                               nsteps, stride, 2024)
    rho = 1.0 - a * dt
    for si in range(1, nsteps // stride + 1):
        k = si * stride
        mean = mu + rho**k * (x0 - mu)
        var = s * s * dt * (1 - rho ** (2 * k)) / (1 - rho * rho)
        X = out[:, si, 0]
        assert abs(X.mean() - mean) < 5 * math.sqrt(var / orbits)
        assert abs(X.var(ddof=1) - var) < 5 * var * math.sqrt(2.0 / (orbits - 1))


# --------------------------------------------------------------------------- GBM
def _brownian(oracle_lib, orbits, dt, nsteps, seed):
    """W(T) driven by the very normals the integrator draws: OU with a = 0,
    s = 1 and X0 = 0 accumulates sum_k sqrt(dt) xi_k."""
    return oracle_lib.integrate("ou", 1, 1, 3, np.zeros((orbits, 1)), [0.0, 0.0, 1.0], 0.0,
                                dt, nsteps, nsteps, seed)[:, -1, 0]


def test_gbm_strong_order_half(oracle_lib):
    """EM for GBM against the exact solution X0 exp((mu - s^2/2) T + s W(T))
    on the same Brownian path: strong error ~ dt^{1/2}."""
    mu, s, x0, T, orbits = 1.0, 0.8, 1.0, 1.0, 2048
    errs, dts = [], []
    for L in range(4, 10):
        nsteps = 2**L
        dt = T / nsteps
        X = oracle_lib.integrate("gbm", 1, 1, 2, np.full((orbits, 1), x0), [mu, s], 0.0, dt,
                                 nsteps, nsteps, 500 + L)[:, -1, 0]
        W = _brownian(oracle_lib, orbits, dt, nsteps, 500 + L)
        exact = x0 * np.exp((mu - 0.5 * s * s) * T + s * W)
        errs.append(np.mean(np.abs(X - exact)))
        dts.append(dt)
    slope = np.polyfit(np.log(dts), np.log(errs), 1)[0]
    assert 0.4 < slope < 0.62, (slope, errs)


def test_gbm_milstein_strong_order_one(oracle_lib):
    """Milstein for GBM against the same exact solution: strong error ~ dt.
    A wrong coefficient of the (dW^2 - dt) correction (or its sign) leaves a
    dt^{1/2} term and drops the slope back to one half."""
    mu, s, x0, T, orbits = 1.0, 0.8, 1.0, 1.0, 2048
    errs, dts = [], []
    for L in range(4, 10):
        nsteps = 2**L
        dt = T / nsteps
        X = oracle_lib.integrate("gbm", 1, 1, 2, np.full((orbits, 1), x0), [mu, s], 0.0, dt,
                                 nsteps, nsteps, 500 + L, method="milstein")[:, -1, 0]
        W = _brownian(oracle_lib, orbits, dt, nsteps, 500 + L)
        exact = x0 * np.exp((mu - 0.5 * s * s) * T + s * W)
        errs.append(np.mean(np.abs(X - exact)))
        dts.append(dt)
    slope = np.polyfit(np.log(dts), np.log(errs), 1)[0]
    assert 0.88 < slope < 1.12, (slope, errs)


def test_gbm_milstein_one_step_closed_form(oracle_lib):
    """One Milstein step of GBM is X0 (1 + mu dt + s dW + s^2 (dW^2 - dt) / 2):
    the second-order Taylor expansion of the exact solution's exponential in
    dW, with dW^2 replaced by its mean where it multiplies mu."""
    mu, s, x0, dt = 0.3, 0.9, 1.7, 0.04
    X = oracle_lib.integrate("gbm", 1, 1, 2, np.full((64, 1), x0), [mu, s], 0.0, dt, 1, 1, 9,
                             method="milstein")[:, -1, 0]
    W = _brownian(oracle_lib, 64, dt, 1, 9)
    want = x0 * (1 + mu * dt + s * W + 0.5 * s * s * (W * W - dt))
    np.testing.assert_allclose(X, want, rtol=1e-14, atol=0)


@pytest.mark.parametrize("model,n,m,d,p", [("ou", 3, 3, 3, [0.7, 0.2, 0.3]),
                                           ("kuramoto", 4, 4, 9, [1.5, 0.1, 0.2, -0.3, 0.4,
                                                                  0.1, 0.2, 0.3, 0.05]),
                                           ("fhn", 6, 3, 5, [0.7, 0.8, 0.08, 0.1, 0.05])])
def test_milstein_equals_em_for_additive_noise(oracle_lib, model, n, m, d, p):
    """With a state-independent diffusion the correction vanishes and the
    Milstein iterates are the Euler-Maruyama iterates, bit for bit."""
    X0 = np.random.default_rng(3).uniform(-1, 1, (5, n))
    a = oracle_lib.integrate(model, n, m, d, X0, p, 0.0, 0.01, 40, 10, 5)
    b = oracle_lib.integrate(model, n, m, d, X0, p, 0.0, 0.01, 40, 10, 5, method="milstein")
    np.testing.assert_array_equal(a, b)


def test_gbm_weak_mean(oracle_lib):
    """E X_K = X0 (1 + mu dt)^K exactly for the EM iterates of GBM."""
    mu, s, x0, dt, K, orbits = 0.5, 0.4, 2.0, 0.01, 100, 65536
    X = oracle_lib.integrate("gbm", 1, 1, 2, np.full((orbits, 1), x0), [mu, s], 0.0, dt, K, K,
                             77)[:, -1, 0]
    mean = x0 * (1 + mu * dt) ** K
    second = x0 * x0 * ((1 + mu * dt) ** 2 + s * s * dt) ** K
    se = math.sqrt((second - mean * mean) / orbits)
    assert abs(X.mean() - mean) < 5 * se


# --------------------------------------------------------------------------- ODE limit
def _adler_exact(psi0, a, b, t):
    """psi' = a - b sin psi with a > b > 0: tan(psi/2) = (b + c tan(c (t - t*)/2)) / a,
    c = sqrt(a^2 - b^2)."""
    c = math.sqrt(a * a - b * b)
    v0 = (a * math.tan(psi0 / 2) - b) / c
    tstar = -2.0 * math.atan(v0) / c
    return 2.0 * math.atan((b + c * math.tan(c * (t - tstar) / 2)) / a)


def _circ(x, y):
    return abs(math.remainder(x - y, 2 * math.pi))


@pytest.mark.parametrize("method,dts,order", [("em", (2e-2, 1e-2, 5e-3), 1.0),
                                              ("rk4", (0.1, 0.05, 0.025), 4.0),
                                              ("implicit_euler", (2e-2, 1e-2, 5e-3), 1.0),
                                              ("implicit_midpoint", (0.1, 0.05, 0.025), 2.0)])
def test_kuramoto_two_oscillators_adler(oracle_lib, method, dts, order):
    """n = 2, g = 0: psi = theta_2 - theta_1 obeys the Adler equation
    psi' = (omega_2 - omega_1) - K sin psi and theta_1 + theta_2 grows at
    omega_1 + omega_2 (a linear invariant every Runge-Kutta method keeps).
    Euler, explicit or implicit, converges with order 1, the implicit
    midpoint rule with order 2, RK4 with order 4."""
    K, w1, w2, T = 3.0, -2.0, 2.0, 2.0
    th0 = np.array([[0.4, 0.7]])
    p = workloads.kuramoto_params([K], [[w1, w2]], [[0.0, 0.0]])[0]
    exact = _adler_exact(0.3, w2 - w1, K, T)
    errs = []
    for dt in dts:
        nsteps = int(round(T / dt))
        out = oracle_lib.integrate("kuramoto", 2, 2, 5, th0, p, 0.0, dt, nsteps, nsteps, 1,
                                   method=method)
        th = out[0, -1]
        errs.append(_circ(th[1] - th[0], exact))
        assert th[0] + th[1] == pytest.approx(1.1 + (w1 + w2) * T, abs=1e-12)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    for r in rates:
        assert abs(r - order) < 0.1 * order, (rates, errs)


@pytest.mark.parametrize("method", ["implicit_euler", "implicit_midpoint"])
def test_implicit_steps_on_a_stiff_linear_decay(oracle_lib, method):
    """OU without noise, x' = -a (x - mu) with a dt = 10 (explicit Euler would
    diverge): implicit Euler multiplies x - mu by 1 / (1 + a dt) per step,
    the midpoint rule by (1 - a dt / 2) / (1 + a dt / 2)."""
    a, mu, dt, K = 1000.0, 0.3, 0.01, 40
    X0 = np.array([[1.7], [-2.0], [0.3]])
    out = oracle_lib.integrate("ou", 1, 1, 3, X0, [a, mu, 0.5], 0.0, dt, K, 1, 4, method=method)
    z = a * dt
    rho = 1.0 / (1.0 + z) if method == "implicit_euler" else (1.0 - z / 2) / (1.0 + z / 2)
    want = mu + (X0[:, 0:1] - mu) * rho ** np.arange(K + 1)[None, :]
    np.testing.assert_allclose(out[:, :, 0], want, rtol=0, atol=2e-14)


@pytest.mark.parametrize("method,c", [("implicit_euler", 1.0), ("implicit_midpoint", 0.5)])
def test_implicit_steps_solve_their_equation(oracle_lib, method, c):
    """FHN chain (nonlinear, coupled): every saved step satisfies
    Y = X + dt f(X + c (Y - X)) with f the separately pinned drift."""
    n, p, dt = 6, np.array([0.7, 0.8, 0.08, 0.1, 0.05]), 0.05
    X0 = np.array([[-1.0, 0.5, 1.2, -0.3, 0.2, 0.1]])
    out = oracle_lib.integrate("fhn", n, 3, 5, X0, p, 0.0, dt, 30, 1, 4, method=method)[0]
    for k in range(30):
        X, Y = out[k], out[k + 1]
        f = oracle_lib.drift("fhn", n, 3, 5, X + c * (Y - X), p)
        np.testing.assert_allclose(Y, X + dt * f, rtol=0, atol=1e-13)


# --------------------------------------------------------------------------- drifts
def test_kuramoto_drift_mean_field_identity(oracle_lib):
    """sum_j sin(t_j - t_i) = cos t_i sum_j sin t_j - sin t_i sum_j cos t_j."""
    rng = np.random.default_rng(3)
    N = 64
    th = rng.uniform(-50, 50, N)
    K, om, sg = 2.5, rng.standard_normal(N), rng.uniform(0, 1, N)
    p = workloads.kuramoto_params([K], om[None], sg[None])[0]
    f = oracle_lib.drift("kuramoto", N, N, 2 * N + 1, th, p)
    mf = om + (K / N) * (np.cos(th) * np.sin(th).sum() - np.sin(th) * np.cos(th).sum())
    np.testing.assert_allclose(f, mf, rtol=0, atol=1e-13)
    # Identical phases: no coupling.
    f = oracle_lib.drift("kuramoto", N, N, 2 * N + 1, np.full(N, 1.3), p)
    np.testing.assert_array_equal(f, om)


def test_kuramoto_diffusion_layout(oracle_lib):
    """g_ij = p_i delta_ij with p_i stored after the frequencies."""
    N = 5
    p = workloads.kuramoto_params([1.0], np.arange(N)[None] * 1.0, (10.0 + np.arange(N))[None])[0]
    xi = np.linspace(-1, 1, N)
    g = oracle_lib.diffusion("kuramoto", N, N, 2 * N + 1, np.zeros(N), p, xi)
    np.testing.assert_array_equal(g, (10.0 + np.arange(N)) * xi)


def test_order_parameter_special_cases(oracle_lib):
    """Eq. (7): r = 1 for identical phases, r = 0 for equally spaced phases,
    r = |cos(phi/2)| for two oscillators at 0 and phi."""
    assert oracle_lib.order_parameter(np.full(64, -2.0)) == pytest.approx(1.0, abs=1e-15)
    for N in (3, 4, 64, 100):
        th = 0.37 + 2 * math.pi * np.arange(N) / N
        assert oracle_lib.order_parameter(th) < 1e-14
    for phi in (0.1, 1.0, 2.5):
        assert oracle_lib.order_parameter([0.0, phi]) == pytest.approx(abs(math.cos(phi / 2)), abs=1e-15)


def test_fhn_fixed_point_invariant(oracle_lib):
    """sigma = 0 and every unit at the fixed point (v*, w*) with
    v*^3 + 3 (1/b - 1) v* + 3 a / b = 0 and w* = (v* + a)/b: nothing moves."""
    a, b, eps, D = 0.7, 0.8, 0.08, 0.1
    roots = np.roots([1.0, 0.0, 3 * (1 / b - 1), 3 * a / b])
    v = float(roots[np.argmin(np.abs(roots.imag))].real)
    assert v == pytest.approx(-1.1994, abs=1e-4)
    w = (v + a) / b
    N = 6
    X0 = np.concatenate([np.full(N, v), np.full(N, w)])[None]
    out = oracle_lib.integrate("fhn", 2 * N, N, 5, X0, [a, b, eps, D, 0.0], 0.0, 1e-2, 1000,
                               1000, 3)
    np.testing.assert_allclose(out[0, -1], X0[0], atol=1e-12)


def test_fhn_uncoupled_units_independent(oracle_lib):
    """D = 0, sigma = 0: a chain is the union of its single units."""
    rng = np.random.default_rng(5)
    N = 4
    v0, w0 = rng.normal(-1, 0.5, N), rng.normal(-0.5, 0.5, N)
    pr = [0.7, 0.8, 0.08, 0.0, 0.0]
    chain = oracle_lib.integrate("fhn", 2 * N, N, 5, np.concatenate([v0, w0])[None], pr, 0.0,
                                 1e-2, 500, 500, 1)[0, -1]
    for i in range(N):
        one = oracle_lib.integrate("fhn", 2, 1, 5, [[v0[i], w0[i]]], pr, 0.0, 1e-2, 500, 500,
                                   1)[0, -1]
        assert chain[i] == one[0] and chain[N + i] == one[1]


def test_fhn_laplacian_no_flux(oracle_lib):
    """The coupling term D (v_{i-1} - 2 v_i + v_{i+1}) with reflected ends sums
    to zero over the chain (no flux through the boundary)."""
    rng = np.random.default_rng(8)
    N = 7
    X = np.concatenate([rng.normal(0, 1, N), np.zeros(N)])
    base = oracle_lib.drift("fhn", 2 * N, N, 5, X, [0.7, 0.8, 0.08, 0.0, 0.0])
    coup = oracle_lib.drift("fhn", 2 * N, N, 5, X, [0.7, 0.8, 0.08, 1.0, 0.0])
    assert abs((coup - base)[:N].sum()) < 1e-13
    lap = np.convolve(np.concatenate([[X[0]], X[:N], [X[N - 1]]]), [1, -2, 1], "valid")
    np.testing.assert_allclose((coup - base)[:N], lap, atol=1e-14)


def _fhn_fixed_point(a, b):
    """Resting state of one FitzHugh-Nagumo unit: the real root of
    v^3 + 3 (1/b - 1) v + 3 a / b = 0, w = (v + a) / b (numpy's polynomial roots)."""
    roots = np.roots([1.0, 0.0, 3 * (1 / b - 1), 3 * a / b])
    v = float(roots[np.argmin(np.abs(roots.imag))].real)
    return v, (v + a) / b


def check_fhn_one_step_drift(oracle_lib):
    """sigma = D = 0, one Euler-Maruyama step from states off the fixed point,
    with a, b and eps all different from each other: the FitzHugh-Nagumo
    equations dv = (v - v^3/3 - w) dt, dw = eps (v + a - b w) dt written out."""
    a, b, eps, dt = 0.55, 1.3, 0.21, 0.01
    v = np.array([0.4, -1.7, 1.1])
    w = np.array([-0.3, 0.9, 0.25])
    N = v.size
    out = oracle_lib.integrate("fhn", 2 * N, N, 5, np.concatenate([v, w])[None],
                               [a, b, eps, 0.0, 0.0], 0.0, dt, 1, 1, 7)
    v1 = v + dt * (v - v ** 3 / 3 - w)
    w1 = w + dt * (eps * (v + a - b * w))
    np.testing.assert_allclose(out[0, 1, :N], v1, rtol=0, atol=1e-14)
    np.testing.assert_allclose(out[0, 1, N:], w1, rtol=0, atol=1e-14)


def check_fhn_noise_on_v_only(oracle_lib):
    """From the fixed point, with coupling on and sigma != eps: one step moves
    each v_i by exactly sigma sqrt(dt) xi_i (xi_i the i-th normal of the
    orbit's step-0 block) and leaves every w_i where it was."""
    a, b, eps, D, sigma, dt, seed = 0.7, 0.8, 0.08, 0.1, 0.37, 0.01, 11
    v, w = _fhn_fixed_point(a, b)
    N = 4
    X0 = np.concatenate([np.full(N, v), np.full(N, w)])[None]
    out = oracle_lib.integrate("fhn", 2 * N, N, 5, X0, [a, b, eps, D, sigma], 0.0, dt, 1, 1, seed)
    xi = oracle_lib.normals(seed, 0, 0, N)
    np.testing.assert_allclose(out[0, 1, :N] - v, sigma * math.sqrt(dt) * xi, rtol=0, atol=1e-14)
    np.testing.assert_allclose(out[0, 1, N:], w, rtol=0, atol=1e-15)


def check_fhn_linearisation(oracle_lib):
    """sigma = D = 0: a perturbation delta of 1e-6 from the fixed point evolves,
    to first order, as (I + dt J)^k delta with the Jacobian
    J = [[1 - v*^2, -1], [eps, -eps b]] of the unit at (v*, w*) -- a stable
    spiral for these parameters, so every entry of J shapes the result."""
    a, b, eps, dt, k = 0.7, 0.8, 0.3, 0.01, 400
    v, w = _fhn_fixed_point(a, b)
    J = np.array([[1 - v * v, -1.0], [eps, -eps * b]])
    A = np.linalg.matrix_power(np.eye(2) + dt * J, k)
    for delta in (np.array([1e-6, 0.0]), np.array([0.0, 1e-6]), np.array([7e-7, -4e-7])):
        X0 = np.array([[v + delta[0], w + delta[1]]])
        out = oracle_lib.integrate("fhn", 2, 1, 5, X0, [a, b, eps, 0.0, 0.0], 0.0, dt, k, k, 3)
        got = out[0, -1] - np.array([v, w])
        want = A @ delta
        assert np.linalg.norm(got - want) <= 1e-4 * np.linalg.norm(want), (got, want)


FHN_CHECKS = (check_fhn_one_step_drift, check_fhn_noise_on_v_only, check_fhn_linearisation)


@pytest.mark.parametrize("check", FHN_CHECKS, ids=lambda f: f.__name__[6:])
def test_fhn_recovery_rate_and_noise(oracle_lib, check):
    check(oracle_lib)


# Mistakes a reading of the FHN parameter layout could make; each replaces
# text of the oracle's source (every pattern occurs exactly once).
FHN_MUTANTS = {
    "recovery_rate_dropped": [("f[N + i] = eps * (v[i] + a - b * w[i]);",
                               "f[N + i] = (v[i] + a - b * w[i]);")],
    "eps_sigma_swapped": [("eps = p[2]", "eps = p[4]"),
                          ("gx[i] = p[4] * xi[i];", "gx[i] = p[2] * xi[i];")],
    "noise_on_w": [("gx[N + i] = 0.0;", "gx[N + i] = p[4] * xi[i];")],
}


@pytest.mark.parametrize("name", sorted(FHN_MUTANTS))
def test_fhn_pins_catch_planted_mistakes(oracle_lib, tmp_path, monkeypatch, name):
    """Compile the oracle with one planted mistake and check that at least one
    of the FHN pins above fails on it (the unaltered oracle passes them all)."""
    with open(oracle_lib.SRC) as f:
        src = f.read()
    for old, new in FHN_MUTANTS[name]:
        assert src.count(old) == 1, old
        src = src.replace(old, new)
    c_path = tmp_path / f"{name}.c"
    c_path.write_text(src)
    so = oracle_lib.build(force=True, src=str(c_path), out=str(tmp_path / f"{name}.so"))
    monkeypatch.setattr(oracle_lib, "_lib", oracle_lib.bind(so))
    failed = []
    for check in FHN_CHECKS:
        try:
            check(oracle_lib)
        except AssertionError:
            failed.append(check.__name__)
    assert failed, f"no FHN pin detects the mutant {name}"


def test_rnn_drift_is_matmul(oracle_lib):
    """f = -X + W tanh X + b equals numpy's matrix product."""
    rng = np.random.default_rng(9)
    n = 24
    W, b, X = rng.normal(0, 0.3, (n, n)), rng.normal(0, 0.3, n), rng.normal(0, 1, n)
    p = np.concatenate([W.ravel(), b, [0.05]])
    f = oracle_lib.drift("rnn", n, n, n * n + n + 1, X, p)
    np.testing.assert_allclose(f, -X + W @ np.tanh(X) + b, rtol=0, atol=1e-13)


def test_rnn_zero_weights_is_ou(oracle_lib):
    """W = 0: dX = (-X + b) dt + sigma dW, an OU process with a = 1, mu = b."""
    n, orbits, dt, K = 3, 4096, 0.05, 40
    b, sg = np.array([0.5, -1.0, 2.0]), 0.3
    p = np.concatenate([np.zeros(n * n), b, [sg]])
    out = oracle_lib.integrate("rnn", n, n, n * n + n + 1, np.zeros((orbits, n)), p, 0.0, dt, K,
                               K, 12)[:, -1]
    ou = oracle_lib.integrate("ou", 1, 1, 3, np.zeros((orbits * n, 1)), [1.0, 0.0, sg], 0.0,
                              dt, K, K, 13)
    rho = 1 - dt
    for i in range(n):
        mean = b[i] * (1 - rho**K)
        var = sg * sg * dt * (1 - rho ** (2 * K)) / (1 - rho * rho)
        assert abs(out[:, i].mean() - mean) < 5 * math.sqrt(var / orbits)
        assert abs(out[:, i].var(ddof=1) - var) < 5 * var * math.sqrt(2 / orbits)
    assert ou.shape == (orbits * n, 2, 1)


# --------------------------------------------------------------------------- addressing
def test_resume_and_shards_bitwise(oracle_lib):
    """Counter-based noise: 2N steps == N steps then N more with step_offset;
    one call == two calls over disjoint orbit ranges with orbit_offset."""
    w = workloads.kuramoto_grid(nK=4, nS=4, n=8, nsteps=200)
    args = ("kuramoto", 8, 8, 17)
    full = oracle_lib.integrate(*args, w["X0"], w["p"], 0.0, 1e-3, 200, 100, 5)
    first = oracle_lib.integrate(*args, w["X0"], w["p"], 0.0, 1e-3, 100, 100, 5)
    second = oracle_lib.integrate(*args, first[:, -1], w["p"], 0.1, 1e-3, 100, 100, 5,
                                  step_offset=100)
    np.testing.assert_array_equal(full[:, 2], second[:, 1])
    a = oracle_lib.integrate(*args, w["X0"][:7], w["p"][:7], 0.0, 1e-3, 200, 100, 5)
    b = oracle_lib.integrate(*args, w["X0"][7:], w["p"][7:], 0.0, 1e-3, 200, 100, 5,
                             orbit_offset=7)
    np.testing.assert_array_equal(np.concatenate([a, b]), full)


# --------------------------------------------------------------------------- paper claim
@pytest.mark.slow
def test_e4_coherence_either_side_of_critical_coupling(oracle_lib):
    """The accuracy section's qualitative outcome for N = 100: incoherence at
    K = 0.02 < K_c and near-synchrony at K = 0.2 > K_c (here dt = 0.2, the
    coarsest step of that protocol, 16 realisations)."""
    with open(os.path.join(GOLDEN, "e4_order_parameter.json")) as f:
        spec = json.load(f)
    assert 2 / (5 * math.pi) == pytest.approx(spec["K_c"], abs=1e-4)
    for case in spec["cases"]:
        w = workloads.kuramoto_e4(case["K"], realisations=16, level=5)
        out = oracle_lib.integrate_parallel("kuramoto", 100, 100, 201, w["X0"], w["p"], 0.0,
                                            w["dt"], w["nsteps"], w["stride"], w["seed"],
                                            threads=8, observable="kuramoto_r")
        r_end = out[:, -1, 0].mean()
        if "r_mean_at_end_below" in case:
            assert r_end < case["r_mean_at_end_below"], r_end
        else:
            assert r_end > case["r_mean_at_end_above"], r_end


# --------------------------------------------------------------------------- adjoint
def _window_R(oracle_lib, n, X0, p, dt, nsteps, lo, hi, seed):
    out = oracle_lib.integrate("kuramoto", n, n, 2 * n + 1, X0, p, 0.0, dt, nsteps, 1, seed,
                               observable="kuramoto_r")
    return out[:, lo:hi + 1, 0].mean(axis=1)


def test_adjoint_matches_central_differences(oracle_lib):
    """The discrete adjoint equals central finite differences of the FP64
    forward map (same noise) for every parameter of every orbit."""
    n, dt, nsteps, lo, hi, seed = 4, 1e-2, 300, 150, 300, 31
    rng = np.random.default_rng(21)
    X0 = rng.uniform(0, 2 * math.pi, (3, n))
    p = workloads.kuramoto_params(rng.uniform(0.5, 3, 3), rng.standard_normal((3, n)),
                                  rng.uniform(0.05, 0.4, (3, n)))
    R, grad, gpo = oracle_lib.kuramoto_adjoint(n, X0, p, 0.0, dt, nsteps, lo, hi, seed)
    np.testing.assert_allclose(R, _window_R(oracle_lib, n, X0, p, dt, nsteps, lo, hi, seed),
                               rtol=0, atol=1e-14)
    h = 1e-6
    fd = np.zeros_like(gpo)
    for q in range(2 * n + 1):
        pp, pm = p.copy(), p.copy()
        pp[:, q] += h
        pm[:, q] -= h
        fd[:, q] = (_window_R(oracle_lib, n, X0, pp, dt, nsteps, lo, hi, seed)
                    - _window_R(oracle_lib, n, X0, pm, dt, nsteps, lo, hi, seed)) / (2 * h)
    np.testing.assert_allclose(gpo, fd, rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(grad, gpo.sum(axis=0), rtol=1e-13)


def test_adjoint_uncoupled_closed_form(oracle_lib):
    """K = 0: the oscillators move independently, dX_i^k/d omega_i = k dt,
    dX_i^k/d p_i = sqrt(dt) sum_{l<k} N_{l,i} and dX_i^k/dK =
    dt/N sum_{l<k} sum_j sin(X_j^l - X_i^l), so dR/dp is a forward sum of
    dr/dX_i = (S cos X_i - C sin X_i)/(N |Z|) along the trajectory."""
    n, dt, nsteps, lo, hi, seed = 5, 2e-2, 200, 100, 200, 8
    rng = np.random.default_rng(5)
    X0 = rng.uniform(0, 2 * math.pi, (1, n))
    p = workloads.kuramoto_params([0.0], rng.standard_normal((1, n)), rng.uniform(0.1, 0.5, (1, n)))
    R, grad, _ = oracle_lib.kuramoto_adjoint(n, X0, p[0], 0.0, dt, nsteps, lo, hi, seed)
    traj = oracle_lib.integrate("kuramoto", n, n, 2 * n + 1, X0, p, 0.0, dt, nsteps, 1, seed)[0]
    xi = np.stack([oracle_lib.normals(seed, 0, k, n) for k in range(nsteps)])
    W = hi - lo + 1
    want = np.zeros(2 * n + 1)
    dXdK = np.zeros(n)
    noise_sum = np.zeros(n)
    for k in range(nsteps + 1):
        X = traj[k]
        if lo <= k <= hi:
            C, S = np.cos(X).sum(), np.sin(X).sum()
            drdx = (S * np.cos(X) - C * np.sin(X)) / (n * math.hypot(C, S))
            want[0] += drdx @ dXdK / W
            want[1:n + 1] += drdx * k * dt / W
            want[n + 1:] += drdx * math.sqrt(dt) * noise_sum / W
        if k < nsteps:
            dXdK += dt / n * np.array([np.sin(X - X[i]).sum() for i in range(n)])
            noise_sum += xi[k]
    np.testing.assert_allclose(grad, want, rtol=1e-10, atol=1e-13)


# --------------------------------------------------------------------------- source-text models
KURAMOTO4_DRIFT = """
const int N = 4;
for (int i = 0; i < N; ++i) {
    real acc = 0;
    for (int j = 0; j < N; ++j) acc = acc + sin(y[j] - y[i]);
    f[i] = acc * (p[0] / N) + p[1 + i];
}
"""
KURAMOTO4_DIFFUSION = "for (int i = 0; i < 4; ++i) gx[i] = p[5 + i] * xi[i];"


@pytest.mark.parametrize("method", ["em", "rk4", "implicit_midpoint"])
def test_custom_model_equals_builtin(oracle_lib, method):
    """The Kuramoto system written as source text (as the paper's users write
    it, Fig. 5) integrates bit for bit like the built-in model."""
    w = workloads.kuramoto_small()
    X0, p = w["X0"][:20], w["p"][:20]
    a = oracle_lib.integrate("kuramoto", 4, 4, 9, X0, p, 0.0, 0.01, 300, 100, 7, method=method)
    b = oracle_lib.integrate("custom", 4, 4, 9, X0, p, 0.0, 0.01, 300, 100, 7, method=method,
                             custom=(KURAMOTO4_DRIFT, KURAMOTO4_DIFFUSION))
    np.testing.assert_array_equal(a, b)


def test_implicit_step_without_a_root_is_nan(oracle_lib):
    """x' = x^2 + 1, dt = 0.1: from x = 100 the implicit Euler equation
    0.1 Y^2 - Y + 100.1 = 0 has no real root, so Newton cannot converge and
    the state becomes NaN; from x = 0 the root (1 - sqrt(0.96)) / 0.2 is found."""
    out = oracle_lib.integrate("custom", 1, 0, 1, [[100.0], [0.0]], [0.0], 0.0, 0.1, 1, 1, 1,
                               method="implicit_euler", custom=("f[0] = y[0] * y[0] + 1;", None))
    assert np.isnan(out[0, 1, 0])
    assert out[1, 1, 0] == pytest.approx((1 - math.sqrt(0.96)) / 0.2, rel=1e-13)


def test_custom_model_time_argument(oracle_lib):
    """dx = a t dt with t_k = t0 + k dt: Euler gives x_K = x0 + a dt (K t0 +
    dt K (K - 1) / 2) exactly in real arithmetic."""
    a, t0, dt, K = 0.5, 2.0, 0.125, 16
    out = oracle_lib.integrate("custom", 1, 0, 1, [[1.0]], [a], t0, dt, K, K, 3,
                               custom=("f[0] = p[0] * t;", None))
    assert out[0, -1, 0] == pytest.approx(1.0 + a * dt * (K * t0 + dt * K * (K - 1) / 2), rel=1e-15)


def test_custom_model_more_noises_than_equations(oracle_lib):
    """n = 1, m = 2: dx = -x dt + s1 dW1 + s2 dW2, three steps by hand with the
    step's first two normals."""
    s1, s2, dt, x = 0.3, 0.7, 0.1, 1.5
    out = oracle_lib.integrate("custom", 1, 2, 2, [[x]], [s1, s2], 0.0, dt, 3, 1, 11,
                               custom=("f[0] = -y[0];", "gx[0] = p[0] * xi[0] + p[1] * xi[1];"))
    for k in range(3):
        xi = oracle_lib.normals(11, 0, k, 2)
        x = x + (-x) * dt + (s1 * xi[0] + s2 * xi[1]) * math.sqrt(dt)
        assert out[0, k + 1, 0] == x

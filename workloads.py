"""Seeded synthetic inputs for the many-orbit SDE workloads.

This module only draws inputs (initial states, parameter grids, seeds) with
numpy's PCG64 generator; it holds none of the integrator's arithmetic and is
shared by the tests, the benchmark and the oracle checks alike.  The noise the
method itself consumes is not drawn here: both the library and the oracle
generate it from the Philox counter (seed, orbit id, step, block).

Every workload mirrors a configuration of the evaluation plan:
  kuramoto_small   n=m=4, 1024 orbits = 32 coupling values x 32 seeds, FP64
  kuramoto_grid    n=m=64, 65,536 orbits on a 256 x 256 (K, sigma) grid, FP32
  rnn_dense        n=m=256 dense random recurrent network, 8192 orbits
  fhn_ragged       4096 FitzHugh-Nagumo chains of uneven size and length
  kuramoto_adjoint n=m=32, 4096 orbits sharing (omega, K, sigma)
  kuramoto_paper   the speed-test protocol of Sec. 2.2.1 (N in {5,10,15})
  kuramoto_e4      the accuracy protocol of Sec. 2.3.1 (N=100)
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 1908038690


def _rng(index: int, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng([BASE_SEED + index, salt])


def kuramoto_params(K, omega, sigma):
    """Parameter rows (K, omega_1..N, sigma_1..N), the layout of the footnote
    of Sec. 2.2.1.  Arguments broadcast over a leading orbit axis."""
    K = np.atleast_1d(np.asarray(K, dtype=np.float64))
    omega = np.atleast_2d(np.asarray(omega, dtype=np.float64))
    sigma = np.atleast_2d(np.asarray(sigma, dtype=np.float64))
    rows = max(K.shape[0], omega.shape[0], sigma.shape[0])
    N = omega.shape[1]
    if sigma.shape[1] == 1:
        sigma = np.repeat(sigma, N, axis=1)
    p = np.empty((rows, 2 * N + 1), dtype=np.float64)
    p[:, 0] = np.broadcast_to(K, (rows,))
    p[:, 1:N + 1] = np.broadcast_to(omega, (rows, N))
    p[:, N + 1:] = np.broadcast_to(sigma, (rows, N))
    return p


def kuramoto_small():
    """n=m=4 Kuramoto, 32 K values in [0,4] x 32 seeds; omega ~ N(0,1) and
    theta0 ~ U[0,2pi) per seed; sigma = 0.1; orbit o = s*32 + iK.  All
    orbits of one seed share its Brownian path (orbit id 0, seed base+s)."""
    n, nK, nS = 4, 32, 32
    rng = _rng(1)
    Ks = np.linspace(0.0, 4.0, nK)
    omega_s = rng.standard_normal((nS, n))
    theta_s = rng.uniform(0.0, 2.0 * math.pi, (nS, n))
    orbits = nK * nS
    X0 = np.repeat(theta_s, nK, axis=0)
    omega = np.repeat(omega_s, nK, axis=0)
    K = np.tile(Ks, nS)
    p = kuramoto_params(K, omega, np.full((orbits, 1), 0.1))
    seed = 7001
    return dict(model="kuramoto", n=n, m=n, d=2 * n + 1, X0=X0, p=p, t0=0.0, dt=1e-3,
                nsteps=10_000, stride=100, seed=seed,
                orbit_ids=np.zeros(orbits, dtype=np.uint32),
                orbit_seeds=(seed + np.arange(nS, dtype=np.uint64)).repeat(nK),
                observable="state", precision=64)


def kuramoto_grid(nK: int = 256, nS: int = 256, n: int = 64, nsteps: int = 20_000):
    """n=m=64 Kuramoto on a K x sigma grid (K in [0,4], sigma in [0.01,0.5],
    K-major: o = iK*nS + iS); omega ~ N(0,1) and theta0 ~ U[0,2pi) shared by
    every orbit; independent noise per orbit; order parameter every 100 steps."""
    rng = _rng(2)
    omega = rng.standard_normal(n)
    theta = rng.uniform(0.0, 2.0 * math.pi, n)
    Ks = np.linspace(0.0, 4.0, nK)
    sig = np.linspace(0.01, 0.5, nS)
    K = np.repeat(Ks, nS)
    sigma = np.tile(sig, nK)[:, None]
    orbits = nK * nS
    p = kuramoto_params(K, np.broadcast_to(omega, (orbits, n)), sigma)
    X0 = np.broadcast_to(theta, (orbits, n)).copy()
    return dict(model="kuramoto", n=n, m=n, d=2 * n + 1, X0=X0, p=p, t0=0.0, dt=1e-3,
                nsteps=nsteps, stride=100, seed=8002, orbit_ids=None, orbit_seeds=None,
                observable="kuramoto_r", precision=32,
                diagonal=np.arange(min(nK, nS)) * (nS + 1) if nK == nS else None)


def kuramoto_adjoint(orbits: int = 4096, n: int = 32):
    """n=m=32 Kuramoto, orbits share (omega[32], K, sigma); theta0 per orbit."""
    rng = _rng(5)
    omega = rng.standard_normal(n)
    theta = rng.uniform(0.0, 2.0 * math.pi, (orbits, n))
    p = kuramoto_params(2.0, omega[None, :], np.full((1, 1), 0.1))[0]
    return dict(model="kuramoto", n=n, m=n, d=2 * n + 1, X0=theta, p=p, t0=0.0, dt=1e-3,
                nsteps=10_000, stride=100, seed=9005, ckpt_every=100, win_lo=5000,
                win_hi=10_000, target=0.6)


def rnn_dense(orbits: int = 8192, n: int = 256):
    """dX = (-X + W tanh X + b) dt + sigma dW; W ~ N(0, 1.5^2/n) and
    b ~ N(0, 0.1) (variance) shared; sigma = 0.05; X0 ~ N(0,1)."""
    rng = _rng(3)
    W = rng.standard_normal((n, n)) * (1.5 / math.sqrt(n))
    b = rng.standard_normal(n) * math.sqrt(0.1)
    p = np.concatenate([W.ravel(), b, [0.05]])
    X0 = rng.standard_normal((orbits, n))
    return dict(model="rnn", n=n, m=n, d=n * n + n + 1, X0=X0, p=p, t0=0.0, dt=1e-2,
                nsteps=5000, stride=100, seed=6003)


def fhn_ragged(count: int = 4096):
    """FitzHugh-Nagumo chains: units ~ logU[2,128], steps ~ logU[1e3,1e5]
    rounded down to a multiple of 100, (a,b,eps,D,sigma) uniform within
    +-20% of (0.7,0.8,0.08,0.1,0.05); v0 = -1.2 + 0.1 z, w0 = -0.62 + 0.1 z."""
    rng = _rng(4)
    units = np.floor(np.exp(rng.uniform(math.log(2), math.log(129), count))).astype(np.int64)
    units = np.clip(units, 2, 128)
    steps = np.exp(rng.uniform(math.log(1e3), math.log(1e5), count))
    steps = np.maximum((steps // 100).astype(np.int64) * 100, 1000)
    base = np.array([0.7, 0.8, 0.08, 0.1, 0.05])
    params = base * rng.uniform(0.8, 1.2, (count, 5))
    X0 = []
    for u in units:
        v = -1.2 + 0.1 * rng.standard_normal(u)
        w = -0.62 + 0.1 * rng.standard_normal(u)
        X0.append(np.concatenate([v, w]))
    return dict(model="fhn", units=units, nsteps=steps, params=params, X0=X0, dt=1e-3,
                stride=100, seed=5004)


def kuramoto_paper(N: int, M: int, nsteps: int = 8000):
    """Speed-test protocol of Sec. 2.2.1: K = 1, omega ~ U[0.01,0.03],
    noise strengths ~ U[0.001,0.003], theta0 ~ U[-pi,pi), dt = 0.05 s."""
    rng = _rng(10, N)
    omega = rng.uniform(0.01, 0.03, (M, N))
    sigma = rng.uniform(0.001, 0.003, (M, N))
    X0 = rng.uniform(-math.pi, math.pi, (M, N))
    p = kuramoto_params(np.ones(M), omega, sigma)
    return dict(model="kuramoto", n=N, m=N, d=2 * N + 1, X0=X0, p=p, t0=0.0, dt=0.05,
                nsteps=nsteps, stride=nsteps // 8 if nsteps >= 8 else 1, seed=4242)


def kuramoto_e4(K: float, realisations: int = 64, N: int = 100, level: int = 5):
    """Accuracy protocol of Sec. 2.3.1: N = 100, omega ~ U(0.2,0.4),
    theta0 ~ U(-pi,pi), noise strengths ~ U(0.01,0.03), 400 s at
    dt = 2^(level-5)/5; one frequency/noise draw per realisation."""
    rng = _rng(11, int(round(K * 1000)))
    omega = rng.uniform(0.2, 0.4, (realisations, N))
    sigma = rng.uniform(0.01, 0.03, (realisations, N))
    X0 = rng.uniform(-math.pi, math.pi, (realisations, N))
    dt = 2.0 ** (level - 5) / 5.0
    nsteps = int(round(400.0 / dt))
    p = kuramoto_params(np.full(realisations, K), omega, sigma)
    return dict(model="kuramoto", n=N, m=N, d=2 * N + 1, X0=X0, p=p, t0=0.0, dt=dt,
                nsteps=nsteps, stride=nsteps // 20, seed=3141)

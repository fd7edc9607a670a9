"""Models given as source text (sode_create_custom): compiled at run time
with hipRTC against the library's own stepper, checked against the built-in
model they restate and against the oracle integrating the same text as C."""
import numpy as np
import pytest

import workloads
from gpu_util import log, threads

pytestmark = pytest.mark.gpu

KURAMOTO4_DRIFT = """
const int N = 4;
for (int i = 0; i < N; ++i) {
    real acc = 0;
    for (int j = 0; j < N; ++j) acc = acc + sin(y[j] - y[i]);
    f[i] = acc * (p[0] / N) + p[1 + i];
}
"""
KURAMOTO4_DIFFUSION = "for (int i = 0; i < 4; ++i) gx[i] = p[5 + i] * xi[i];"

# Forced, damped pair with three Wiener processes (one shared): n = 2, m = 3.
FORCED_DRIFT = "f[0] = -p[0] * y[0] + sin(t); f[1] = -p[0] * y[1] + cos(t) * y[0];"
FORCED_DIFFUSION = "gx[0] = p[1] * xi[0] + p[2] * xi[2]; gx[1] = p[1] * xi[1] + p[2] * xi[2];"

# Stiff van der Pol oscillator (ODE).
VDP_DRIFT = "f[0] = y[1]; f[1] = p[0] * ((1 - y[0] * y[0]) * y[1] - y[0]);"


def _run(drift, diffusion, n, m, d, X0, p, t0, dt, nsteps, stride, seed, *, precision=64,
         method="em", orbit_offset=0, orbit_ids=None, orbit_seeds=None):
    import torch
    import paper_1908_03869_amd as sode
    it = sode.Integrator.custom(drift, diffusion, n, m, d, precision=precision, method=method,
                                shared_params=int(np.asarray(p).ndim == 1),
                                ode_limit=int(method in ("rk4", "implicit_euler", "implicit_midpoint")))
    dtype = torch.float64 if precision == 64 else torch.float32
    X0_t = torch.tensor(np.ascontiguousarray(X0), dtype=dtype, device="cuda")
    p_t = torch.tensor(np.ascontiguousarray(p), dtype=dtype, device="cuda")
    ids = None if orbit_ids is None else torch.tensor(
        np.asarray(orbit_ids, dtype=np.int64).astype(np.int32), device="cuda")
    sds = None if orbit_seeds is None else torch.tensor(
        np.asarray(orbit_seeds, dtype=np.uint64).astype(np.int64), device="cuda")
    out = it.integrate(X0_t, p_t, t0, dt, nsteps, stride, seed, orbit_offset=orbit_offset,
                       orbit_ids=ids, orbit_seeds=sds)
    it.sync()
    res = out.double().cpu().numpy()
    it.close()
    return res


def _oracle(drift, diffusion, n, m, d, X0, p, t0, dt, nsteps, stride, seed, method="em",
            orbit_ids=None, orbit_seeds=None):
    import oracle
    return oracle.integrate_parallel("custom", n, m, d, X0, p, t0, dt, nsteps, stride, seed,
                                     threads=threads(), method=method, custom=(drift, diffusion),
                                     orbit_ids=orbit_ids, orbit_seeds=orbit_seeds)


def test_kuramoto_text_matches_builtin_and_oracle(gpu):
    """The small Kuramoto ensemble (1024 orbits, binary64) written as source text."""
    from gpu_util import run_library
    w = workloads.kuramoto_small()
    w = dict(w, nsteps=2000, stride=100)
    log("custom kuramoto n=4 fp64")
    noise = dict(orbit_ids=w["orbit_ids"], orbit_seeds=w["orbit_seeds"])
    got = _run(KURAMOTO4_DRIFT, KURAMOTO4_DIFFUSION, 4, 4, 9, w["X0"], w["p"], 0.0, w["dt"],
               2000, 100, w["seed"], **noise)
    builtin = run_library(w, precision=64, kernel="plain", wrap=0)  # the text does not wrap
    assert np.abs(got - builtin).max() <= 1e-12
    want = _oracle(KURAMOTO4_DRIFT, KURAMOTO4_DIFFUSION, 4, 4, 9, w["X0"], w["p"], 0.0, w["dt"],
                   2000, 100, w["seed"], **noise)
    assert np.abs(got - want).max() <= 1e-10


@pytest.mark.parametrize("precision,tol", [(64, 1e-10), (32, 1e-4)])
@pytest.mark.parametrize("method", ["em", "rk4"])
def test_forced_model_with_more_noises(gpu, precision, tol, method):
    """Time-dependent drift (sin t, cos t) and m = 3 > n = 2; 300 orbits."""
    rng = np.random.default_rng(17)
    X0 = rng.uniform(-1, 1, (300, 2))
    p = np.column_stack([rng.uniform(0.5, 2.0, 300), np.full(300, 0.2), np.full(300, 0.1)])
    if precision == 32:
        X0 = X0.astype(np.float32).astype(np.float64)
        p = p.astype(np.float32).astype(np.float64)
    log(f"custom forced model {method} fp{precision}")
    got = _run(FORCED_DRIFT, FORCED_DIFFUSION, 2, 3, 3, X0, p, 0.5, 0.01, 1000, 100, 99,
               precision=precision, method=method)
    want = _oracle(FORCED_DRIFT, FORCED_DIFFUSION, 2, 3, 3, X0, p, 0.5, 0.01, 1000, 100, 99,
                   method=method)
    assert np.abs(got - want).max() <= tol


@pytest.mark.parametrize("method", ["implicit_euler", "implicit_midpoint"])
def test_stiff_van_der_pol_implicit(gpu, method):
    """mu = 30, dt = 0.01 over 3 s, through the fast relaxation jumps:
    implicit steps against the oracle's."""
    rng = np.random.default_rng(5)
    X0 = np.column_stack([rng.uniform(-2, 2, 70), rng.uniform(-1, 1, 70)])
    log(f"custom van der Pol {method}")
    got = _run(VDP_DRIFT, None, 2, 0, 1, X0, np.array([30.0]), 0.0, 0.01, 300, 30, 1,
               method=method)
    want = _oracle(VDP_DRIFT, None, 2, 0, 1, X0, np.array([30.0]), 0.0, 0.01, 300, 30, 1,
                   method=method)
    assert np.all(np.isfinite(got))
    assert np.abs(got - want).max() <= 1e-8


def test_implicit_step_without_a_root_gives_nan(gpu):
    """x' = x^2 + 1 from x = 100 with dt = 0.1: the implicit Euler equation
    dt Y^2 - Y + X + dt = 0 has no real root, Newton cannot converge and the
    state becomes NaN (the oracle does the same); the other orbit, x = 0,
    has a root and stays finite."""
    import torch
    import paper_1908_03869_amd as sode
    X0 = np.array([[100.0], [0.0]])
    log("implicit step without a root")
    it = sode.Integrator.custom("f[0] = y[0] * y[0] + 1;", None, 1, 0, 1, precision=64,
                                method="implicit_euler", shared_params=1)
    out = it.integrate(torch.tensor(X0, device="cuda"), torch.zeros(1, dtype=torch.float64,
                       device="cuda"), 0.0, 0.1, 1, 1, 1)
    with pytest.raises(sode.SodeError) as e:  # the NaN is reported at the sync
        it.sync()
    assert e.value.status == sode.abi.SODE_ENONFINITE
    got = out.cpu().numpy()
    it.close()
    want = _oracle("f[0] = y[0] * y[0] + 1;", None, 1, 0, 1, X0, np.array([0.0]), 0.0, 0.1, 1,
                   1, 1, method="implicit_euler")
    assert np.isnan(want[0, 1, 0]) and np.isnan(got[0, 1, 0])
    assert np.isfinite(got[1, 1, 0]) and abs(got[1, 1, 0] - want[1, 1, 0]) <= 1e-12


def test_shards_equal_one_call(gpu):
    rng = np.random.default_rng(8)
    X0 = rng.uniform(-1, 1, (200, 2))
    p = np.column_stack([rng.uniform(0.5, 2.0, 200), np.full(200, 0.2), np.full(200, 0.1)])
    args = (0.0, 0.01, 400, 100, 3)
    log("custom shards")
    full = _run(FORCED_DRIFT, FORCED_DIFFUSION, 2, 3, 3, X0, p, *args)
    a = _run(FORCED_DRIFT, FORCED_DIFFUSION, 2, 3, 3, X0[:77], p[:77], *args)
    b = _run(FORCED_DRIFT, FORCED_DIFFUSION, 2, 3, 3, X0[77:], p[77:], *args, orbit_offset=77)
    np.testing.assert_array_equal(np.concatenate([a, b]), full)

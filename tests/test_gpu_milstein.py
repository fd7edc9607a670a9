"""Milstein stepper (method 2, plain kernel) against the FP64 oracle's
Milstein scheme, and its strong order one on the GPU itself."""
import numpy as np
import pytest

from gpu_util import log, run_library, run_oracle

pytestmark = pytest.mark.gpu


def _gbm(n, orbits, nsteps, dt, mu=0.5, s=0.4, stride=None):
    X0 = np.random.default_rng(n * 1000 + orbits).uniform(0.5, 2.0, (orbits, n))
    return dict(model="gbm", n=n, m=n, d=2, X0=X0, p=np.array([mu, s]), t0=0.0, dt=dt,
                nsteps=nsteps, stride=stride or nsteps // 10, seed=20240611,
                observable="state")


@pytest.mark.parametrize("n", [1, 3])
def test_gbm_fp64_matches_oracle(gpu, n):
    """n = 1 takes the compile-time-size kernel, n = 3 the runtime-size one;
    1000 orbits leave a ragged last block."""
    w = _gbm(n, 1000, 500, 2e-3)
    log(f"milstein gbm fp64 n={n}")
    got = run_library(w, precision=64, kernel="plain", method="milstein")
    want = run_oracle(w, method="milstein")
    rel = np.abs(got - want) / np.abs(want)
    assert rel.max() <= 1e-12, rel.max()


def test_gbm_fp32_matches_oracle(gpu):
    w = _gbm(1, 4096, 1000, 1e-3)
    log("milstein gbm fp32")
    got = run_library(w, precision=32, kernel="plain", method="milstein")
    want = run_oracle(w, method="milstein", precision=32)
    rel = np.abs(got - want) / np.abs(want)
    assert rel.max() <= 1e-4, rel.max()


@pytest.mark.parametrize("model,n,m,d,p", [("ou", 2, 2, 3, [0.7, 0.2, 0.3]),
                                           ("kuramoto", 4, 4, 9, [1.5, 0.1, 0.2, -0.3, 0.4,
                                                                  0.1, 0.2, 0.3, 0.05])])
def test_additive_noise_milstein_is_em(gpu, model, n, m, d, p):
    X0 = np.random.default_rng(4).uniform(-1, 1, (130, n))
    w = dict(model=model, n=n, m=m, d=d, X0=X0, p=np.array(p), t0=0.0, dt=1e-2, nsteps=200,
             stride=20, seed=99, observable="state")
    log(f"milstein == em for {model}")
    a = run_library(w, precision=64, kernel="plain", method="em")
    b = run_library(w, precision=64, kernel="plain", method="milstein")
    np.testing.assert_array_equal(a, b)


def test_gbm_strong_order_one_on_gpu(gpu):
    """65,536 orbits per level: the mean absolute error against the exact
    solution X0 exp((mu - s^2/2) T + s W(T)), with W(T) integrated by the
    library from the same normals (OU with a = 0, s = 1), falls like dt;
    Euler-Maruyama on the same paths falls like dt^(1/2)."""
    mu, s, T, orbits = 1.0, 0.8, 1.0, 65536
    X0 = np.ones((orbits, 1))
    slopes = {}
    for method in ("milstein", "em"):
        errs, dts = [], []
        for L in range(4, 10):
            nsteps = 2**L
            dt = T / nsteps
            w = dict(model="gbm", n=1, m=1, d=2, X0=X0, p=np.array([mu, s]), t0=0.0, dt=dt,
                     nsteps=nsteps, stride=nsteps, seed=700 + L, observable="state")
            log(f"strong order {method} L={L}")
            X = run_library(w, precision=64, kernel="plain", method=method)[:, -1, 0]
            bw = dict(w, model="ou", d=3, X0=np.zeros((orbits, 1)), p=np.array([0.0, 0.0, 1.0]))
            W = run_library(bw, precision=64, kernel="plain")[:, -1, 0]
            exact = np.exp((mu - 0.5 * s * s) * T + s * W)
            errs.append(np.mean(np.abs(X - exact)))
            dts.append(dt)
        slopes[method] = np.polyfit(np.log(dts), np.log(errs), 1)[0]
    print(f"strong-order slopes: {slopes}")
    assert 0.9 < slopes["milstein"] < 1.1, slopes
    assert 0.4 < slopes["em"] < 0.6, slopes

"""Implicit Euler and implicit midpoint ODE steppers (methods 3, 4) of the
one-orbit-per-lane kernel against the oracle's steppers.  Both sides solve
the same implicit equation by Newton's method to a relative correction of
64 eps, so they agree to a few times that bound per step; binary64 cases
are held to 1e-10, binary32 to 1e-4."""
import numpy as np
import pytest

import workloads
from gpu_util import circular_diff, log, run_library, run_oracle

pytestmark = pytest.mark.gpu


def _case(model, n, m, d, p, orbits=130, dt=0.05, nsteps=200, stride=20, scale=1.0):
    X0 = np.random.default_rng(n * 7 + orbits).uniform(-scale, scale, (orbits, n))
    return dict(model=model, n=n, m=m, d=d, X0=X0, p=np.asarray(p, dtype=np.float64), t0=0.0,
                dt=dt, nsteps=nsteps, stride=stride, seed=5, observable="state")


CASES = {
    "ou_stiff_n1": ("ou", 1, 1, 3, [1000.0, 0.3, 0.5], 0.01),
    "ou_stiff_n3": ("ou", 3, 3, 3, [1000.0, 0.3, 0.5], 0.01),
    "kuramoto_n2": ("kuramoto", 2, 2, 5, [3.0, -2.0, 2.0, 0.0, 0.0], 0.05),
    "fhn_n6": ("fhn", 6, 3, 5, [0.7, 0.8, 0.08, 0.1, 0.05], 0.05),
    "rnn_n6": ("rnn", 6, 6, 43, None, 0.05),
}


def _params(name):
    model, n, m, d, p, dt = CASES[name]
    if p is None:  # dense network: W ~ N(0, 1.5^2 / n), b ~ N(0, 0.1), sigma
        rng = np.random.default_rng(3)
        W = rng.normal(0.0, 1.5 / np.sqrt(n), (n, n))
        p = np.concatenate([W.ravel(), rng.normal(0.0, np.sqrt(0.1), n), [0.05]])
    return model, n, m, d, p, dt


@pytest.mark.parametrize("method", ["implicit_euler", "implicit_midpoint"])
@pytest.mark.parametrize("name", list(CASES))
def test_fp64_matches_oracle(gpu, name, method):
    model, n, m, d, p, dt = _params(name)
    w = _case(model, n, m, d, p, dt=dt)
    log(f"{method} fp64 {name}")
    got = run_library(w, precision=64, kernel="plain", method=method)
    want = run_oracle(w, method=method)
    # Kuramoto phases come back reduced to [-pi, pi]; the oracle never wraps.
    diff = circular_diff(got, want) if model == "kuramoto" else np.abs(got - want)
    assert diff.max() <= 1e-10


@pytest.mark.parametrize("method", ["implicit_euler", "implicit_midpoint"])
def test_fp32_matches_oracle(gpu, method):
    model, n, m, d, p, dt = _params("fhn_n6")
    w = _case(model, n, m, d, p, dt=dt)
    log(f"{method} fp32 fhn")
    got = run_library(w, precision=32, kernel="plain", method=method)
    want = run_oracle(w, method=method, precision=32)
    assert np.abs(got - want).max() <= 1e-4


def test_largest_size(gpu):
    """n = 16, the largest the implicit steppers take (16 x 16 Newton matrix per lane)."""
    w = workloads.kuramoto_grid(nK=3, nS=5, n=16, nsteps=100)
    w = dict(w, observable="state", nsteps=100, stride=20)
    log("implicit midpoint fp64 kuramoto n=16")
    got = run_library(w, precision=64, kernel="plain", method="implicit_midpoint")
    want = run_oracle(w, method="implicit_midpoint")
    assert circular_diff(got, want).max() <= 1e-10

"""Coupled binary32 kernel at sizes that are not multiples of 16: the row is
padded with oscillators frozen at phase 0 whose coupling is cancelled.
Checked against the FP64 oracle of the unpadded N-oscillator system with the
bounds of the unpadded kernel (1e-3 on phases over 2000 steps, 1e-4 on r)."""
import numpy as np
import pytest

import workloads
from gpu_util import circular_diff, log, run_library, run_oracle

pytestmark = pytest.mark.gpu


def _grid(n, nsteps, nK=7, nS=11):
    return workloads.kuramoto_grid(nK=nK, nS=nS, n=n, nsteps=nsteps)


@pytest.mark.parametrize("n", [1, 5, 15, 33, 50, 100, 127])
def test_padded_state(gpu, n):
    """P = 1..8 oscillators per lane (every lane_normals layout), 77 orbits."""
    w = dict(_grid(n, 2000), observable="state")
    log(f"padded coupled state n={n}")
    got = run_library(w, precision=32, kernel="coupled")
    assert got.shape == (77, 21, n)
    want = run_oracle(w, precision=32)
    assert circular_diff(got, want).max() <= 1e-3


@pytest.mark.parametrize("n", [5, 100])
def test_padded_order_parameter(gpu, n):
    w = _grid(n, 4000, nK=9, nS=9)
    log(f"padded coupled r n={n}")
    got = run_library(w, precision=32, kernel="coupled")
    want = run_oracle(w, precision=32)
    assert np.abs(got - want).max() <= 1e-4


@pytest.mark.parametrize("n", [15, 100])
def test_padded_mean_field(gpu, n):
    w = dict(_grid(n, 2000), observable="state")
    log(f"padded coupled mean-field n={n}")
    got = run_library(w, precision=32, kernel="coupled", drift=1)
    want = run_oracle(w, precision=32)
    assert circular_diff(got, want).max() <= 1e-3


def test_padded_uncompensated(gpu):
    w = dict(_grid(100, 2000), observable="state")
    log("padded coupled n=100 without compensation")
    got = run_library(w, precision=32, kernel="coupled", compensated=0)
    want = run_oracle(w, precision=32)
    assert circular_diff(got, want).max() <= 1e-3


def test_accuracy_study_workload(gpu):
    """The Sec. 2.3.1 system (N = 100, omega ~ U(0.2, 0.4), K = 0.2) over its
    full 400 s at dt = 0.05 (level 3), 16 realisations: r(t) within 1e-4."""
    w = workloads.kuramoto_e4(0.2, realisations=16, level=3)
    w = dict(w, observable="kuramoto_r")
    log("padded coupled E4 workload K=0.2 level 3")
    got = run_library(w, precision=32, kernel="coupled")
    want = run_oracle(w, precision=32)
    assert np.abs(got - want).max() <= 1e-4

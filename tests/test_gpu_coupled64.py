"""Binary64 16-lane Kuramoto kernel (kernel "coupled", precision 64) against
the FP64 oracle.  The kernel evaluates each unordered pair once and sums in
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

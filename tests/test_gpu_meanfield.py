"""The mean-field form of the Kuramoto coupling (drift option 1) against the
FP64 oracle, which evaluates the pairwise sines of Eq. (5): the two forms
are the same function in real arithmetic, so the bounds are those of the
pairwise kernels - 1e-10 for binary64, 1e-4 on r and 1e-3 on phases for
binary32."""
import numpy as np
import pytest

import workloads
from gpu_util import as_received, circular_diff, log, run_library, run_oracle, threads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N", [5, 10, 15, 64])
def test_plain_fp64_paper_shapes(gpu, N):
    """The paper's speed-test systems (Sec. 2.2.1; N = 5, 10, 15) and a
    runtime-N case, 97 orbits (ragged last block), 2000 steps of dt = 0.05."""
    w = dict(workloads.kuramoto_paper(N, 97, nsteps=2000), observable="state")
    log(f"mean-field plain fp64 N={N}")
    got = run_library(w, precision=64, kernel="plain", drift=1)
    want = run_oracle(w)
    assert circular_diff(got, want).max() <= 1e-10


@pytest.mark.parametrize("N", [5, 15])
def test_plain_fp32_paper_shapes(gpu, N):
    w = dict(workloads.kuramoto_paper(N, 97, nsteps=2000), observable="state")
    log(f"mean-field plain fp32 N={N}")
    got = run_library(w, precision=32, kernel="plain", drift=1)
    want = run_oracle(w, precision=32)
    assert circular_diff(got, want).max() <= 1e-3


@pytest.mark.parametrize("n", [16, 64, 128])
def test_coupled_fp32_state(gpu, n):
    w = dict(workloads.kuramoto_grid(nK=7, nS=11, n=n, nsteps=2000), observable="state")
    log(f"mean-field coupled fp32 state n={n}")
    got = run_library(w, precision=32, kernel="coupled", drift=1)
    want = run_oracle(w, precision=32)
    assert circular_diff(got, want).max() <= 1e-3


def test_coupled_fp32_order_parameter(gpu):
    w = workloads.kuramoto_grid(nK=9, nS=9, n=64, nsteps=4000)
    log("mean-field coupled fp32 r n=64, 81 orbits x 4000 steps")
    got = run_library(w, precision=32, kernel="coupled", drift=1)
    want = run_oracle(w, precision=32)
    assert np.abs(got - want).max() <= 1e-4


def test_full_grid_sampled(gpu):
    """The full n = 64 grid (65,536 orbits, 2x10^4 steps) with the mean-field
    drift, sampled on the grid diagonal like the pairwise test."""
    w = workloads.kuramoto_grid()
    log("mean-field kuramoto_grid full size")
    got = run_library(w, precision=32, drift=1)
    rows = w["diagonal"][::11]
    want = run_oracle(w, rows=rows, precision=32)
    err = np.abs(got[rows] - want)
    assert err[:, -1].max() <= 1e-4, err[:, -1].max()
    assert err.max() <= 1e-3, err.max()


def test_adjoint_with_mean_field_recompute(gpu):
    """The adjoint recomputes each segment with the same drift form as its
    forward pass; the gradient meets the pairwise oracle adjoint's bound."""
    import torch
    import oracle
    import paper_1908_03869_amd as sode
    w = workloads.kuramoto_adjoint()
    rows = np.arange(64)
    X0 = torch.tensor(np.ascontiguousarray(w["X0"][rows]), dtype=torch.float32, device="cuda")
    p = torch.tensor(w["p"], dtype=torch.float32, device="cuda")
    it = sode.Integrator("kuramoto", 32, 32, 65, precision=32, shared_params=1, drift=1)
    args = (0.0, w["dt"], w["nsteps"], w["ckpt_every"], w["win_lo"], w["win_hi"], w["seed"])
    log("mean-field adjoint vs oracle, 64 orbits x 1e4 steps")
    ckpt, R = it.forward_ckpt(X0, p, *args)
    dLdR = 2.0 * (R - w["target"]) / len(rows)
    grad, _ = it.adjoint(p, ckpt, *args, dL_dR=dLdR)
    it.sync()
    Rg = R.cpu().numpy()
    Rref, gref, _ = oracle.kuramoto_adjoint_parallel(
        32, as_received(w["X0"][rows], 32), as_received(w["p"], 32), 0.0, w["dt"], w["nsteps"],
        w["win_lo"], w["win_hi"], w["seed"], dL_dR=2.0 * (Rg - w["target"]) / len(rows),
        threads=threads())
    it.close()
    assert np.max(np.abs(Rg - Rref)) <= 1e-4
    g = grad.cpu().numpy()
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    print(f"relative L2 error of the summed gradient: {rel:.3e}")
    assert rel <= 1e-3, rel

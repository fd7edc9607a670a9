"""Runs that end, save or resume inside a group of steps that share one
Philox block.  At one or two oscillators per lane the 16-lane Kuramoto
kernels (binary32 and binary64, integrate, forward_ckpt and adjoint) draw
the normals of 4 / P consecutive steps together; these cases put the step
count, the save stride, the checkpoint interval and the step offset at
values that are not multiples of 4 or 2.

Bounds: 35 steps from the oracle's own inputs, so binary32 phases are held
to 1e-4 (the rounding of a few dozen compensated steps is ~1e-6; one normal
drawn for the wrong step moves a phase by sigma sqrt(dt) ~ 1e-2 on the
largest-sigma orbits) and binary64 to 1e-10 as in the other binary64 tests.
The stride-independence and split-run checks are bitwise: the path an orbit
takes cannot depend on where it is saved or resumed."""
import numpy as np
import pytest

import workloads
from gpu_util import as_received, circular_diff, log, run_library, run_oracle

pytestmark = pytest.mark.gpu

# (precision, n): P = 1 and 2 oscillators per lane, padded and unpadded, and
# one P = 4 row, whose steps draw their own blocks, as a control.
SIZES = [(32, 5), (32, 16), (32, 20), (32, 32), (32, 64),
         (64, 8), (64, 16), (64, 24), (64, 32), (64, 64)]


def _grid(n, nsteps, stride):
    w = workloads.kuramoto_grid(nK=5, nS=8, n=n, nsteps=nsteps)
    return dict(w, stride=stride, observable="state")


@pytest.mark.parametrize("drift", [0, 1])
@pytest.mark.parametrize("precision,n", SIZES)
def test_ragged_step_groups_match_oracle(gpu, precision, n, drift):
    """35 steps saved every 7: five saves land at different positions in a
    group and the run ends one (P = 2) or three (P = 1) steps into a group."""
    w = _grid(n, 35, 7)
    log(f"tails vs oracle fp{precision} n={n} drift={drift}")
    got = run_library(w, precision=precision, kernel="coupled", drift=drift)
    want = run_oracle(w, precision=precision)
    assert got.shape == (40, 6, n)
    bound = 1e-4 if precision == 32 else 1e-10
    assert circular_diff(got, want).max() <= bound


@pytest.mark.parametrize("precision,n", SIZES)
def test_stride_does_not_change_the_path(gpu, precision, n):
    """Saving every step and saving every 7th give the same states, bitwise."""
    w = _grid(n, 35, 7)
    log(f"tails stride independence fp{precision} n={n}")
    every = run_library(w, precision=precision, kernel="coupled", stride=1)
    sparse = run_library(w, precision=precision, kernel="coupled")
    np.testing.assert_array_equal(sparse, every[:, ::7])


@pytest.mark.parametrize("precision,n", SIZES)
def test_resume_inside_a_group(gpu, precision, n):
    """13 steps, then 22 more from step_offset = 13, equal the 35-step run
    bitwise (binary32 with a single rounded phase: a compensated resume
    restarts its trailing part)."""
    w = _grid(n, 35, 35)
    kw = dict(precision=precision, kernel="coupled", compensated=0)
    log(f"tails resume at step 13 fp{precision} n={n}")
    full = run_library(w, **kw)
    head = run_library(w, nsteps=13, stride=13, **kw)
    rest = run_library(w, X0=head[:, -1], nsteps=22, stride=22, step_offset=13,
                       t0=13 * w["dt"], **kw)
    np.testing.assert_array_equal(rest[:, -1], full[:, -1])


@pytest.mark.parametrize("n", [16, 32])
def test_adjoint_with_odd_checkpoint_interval(gpu, n):
    """Checkpoints every 7 steps, 63 steps from step_offset = 5, window
    [10, 61]: without compensation the checkpoints equal integrate's states
    bitwise; with it (the default) each checkpoint is what integrate gives
    when restarted from the one before it; R is within 1e-5 of the oracle's
    and the gradient within 1e-3 relative of the FP64 oracle adjoint (the
    adjoint workload's bound)."""
    import torch
    import oracle
    import paper_1908_03869_amd as sode

    w = workloads.kuramoto_adjoint(orbits=40, n=n)
    nsteps, every, lo, hi, off = 63, 7, 10, 61, 5
    X0 = torch.tensor(np.ascontiguousarray(w["X0"]), dtype=torch.float32, device="cuda")
    p = torch.tensor(w["p"], dtype=torch.float32, device="cuda")
    args = (0.0, w["dt"], nsteps, every, lo, hi, w["seed"])
    log(f"tails adjoint n={n} every={every} offset={off}")
    it0 = sode.Integrator("kuramoto", n, n, 2 * n + 1, precision=32, shared_params=1,
                          compensated=0)
    ckpt0, _ = it0.forward_ckpt(X0, p, *args, step_offset=off)
    it0.sync()
    states = run_library(dict(w, observable="state"), precision=32, kernel="coupled",
                         nsteps=nsteps, stride=every, step_offset=off, shared=True,
                         compensated=0)
    np.testing.assert_array_equal(ckpt0.double().cpu().numpy(), states)
    it = sode.Integrator("kuramoto", n, n, 2 * n + 1, precision=32, shared_params=1)
    ckpt, R = it.forward_ckpt(X0, p, *args, step_offset=off)
    grad, _ = it.adjoint(p, ckpt, *args, step_offset=off)
    it.sync()
    ck = ckpt.double().cpu().numpy()
    for c in range(ck.shape[1] - 1):
        seg = run_library(dict(w, observable="state"), precision=32, kernel="coupled",
                          X0=ck[:, c], nsteps=every, stride=every, step_offset=off + c * every,
                          t0=c * every * w["dt"], shared=True)
        np.testing.assert_array_equal(seg[:, -1], ck[:, c + 1], err_msg=f"checkpoint {c + 1}")

    Rref, gref, _ = oracle.kuramoto_adjoint(n, as_received(w["X0"], 32),
                                            as_received(w["p"], 32), 0.0, w["dt"], nsteps,
                                            lo, hi, w["seed"], step_offset=off, per_orbit=False)
    assert np.max(np.abs(R.cpu().numpy() - Rref)) <= 1e-5
    g = grad.cpu().numpy()
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    assert rel <= 1e-3, rel

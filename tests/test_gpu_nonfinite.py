"""The non-finite flag: a NaN or infinite saved value makes the next
sode_sync return SODE_ENONFINITE (the Python layer raises), for every
integrate path; the sync clears the flag."""
import numpy as np
import pytest

import workloads
from gpu_util import log

pytestmark = pytest.mark.gpu


def _sync_status(it):
    import paper_1908_03869_amd as sode
    try:
        it.sync()
        return sode.abi.SODE_OK
    except sode.SodeError as e:
        return e.status


def test_unstable_explicit_step_then_clean_run(gpu):
    """OU with a dt = 10: Euler-Maruyama multiplies x - mu by -9 per step and
    overflows binary32 within 50 steps; a stable run afterwards is clean."""
    import torch
    import paper_1908_03869_amd as sode
    it = sode.Integrator("ou", 1, 1, 3, precision=32, shared_params=1)
    X0 = torch.ones(100, 1, device="cuda")
    log("non-finite: unstable OU")
    it.integrate(X0, torch.tensor([1000.0, 0.0, 0.1], device="cuda"), 0.0, 0.01, 100, 10, 1)
    assert _sync_status(it) == sode.abi.SODE_ENONFINITE
    it.integrate(X0, torch.tensor([1.0, 0.0, 0.1], device="cuda"), 0.0, 0.01, 100, 10, 1)
    assert _sync_status(it) == sode.abi.SODE_OK
    it.close()


@pytest.mark.parametrize("precision,kernel,n", [(32, "coupled", 64), (64, "coupled", 16),
                                                (64, "plain", 4), (32, "coupled", 5)])
def test_nan_input_is_reported(gpu, precision, kernel, n):
    import torch
    import paper_1908_03869_amd as sode
    w = workloads.kuramoto_grid(nK=2, nS=3, n=n, nsteps=100)
    dtype = torch.float32 if precision == 32 else torch.float64
    X0 = torch.tensor(w["X0"], dtype=dtype, device="cuda")
    X0[3, n // 2] = float("nan")
    it = sode.Integrator("kuramoto", n, n, 2 * n + 1, precision=precision, kernel=kernel)
    log(f"non-finite: NaN input {precision} {kernel} n={n}")
    it.integrate(X0, torch.tensor(w["p"], dtype=dtype, device="cuda"), 0.0, 1e-3, 100, 50, 1)
    assert _sync_status(it) == sode.abi.SODE_ENONFINITE
    it.close()


def test_dense_network_and_ragged_report(gpu):
    import torch
    import paper_1908_03869_amd as sode
    w = workloads.rnn_dense()
    X0 = torch.tensor(w["X0"][:64], dtype=torch.float32, device="cuda")
    X0[7, 3] = float("inf")
    it = sode.Integrator("rnn", 256, 256, w["d"], precision=32, shared_params=1,
                         kernel="matrix")
    log("non-finite: dense network")
    it.integrate(X0, torch.tensor(w["p"], dtype=torch.float32, device="cuda"), 0.0, w["dt"], 20,
                 10, 1)
    assert _sync_status(it) == sode.abi.SODE_ENONFINITE
    it.close()

    n = np.array([8, 20])
    batch = sode.RaggedBatch(n, nsteps=np.array([100, 200]), stride=50, seeds=5,
                             orbit_ids=np.arange(2), d=5)
    X0 = torch.zeros(batch.x0_len, device="cuda")
    X0[3] = float("nan")
    p = torch.tensor(np.tile([0.7, 0.8, 0.08, 0.1, 0.05], 2), dtype=torch.float32, device="cuda")
    rg = sode.Integrator("fhn", 20, 10, 5, precision=32)
    log("non-finite: ragged")
    rg.integrate_ragged(batch, X0, p, 0.0, 1e-3)
    assert _sync_status(rg) == sode.abi.SODE_ENONFINITE
    rg.close()

"""Dense random networks with the drift's matrix product on MFMA, against
the FP64 oracle.

Workload: n = m = 256, W ~ N(0, 1.5^2/n) and b ~ N(0, 0.1) shared,
sigma = 0.05, 8192 orbits, dt = 1e-2, 5000 steps, state saved every 100
steps.  Error: relative L2 norm of the final-state difference per orbit, max over
64 orbits; the workload's bound is 1e-2.  The split (bf16x3, the default)
and binary32 products meet it with a wide margin and are held to 1e-3 and
1e-4.  The plain bfloat16 product does NOT meet it on this workload (max
~5e-2, median ~1e-2: rounding W alone to bfloat16 already moves the
trajectories by ~1e-2); its test pins that measured envelope instead.
"""
import numpy as np
import pytest

import workloads
from gpu_util import log, run_library, run_oracle

pytestmark = pytest.mark.gpu

BOUND = {"bf16": 1e-2, "bf16x3": 1e-3, "fp32": 1e-4}
ENVELOPE_BF16 = {"max": 0.1, "median": 2e-2}


def _rel_final(got, ref):
    d = np.linalg.norm(got[:, -1] - ref[:, -1], axis=1)
    return d / np.linalg.norm(ref[:, -1], axis=1)


def _run(w, gemm, **kw):
    import torch
    import paper_1908_03869_amd as sode
    it = sode.Integrator("rnn", w["n"], w["m"], w["d"], precision=32, shared_params=1,
                         kernel="matrix", gemm=gemm)
    X0 = torch.tensor(w["X0"], dtype=torch.float32, device="cuda")
    p = torch.tensor(w["p"], dtype=torch.float32, device="cuda")
    out = it.integrate(X0, p, 0.0, w["dt"], w["nsteps"], w["stride"], w["seed"], **kw)
    it.sync()
    res = out.double().cpu().numpy()
    it.close()
    return res


@pytest.fixture(scope="module")
def full_reference():
    w = workloads.rnn_dense()
    rows = np.arange(0, 8192, 128)
    ref = run_oracle(w, rows=rows, precision=32)
    return w, rows, ref


@pytest.mark.parametrize("gemm", ["bf16", "bf16x3", "fp32"])
def test_full_workload_against_oracle(gpu, full_reference, gemm):
    w, rows, ref = full_reference
    log(f"rnn n=256 8192 orbits x 5000 steps, gemm={gemm}")
    got = _run(w, gemm)
    assert got.shape == (8192, 51, 256)
    assert np.all(np.isfinite(got))
    rel = _rel_final(got[rows], ref)
    print(f"{gemm}: final-state relative L2 error over 64 orbits: max {rel.max():.2e}, "
          f"median {np.median(rel):.2e}")
    if gemm == "bf16":
        assert rel.max() <= ENVELOPE_BF16["max"] and np.median(rel) <= ENVELOPE_BF16["median"]
    else:
        assert rel.max() <= BOUND[gemm]


@pytest.mark.parametrize("n", [64, 128])
@pytest.mark.parametrize("gemm", ["bf16", "bf16x3", "fp32"])
def test_smaller_networks_ragged_orbit_tail(gpu, n, gemm):
    """45 orbits: one full 32-orbit block and a partial one."""
    w = workloads.rnn_dense(orbits=45, n=n)
    w = dict(w, nsteps=600, stride=100)
    log(f"rnn n={n} 45 orbits, gemm={gemm}")
    got = _run(w, gemm)
    ref = run_oracle(w, precision=32)
    rel = np.linalg.norm(got - ref, axis=2) / np.linalg.norm(ref, axis=2)
    assert rel.max() <= BOUND[gemm], rel.max()


def test_repeatable_and_shardable(gpu):
    w = workloads.rnn_dense(orbits=70, n=128)
    w = dict(w, nsteps=300, stride=100)
    log("rnn replay and shards")
    a = _run(w, "bf16x3")
    b = _run(w, "bf16x3")
    np.testing.assert_array_equal(a, b)
    lo = _run(dict(w, X0=w["X0"][:40]), "bf16x3")
    hi = _run(dict(w, X0=w["X0"][40:]), "bf16x3", orbit_offset=40)
    np.testing.assert_array_equal(np.concatenate([lo, hi]), a)

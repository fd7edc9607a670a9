"""Binary64 ensemble statistics over orbits (mean and sample standard
deviation per saved column) against numpy on the same arrays."""
import numpy as np
import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu


def _stats(x, precision):
    import torch
    import paper_1908_03869_amd as sode
    it = sode.Integrator("kuramoto", 4, 4, 9, precision=precision)
    t = torch.tensor(x, dtype=torch.float32 if precision == 32 else torch.float64, device="cuda")
    m, s = it.ensemble_stats(t)
    it.sync()
    out = m.cpu().numpy(), s.cpu().numpy()
    it.close()
    return out


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("orbits,shape", [(1000, (201, 1)), (37, (5, 64)), (1, (3, 7)),
                                          (65536, (2, 300))])
def test_matches_numpy(gpu, precision, orbits, shape):
    rng = np.random.default_rng(orbits)
    x = 3.0 + rng.standard_normal((orbits,) + shape) * rng.uniform(0.1, 2.0, shape)
    if precision == 32:
        x = x.astype(np.float32).astype(np.float64)
    log(f"stats {precision} {orbits} {shape}")
    m, s = _stats(x, precision)
    np.testing.assert_allclose(m, x.mean(axis=0), rtol=1e-13, atol=1e-13)
    want = x.std(axis=0, ddof=1) if orbits > 1 else np.zeros(shape)
    np.testing.assert_allclose(s, want, rtol=1e-11, atol=1e-13)


def test_reproducible(gpu):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4096, 201))
    a = _stats(x, 64)
    b = _stats(x, 64)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_accuracy_study_statistics(gpu):
    """The Sec. 2.3.1 statistics end to end: r(t) of 16 realisations of the
    N = 100 system (K = 0.02, dt = 0.2, 400 s) from the padded 16-lane
    kernel, reduced on the GPU, against numpy's mean and standard deviation
    of the FP64 oracle's r(t) on the same realisations."""
    import torch
    import paper_1908_03869_amd as sode
    import workloads
    from gpu_util import run_oracle
    w = dict(workloads.kuramoto_e4(0.02, realisations=16, level=5), observable="kuramoto_r")
    log("accuracy-study statistics K=0.02 level 5")
    it = sode.Integrator("kuramoto", 100, 100, 201, precision=32, kernel="coupled",
                         observable="kuramoto_r")
    X0 = torch.tensor(w["X0"], dtype=torch.float32, device="cuda")
    p = torch.tensor(w["p"], dtype=torch.float32, device="cuda")
    r = it.integrate(X0, p, 0.0, w["dt"], w["nsteps"], w["stride"], w["seed"])
    mean, std = it.ensemble_stats(r)
    it.sync()
    mean, std = mean.cpu().numpy()[:, 0], std.cpu().numpy()[:, 0]
    it.close()
    ref = run_oracle(w, precision=32)[:, :, 0]
    np.testing.assert_allclose(mean, ref.mean(axis=0), rtol=0, atol=1e-4)
    np.testing.assert_allclose(std, ref.std(axis=0, ddof=1), rtol=0, atol=1e-4)

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

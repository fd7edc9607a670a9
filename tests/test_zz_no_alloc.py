"""sode_ensemble_stats_noalloc, the entry point that never allocates device
memory, against sode_ensemble_stats on the same arrays: both run the same two
fixed-order kernels over the same orbit chunks, so the results must agree
bit for bit.  Two calls in a row (the second on fewer orbits and columns,
so stale partials of the first call would show), in binary32 and binary64,
and the column limit refused with SODE_ETOOBIG."""
import numpy as np
import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu


def _both(it, t):
    import torch
    from paper_1908_03869_amd import abi
    orbits = t.shape[0]
    cols = t[0].numel()
    res = []
    for fn in (abi.sode_ensemble_stats, abi.sode_ensemble_stats_noalloc):
        mean = torch.full((cols,), float("nan"), dtype=torch.float64, device=t.device)
        std = torch.full((cols,), float("nan"), dtype=torch.float64, device=t.device)
        st = fn(it.handle, t.data_ptr(), orbits, cols, mean.data_ptr(), std.data_ptr(),
                torch.cuda.current_stream().cuda_stream)
        assert st == abi.SODE_OK, (fn.__name__, abi.sode_strerror(st))
        it.sync()
        res.append((mean.cpu().numpy(), std.cpu().numpy()))
    return res


@pytest.mark.parametrize("precision", [32, 64])
def test_noalloc_matches_allocating_entry_point(gpu, precision):
    import torch
    import paper_1908_03869_amd as sode
    dtype = torch.float32 if precision == 32 else torch.float64
    it = sode.Integrator("kuramoto", 4, 4, 9, precision=precision)
    rng = np.random.default_rng(precision)
    for orbits, cols in ((5000, 2048), (77, 301)):
        x = 0.5 + rng.standard_normal((orbits, cols)) * rng.uniform(0.1, 2.0, cols)
        log(f"stats noalloc vs allocating, fp{precision}, {orbits} x {cols}")
        t = torch.tensor(x, dtype=dtype, device="cuda")
        (m0, s0), (m1, s1) = _both(it, t)
        np.testing.assert_array_equal(m1, m0)
        np.testing.assert_array_equal(s1, s0)
        xr = x.astype(np.float32).astype(np.float64) if precision == 32 else x
        np.testing.assert_allclose(m1, xr.mean(axis=0), rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(s1, xr.std(axis=0, ddof=1), rtol=1e-11, atol=1e-13)
    it.close()


def test_noalloc_refuses_too_many_columns(gpu):
    import torch
    import paper_1908_03869_amd as sode
    from paper_1908_03869_amd import abi
    it = sode.Integrator("kuramoto", 4, 4, 9, precision=64)
    cols = abi.SODE_STATS_NOALLOC_MAX_COLS + 1
    t = torch.zeros((3, cols), dtype=torch.float64, device="cuda")
    mean = torch.empty(cols, dtype=torch.float64, device="cuda")
    st = abi.sode_ensemble_stats_noalloc(it.handle, t.data_ptr(), 3, cols, mean.data_ptr(), None,
                                         None)
    assert st == abi.SODE_ETOOBIG
    it.close()

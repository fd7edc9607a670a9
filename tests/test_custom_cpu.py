"""Models given as source text: argument checks and run-time compilation on
the host (hipRTC needs no GPU), through the C ABI."""
import ctypes

import pytest

import paper_1908_03869_amd as sode
from paper_1908_03869_amd import abi

DRIFT = "for (int i = 0; i < 2; ++i) f[i] = -p[0] * y[i] + sin(t);"
DIFFUSION = "gx[0] = p[1] * xi[0]; gx[1] = p[1] * xi[1];"
FAKE = ctypes.c_void_p(16)


def test_create_custom_rejects_bad_arguments():
    assert abi.sode_create_custom(DRIFT, DIFFUSION, 0, 2, 2)[0] == abi.SODE_EINVAL
    assert abi.sode_create_custom(DRIFT, DIFFUSION, 129, 2, 2)[0] == abi.SODE_EINVAL
    assert abi.sode_create_custom(DRIFT, DIFFUSION, 2, -1, 2)[0] == abi.SODE_EINVAL
    assert abi.sode_create_custom(DRIFT, DIFFUSION, 2, 2, -1)[0] == abi.SODE_EINVAL
    assert abi.sode_create_custom(DRIFT, None, 2, 2, 2)[0] == abi.SODE_EINVAL  # m > 0 needs g
    st, h = abi.sode_create_custom(DRIFT, None, 2, 0, 2)  # an ODE needs none
    assert st == abi.SODE_OK
    abi.sode_destroy(h)
    L = abi.load()
    assert L.sode_create_custom(None, None, 1, 0, 0, ctypes.byref(ctypes.c_void_p())) == abi.SODE_EINVAL


def test_build_compiles_and_reports_errors():
    it = sode.Integrator.custom(DRIFT, DIFFUSION, 2, 2, 2, precision=64)
    it.build()
    it.set_option("precision", 32)
    it.build()
    it.close()
    bad = sode.Integrator.custom("f[0] = y[0] +;\nf[1] = 0;", None, 2, 0, 0)
    with pytest.raises(sode.SodeError) as e:
        bad.build()
    assert e.value.status == abi.SODE_EBUILD
    log = bad.build_log()
    assert "drift:1" in log and "error" in log
    bad.close()


def test_option_support():
    st, h = abi.sode_create_custom(DRIFT, DIFFUSION, 2, 2, 2)
    call = lambda: abi.sode_integrate(h, FAKE, FAKE, 1, 0.0, 0.01, 10, 10, 1, FAKE, None)
    assert abi.sode_set_option(h, "observable", 1) == abi.SODE_EINVAL  # r is Kuramoto only
    abi.sode_set_option(h, "method", 2)  # Milstein needs dg/dx, unknown for source text
    assert call() == abi.SODE_EUNSUPPORTED
    abi.sode_set_option(h, "method", 0)
    abi.sode_set_option(h, "kernel", 2)
    assert call() == abi.SODE_EUNSUPPORTED
    abi.sode_set_option(h, "kernel", 0)
    assert abi.sode_integrate(h, FAKE, FAKE, 0, 0.0, 0.01, 10, 10, 1, FAKE, None) == abi.SODE_OK
    abi.sode_destroy(h)
    st, h = abi.sode_create_custom("for (int i = 0; i < 17; ++i) f[i] = -y[i];", None, 17, 0, 0)
    abi.sode_set_option(h, "method", 4)  # implicit steppers: n <= 16
    assert abi.sode_integrate(h, FAKE, FAKE, 1, 0.0, 0.01, 10, 10, 1, FAKE, None) == abi.SODE_EUNSUPPORTED
    abi.sode_destroy(h)

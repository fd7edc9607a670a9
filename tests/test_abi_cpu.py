"""The C ABI without a GPU: the library loads, exports every symbol that
include/sode.h declares, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re

import pytest

import paper_1908_03869_amd as sode
from paper_1908_03869_amd import abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sode.h")

# A non-null placeholder address; validation rejects every call below before
# the pointer could be used.
FAKE = 0x1000


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sode_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert sorted(abi.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    L = abi.load()
    for name in _declared():
        assert hasattr(L, name), name
    assert abi.sode_version() >= 100


def test_strerror_covers_every_status():
    for st in (0, -1, -2, -3, -4, -5, -6, -7):
        assert abi.sode_strerror(st) and abi.sode_strerror(st) != "unknown status"
    assert abi.sode_strerror(-99) == "unknown status"


@pytest.mark.parametrize("model,n,m,d,ok", [
    ("kuramoto", 4, 4, 9, True), ("kuramoto", 4, 4, 8, False), ("kuramoto", 4, 3, 9, False),
    ("ou", 3, 3, 3, True), ("ou", 3, 3, 2, False), ("gbm", 1, 1, 2, True),
    ("fhn", 8, 4, 5, True), ("fhn", 7, 3, 5, False), ("rnn", 3, 3, 13, True),
    ("rnn", 3, 3, 12, False), ("nonesuch", 4, 4, 9, False), ("kuramoto", 0, 0, 1, False),
])
def test_create_checks_model_dimensions(model, n, m, d, ok):
    st, h = abi.sode_create(model, n, m, d)
    assert (st == abi.SODE_OK) == ok
    assert (h is not None) == ok
    if h:
        assert abi.sode_destroy(h) == 0


def test_create_rejects_null_output():
    L = abi.load()
    assert L.sode_create(b"kuramoto", 4, 4, 9, None) == abi.SODE_EINVAL
    assert L.sode_create(None, 4, 4, 9, ctypes.byref(ctypes.c_void_p())) == abi.SODE_EINVAL


def test_options_round_trip_and_reject_unknown():
    st, h = abi.sode_create("kuramoto", 64, 64, 129)
    assert st == 0
    try:
        for key, val in (("precision", 64), ("method", 1), ("observable", 1), ("kernel", 2),
                         ("shared_params", 1), ("drift", 1)):
            assert abi.sode_set_option(h, key, val) == 0
            assert abi.sode_get_option(h, key) == (0, val)
        assert abi.sode_set_option(h, "precision", 16) == abi.SODE_EINVAL
        assert abi.sode_set_option(h, "method", 5) == abi.SODE_EINVAL
        assert abi.sode_set_option(h, "kernel", 7) == abi.SODE_EINVAL
        assert abi.sode_set_option(h, "drift", 2) == abi.SODE_EINVAL
        assert abi.sode_set_option(h, "bogus", 1) == abi.SODE_EINVAL
        assert abi.sode_get_option(h, "bogus")[0] == abi.SODE_EINVAL
        assert abi.sode_get_option(h, "precision") == (0, 64)
    finally:
        abi.sode_destroy(h)
    st, h = abi.sode_create("ou", 2, 2, 3)
    assert abi.sode_set_option(h, "observable", 1) == abi.SODE_EINVAL  # r is Kuramoto only
    abi.sode_destroy(h)


def _call(h, **kw):
    a = dict(X0=FAKE, p=FAKE, orbits=16, t0=0.0, dt=1e-3, nsteps=100, stride=10, seed=1,
             orbit_offset=0, step_offset=0, orbit_ids=None, orbit_seeds=None, out=FAKE,
             stream=None)
    a.update(kw)
    return abi.sode_integrate_ex(h, a["X0"], a["p"], a["orbits"], a["t0"], a["dt"], a["nsteps"],
                                 a["stride"], a["seed"], a["orbit_offset"], a["step_offset"],
                                 a["orbit_ids"], a["orbit_seeds"], a["out"], a["stream"])


@pytest.mark.parametrize("bad", [
    dict(orbits=-1), dict(nsteps=-5), dict(stride=0), dict(nsteps=105, stride=10),
    dict(dt=0.0), dict(dt=-1e-3), dict(dt=float("nan")), dict(t0=float("inf")),
    dict(X0=None), dict(p=None), dict(out=None), dict(step_offset=2**32 - 50),
    dict(orbits=2**27 + 1),
])
def test_integrate_rejects_bad_arguments(bad):
    st, h = abi.sode_create("kuramoto", 4, 4, 9)
    try:
        assert _call(h, **bad) == abi.SODE_EINVAL
    finally:
        abi.sode_destroy(h)


def test_integrate_null_handle_and_zero_orbits():
    assert _call(None) == abi.SODE_EINVAL
    st, h = abi.sode_create("kuramoto", 4, 4, 9)
    # Nothing to do: succeeds without touching the device or the pointers.
    assert _call(h, orbits=0, X0=None, p=None, out=None) == abi.SODE_OK
    assert abi.sode_sync(h) == abi.SODE_OK
    abi.sode_destroy(h)


def test_unsupported_kernel_requests():
    st, h = abi.sode_create("kuramoto", 130, 130, 261)
    abi.sode_set_option(h, "kernel", 2)  # coupled needs n <= 128
    assert _call(h) == abi.SODE_EUNSUPPORTED
    abi.sode_destroy(h)
    st, h = abi.sode_create("kuramoto", 64, 64, 129)
    abi.sode_set_option(h, "kernel", 2)
    abi.sode_set_option(h, "method", 1)  # coupled is Euler-Maruyama only
    assert _call(h) == abi.SODE_EUNSUPPORTED
    abi.sode_destroy(h)
    st, h = abi.sode_create("ou", 200, 200, 3)  # beyond the plain kernel's 128 states
    assert _call(h) == abi.SODE_EUNSUPPORTED
    abi.sode_destroy(h)
    st, h = abi.sode_create("ou", 17, 17, 3)
    abi.sode_set_option(h, "method", 3)  # implicit steppers hold n x n per lane: n <= 16
    assert _call(h) == abi.SODE_EUNSUPPORTED
    abi.sode_set_option(h, "method", 4)
    assert _call(h) == abi.SODE_EUNSUPPORTED
    abi.sode_destroy(h)
    st, h = abi.sode_create("rnn", 256, 256, 256 * 256 + 257)
    assert _call(h) == abi.SODE_EUNSUPPORTED  # n = 256 needs the matrix kernel: shared W
    abi.sode_set_option(h, "shared_params", 1)
    abi.sode_set_option(h, "kernel", 3)
    abi.sode_set_option(h, "observable", 0)
    abi.sode_set_option(h, "precision", 64)
    assert _call(h) == abi.SODE_EUNSUPPORTED  # matrix kernel is binary32
    assert abi.sode_set_option(h, "gemm", 3) == abi.SODE_EINVAL
    for g in (0, 1, 2):
        assert abi.sode_set_option(h, "gemm", g) == 0 and abi.sode_get_option(h, "gemm") == (0, g)
    abi.sode_destroy(h)


def test_python_layer_raises_on_error():
    with pytest.raises(sode.SodeError):
        sode.Integrator("kuramoto", 4, 4, 10)
    it = sode.Integrator("kuramoto", 4, 4, 9, precision=64, method="rk4")
    assert it.options["precision"] == 64 and it.options["method"] == 1
    with pytest.raises(sode.SodeError):
        it.set_option("precision", 8)
    it.close()


def test_destroy_accepts_null():
    assert abi.sode_destroy(None) == 0


def _ckpt(h, **kw):
    a = dict(X0=FAKE, p=FAKE, orbits=16, t0=0.0, dt=1e-3, nsteps=1000, every=100, lo=500,
             hi=1000, seed=1, ckpt=FAKE, R=FAKE)
    a.update(kw)
    return abi.sode_forward_ckpt(h, a["X0"], a["p"], a["orbits"], a["t0"], a["dt"], a["nsteps"],
                                 a["every"], a["lo"], a["hi"], a["seed"], 0, 0, a["ckpt"], a["R"],
                                 None)


def _adj(h, **kw):
    a = dict(p=FAKE, orbits=16, t0=0.0, dt=1e-3, nsteps=1000, every=100, lo=500, hi=1000,
             seed=1, ckpt=FAKE, dLdR=None, grad=FAKE, rows=None)
    a.update(kw)
    return abi.sode_adjoint(h, a["p"], a["orbits"], a["t0"], a["dt"], a["nsteps"], a["every"],
                            a["lo"], a["hi"], a["seed"], 0, 0, a["ckpt"], a["dLdR"], a["grad"],
                            a["rows"], None)


@pytest.mark.parametrize("bad", [
    dict(nsteps=0), dict(every=0), dict(nsteps=1050), dict(lo=-1), dict(hi=1001),
    dict(lo=600, hi=500), dict(dt=0.0), dict(orbits=-2), dict(t0=float("nan")),
])
def test_adjoint_entry_points_reject_bad_arguments(bad):
    st, h = abi.sode_create("kuramoto", 32, 32, 65)
    try:
        assert _ckpt(h, **bad) == abi.SODE_EINVAL
        assert _adj(h, **bad) == abi.SODE_EINVAL
    finally:
        abi.sode_destroy(h)


def test_adjoint_entry_points_pointers_and_support():
    st, h = abi.sode_create("kuramoto", 32, 32, 65)
    assert _ckpt(h, X0=None) == abi.SODE_EINVAL
    assert _ckpt(h, R=None) == abi.SODE_EINVAL
    assert _adj(h, grad=None, rows=None) == abi.SODE_EINVAL
    assert _ckpt(h, orbits=0, X0=None, p=None, ckpt=None, R=None) == abi.SODE_OK
    abi.sode_set_option(h, "precision", 64)
    assert _ckpt(h) == abi.SODE_EUNSUPPORTED
    assert _adj(h) == abi.SODE_EUNSUPPORTED
    abi.sode_destroy(h)
    st, h = abi.sode_create("kuramoto", 12, 12, 25)
    assert _ckpt(h) == abi.SODE_EUNSUPPORTED
    abi.sode_destroy(h)
    st, h = abi.sode_create("ou", 4, 4, 3)
    assert _adj(h) == abi.SODE_EUNSUPPORTED
    abi.sode_destroy(h)


@pytest.mark.parametrize("model,n,m,d", [("kuramoto", 4, 4, 9), ("ou", 3, 3, 3), ("fhn", 6, 3, 5),
                                         ("gbm", 2, 2, 2), ("rnn", 3, 3, 13)])
@pytest.mark.parametrize("method", [1, 3, 4])
def test_ode_methods_need_ode_limit_on_models_with_noise(model, n, m, d, method):
    """RK4 and the implicit steppers integrate the ODE limit g = 0: a model
    with a diffusion is refused unless "ode_limit" is set.  Zero orbits reach
    the kernel choice without touching the device."""
    st, h = abi.sode_create(model, n, m, d)
    try:
        assert abi.sode_get_option(h, "ode_limit") == (0, 0)
        abi.sode_set_option(h, "method", method)
        assert _call(h, orbits=0) == abi.SODE_EUNSUPPORTED
        assert _call(h) == abi.SODE_EUNSUPPORTED
        assert abi.sode_set_option(h, "ode_limit", 1) == 0
        assert abi.sode_get_option(h, "ode_limit") == (0, 1)
        assert _call(h, orbits=0) == abi.SODE_OK
        abi.sode_set_option(h, "method", 0)  # Euler-Maruyama never needs it
        abi.sode_set_option(h, "ode_limit", 0)
        assert _call(h, orbits=0) == abi.SODE_OK
        assert abi.sode_set_option(h, "ode_limit", 2) == abi.SODE_EINVAL
    finally:
        abi.sode_destroy(h)


def test_ode_methods_on_source_text_models():
    """A source-text ODE (m = 0) takes RK4 and the implicit steppers as is;
    with Wiener processes it needs "ode_limit" like the built-in models."""
    for m, diffusion in ((0, None), (1, "gx[0] = p[0] * xi[0];")):
        st, h = abi.sode_create_custom("f[0] = -y[0];", diffusion, 1, m, 1)
        assert st == 0
        try:
            for method in (1, 3, 4):
                abi.sode_set_option(h, "method", method)
                assert _call(h, orbits=0) == (abi.SODE_OK if m == 0 else abi.SODE_EUNSUPPORTED)
                abi.sode_set_option(h, "ode_limit", 1)
                assert _call(h, orbits=0) == abi.SODE_OK
                abi.sode_set_option(h, "ode_limit", 0)
        finally:
            abi.sode_destroy(h)


def test_wrap_option_fixes_the_phase_convention():
    """"wrap" 1 (default): every kernel returns reduced phases.  "wrap" 0
    (continuous phases) is served by the one-orbit-per-lane kernel only:
    auto selection takes it, an explicit 16-lane request and the
    checkpointed forward pass / adjoint (whose checkpoints are reduced) are
    refused."""
    st, h = abi.sode_create("kuramoto", 64, 64, 129)
    try:
        assert abi.sode_get_option(h, "wrap") == (0, 1)
        abi.sode_set_option(h, "kernel", 2)
        assert _call(h, orbits=0) == abi.SODE_OK
        assert abi.sode_set_option(h, "wrap", 0) == 0
        assert abi.sode_get_option(h, "wrap") == (0, 0)
        assert _call(h, orbits=0) == abi.SODE_EUNSUPPORTED
        abi.sode_set_option(h, "kernel", 0)
        assert _call(h, orbits=0) == abi.SODE_OK
        abi.sode_set_option(h, "precision", 64)
        assert _call(h, orbits=0) == abi.SODE_OK
        assert abi.sode_set_option(h, "wrap", 3) == abi.SODE_EINVAL
    finally:
        abi.sode_destroy(h)
    st, h = abi.sode_create("kuramoto", 32, 32, 65)
    try:
        assert _ckpt(h, orbits=0, X0=None, p=None, ckpt=None, R=None) == abi.SODE_OK
        abi.sode_set_option(h, "wrap", 0)
        assert _ckpt(h) == abi.SODE_EUNSUPPORTED
        assert _adj(h) == abi.SODE_EUNSUPPORTED
    finally:
        abi.sode_destroy(h)


def test_noise_waves_option():
    """"noise_waves": -1 (by ensemble size, the default), 0, 1 or 2 waves
    drawing the normals of the binary64 four-lane form; anything else is
    refused and leaves the handle unchanged."""
    st, h = abi.sode_create("kuramoto", 4, 4, 9)
    try:
        assert abi.sode_get_option(h, "noise_waves") == (0, -1)
        for v in (0, 1, 2, -1):
            assert abi.sode_set_option(h, "noise_waves", v) == 0
            assert abi.sode_get_option(h, "noise_waves") == (0, v)
        abi.sode_set_option(h, "noise_waves", 2)
        for v in (-2, 3, 64):
            assert abi.sode_set_option(h, "noise_waves", v) == abi.SODE_EINVAL
        assert abi.sode_get_option(h, "noise_waves") == (0, 2)
        abi.sode_set_option(h, "precision", 64)
        assert _call(h, orbits=0) == abi.SODE_OK
    finally:
        abi.sode_destroy(h)


def _ragged(h, descs, x0_len=1000, p_len=1000, out_len=10**7, dt=1e-3):
    arr = (abi.SodeInstance * len(descs))(*descs) if descs else None
    return abi.sode_integrate_ragged(h, arr, len(descs), FAKE, x0_len, FAKE, p_len, FAKE, out_len,
                                     0.0, dt, None)


def _desc(**kw):
    d = dict(n=8, nsteps=100, stride=10, x0_offset=0, p_offset=0, out_offset=0, seed=1,
             orbit_id=0)
    d.update(kw)
    e = abi.SodeInstance()
    for k, v in d.items():
        setattr(e, k, v)
    return e


@pytest.mark.parametrize("bad", [
    dict(n=7), dict(n=0), dict(n=258), dict(nsteps=-1), dict(stride=0), dict(nsteps=105),
    dict(x0_offset=995), dict(p_offset=996), dict(out_offset=10**7 - 50), dict(x0_offset=-1),
    dict(reserved0=1), dict(reserved1=2), dict(nsteps=2**32, stride=1),
])
def test_ragged_rejects_bad_descriptors(bad):
    st, h = abi.sode_create("fhn", 256, 128, 5)
    try:
        assert _ragged(h, [_desc(), _desc(**bad)]) == abi.SODE_EINVAL
    finally:
        abi.sode_destroy(h)


def test_ragged_support_and_trivial_calls():
    st, h = abi.sode_create("fhn", 16, 8, 5)
    assert _ragged(h, [_desc(n=18)]) == abi.SODE_EINVAL      # above the handle's n
    assert _ragged(h, []) == abi.SODE_OK                      # nothing to do
    assert _ragged(h, [_desc()], dt=0.0) == abi.SODE_EINVAL
    abi.sode_set_option(h, "method", 1)                       # RK4: no ragged kernel
    assert _ragged(h, [_desc()]) == abi.SODE_EUNSUPPORTED
    abi.sode_set_option(h, "method", 0)
    abi.sode_set_option(h, "precision", 64)
    assert _ragged(h, [_desc()]) == abi.SODE_EUNSUPPORTED
    abi.sode_destroy(h)
    st, h = abi.sode_create("kuramoto", 4, 4, 9)
    assert _ragged(h, [_desc()]) == abi.SODE_EUNSUPPORTED
    for key, val in (("waves_per_cu", 8), ("units_per_lane", 4), ("graph", 0), ("persistent", 0)):
        assert abi.sode_set_option(h, key, val) == 0
        assert abi.sode_get_option(h, key) == (0, val)
    assert abi.sode_set_option(h, "units_per_lane", 3) == abi.SODE_EINVAL
    assert abi.sode_set_option(h, "waves_per_cu", 64) == abi.SODE_EINVAL
    abi.sode_destroy(h)


def test_ensemble_stats_argument_checks():
    st, h = abi.sode_create("kuramoto", 4, 4, 9)
    assert abi.sode_ensemble_stats(h, FAKE, -1, 10, FAKE, None, None) == abi.SODE_EINVAL
    assert abi.sode_ensemble_stats(h, FAKE, 10, -1, FAKE, None, None) == abi.SODE_EINVAL
    assert abi.sode_ensemble_stats(h, None, 10, 10, FAKE, None, None) == abi.SODE_EINVAL
    assert abi.sode_ensemble_stats(h, FAKE, 10, 10, None, None, None) == abi.SODE_EINVAL
    assert abi.sode_ensemble_stats(h, FAKE, 10, 0, None, None, None) == abi.SODE_OK
    assert abi.sode_ensemble_stats(None, FAKE, 10, 10, FAKE, None, None) == abi.SODE_EINVAL
    abi.sode_destroy(h)


def test_ensemble_stats_noalloc_argument_checks():
    """Same checks as sode_ensemble_stats, plus the fixed capacity: more than
    SODE_STATS_NOALLOC_MAX_COLS columns is refused before any HIP call."""
    st, h = abi.sode_create("kuramoto", 4, 4, 9)
    f = abi.sode_ensemble_stats_noalloc
    assert f(h, FAKE, -1, 10, FAKE, None, None) == abi.SODE_EINVAL
    assert f(h, FAKE, 10, -1, FAKE, None, None) == abi.SODE_EINVAL
    assert f(h, None, 10, 10, FAKE, None, None) == abi.SODE_EINVAL
    assert f(h, FAKE, 10, 10, None, None, None) == abi.SODE_EINVAL
    assert f(h, FAKE, 10, 0, None, None, None) == abi.SODE_OK
    assert f(None, FAKE, 10, 10, FAKE, None, None) == abi.SODE_EINVAL
    big = abi.SODE_STATS_NOALLOC_MAX_COLS + 1
    assert f(h, FAKE, 10, big, FAKE, None, None) == abi.SODE_ETOOBIG
    assert f(h, FAKE, 1 << 20, big, FAKE, FAKE, None) == abi.SODE_ETOOBIG
    assert "fixed capacity" in abi.sode_strerror(abi.SODE_ETOOBIG)
    abi.sode_destroy(h)


def test_noalloc_column_limit_matches_header():
    text = open(HEADER).read()
    m = re.search(r"#define SODE_STATS_NOALLOC_MAX_COLS (\d+)", text)
    assert m and int(m.group(1)) == abi.SODE_STATS_NOALLOC_MAX_COLS

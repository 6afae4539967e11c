"""The C-ABI library on a machine without a GPU: it loads, exports every declared symbol, and
rejects invalid arguments before any device call."""
import ctypes as C
import os

import numpy as np
import pytest

from paper_2105_07372_amd import binding as B


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2105_07372_amd import build
        build.build()
    return B.load()


def test_exports_every_declared_symbol(lib):
    names = B.header_symbols()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert lib.em_version().decode().startswith("synchem")


def _params(**kw):
    p = B.EmParams()
    p.n_obs, p.K, p.Q, p.L, p.window_lo, p.window_count = 100, 4, 4, 36, -3, 7
    p.sigma2, p.gamma, p.update_rho, p.precision, p.flags = 1.0, 0.0, 1, 1, 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


FAKE = C.c_void_p(0x1000)     # never dereferenced: validation fails first


@pytest.mark.parametrize("kw,status,text", [
    (dict(n_obs=0), B.EM_EINVAL, "n_obs"),
    (dict(K=0), B.EM_EINVAL, "K and Q"),
    (dict(L=0, window_count=1), B.EM_EINVAL, "L must"),
    (dict(window_count=0), B.EM_EINVAL, "window_count"),
    (dict(window_count=37), B.EM_EINVAL, "window_count"),
    (dict(sigma2=0.0), B.EM_EINVAL, "sigma2"),
    (dict(sigma2=float("nan")), B.EM_EINVAL, "sigma2"),
    (dict(gamma=-1.0), B.EM_EINVAL, "gamma"),
    (dict(update_rho=2), B.EM_EINVAL, "update_rho"),
    (dict(precision=9), B.EM_EINVAL, "precision"),
    (dict(flags=1 << 7), B.EM_EINVAL, "flag"),
    (dict(K=64, Q=64), B.EM_EUNSUPPORTED, "2048"),
    (dict(K=600, Q=1), B.EM_EUNSUPPORTED, "K above"),
    (dict(L=5000, window_count=1500), B.EM_EUNSUPPORTED, "window above"),
])
def test_init_rejects_invalid_params_without_device_work(lib, kw, status, text):
    ctx = C.c_void_p()
    p = _params(**kw)
    st = lib.em_init(C.byref(ctx), C.byref(p), FAKE, None, None)
    assert st == status
    assert ctx.value is None
    assert text in lib.em_last_error(None).decode()


def test_init_rejects_bad_prior_and_pointers(lib):
    ctx = C.c_void_p()
    p = _params()
    bad = np.array([0.1, -0.2, 0.3, 0.1, 0.1, 0.1, 0.1])
    assert lib.em_init(C.byref(ctx), C.byref(p), FAKE, B._dptr(bad), None) == B.EM_EINVAL
    assert "prior" in lib.em_last_error(None).decode()
    zero = np.zeros(7)
    assert lib.em_init(C.byref(ctx), C.byref(p), FAKE, B._dptr(zero), None) == B.EM_EINVAL
    assert lib.em_init(C.byref(ctx), C.byref(p), None, None, None) == B.EM_EINVAL
    assert lib.em_init(None, C.byref(p), FAKE, None, None) == B.EM_EINVAL
    gai = np.full(16, -1.0)
    p.gamma_a_inv = B._dptr(gai)
    assert lib.em_init(C.byref(ctx), C.byref(p), FAKE, None, None) == B.EM_EINVAL
    a0 = np.full(32, np.inf)
    p = _params()
    p.a0 = B._dptr(a0)
    assert lib.em_init(C.byref(ctx), C.byref(p), FAKE, None, None) == B.EM_EINVAL


def test_init_validates_angle_lists(lib):
    """The refined-resolution window: finite angles, window_lo 0; W is not bounded by L."""
    ctx = C.c_void_p()
    p = _params()                              # window_lo = -3
    ang = np.linspace(-0.2, 0.2, 7)
    p.angles = B._dptr(ang)
    assert lib.em_init(C.byref(ctx), C.byref(p), FAKE, None, None) == B.EM_EINVAL
    assert "window_lo" in lib.em_last_error(None).decode()
    p.window_lo = 0
    bad = ang.copy()
    bad[3] = np.nan
    p.angles = B._dptr(bad)
    assert lib.em_init(C.byref(ctx), C.byref(p), FAKE, None, None) == B.EM_EINVAL
    assert "angles" in lib.em_last_error(None).decode()
    many = np.linspace(-0.5, 0.5, 48)           # W = 48 > L = 36 is allowed with angles
    p.window_count = 48
    p.angles = B._dptr(many)
    p.sigma2 = 0.0                               # ... so the check after the window's fails
    assert lib.em_init(C.byref(ctx), C.byref(p), FAKE, None, None) == B.EM_EINVAL
    assert "sigma2" in lib.em_last_error(None).decode()


def test_sync_calls_validate_before_device_work(lib):
    """Synchronize and Match entry points reject bad sizes and pointers without touching the
    device (FAKE is never dereferenced)."""
    st = B.STATUS_NAMES
    ok = FAKE
    assert lib.em_relative_rotations(None, 8, 4, 4, 36, ok, None, None, None) == B.EM_EINVAL
    assert lib.em_relative_rotations(ok, 1, 4, 4, 36, ok, None, None, None) == B.EM_EINVAL
    assert lib.em_relative_rotations(ok, 8, 4, 4, 0, ok, None, None, None) == B.EM_EINVAL
    assert lib.em_relative_rotations(ok, 9000, 4, 4, 36, ok, None, None, None) == B.EM_EUNSUPPORTED
    assert lib.em_relative_rotations(ok, 8, 64, 64, 36, ok, None, None, None) == B.EM_EUNSUPPORTED
    assert lib.em_ppm(None, 8, 36, 5, ok, None) == B.EM_EINVAL
    assert lib.em_ppm(ok, 8, 36, -1, ok, None) == B.EM_EINVAL
    assert lib.em_nearest(ok, 100, 4, 4, 1, ok, None, None) == B.EM_EINVAL
    assert lib.em_nearest(ok, 100, 4, 4, 101, ok, None, None) == B.EM_EINVAL
    assert lib.em_nearest(ok, 100, 3, 3, 10, ok, None, None) == B.EM_EUNSUPPORTED
    assert "multiple of 8" in lib.em_last_error(None).decode()
    assert lib.em_sync_match(ok, 100, 4, 4, 36, 10, 5, None, None, None) == B.EM_EINVAL
    assert lib.em_sync_match(ok, 100, 4, 4, 5000, 10, 5, ok, None, None) == B.EM_EINVAL
    assert lib.em_align(ok, 0, 4, 4, ok, ok, None) == B.EM_EINVAL
    assert lib.em_align(ok, 10, 4, 4, None, ok, None) == B.EM_EINVAL
    for fn in (lib.em_aligned_mean, lib.em_aligned_mean_noalloc):
        assert fn(ok, 0, 4, 4, ok, ok, None) == B.EM_EINVAL
        assert fn(ok, 10, 4, 4, None, ok, None) == B.EM_EINVAL
        assert fn(ok, 10, 4, 4, ok, None, None) == B.EM_EINVAL
        assert fn(ok, 10, 64, 64, ok, ok, None) == B.EM_EUNSUPPORTED    # D above the scratch
        assert "2048" in lib.em_last_error(None).decode()
    assert st[B.EM_EINVAL]


def test_null_context_calls_are_rejected(lib):
    d = C.c_double(0.0)
    assert lib.em_step(None, 1, 0.0, None, None) == B.EM_EINVAL
    assert lib.em_loglik(None, C.byref(d)) == B.EM_EINVAL
    assert lib.em_posterior(None, 0, 1, None, None, None) == B.EM_EINVAL
    assert lib.em_get_state(None, None, None, None) == B.EM_EINVAL
    assert lib.em_loglik_bwd(None, 1.0, None, None, None) == B.EM_EINVAL
    lib.em_destroy(None)


def test_learn_prior_validates_before_device_work(lib):
    rb = np.zeros(5)
    assert lib.em_learn_prior(FAKE, 10, 0, 0, 5, B._dptr(rb), None, None, None) == B.EM_EINVAL
    assert lib.em_learn_prior(FAKE, 10, 36, 0, 40, B._dptr(rb), None, None, None) == B.EM_EINVAL
    assert lib.em_learn_prior(None, 10, 36, 0, 5, B._dptr(rb), None, None, None) == B.EM_EINVAL
    assert lib.em_learn_prior(FAKE, -1, 36, 0, 5, B._dptr(rb), None, None, None) == B.EM_EINVAL
    assert "n must" in lib.em_last_error(None).decode()


def test_struct_layout_matches_header():
    assert C.sizeof(B.EmParams) == 88
    assert B.EmParams.sigma2.offset == 32 and B.EmParams.flags.offset == 56
    assert B.EmParams.a0.offset == 72 and B.EmParams.angles.offset == 80

"""Argument errors the library detects on the host, before any device work
(no GPU needed): every case below fails validation, so no pointer in it is
ever dereferenced and nothing is launched."""
import ctypes
import os

import pytest

from paper_1208_4830_amd import sblm

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1208_4830_amd", "libsblm.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsblm.so not built")

OK, EINVAL, ESTATE, ERANGE = 0, -1, -4, -5
FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def _lcs(n_lc):
    return sblm.sblm_lcs(n_lc, FAKE.value, FAKE.value, FAKE.value, FAKE.value)


def _expect(rc, code, *words):
    assert rc == code, (rc, code)
    msg = sblm.load().sblm_last_error().decode()
    for w in words:
        assert w in msg, (w, msg)


def test_magnify_and_chi2_arguments():
    lib = sblm.load()
    _expect(lib.sblm_magnify(FAKE, 4, FAKE, 10, 7, FAKE, None, None, None), EINVAL,
            "sblm_magnify", "mode")
    _expect(lib.sblm_magnify(FAKE, 0, FAKE, 10, 0, FAKE, None, None, None), EINVAL, "n = 0")
    _expect(lib.sblm_magnify(FAKE, 4, FAKE, -1, 0, FAKE, None, None, None), EINVAL, "n_t")
    _expect(lib.sblm_magnify(FAKE, (1 << 26) + 1, FAKE, 10, 0, FAKE, None, None, None),
            ERANGE, "beyond")
    _expect(lib.sblm_magnify(None, 4, FAKE, 10, 0, FAKE, None, None, None), EINVAL, "null")
    assert lib.sblm_magnify(None, 4, None, 0, 0, None, None, None, None) == OK  # no epochs
    lc = _lcs(3)
    _expect(lib.sblm_chi2(ctypes.byref(lc), FAKE, 4, 9, FAKE, FAKE, FAKE, None, None), EINVAL,
            "mode")
    _expect(lib.sblm_chi2(None, FAKE, 4, 0, FAKE, FAKE, FAKE, None, None), EINVAL, "null")
    _expect(lib.sblm_chi2(ctypes.byref(lc), FAKE, 0, 0, FAKE, FAKE, FAKE, None, None), EINVAL,
            "pop = 0")
    big = _lcs((1 << 20) + 1)
    _expect(lib.sblm_chi2(ctypes.byref(big), FAKE, 4, 0, FAKE, FAKE, FAKE, None, None), ERANGE,
            "beyond")
    _expect(lib.sblm_chi2(ctypes.byref(lc), None, 4, 0, FAKE, FAKE, FAKE, None, None), EINVAL,
            "null theta")


def _cfg(**kw):
    cfg = sblm.ea_default_config()
    for k, v in kw.items():
        setattr(cfg, k, v)
    return cfg


@pytest.mark.parametrize("field,value,code,word", [
    ("pop", 1, ERANGE, "pop"), ("pop", 1025, ERANGE, "pop"),
    ("n_tourn", 300, EINVAL, "n_tourn"), ("p_mut0", 1.5, EINVAL, "probabilities"),
    ("stag_window", 0, ERANGE, "stag_window"), ("restart_after", 0, EINVAL, "restart_after"),
    ("mode", 3, EINVAL, "mode"), ("n_islands", 0, ERANGE, "n_islands"),
    ("n_islands", 257, ERANGE, "n_islands"), ("mig_every", -1, EINVAL, "mig_every"),
    ("n_migrants", 129, EINVAL, "n_migrants"),
])
def test_ea_config_errors(field, value, code, word):
    lib = sblm.load()
    cfg = _cfg(**{field: value})
    h = ctypes.c_void_p()
    lc = _lcs(2)
    _expect(lib.ea_create(ctypes.byref(cfg), ctypes.byref(lc), 1, ctypes.byref(h)), code, word)
    assert not h.value


def test_ea_domain_and_state_errors():
    lib = sblm.load()
    cfg = _cfg()
    cfg.lo[1], cfg.hi[1] = 2.0, 0.5  # empty domain
    h = ctypes.c_void_p()
    lc = _lcs(2)
    _expect(lib.ea_create(ctypes.byref(cfg), ctypes.byref(lc), 1, ctypes.byref(h)), EINVAL,
            "domain")
    _expect(lib.ea_create(None, ctypes.byref(lc), 1, ctypes.byref(h)), EINVAL, "null")
    for call in (lambda: lib.ea_generation(None, FAKE, FAKE, FAKE, None),
                 lambda: lib.ea_fit(None, 1, None, None),
                 lambda: lib.ea_migrate(None, None, None, None, None),
                 lambda: lib.ea_refine(None, None, None, None, None),
                 lambda: lib.ea_autotune_cached(None, b"/tmp/x", None, None, 0, None),
                 lambda: lib.ea_freeze(None, None, 0, None)):
        assert call() == ESTATE


def test_simplex_arguments():
    lib = sblm.load()
    lo = (ctypes.c_double * 6)(*[0.0] * 6)
    hi = (ctypes.c_double * 6)(*[1.0] * 6)
    lc = _lcs(3)
    cfg = sblm.nm_default_config()
    bad = sblm.nm_default_config()
    bad.tol_x = -1.0
    _expect(lib.nm_refine(ctypes.byref(lc), lo, hi, FAKE, ctypes.byref(bad), FAKE, None, None,
                          None, None, None, None), EINVAL, "tolerance")
    bad = sblm.nm_default_config()
    bad.max_iter = 2000000
    _expect(lib.nm_refine(ctypes.byref(lc), lo, hi, FAKE, ctypes.byref(bad), FAKE, None, None,
                          None, None, None, None), EINVAL, "max_iter")
    _expect(lib.nm_refine(ctypes.byref(lc), lo, hi, FAKE, None, FAKE, None, None, None, None,
                          None, None), EINVAL, "null config")
    _expect(lib.nm_refine_multi(ctypes.byref(lc), 0, lo, hi, FAKE, ctypes.byref(cfg), FAKE,
                                None, None, None, None, None, None), EINVAL, "reps")
    _expect(lib.nm_refine_multi(ctypes.byref(lc), 1 << 23, lo, hi, FAKE, ctypes.byref(cfg),
                                FAKE, None, None, None, None, None, None), ERANGE, "2^24")
    _expect(lib.nm_refine(ctypes.byref(lc), hi, lo, FAKE, ctypes.byref(cfg), FAKE, None, None,
                          None, None, None, None), EINVAL, "hi[")
    _expect(lib.nm_iterated(ctypes.byref(lc), 2, 0, 1, lo, hi, ctypes.byref(cfg), FAKE, None,
                            None, None, None, None, None), EINVAL, "runs = 0")
    long_cfg = sblm.nm_default_config()
    long_cfg.max_iter = 1000000
    _expect(lib.nm_iterated(ctypes.byref(lc), 2, 5000, 1, lo, hi, ctypes.byref(long_cfg), FAKE,
                            None, None, None, None, None, None), ERANGE, "per slot")
    # more than 2^31 - 1 starts per lightcurve (the start counter is 32-bit)
    _expect(lib.nm_iterated(ctypes.byref(lc), 1 << 10, 1 << 21, 1, lo, hi, ctypes.byref(cfg),
                            FAKE, None, None, None, None, None, None), ERANGE, "starts")
    # more slots per lightcurve than the per-round ranking loop is built for
    _expect(lib.nm_iterated(ctypes.byref(lc), 1025, 1, 1, lo, hi, ctypes.byref(cfg),
                            FAKE, None, None, None, None, None, None), ERANGE, "beyond 1024")
    # the no-alloc simplex: beyond its static array, and the usual checks
    big = sblm.sblm_lcs(10380, FAKE, FAKE, FAKE, FAKE)
    _expect(lib.nm_refine_noalloc(ctypes.byref(big), lo, hi, FAKE, ctypes.byref(cfg), FAKE,
                                  None, None, None, None, None, None), ERANGE, "9936")
    _expect(lib.nm_refine_noalloc(ctypes.byref(lc), hi, lo, FAKE, ctypes.byref(cfg), FAKE,
                                  None, None, None, None, None, None), EINVAL, "hi[")
    _expect(lib.nm_refine_noalloc(ctypes.byref(lc), lo, hi, None, ctypes.byref(cfg), FAKE,
                                  None, None, None, None, None, None), EINVAL, "null")


def test_network_arguments():
    lib = sblm.load()
    h = ctypes.c_void_p()
    _expect(lib.mlp_create(100, 0, ctypes.byref(h)), EINVAL, "multiple of 64")
    _expect(lib.mlp_create(1 << 21, 0, ctypes.byref(h)), ERANGE, "2^20")
    _expect(lib.mlp_create(64, 0, None), EINVAL, "null")

"""ctypes binding of the C oracle (sblm_oracle.c, ea_oracle.c).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Functions take and
return numpy float64 / int arrays; the parameter layout is the library's:
six planes (log10 q, d, u0, alpha, tE, t0), plane j = theta[j].
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsblm_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i8p = ctypes.POINTER(ctypes.c_int8)


class EAConfig(ctypes.Structure):
    _fields_ = [("pop", ctypes.c_int32), ("n_tourn", ctypes.c_int32),
                ("p_mut0", ctypes.c_double), ("p_mut_min", ctypes.c_double),
                ("p_mut_max", ctypes.c_double), ("stag_frac", ctypes.c_double),
                ("stag_window", ctypes.c_int32), ("restart_after", ctypes.c_int32)]


class EALCState(ctypes.Structure):
    _fields_ = [("gen", ctypes.c_int64), ("gen_restart", ctypes.c_int64),
                ("best_gen", ctypes.c_int64), ("p_mut", ctypes.c_double),
                ("stag_count", ctypes.c_int32), ("n_restarts", ctypes.c_int32),
                ("best_chi2", ctypes.c_double), ("best_Fs", ctypes.c_double),
                ("best_Fb", ctypes.c_double), ("best_p", ctypes.c_double * 6),
                ("hist", ctypes.c_double * 64)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from .build_oracle import build
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_source_position.argtypes = [ctypes.c_double] * 5 + [_dp, _dp]
    lib.orc_lens_poly.argtypes = [ctypes.c_double] * 4 + [_dp, _dp]
    lib.orc_poly_roots.argtypes = [_dp, _dp, ctypes.c_int, _dp, _dp]
    lib.orc_poly_roots.restype = ctypes.c_int
    lib.orc_images.argtypes = [ctypes.c_double] * 4 + [_dp] * 4
    lib.orc_images.restype = ctypes.c_int
    lib.orc_point_magnification.argtypes = [ctypes.c_double] * 4 + [ctypes.POINTER(ctypes.c_int)]
    lib.orc_point_magnification.restype = ctypes.c_double
    lib.orc_magnify.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int64, _dp, _i8p, ctypes.c_int]
    lib.orc_lsq_chi2.argtypes = [_dp, _dp, _dp, ctypes.c_int64, _dp, _dp, _dp]
    lib.orc_chi2.argtypes = [_i64p, ctypes.c_int32, _dp, _dp, _dp, _dp, ctypes.c_int32,
                             _dp, _dp, _dp, ctypes.c_int]
    lib.orc_decode.argtypes = [_dp, ctypes.c_int64, _dp, _dp, _dp]
    lib.orc_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
    lib.orc_draw.argtypes = [ctypes.c_uint64] * 6
    lib.orc_draw.restype = ctypes.c_uint64
    lib.orc_u01.argtypes = [ctypes.c_uint64]
    lib.orc_u01.restype = ctypes.c_double
    lib.orc_below.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
    lib.orc_below.restype = ctypes.c_uint32
    lib.orc_exp2_neg.argtypes = [ctypes.c_double]
    lib.orc_exp2_neg.restype = ctypes.c_double
    lib.orc_ea_init.argtypes = [ctypes.POINTER(EAConfig), ctypes.c_uint64, ctypes.c_int64, _dp,
                                ctypes.POINTER(EALCState)]
    lib.orc_ea_generation.argtypes = [ctypes.POINTER(EAConfig), ctypes.c_uint64, ctypes.c_int64,
                                      _dp, _dp, _dp, _dp, ctypes.POINTER(EALCState), _i32p]
    lib.orc_ea_init.restype = ctypes.c_int
    lib.orc_ea_generation.restype = ctypes.c_int
    _lib = lib
    return lib


def default_threads():
    """Host threads for the oracle: the CPUs this process may use, at most 16
    (one GPU's share of a shared host)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


# ----------------------------------------------------------------------------
# Forward model (Sec. 2.2)
# ----------------------------------------------------------------------------

def source_position(t, u0, alpha, tE, t0):
    lib = _load()
    zr, zi = ctypes.c_double(), ctypes.c_double()
    lib.orc_source_position(t, u0, alpha, tE, t0, ctypes.byref(zr), ctypes.byref(zi))
    return complex(zr.value, zi.value)


def lens_poly(zeta, d, q):
    """Coefficients c[0..5] (c[j] multiplies z**j) as a complex array."""
    lib = _load()
    cr, ci = np.zeros(6), np.zeros(6)
    lib.orc_lens_poly(zeta.real, zeta.imag, d, q, _p(cr), _p(ci))
    return cr + 1j * ci


def poly_roots(c, deg=None):
    lib = _load()
    c = np.asarray(c, dtype=complex)
    deg = len(c) - 1 if deg is None else deg
    cr, ci = _f64(c.real), _f64(c.imag)
    rr, ri = np.zeros(5), np.zeros(5)
    lib.orc_poly_roots(_p(cr), _p(ci), deg, _p(rr), _p(ri))
    return (rr + 1j * ri)[:deg]


def images(zeta, d, q):
    """(image positions, det J per image, sorted residuals of all roots)."""
    lib = _load()
    ir, ii, dj, rs = np.zeros(5), np.zeros(5), np.zeros(5), np.zeros(5)
    n = lib.orc_images(zeta.real, zeta.imag, d, q, _p(ir), _p(ii), _p(dj), _p(rs))
    return (ir + 1j * ii)[:n], dj[:n], rs


def point_magnification(zeta, d, q):
    """(A, n_img) at one source position."""
    lib = _load()
    n = ctypes.c_int()
    A = lib.orc_point_magnification(zeta.real, zeta.imag, d, q, ctypes.byref(n))
    return A, n.value


def magnify(theta, t, nthreads=None):
    """A[n][n_t], n_img[n][n_t] for theta[6][n] and shared epochs t[n_t]."""
    lib = _load()
    theta = _f64(theta)
    t = _f64(t)
    n, n_t = theta.shape[1], t.shape[0]
    A = np.zeros((n, n_t))
    ni = np.zeros((n, n_t), dtype=np.int8)
    lib.orc_magnify(_p(theta), n, _p(t), n_t, _p(A), _p(ni, _i8p),
                    nthreads or default_threads())
    return A, ni


def lsq_chi2(A, y, w):
    """(chi2, Fs, Fb) of one lightcurve given its magnifications."""
    lib = _load()
    A, y, w = _f64(A), _f64(y), _f64(w)
    c, fs, fb = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib.orc_lsq_chi2(_p(A), _p(y), _p(w), A.shape[0], ctypes.byref(c), ctypes.byref(fs),
                     ctypes.byref(fb))
    return c.value, fs.value, fb.value


def chi2(off, t, y, w, theta, pop, nthreads=None):
    """chi2, Fs, Fb [n_lc*pop] for a CSR batch (individual i -> lc i // pop)."""
    lib = _load()
    off = np.ascontiguousarray(off, dtype=np.int64)
    t, y, w, theta = _f64(t), _f64(y), _f64(w), _f64(theta)
    n_lc = off.shape[0] - 1
    n = n_lc * pop
    assert theta.shape == (6, n)
    c, fs, fb = np.zeros(n), np.zeros(n), np.zeros(n)
    lib.orc_chi2(_p(off, _i64p), n_lc, _p(t), _p(y), _p(w), _p(theta), pop,
                 _p(c), _p(fs), _p(fb), nthreads or default_threads())
    return c, fs, fb


def decode(P, lo, hi):
    """Eq. (EMMA-encoding) for P[6][n]."""
    lib = _load()
    P = _f64(P)
    lo, hi = _f64(lo), _f64(hi)
    out = np.zeros_like(P)
    lib.orc_decode(_p(P), P.shape[1], _p(lo), _p(hi), _p(out))
    return out


# ----------------------------------------------------------------------------
# Random numbers and the EA (Appendix A)
# ----------------------------------------------------------------------------

def philox4x64_10(ctr, key):
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib.orc_philox4x64_10(_p(c, _u64p), _p(k, _u64p), _p(out, _u64p))
    return out


def draw(seed, lc, gen, purpose, row, j):
    return _load().orc_draw(seed, lc, gen, purpose, row, j)


def u01(x):
    return _load().orc_u01(x)


def below(x, n):
    return _load().orc_below(x, n)


def exp2_neg(v):
    return _load().orc_exp2_neg(v)


class EA:
    """One lightcurve's EA state; P is the [pop][6] encoded population."""

    def __init__(self, pop, seed, lc, n_tourn=0, p_mut0=0.01, p_mut_min=1e-4, p_mut_max=0.5,
                 stag_frac=0.01, stag_window=10, restart_after=10):
        self.cfg = EAConfig(pop, n_tourn, p_mut0, p_mut_min, p_mut_max, stag_frac,
                            stag_window, restart_after)
        self.seed, self.lc, self.pop = seed, lc, pop
        self.P = np.zeros((pop, 6))
        self.st = EALCState()
        rc = _load().orc_ea_init(ctypes.byref(self.cfg), seed, lc, _p(self.P),
                                 ctypes.byref(self.st))
        if rc != 0:
            raise ValueError("orc_ea_init rejected the configuration")

    def generation(self, chi2, Fs=None, Fb=None):
        """Advance one generation; returns the parent ranks of every pairing."""
        chi2 = _f64(chi2)
        Fs = _f64(np.zeros(self.pop) if Fs is None else Fs)
        Fb = _f64(np.zeros(self.pop) if Fb is None else Fb)
        parents = np.zeros(2 * (self.pop // 2), dtype=np.int32)
        rc = _load().orc_ea_generation(ctypes.byref(self.cfg), self.seed, self.lc,
                                       _p(self.P), _p(chi2), _p(Fs), _p(Fb),
                                       ctypes.byref(self.st), _p(parents, _i32p))
        if rc != 0:
            raise ValueError("orc_ea_generation rejected the configuration")
        return parents

    def summary(self):
        s = self.st
        return dict(gen=s.gen, gen_restart=s.gen_restart, best_gen=s.best_gen, p_mut=s.p_mut,
                    stag_count=s.stag_count, n_restarts=s.n_restarts, best_chi2=s.best_chi2,
                    best_Fs=s.best_Fs, best_Fb=s.best_Fb, best_p=np.array(s.best_p[:]))


def caustic_points(d, q, n_phi, rng):
    """Points on the caustic of the lens (d, q) for phases phi ~ U[0, 2 pi).

    The critical curve is |1/conj(z)^2 + q/(d - conj(z))^2| = 1 (det J = 0);
    with 1/z^2 + q/(d - z)^2 = exp(i phi) it is the set of roots of the
    quartic exp(i phi) z^2 (z - d)^2 - (z - d)^2 - q z^2 = 0, mapped to the
    source plane by Eq. (lensing) to give the caustic.  Returns (zeta_c, z_c).
    """
    phis = rng.uniform(0.0, 2.0 * np.pi, n_phi)
    zs, zetas = [], []
    for phi in phis:
        e = np.exp(1j * phi)
        # e z^2 (z^2 - 2 d z + d^2) - (z^2 - 2 d z + d^2) - q z^2
        c = np.array([-d * d, 2 * d, e * d * d - 1 - q, -2 * d * e, e], dtype=complex)
        roots = poly_roots(c, 4)
        k = rng.integers(0, 4)
        z = roots[k]
        zb = np.conj(z)
        zs.append(z)
        zetas.append(z - 1 / zb + q / (d - zb))
    return np.array(zetas), np.array(zs)

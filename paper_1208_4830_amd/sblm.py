"""Thin ctypes binding of libsblm (C ABI declared in include/sblm.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device arrays are torch CUDA tensors (float64 / int64 / int8,
contiguous); PyTorch supplies device memory and the stream.  There is no
fallback: `load()` raises if libsblm.so is missing or fails to load.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# SBLM_LIB selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("SBLM_LIB", os.path.join(_HERE, "libsblm.so"))
NPAR = 6
FP64, MIXED = 0, 1
# proposal network sizes (include/sblm.h)
NBINS, NOUT, NOUT_PAD, NTARGET, NPARAMS = 256, 120, 128, 7, 455800
SEED_AT_RESTARTS = 1
SEED_WINDOW_ONLY = 2

_lib = None


class SblmError(RuntimeError):
    pass


class sblm_lcs(ctypes.Structure):
    _fields_ = [("n_lc", ctypes.c_int32), ("off", ctypes.c_void_p), ("t", ctypes.c_void_p),
                ("y", ctypes.c_void_p), ("w", ctypes.c_void_p)]


class ea_config(ctypes.Structure):
    _fields_ = [("pop", ctypes.c_int32), ("n_tourn", ctypes.c_int32),
                ("p_mut0", ctypes.c_double), ("p_mut_min", ctypes.c_double),
                ("p_mut_max", ctypes.c_double), ("stag_frac", ctypes.c_double),
                ("stag_window", ctypes.c_int32), ("restart_after", ctypes.c_int32),
                ("lo", ctypes.c_double * NPAR), ("hi", ctypes.c_double * NPAR),
                ("mode", ctypes.c_int32), ("n_islands", ctypes.c_int32),
                ("mig_every", ctypes.c_int32), ("n_migrants", ctypes.c_int32)]


class nm_config(ctypes.Structure):
    _fields_ = [("tol_x", ctypes.c_double), ("tol_f", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("mode", ctypes.c_int32)]


class ea_lc_summary(ctypes.Structure):
    _fields_ = [("best_chi2", ctypes.c_double), ("best_Fs", ctypes.c_double),
                ("best_Fb", ctypes.c_double), ("best_theta", ctypes.c_double * NPAR),
                ("best_gen", ctypes.c_int64), ("p_mut", ctypes.c_double),
                ("stag_count", ctypes.c_int32), ("n_restarts", ctypes.c_int32),
                ("gen", ctypes.c_int64), ("gen_restart", ctypes.c_int64)]


STATS_FIELDS = ("n_solves", "n_iter", "n_capped", "n_fallback", "n_degree4", "n_degenerate",
                "n_wave_iter", "n_iter_fp32", "n_polished", "n_retried",
                "n_unsettled", "n_newton")

_SIGS = {
    "sblm_magnify": [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                     ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                     ctypes.c_void_p],
    "sblm_chi2": [ctypes.POINTER(sblm_lcs), ctypes.c_void_p, ctypes.c_int32, ctypes.c_int,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p],
    "ea_default_config": [ctypes.POINTER(ea_config)],
    "ea_create": [ctypes.POINTER(ea_config), ctypes.POINTER(sblm_lcs), ctypes.c_uint64,
                  ctypes.POINTER(ctypes.c_void_p)],
    "ea_generation": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_void_p],
    "ea_evaluate": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "ea_fit": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p],
    "ea_buffers": [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_void_p)] * 4,
    "ea_summary": [ctypes.c_void_p, ctypes.POINTER(ea_lc_summary), ctypes.c_void_p],
    "ea_save": [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t),
                ctypes.c_void_p],
    "ea_load": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "ea_destroy": [ctypes.c_void_p],
    "ea_autotune": [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_size_t, ctypes.c_void_p],
    "ea_autotune_cached": [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32),
                           ctypes.c_char_p, ctypes.c_size_t, ctypes.c_void_p],
    "ea_get_schedule": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)],
    "ea_time_fitness": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p],
    "ea_fitness_time": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                        ctypes.POINTER(ctypes.c_int64)],
    "ea_set_schedule": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)],
    "ea_draws": [ctypes.c_uint64] * 6 + [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p],
    "ea_generation_traced": [ctypes.c_void_p] * 6,
    "ea_migrate": [ctypes.c_void_p] * 5,
    "sblm_last_error": [],
    "sblm_resample": [ctypes.POINTER(sblm_lcs), ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_void_p],
    "mlp_make_data": [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "mlp_create": [ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p)],
    "mlp_destroy": [ctypes.c_void_p],
    "mlp_set_params": [ctypes.c_void_p, ctypes.c_void_p],
    "mlp_get_params": [ctypes.c_void_p, ctypes.c_void_p],
    "mlp_forward": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                    ctypes.c_void_p],
    "mlp_loss_grad": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                      ctypes.c_void_p, ctypes.c_void_p],
    "mlp_get_grad": [ctypes.c_void_p, ctypes.c_void_p],
    "mlp_set_grad": [ctypes.c_void_p, ctypes.c_void_p],
    "mlp_adam_step": [ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p],
    "mlp_train": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                  ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                  ctypes.c_void_p, ctypes.c_void_p],
    "nm_default_config": [ctypes.POINTER(nm_config)],
    "nm_refine": [ctypes.POINTER(sblm_lcs), ctypes.POINTER(ctypes.c_double),
                  ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.POINTER(nm_config),
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "nm_refine_multi": [ctypes.POINTER(sblm_lcs), ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                        ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                        ctypes.POINTER(nm_config), ctypes.c_void_p, ctypes.c_void_p,
                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                        ctypes.c_void_p],
    "nm_refine_noalloc": [ctypes.POINTER(sblm_lcs), ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                          ctypes.POINTER(nm_config), ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_void_p],
    "nm_iterated": [ctypes.POINTER(sblm_lcs), ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                    ctypes.POINTER(nm_config)] + [ctypes.c_void_p] * 7,
    "ea_best": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "ea_freeze": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                  ctypes.c_void_p],
    "ea_records": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "ea_refine": [ctypes.c_void_p, ctypes.POINTER(nm_config), ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p],
    "ea_seed": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                ctypes.c_int32, ctypes.c_void_p],
}
EXPORTS = tuple(_SIGS)


def load():
    """Load libsblm.so (once).  Raises SblmError if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SblmError(f"{LIB_PATH} not built: run paper_1208_4830_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.sblm_last_error.restype = ctypes.c_char_p
    lib.ea_default_config.restype = None
    lib.ea_destroy.restype = None
    lib.mlp_destroy.restype = None
    lib.nm_default_config.restype = None
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        msg = load().sblm_last_error().decode()
        raise SblmError(f"libsblm error {rc}: {msg}")


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(x, dtype=torch.float64):
    if x is None:
        return None
    if not (x.is_cuda and x.dtype == dtype and x.is_contiguous()):
        raise SblmError(f"expected a contiguous CUDA {dtype} tensor, got {x.dtype} on {x.device}")
    return x


def _ptr(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None else None


class _CudaArray:
    def __init__(self, ptr, shape, typestr):
        self.__cuda_array_interface__ = {"shape": shape, "typestr": typestr,
                                         "data": (ptr, False), "version": 2, "strides": None}


def _device_view(ptr, shape, typestr="<f8"):
    return torch.as_tensor(_CudaArray(ptr, tuple(shape), typestr), device="cuda")


def new_stats(device="cuda"):
    """Zeroed sblm_stats block (one uint64 per field) as an int64 device tensor."""
    return torch.zeros(len(STATS_FIELDS), dtype=torch.int64, device=device)


def stats_dict(st):
    return dict(zip(STATS_FIELDS, st.cpu().tolist()))


def sblm_magnify(theta, t, mode=FP64, A=None, n_img=None, stats=None, stream=None):
    """A[n][n_t] (and n_img[n][n_t] if given) for theta[6][n], epochs t[n_t]."""
    lib = load()
    theta, t = _dev(theta), _dev(t)
    n, n_t = theta.shape[1], t.shape[0]
    if A is None:
        A = torch.empty((n, n_t), dtype=torch.float64, device=theta.device)
    _dev(A), _dev(n_img, torch.int8), _dev(stats, torch.int64)
    _check(lib.sblm_magnify(_ptr(theta), n, _ptr(t), n_t, mode, _ptr(A), _ptr(n_img),
                            _ptr(stats), _stream(stream)))
    return A


class Lightcurves:
    """Device CSR batch (keeps the tensors alive for the descriptor)."""

    def __init__(self, off, t, y, w):
        self.off = _dev(off, torch.int64)
        self.t, self.y, self.w = _dev(t), _dev(y), _dev(w)
        self.n_lc = self.off.shape[0] - 1
        self.desc = sblm_lcs(self.n_lc, self.off.data_ptr(), self.t.data_ptr(),
                             self.y.data_ptr(), self.w.data_ptr())


def sblm_chi2(lcs, theta, pop, mode=FP64, chi2=None, Fs=None, Fb=None, stats=None,
              stream=None):
    """(chi2, Fs, Fb)[n_lc*pop] for decoded theta[6][n_lc*pop]."""
    lib = load()
    theta = _dev(theta)
    n = lcs.n_lc * pop
    outs = []
    for x in (chi2, Fs, Fb):
        outs.append(torch.empty(n, dtype=torch.float64, device=theta.device) if x is None
                    else _dev(x))
    _dev(stats, torch.int64)
    _check(lib.sblm_chi2(ctypes.byref(lcs.desc), _ptr(theta), pop, mode, _ptr(outs[0]),
                         _ptr(outs[1]), _ptr(outs[2]), _ptr(stats), _stream(stream)))
    return tuple(outs)


def ea_draws(seed, lc, gen, purpose, row, j0, n, device="cuda", stream=None):
    """Raw Philox words of the EA's streams as an int64 tensor (bit pattern)."""
    out = torch.empty(n, dtype=torch.int64, device=device)
    _check(load().ea_draws(seed, lc, gen, purpose, row, j0, n, _ptr(out), _stream(stream)))
    return out


class SnapHeader(ctypes.Structure):
    _fields_ = [("magic", ctypes.c_uint64), ("seed", ctypes.c_uint64), ("n_lc", ctypes.c_int32),
                ("pop", ctypes.c_int32), ("cfg", ea_config), ("rec_size", ctypes.c_uint64)]


def parse_snapshot(blob):
    """(header, P[6][n_lc*pop], per-lightcurve records) from an ea_save blob."""
    import numpy as np
    hd = SnapHeader.from_buffer_copy(blob[:ctypes.sizeof(SnapHeader)])
    n = hd.n_lc * hd.pop
    o = ctypes.sizeof(SnapHeader)
    P = np.frombuffer(blob, dtype=np.float64, count=6 * n, offset=o).reshape(6, n)
    rec = np.dtype([("gen", "<i8"), ("gen_restart", "<i8"), ("best_gen", "<i8"),
                    ("p_mut", "<f8"), ("stag_count", "<i4"), ("n_restarts", "<i4"),
                    ("best_chi2", "<f8"), ("best_Fs", "<f8"), ("best_Fb", "<f8"),
                    ("best_p", "<f8", (6,)), ("hist", "<f8", (64,))])
    assert rec.itemsize == hd.rec_size
    recs = np.frombuffer(blob, dtype=rec, count=hd.n_lc, offset=o + 6 * n * 8)
    return hd, P.copy(), recs.copy()


def ea_default_config():
    cfg = ea_config()
    load().ea_default_config(ctypes.byref(cfg))
    return cfg


class EAState:
    """Owner of an ea_state* (device workspace of one batched fit)."""

    def __init__(self, cfg, lcs, seed):
        lib = load()
        self.lcs = lcs  # keep the device arrays alive
        self.cfg = cfg
        h = ctypes.c_void_p()
        _check(lib.ea_create(ctypes.byref(cfg), ctypes.byref(lcs.desc), seed, ctypes.byref(h)))
        self.h = h
        P, c, fs, fb = (ctypes.c_void_p() for _ in range(4))
        _check(lib.ea_buffers(self.h, ctypes.byref(P), ctypes.byref(c), ctypes.byref(fs),
                              ctypes.byref(fb)))
        self._ptrs = dict(P=P.value, chi2=c.value, Fs=fs.value, Fb=fb.value)

    def ptr(self, name):
        return self._ptrs[name]

    def view(self, name):
        """Zero-copy torch view of a state buffer ('P' [6][n], 'chi2', 'Fs',
        'Fb' [n], n = n_lc * n_islands * pop, island-major within each
        lightcurve); valid until close()."""
        n = self.lcs.n_lc * self.cfg.n_islands * self.cfg.pop
        shape = (NPAR, n) if name == "P" else (n,)
        return _device_view(self._ptrs[name], shape)

    def generation(self, chi2, Fs, Fb, stream=None):
        _check(load().ea_generation(self.h, _ptr(_dev(chi2)), _ptr(_dev(Fs)), _ptr(_dev(Fb)),
                                    _stream(stream)))

    def generation_traced(self, chi2, Fs, Fb, parents, stream=None):
        _check(load().ea_generation_traced(self.h, _ptr(_dev(chi2)), _ptr(_dev(Fs)),
                                           _ptr(_dev(Fb)), _ptr(_dev(parents, torch.int32)),
                                           _stream(stream)))

    def migrate(self, chi2=None, Fs=None, Fb=None, stream=None):
        """One ring migration among every lightcurve's islands now, on the
        given fitness arrays (modified in place) or the state's own."""
        if chi2 is None:
            args = (None, None, None)
        else:
            args = tuple(_ptr(a) for a in (chi2, Fs, Fb))
        _check(load().ea_migrate(self.h, *args, _stream(stream)))

    def evaluate(self, stats=None, stream=None):
        _check(load().ea_evaluate(self.h, _ptr(stats), _stream(stream)))

    def fit(self, n_gen, stats=None, stream=None):
        _check(load().ea_fit(self.h, n_gen, _ptr(stats), _stream(stream)))

    def time_fitness(self, enable=True, stream=None):
        """Stamp the device clock around the fitness kernel of every replayed
        generation (and clear the sums)."""
        _check(load().ea_time_fitness(self.h, 1 if enable else 0, _stream(stream)))

    def fitness_time(self):
        """(milliseconds summed over the timed fitness launches, launches)."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(load().ea_fitness_time(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def autotune(self, stream=None, cache=None):
        """Time the candidate schedules; returns the report text.  With
        `cache` (a file path) a choice kept there for this device and
        workload is installed instead, or the new choice is appended."""
        buf = ctypes.create_string_buffer(4096)
        if cache is None:
            _check(load().ea_autotune(self.h, buf, len(buf), _stream(stream)))
        else:
            tuned = ctypes.c_int32(-1)
            _check(load().ea_autotune_cached(self.h, os.fsencode(cache), ctypes.byref(tuned),
                                             buf, len(buf), _stream(stream)))
        return buf.value.decode()

    def schedule(self):
        """(lanes per individual, waves per block, persistent, asynchronous)."""
        out = (ctypes.c_int32 * 4)()
        _check(load().ea_get_schedule(self.h, out))
        return tuple(out)

    def set_schedule(self, lanes, wpb, persistent, asynchronous=1):
        _check(load().ea_set_schedule(self.h, (ctypes.c_int32 * 4)(lanes, wpb, persistent,
                                                                     asynchronous)))

    def summary(self, stream=None):
        out = (ea_lc_summary * self.lcs.n_lc)()
        _check(load().ea_summary(self.h, out, _stream(stream)))
        return out

    def save(self, stream=None):
        n = ctypes.c_size_t()
        _check(load().ea_save(self.h, None, ctypes.byref(n), _stream(stream)))
        buf = ctypes.create_string_buffer(n.value)
        _check(load().ea_save(self.h, buf, ctypes.byref(n), _stream(stream)))
        return buf.raw

    def load(self, blob, stream=None):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(load().ea_load(self.h, buf, len(blob), _stream(stream)))

    def seed(self, out, n_seed, at_restarts=False, stream=None):
        """Overwrite rows [0, n_seed) of every lightcurve's population with
        draws from the proposal mixture out[n_lc][>=120] (float32); with
        at_restarts, every later restart re-draws them (out is kept alive
        here while attached)."""
        out = _dev(out, torch.float32)
        _check(load().ea_seed(self.h, _ptr(out), out.shape[1], n_seed,
                              SEED_AT_RESTARTS if at_restarts else 0, _stream(stream)))
        self._proposals = out if (at_restarts and n_seed > 0) else None

    def seed_window(self, n_seed, at_restarts=False, stream=None):
        """As seed, with rows drawn from the observation window alone: t0 at
        the middle of the observed span, tE a quarter of it, the other genes
        uniform (the ablation of the learned form)."""
        _check(load().ea_seed(self.h, None, 0, n_seed,
                              SEED_WINDOW_ONLY | (SEED_AT_RESTARTS if at_restarts else 0),
                              _stream(stream)))
        self._proposals = None

    def freeze(self, mask, stream=None):
        """Freeze (nonzero) or resume (0) the EA of each lightcurve: mask of
        n_lc host ints."""
        import numpy as np
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.int32).reshape(-1))
        _check(load().ea_freeze(self.h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                m.size, _stream(stream)))

    def best(self, stream=None):
        """(x [6][n_lc] encoded, chi2 [n_lc]) of every lightcurve's record."""
        n = self.lcs.n_lc
        x = torch.empty((NPAR, n), dtype=torch.float64, device=self.lcs.t.device)
        c = torch.empty(n, dtype=torch.float64, device=self.lcs.t.device)
        _check(load().ea_best(self.h, _ptr(x), _ptr(c), _stream(stream)))
        return x, c

    def records(self, stream=None):
        """(x [6][n], chi2 [n]) of every island's record, n = n_lc * n_islands."""
        n = self.lcs.n_lc * self.cfg.n_islands
        x = torch.empty((NPAR, n), dtype=torch.float64, device=self.lcs.t.device)
        c = torch.empty(n, dtype=torch.float64, device=self.lcs.t.device)
        _check(load().ea_records(self.h, _ptr(x), _ptr(c), _stream(stream)))
        return x, c

    def refine(self, cfg=None, stats=None, stream=None):
        """Simplex fine-tuning of every record (one per island); returns the
        steps taken [n_lc * n_islands]."""
        cfg = cfg or nm_default_config()
        it = torch.empty(self.lcs.n_lc * self.cfg.n_islands, dtype=torch.int32,
                         device=self.lcs.t.device)
        _check(load().ea_refine(self.h, ctypes.byref(cfg), _ptr(it), _ptr(stats),
                                _stream(stream)))
        return it

    def close(self):
        if self.h:
            load().ea_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- simplex

def nm_default_config():
    cfg = nm_config()
    load().nm_default_config(ctypes.byref(cfg))
    return cfg


def nm_refine(lcs, lo, hi, x0, cfg=None, stats=None, stream=None, reps=1):
    """(x [6][n], chi2, Fs, Fb [n], steps [n] int32) from encoded start
    points x0 [6][n] in the domain [lo, hi], n = n_lc * reps: `reps`
    simplices per lightcurve (simplex k * reps + i on lightcurve k)."""
    cfg = cfg or nm_default_config()
    x0 = _dev(x0)
    n = lcs.n_lc * reps
    if x0.shape != (NPAR, n):
        raise SblmError(f"x0 must be [6][{n}], got {tuple(x0.shape)}")
    dev = x0.device
    x = torch.empty_like(x0)
    c, fs, fb = (torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3))
    it = torch.empty(n, dtype=torch.int32, device=dev)
    lo_ = (ctypes.c_double * NPAR)(*[float(v) for v in lo])
    hi_ = (ctypes.c_double * NPAR)(*[float(v) for v in hi])
    _check(load().nm_refine_multi(ctypes.byref(lcs.desc), reps, lo_, hi_, _ptr(x0),
                                  ctypes.byref(cfg), _ptr(x), _ptr(c), _ptr(fs), _ptr(fb),
                                  _ptr(it), _ptr(stats), _stream(stream)))
    return x, c, fs, fb, it


def nm_refine_noalloc(lcs, lo, hi, x0, cfg=None, out=None, stats=None, stream=None):
    """nm_refine (one simplex per lightcurve) through the entry point that
    allocates no device memory.  `out` = (x, chi2, Fs, Fb, steps): caller
    tensors ([6][n_lc] float64, three [n_lc] float64, [n_lc] int32) written
    in place; allocated here when None."""
    cfg = cfg or nm_default_config()
    x0 = _dev(x0)
    n = lcs.n_lc
    if x0.shape != (NPAR, n):
        raise SblmError(f"x0 must be [6][{n}], got {tuple(x0.shape)}")
    if out is None:
        dev = x0.device
        out = (torch.empty_like(x0),) + tuple(torch.empty(n, dtype=torch.float64, device=dev)
                                              for _ in range(3)) + \
            (torch.empty(n, dtype=torch.int32, device=dev),)
    x, c, fs, fb, it = out
    lo_ = (ctypes.c_double * NPAR)(*[float(v) for v in lo])
    hi_ = (ctypes.c_double * NPAR)(*[float(v) for v in hi])
    _check(load().nm_refine_noalloc(ctypes.byref(lcs.desc), lo_, hi_, _ptr(x0),
                                    ctypes.byref(cfg), _ptr(_dev(x)), _ptr(_dev(c)),
                                    _ptr(_dev(fs)), _ptr(_dev(fb)), _ptr(_dev(it, torch.int32)),
                                    _ptr(stats), _stream(stream)))
    return x, c, fs, fb, it


def nm_iterated(lcs, lo, hi, reps, runs, seed, cfg=None, stats=None, stream=None,
                device="cuda"):
    """Iterated simplex: (x [6][n_lc] encoded, chi2, Fs, Fb [n_lc], steps
    [n_lc] int64) best over reps * runs random starts per lightcurve."""
    cfg = cfg or nm_default_config()
    n = lcs.n_lc
    dev = lcs.t.device if lcs.t is not None else device
    x = torch.empty((NPAR, n), dtype=torch.float64, device=dev)
    c, fs, fb = (torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3))
    it = torch.empty(n, dtype=torch.int64, device=dev)
    lo_ = (ctypes.c_double * NPAR)(*[float(v) for v in lo])
    hi_ = (ctypes.c_double * NPAR)(*[float(v) for v in hi])
    _check(load().nm_iterated(ctypes.byref(lcs.desc), reps, runs, seed, lo_, hi_,
                              ctypes.byref(cfg), _ptr(x), _ptr(c), _ptr(fs), _ptr(fb),
                              _ptr(it), _ptr(stats), _stream(stream)))
    return x, c, fs, fb, it


# ---------------------------------------------------------------- proposal network

def sblm_resample(lcs, want_f32=False, want_bf16=True, stream=None):
    """(xb [n_lc][256] bfloat16 or None, xf [n_lc][256] float32 or None)."""
    dev = lcs.t.device
    xb = torch.empty((lcs.n_lc, NBINS), dtype=torch.bfloat16, device=dev) if want_bf16 else None
    xf = torch.empty((lcs.n_lc, NBINS), dtype=torch.float32, device=dev) if want_f32 else None
    _check(load().sblm_resample(ctypes.byref(lcs.desc), _ptr(xf), _ptr(xb), _stream(stream)))
    return xb, xf


def mlp_make_data(seed, first, n, want_f32=False, device="cuda", stream=None):
    """Training samples first..first+n-1: (xb bfloat16 [n][256], xf float32
    [n][256] or None, y float32 [n][7])."""
    xb = torch.empty((n, NBINS), dtype=torch.bfloat16, device=device)
    xf = torch.empty((n, NBINS), dtype=torch.float32, device=device) if want_f32 else None
    y = torch.empty((n, NTARGET), dtype=torch.float32, device=device)
    _check(load().mlp_make_data(seed, first, n, _ptr(xb), _ptr(xf), _ptr(y), _stream(stream)))
    return xb, xf, y


class MLP:
    """Owner of an mlp_net* (weights, Adam moments and activation buffers)."""

    def __init__(self, batch_max=1024, seed=0):
        h = ctypes.c_void_p()
        _check(load().mlp_create(batch_max, seed, ctypes.byref(h)))
        self.h = h
        self.batch_max = batch_max

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == NPARAMS
        _check(load().mlp_set_params(self.h, p.ctypes.data_as(ctypes.c_void_p)))

    def get_params(self):
        import numpy as np
        p = np.empty(NPARAMS, dtype=np.float32)
        _check(load().mlp_get_params(self.h, p.ctypes.data_as(ctypes.c_void_p)))
        return p

    def grad(self):
        import numpy as np
        g = np.empty(NPARAMS, dtype=np.float32)
        _check(load().mlp_get_grad(self.h, g.ctypes.data_as(ctypes.c_void_p)))
        return g

    def set_grad(self, grad):
        import numpy as np
        g = np.ascontiguousarray(grad, dtype=np.float32)
        assert g.size == NPARAMS
        _check(load().mlp_set_grad(self.h, g.ctypes.data_as(ctypes.c_void_p)))

    def forward(self, xb, out=None, stream=None):
        xb = _dev(xb, torch.bfloat16)
        if out is None:
            out = torch.empty((xb.shape[0], NOUT_PAD), dtype=torch.float32, device=xb.device)
        _check(load().mlp_forward(self.h, _ptr(xb), xb.shape[0], _ptr(_dev(out, torch.float32)),
                                  _stream(stream)))
        return out

    def loss_grad(self, xb, y, stream=None):
        xb, y = _dev(xb, torch.bfloat16), _dev(y, torch.float32)
        loss = torch.zeros(1, dtype=torch.float32, device=xb.device)
        _check(load().mlp_loss_grad(self.h, _ptr(xb), _ptr(y), xb.shape[0], _ptr(loss),
                                    _stream(stream)))
        return loss

    def adam_step(self, lr, stream=None):
        _check(load().mlp_adam_step(self.h, lr, _stream(stream)))

    def train(self, xb, y, batch=1024, epochs=1, lr0=1e-3, lr1=1e-5, stream=None):
        """Returns the per-step losses (float32 device tensor)."""
        xb, y = _dev(xb, torch.bfloat16), _dev(y, torch.float32)
        steps = epochs * (xb.shape[0] // batch)
        loss = torch.zeros(max(steps, 1), dtype=torch.float32, device=xb.device)
        _check(load().mlp_train(self.h, _ptr(xb), _ptr(y), xb.shape[0], batch, epochs, lr0,
                                lr1, _ptr(loss), _stream(stream)))
        return loss[:steps]

    def close(self):
        if self.h:
            load().mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""The paper's fitting experiments (Sec. 4.2-4.4, Tables 2 and 3) as a
measurement harness around the library.

Lightcurves are drawn by `inputs.paper_workload` (Table 1 ranges, 100 points
between the t_start and t_end windows; experiment 1 uniform and noise-free,
experiment 2 random times, magnitude noise and blending).  Every
magnification and every fit runs in the library on the GPU; this module only
does the bookkeeping around them in numpy:
  - observations: m = m0 - 2.5 log10(f A + 1 - f) (Eq. A_s, Eq. blend);
    sigma = 0.01 mag (experiment 1) or log10 sigma = 0.3416 m - 7.7095 at the
    true magnitude (Eq. noiseModel, experiment 2);
  - fitting in flux: F = 10^(-0.4 (m - 20)) with sigma_F = 0.4 ln 10 F sigma,
    so that the library's profiled (Fs, Fb) are (m0, f) in flux form:
    m0 = 20 - 2.5 log10(Fs + Fb), f = Fs / (Fs + Fb);
  - success (Sec. 4.2): Delta chi^2 / nu < 1 in magnitudes (nu = N - 7, or
    N - 8 with blending), and for the strict form every parameter within
    10% (q, a, b, tE, m0, f relative to the true value; tm relative to tE;
    the wrapped angle relative to 2 pi); also reported, the strict form on
    the six lens and trajectory parameters alone (m0 and f are profiled
    here, not searched, and with the noise of Eq. noiseModel at 18-22 mag
    the profiled f of the true model itself misses 10% on many lightcurves);
  - peak classes (Tables 2-3): maxima of the source magnification on a
    4000-point grid over [t_start, t_end] with a prominence of at least 0.01
    mag, classes 1, 2, 3 and 4 or more.
"""
import math
import time

import numpy as np

from . import inputs

ZP = 20.0
SIGMA_EXP1 = 0.01
GRID = 4000
PROMINENCE = 0.01


def _magnify_each(sblm, torch, theta, times):
    """A of column k of theta at its own epochs times[k] (one call each)."""
    out = []
    for k, t in enumerate(times):
        th = torch.as_tensor(np.ascontiguousarray(theta[:, k:k + 1]), device="cuda")
        A = sblm.sblm_magnify(th, torch.as_tensor(np.ascontiguousarray(t), device="cuda"))
        out.append(A[0].cpu().numpy())
    return out


def observations(sblm, torch, wl):
    """Magnitudes and device lightcurves in flux for a PaperWorkload:
    dict(lcs, m_true, m_obs, sigma) with per-point arrays in CSR order."""
    times = [wl.t[wl.off[k]:wl.off[k + 1]] for k in range(wl.n_lc)]
    A = np.concatenate(_magnify_each(sblm, torch, wl.theta, times))
    lc_of = np.repeat(np.arange(wl.n_lc), np.diff(wl.off))
    f, m0 = wl.f[lc_of], wl.m0[lc_of]
    m_true = m0 - 2.5 * np.log10(f * A + (1.0 - f))
    if wl.experiment == 1:
        sigma = np.full(m_true.shape, SIGMA_EXP1)
        m_obs = m_true.copy()
    else:
        sigma = 10.0 ** (0.3416 * m_true - 7.7095)
        m_obs = m_true + sigma * wl.noise
    y = 10.0 ** (-0.4 * (m_obs - ZP))
    w = 1.0 / (0.4 * math.log(10.0) * y * sigma) ** 2
    cu = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt,
                                                     device="cuda")
    lcs = sblm.Lightcurves(cu(wl.off, torch.int64), cu(wl.t), cu(y), cu(w))
    return dict(lcs=lcs, m_true=m_true, m_obs=m_obs, sigma=sigma)


def count_peaks(A):
    """Maxima of A with a prominence of at least 0.01 mag."""
    M = 2.5 * np.log10(np.asarray(A, float))
    n = len(M)
    d = np.diff(M)
    count = 0
    i = 1
    while i < n - 1:
        if d[i - 1] <= 0:
            i += 1
            continue
        j = i  # end of a run of equal values starting at i
        while j < n - 1 and d[j] == 0:
            j += 1
        if j < n - 1 and d[j] < 0:
            higher_l = np.nonzero(M[:i] > M[i])[0]
            higher_r = np.nonzero(M[j + 1:] > M[i])[0]
            lo = higher_l[-1] + 1 if higher_l.size else 0
            hi = j + 1 + higher_r[0] if higher_r.size else n
            base = max(M[lo:i].min(), M[j + 1:hi].min())
            if M[i] - base >= PROMINENCE:
                count += 1
        i = j + 1
    return count


def peak_classes(sblm, torch, wl):
    """Class 1..4 (4 = four or more peaks) of every lightcurve."""
    grids = [np.linspace(wl.t_start[k], wl.t_end[k], GRID) for k in range(wl.n_lc)]
    A = _magnify_each(sblm, torch, wl.theta, grids)
    return np.array([min(max(count_peaks(a), 1), 4) for a in A])


def evaluate(sblm, torch, wl, obs, theta_fit, Fs, Fb, lens_only=False):
    """(weak, strict, Delta chi^2 / nu) arrays for fitted parameters
    theta_fit[6][n_lc] with profiled fluxes Fs, Fb [n_lc].  lens_only: the
    strict test on the six lens and trajectory parameters alone (m0 and f
    are profiled by the fit, not searched)."""
    times = [wl.t[wl.off[k]:wl.off[k + 1]] for k in range(wl.n_lc)]
    A_fit = _magnify_each(sblm, torch, theta_fit, times)
    n_par = 7 if wl.experiment == 1 else 8
    weak = np.zeros(wl.n_lc, bool)
    strict = np.zeros(wl.n_lc, bool)
    dchi = np.full(wl.n_lc, np.inf)
    for k in range(wl.n_lc):
        sl = slice(wl.off[k], wl.off[k + 1])
        tot = Fs[k] + Fb[k]
        if not tot > 0:
            continue
        m0_fit, f_fit = ZP - 2.5 * math.log10(tot), Fs[k] / tot
        flux = f_fit * A_fit[k] + (1.0 - f_fit)
        if np.any(flux <= 0):
            continue
        r_fit = (obs["m_obs"][sl] - (m0_fit - 2.5 * np.log10(flux))) / obs["sigma"][sl]
        r_true = (obs["m_obs"][sl] - obs["m_true"][sl]) / obs["sigma"][sl]
        dchi[k] = (r_fit @ r_fit - r_true @ r_true) / (sl.stop - sl.start - n_par)
        tt, tf = wl.theta[:, k], theta_fit[:, k]
        rel = [abs(10 ** tf[0] - 10 ** tt[0]) / 10 ** tt[0],
               abs(tf[1] - tt[1]) / tt[1], abs(tf[2] - tt[2]) / tt[2],
               abs(tf[4] - tt[4]) / tt[4], abs(tf[5] - tt[5]) / tt[4],
               min((tf[3] - tt[3]) % (2 * math.pi), (tt[3] - tf[3]) % (2 * math.pi))
               / (2 * math.pi)]
        if not lens_only:
            rel.append(abs(m0_fit - wl.m0[k]) / wl.m0[k])
            if wl.experiment == 2:
                rel.append(abs(f_fit - wl.f[k]) / wl.f[k])
        weak[k] = dchi[k] < 1.0
        strict[k] = weak[k] and max(rel) < 0.1
    return weak, strict, dchi


def _decode(x, lo, hi):
    return lo[:, None] + (hi - lo)[:, None] * x


def _rates(ok, classes):
    """Overall and per-class success fractions."""
    out = {"all": round(float(np.mean(ok)), 4)}
    for c in (1, 2, 3, 4):
        sel = classes == c
        out[f"{c}_peak" + ("s" if c > 1 else "")] = (round(float(np.mean(ok[sel])), 4)
                                                   if sel.any() else None)
    return out


def run_experiment(sblm, torch, experiment, n_lc=512, pop=1000, checkpoints=(250, 500, 1000),
                   passes=3, iterated=(16, 2, 10000), seed=11, sched=(16, 4, 1, 0)):
    """One experiment: the EA alone and with simplex fine-tuning at every
    checkpoint, and the iterated simplex; success rates (strict and weak),
    by peak class, with the GPU seconds they took."""
    lo, hi = inputs.PAPER_LO, inputs.PAPER_HI
    wl = inputs.paper_workload(seed, n_lc, experiment)
    obs = observations(sblm, torch, wl)
    classes = peak_classes(sblm, torch, wl)
    lcs = obs["lcs"]
    cfg = sblm.ea_default_config()
    cfg.pop = pop
    for j in range(6):
        cfg.lo[j], cfg.hi[j] = float(lo[j]), float(hi[j])
    state = sblm.EAState(cfg, lcs, seed)
    state.set_schedule(*sched)
    nm_cfg = sblm.nm_default_config()
    sync = torch.cuda.synchronize
    ea_s, gens, rows = 0.0, 0, []
    for cp in checkpoints:
        sync()
        t0 = time.perf_counter()
        state.fit(cp - gens)
        sync()
        ea_s += time.perf_counter() - t0
        gens = cp
        summ = state.summary()
        th_ea = np.array([s.best_theta[:] for s in summ]).T
        fs_ea = np.array([s.best_Fs for s in summ])
        fb_ea = np.array([s.best_Fb for s in summ])
        x, c_best = state.best()
        sync()
        t0 = time.perf_counter()
        best = (x, c_best, torch.as_tensor(fs_ea, device="cuda"),
                torch.as_tensor(fb_ea, device="cuda"))
        for _ in range(passes):
            x, c, fs, fb, _ = sblm.nm_refine(lcs, lo, hi, x, nm_cfg)
            better = c < best[1]
            best = tuple(torch.where(better, a, b) for a, b in
                         ((x, best[0]), (c, best[1]), (fs, best[2]), (fb, best[3])))
        sync()
        nm_s = time.perf_counter() - t0
        th_nm = _decode(best[0].cpu().numpy(), lo, hi)
        fs_nm, fb_nm = best[2].cpu().numpy(), best[3].cpu().numpy()
        w_ea, s_ea, _ = evaluate(sblm, torch, wl, obs, th_ea, fs_ea, fb_ea)
        _, l_ea, _ = evaluate(sblm, torch, wl, obs, th_ea, fs_ea, fb_ea, lens_only=True)
        w_nm, s_nm, _ = evaluate(sblm, torch, wl, obs, th_nm, fs_nm, fb_nm)
        _, l_nm, _ = evaluate(sblm, torch, wl, obs, th_nm, fs_nm, fb_nm, lens_only=True)
        rows.append(dict(gen=cp, ea_seconds=round(ea_s, 3), amoeba_seconds=round(nm_s, 3),
                         ea=dict(strict=_rates(s_ea, classes), weak=_rates(w_ea, classes),
                                 strict_lens=_rates(l_ea, classes)),
                         ea_amoeba=dict(strict=_rates(s_nm, classes),
                                        weak=_rates(w_nm, classes),
                                        strict_lens=_rates(l_nm, classes))))
    state.close()
    # ceiling: the true parameters with their fluxes profiled on the noisy
    # data (what the information in the lightcurves allows)
    _, fs_t, fb_t = sblm.sblm_chi2(lcs, torch.as_tensor(np.ascontiguousarray(wl.theta),
                                                        device="cuda"), 1)
    fs_t, fb_t = fs_t.cpu().numpy(), fb_t.cpu().numpy()
    w_t, s_t, _ = evaluate(sblm, torch, wl, obs, wl.theta, fs_t, fb_t)
    _, l_t, _ = evaluate(sblm, torch, wl, obs, wl.theta, fs_t, fb_t, lens_only=True)
    out = dict(experiment=experiment, lightcurves=n_lc, points=100, pop=pop,
               classes={str(c): int(np.sum(classes == c)) for c in (1, 2, 3, 4)},
               truth_profiled=dict(strict=_rates(s_t, classes), weak=_rates(w_t, classes),
                                   strict_lens=_rates(l_t, classes)),
               checkpoints=rows)
    if iterated:
        reps, runs, max_iter = iterated
        it_cfg = sblm.nm_default_config()
        it_cfg.max_iter = max_iter
        sync()
        t0 = time.perf_counter()
        x, c, fs, fb, _ = sblm.nm_iterated(lcs, lo, hi, reps, runs, seed, it_cfg)
        sync()
        dt = time.perf_counter() - t0
        th_it, fs_it, fb_it = _decode(x.cpu().numpy(), lo, hi), fs.cpu().numpy(), fb.cpu().numpy()
        w_it, s_it, _ = evaluate(sblm, torch, wl, obs, th_it, fs_it, fb_it)
        _, l_it, _ = evaluate(sblm, torch, wl, obs, th_it, fs_it, fb_it, lens_only=True)
        out["iterated_simplex"] = dict(starts=reps * runs, max_steps_per_run=max_iter,
                                       gpu_seconds=round(dt, 3),
                                       strict=_rates(s_it, classes), weak=_rates(w_it, classes),
                                       strict_lens=_rates(l_it, classes))
    return out

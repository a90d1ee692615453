"""GPU parity of the batched simplex refinement against the simplex oracle
driven by the oracle's chi^2, and the EA-with-amoeba record update."""
import numpy as np
import pytest
import torch

from oracle import nm_oracle as NM
from oracle import oracle as O
from paper_1208_4830_amd import inputs
from tests.helpers import oracle_lightcurves

pytestmark = pytest.mark.gpu

LO, HI = inputs.PRIOR_LO, inputs.PRIOR_HI


def oracle_f(t, y, w):
    off = np.array([0, t.size], np.int64)

    def f(x):
        th = O.decode(np.asarray(x, float)[:, None], LO, HI)
        return O.chi2(off, t, y, w, th, 1, nthreads=1)[0][0]
    return f


def device_lcs(hip, wl, y, w):
    cu = lambda a, dt=torch.float64: torch.tensor(a, dtype=dt, device="cuda")
    return hip.Lightcurves(cu(wl.off, torch.int64), cu(wl.t), cu(y), cu(w))


# SBLM_NM_SPEC_MAX: "0" evaluates one point of a step per round (the
# reflection, then the one other point it asks for), a large value all four
# at once; the sequence of simplices is the same
ONE, FOUR = "0", "1000000000"
_ORACLE_RUNS = {}


def _oracle_minimise(key, f, x0, cfg):
    if key not in _ORACLE_RUNS:
        _ORACLE_RUNS[key] = NM.minimise(f, x0, cfg.tol_x, cfg.tol_f, cfg.max_iter)
    return _ORACLE_RUNS[key]


@pytest.mark.parametrize("mode,lanes,form", [(0, "256", FOUR), (0, "256", ONE), (1, "256", ONE),
                                             (1, "256", FOUR), (0, "128", ONE), (0, "64", ONE),
                                             (0, "64", FOUR)])
def test_simplex_matches_oracle(hip, mode, lanes, form, monkeypatch):
    # lanes: trial points spread over 4, 2 or 1 waves (merged across waves)
    monkeypatch.setenv("SBLM_NM_LANES", lanes)
    monkeypatch.setenv("SBLM_NM_SPEC_MAX", form)
    # ragged lengths including an empty lightcurve; starts near the truth,
    # one start on the domain's edges (0 and 1 coordinates)
    lengths = [300, 0, 257, 64, 300, 120, 300, 33]
    wl = inputs.uniform_workload(41, len(lengths), 300)
    ts, off = [], [0]
    for k, L in enumerate(lengths):
        ts.append(wl.t[k * 300:k * 300 + L])
        off.append(off[-1] + L)
    wl.t, wl.off = np.concatenate(ts), np.array(off, np.int64)
    wl.sfrac, wl.noise = wl.sfrac[:wl.t.size], wl.noise[:wl.t.size]
    y, w = oracle_lightcurves(wl)
    lcs = device_lcs(hip, wl, y, w)
    rng = np.random.default_rng(3)
    x0 = np.clip((wl.theta - LO[:, None]) / (HI - LO)[:, None]
                 + rng.normal(scale=0.02, size=wl.theta.shape), 0, 1)
    x0[:, 3] = [0.0, 1.0, 0.5, 1.0, 0.0, 0.4]
    cfg = hip.nm_default_config()
    cfg.max_iter, cfg.mode = 150, mode
    st = hip.new_stats()
    x, c, fs, fb, it = hip.nm_refine(lcs, LO, HI, torch.tensor(x0, device="cuda"), cfg,
                                     stats=st)
    x, c, fs, fb, it = (a.cpu().numpy() for a in (x, c, fs, fb, it))
    # every warm-started solve converged (or was solved again from the cold
    # start): no NaN magnification entered a chi^2
    assert hip.stats_dict(st)["n_capped"] == 0
    for k in range(len(lengths)):
        sl = slice(off[k], off[k + 1])
        xr, fr, steps, _, _ = _oracle_minimise(("matches", k), oracle_f(wl.t[sl], y[sl], w[sl]),
                                               x0[:, k], cfg)
        # the simplices follow from the accept/shrink decisions alone: the
        # same decisions give bit-identical vertices
        assert it[k] == steps, (k, it[k], steps)
        assert np.array_equal(x[:, k], xr), (k, x[:, k] - xr)
        tol = 1e-8 if mode == 0 else 1e-6
        assert abs(c[k] - fr) <= tol * max(abs(fr), 1e-300) + 1e-14 * np.sum(w[sl] * y[sl] ** 2)
    assert np.all(c <= np.array([oracle_f(wl.t[off[k]:off[k + 1]], y[off[k]:off[k + 1]],
                                          w[off[k]:off[k + 1]])(x0[:, k]) + 1e-9
                                 for k in range(len(lengths))]))


def test_ea_refine_improves_records_only(hip):
    wl = inputs.uniform_workload(42, 32, 400)
    y, w = oracle_lightcurves(wl)
    lcs = device_lcs(hip, wl, y, w)
    cfg = hip.ea_default_config()
    cfg.pop = 48
    st = hip.EAState(cfg, lcs, 5)
    st.fit(30)
    before = [(s.best_chi2, tuple(s.best_theta)) for s in st.summary()]
    P0 = st.view("P").clone()
    x0, c0 = st.best()
    it = st.refine()
    torch.cuda.synchronize()
    after = st.summary()
    assert torch.equal(P0, st.view("P"))  # the population is not touched
    th = torch.tensor(np.array([s.best_theta[:] for s in after]).T.copy(), device="cuda")
    c_new, fs_new, _ = hip.sblm_chi2(lcs, th, 1)
    c_new = c_new.cpu().numpy()
    n_better = 0
    for k, s in enumerate(after):
        assert s.best_chi2 <= before[k][0]
        if s.best_chi2 < before[k][0]:
            n_better += 1
            # the record is consistent: its chi^2 is that of its parameters
            assert abs(c_new[k] - s.best_chi2) <= 1e-9 * s.best_chi2
        else:
            assert tuple(s.best_theta) == before[k][1]
    assert n_better >= 16 and int(it.max()) > 0
    c_true = hip.sblm_chi2(lcs, torch.tensor(wl.theta.copy(), device="cuda"), 1)[0].cpu().numpy()
    ok_before = np.mean(np.array([b[0] for b in before]) <= c_true + 10)
    ok_after = np.mean(np.array([s.best_chi2 for s in after]) <= c_true + 10)
    print(f"success before/after the simplex: {ok_before:.3f} / {ok_after:.3f}")
    assert ok_after >= ok_before
    st.close()


@pytest.mark.parametrize("form", [ONE, FOUR])
def test_several_simplices_per_lightcurve(hip, form, monkeypatch):
    # nm_refine_multi: three starts per lightcurve (one lightcurve empty);
    # simplex k * 3 + i follows the oracle simplex on lightcurve k, with a
    # step's points evaluated one per round or all four at once
    monkeypatch.setenv("SBLM_NM_SPEC_MAX", form)
    lengths, reps = [200, 0, 150], 3
    wl = inputs.uniform_workload(43, len(lengths), 200)
    ts, off = [], [0]
    for k, L in enumerate(lengths):
        ts.append(wl.t[k * 200:k * 200 + L])
        off.append(off[-1] + L)
    wl.t, wl.off = np.concatenate(ts), np.array(off, np.int64)
    wl.sfrac, wl.noise = wl.sfrac[:wl.t.size], wl.noise[:wl.t.size]
    y, w = oracle_lightcurves(wl)
    lcs = device_lcs(hip, wl, y, w)
    rng = np.random.default_rng(8)
    x0 = rng.uniform(0.05, 0.95, (6, len(lengths) * reps))
    cfg = hip.nm_default_config()
    cfg.max_iter = 120
    x, c, fs, fb, it = (a.cpu().numpy() for a in
                        hip.nm_refine(lcs, LO, HI, torch.tensor(x0, device="cuda"), cfg,
                                      reps=reps))
    for k in range(len(lengths)):
        sl = slice(off[k], off[k + 1])
        for i in range(reps):
            j = k * reps + i
            xr, fr, steps, _, _ = _oracle_minimise(("several", j), oracle_f(wl.t[sl], y[sl], w[sl]),
                                                   x0[:, j], cfg)
            assert it[j] == steps, (k, i, it[j], steps)
            assert np.array_equal(x[:, j], xr), (k, i)
            assert abs(c[j] - fr) <= 1e-8 * max(abs(fr), 1e-300) + 1e-14 * np.sum(w[sl] * y[sl] ** 2)
    with pytest.raises(hip.SblmError):  # start points of the wrong shape
        hip.nm_refine(lcs, LO, HI, torch.tensor(x0[:, :4], device="cuda"), cfg, reps=reps)


@pytest.mark.parametrize("form", [ONE, FOUR])
def test_iterated_simplex_matches_oracle(hip, form, monkeypatch):
    # nm_iterated: 2 slots x 2 runs per lightcurve from Philox starts; the
    # best run, its start index order on ties and the total steps follow the
    # oracle's sequential loop over the same starts
    monkeypatch.setenv("SBLM_NM_SPEC_MAX", form)
    lengths = [180, 0, 120]
    wl = inputs.uniform_workload(44, len(lengths), 180)
    ts, off = [], [0]
    for k, L in enumerate(lengths):
        ts.append(wl.t[k * 180:k * 180 + L])
        off.append(off[-1] + L)
    wl.t, wl.off = np.concatenate(ts), np.array(off, np.int64)
    wl.sfrac, wl.noise = wl.sfrac[:wl.t.size], wl.noise[:wl.t.size]
    y, w = oracle_lightcurves(wl)
    lcs = device_lcs(hip, wl, y, w)
    cfg = hip.nm_default_config()
    cfg.max_iter = 60
    reps, runs, seed = 2, 2, 1234
    st = hip.new_stats()
    x, c, fs, fb, it = (a.cpu().numpy() for a in
                        hip.nm_iterated(lcs, LO, HI, reps, runs, seed, cfg, stats=st))
    assert hip.stats_dict(st)["n_capped"] == 0
    for k in range(len(lengths)):
        sl = slice(off[k], off[k + 1])
        xr, fr, total, s = NM.iterated(oracle_f(wl.t[sl], y[sl], w[sl]), seed, k, reps * runs,
                                       cfg.tol_x, cfg.tol_f, cfg.max_iter)
        assert it[k] == total, (k, it[k], total)
        assert np.array_equal(x[:, k], xr), (k, s)
        assert abs(c[k] - fr) <= 1e-8 * max(abs(fr), 1e-300) + 1e-14 * np.sum(w[sl] * y[sl] ** 2)
    with pytest.raises(hip.SblmError):
        hip.nm_iterated(lcs, LO, HI, 0, runs, seed, cfg)


def test_multi_and_iterated_full_size_sampled(hip):
    # the batched set (256 lightcurves x 1000 epochs) in the bench's launch
    # configurations: 8 simplices per lightcurve (the islands' fine-tuning),
    # sampled simplices against the oracle; the iterated simplex with 16
    # slots x 4 runs of up to 10^4 steps, checked by properties on samples
    wl = inputs.uniform_workload(2, 256, 1000)
    y, w = oracle_lightcurves(wl)
    lcs = device_lcs(hip, wl, y, w)
    rng = np.random.default_rng(12)
    reps = 8
    # starts near the truth, as the islands' records are: from random starts
    # a simplex can meet chi^2 values equal to rounding (flat regions far from
    # the data), where the accept decisions of two correct evaluations differ;
    # random starts are covered by the property checks below
    x_true = (wl.theta - LO[:, None]) / (HI - LO)[:, None]
    x0 = np.clip(np.repeat(x_true, reps, axis=1)
                 + rng.normal(scale=0.02, size=(6, wl.n_lc * reps)), 0, 1)
    cfg = hip.nm_default_config()
    x, c, fs, fb, it = (a.cpu().numpy() for a in
                        hip.nm_refine(lcs, LO, HI, torch.tensor(x0, device="cuda"), cfg,
                                      reps=reps))
    for j in (5, 1000, 2047):
        k = j // reps
        sl = slice(wl.off[k], wl.off[k + 1])
        xr, fr, steps, _, _ = NM.minimise(oracle_f(wl.t[sl], y[sl], w[sl]), x0[:, j],
                                          cfg.tol_x, cfg.tol_f, cfg.max_iter)
        assert it[j] == steps, (j, it[j], steps)
        assert np.array_equal(x[:, j], xr), j
        assert abs(c[j] - fr) <= 1e-8 * fr
    cfg.max_iter = 10000
    reps, runs, seed = 16, 4, 7
    st = hip.new_stats()
    x, c, fs, fb, it = (a.cpu().numpy() for a in
                        hip.nm_iterated(lcs, LO, HI, reps, runs, seed, cfg, stats=st))
    # from random starts far from the data, some sources cross caustics,
    # where two images merge and the root iteration stalls at the rounding
    # level next to a near-double root: those solves reach the cap with
    # settled roots; none may be unsettled (a NaN chi^2)
    s = hip.stats_dict(st)
    print(f"iterated simplex, full size: {s}")
    assert s["n_unsettled"] == 0 and s["n_capped"] <= 1e-4 * s["n_solves"]
    for k in (0, 128, 255):
        sl = slice(wl.off[k], wl.off[k + 1])
        f = oracle_f(wl.t[sl], y[sl], w[sl])
        # the reported point has the reported chi^2, no start is fitter than
        # the result, and every run took at least one step
        assert abs(f(x[:, k]) - c[k]) <= 1e-8 * c[k]
        for s in range(reps * runs):
            assert c[k] <= f(NM.start_point(seed, k, s)) * (1 + 1e-12)
        assert it[k] >= reps * runs


def test_iterated_simplex_repeatable_and_complete(hip):
    # slots take the next unstarted start of their lightcurve as their runs
    # end (3 slots x 3 runs, runs of different lengths): two calls agree bit
    # for bit, and the result is the oracle's best over all nine starts
    lengths = [150, 90]
    wl = inputs.uniform_workload(45, len(lengths), 150)
    ts, off = [], [0]
    for k, L in enumerate(lengths):
        ts.append(wl.t[k * 150:k * 150 + L])
        off.append(off[-1] + L)
    wl.t, wl.off = np.concatenate(ts), np.array(off, np.int64)
    wl.sfrac, wl.noise = wl.sfrac[:wl.t.size], wl.noise[:wl.t.size]
    y, w = oracle_lightcurves(wl)
    lcs = device_lcs(hip, wl, y, w)
    cfg = hip.nm_default_config()
    cfg.max_iter = 40
    reps, runs, seed = 3, 3, 99
    first = [a.cpu().numpy() for a in hip.nm_iterated(lcs, LO, HI, reps, runs, seed, cfg)]
    second = [a.cpu().numpy() for a in hip.nm_iterated(lcs, LO, HI, reps, runs, seed, cfg)]
    for a, b in zip(first, second):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    x, c, _, _, it = first
    for k in range(len(lengths)):
        sl = slice(off[k], off[k + 1])
        xr, fr, total, s = NM.iterated(oracle_f(wl.t[sl], y[sl], w[sl]), seed, k, reps * runs,
                                       cfg.tol_x, cfg.tol_f, cfg.max_iter)
        assert it[k] == total, (k, it[k], total)
        assert np.array_equal(x[:, k], xr), (k, s)
        assert abs(c[k] - fr) <= 1e-8 * max(abs(fr), 1e-300) + 1e-14 * np.sum(w[sl] * y[sl] ** 2)


def test_iterated_simplex_independent_of_slots(hip):
    # the same 4 starts per lightcurve run as (slots, runs) = (1, 4), (2, 2)
    # and (4, 1): every run begins its root solves cold, so a start's run,
    # its chi^2 values and steps do not depend on the slot that ran it or on
    # what ran there before -- bit-identical best point, chi^2 and steps
    lengths = [160, 0, 97, 160]
    wl = inputs.uniform_workload(46, len(lengths), 160)
    ts, off = [], [0]
    for k, L in enumerate(lengths):
        ts.append(wl.t[k * 160:k * 160 + L])
        off.append(off[-1] + L)
    wl.t, wl.off = np.concatenate(ts), np.array(off, np.int64)
    wl.sfrac, wl.noise = wl.sfrac[:wl.t.size], wl.noise[:wl.t.size]
    y, w = oracle_lightcurves(wl)
    lcs = device_lcs(hip, wl, y, w)
    cfg = hip.nm_default_config()
    cfg.max_iter = 50
    seed = 321
    outs = []
    for reps, runs in ((1, 4), (2, 2), (4, 1)):
        st = hip.new_stats()
        outs.append([a.cpu().numpy() for a in
                     hip.nm_iterated(lcs, LO, HI, reps, runs, seed, cfg, stats=st)])
        assert hip.stats_dict(st)["n_capped"] == 0
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    with pytest.raises(hip.SblmError):
        hip.nm_iterated(lcs, LO, HI, 1025, 1, seed, cfg)


def test_work_order_packing_beyond_one_block(hip, monkeypatch):
    # 4200 lightcurves x 4 simplices = 67 200 trial slots, beyond what one
    # block packs (65 536): the two-launch packing.  At 64 lanes (no saved
    # roots) a simplex's chi^2 values depend on its points alone, so every
    # simplex must match, bit for bit, the same simplex run in a small call
    # (one-block packing, four points per step), and one the oracle
    monkeypatch.setenv("SBLM_NM_LANES", "64")
    n_lc, L, reps = 4200, 40, 4
    wl = inputs.uniform_workload(47, n_lc, L)
    y, w = oracle_lightcurves(wl)
    lcs = device_lcs(hip, wl, y, w)
    rng = np.random.default_rng(14)
    x_true = (wl.theta - LO[:, None]) / (HI - LO)[:, None]
    x0 = np.clip(np.repeat(x_true, reps, axis=1)
                 + rng.normal(scale=0.05, size=(6, n_lc * reps)), 0, 1)
    cfg = hip.nm_default_config()
    cfg.max_iter = 40
    big = [a.cpu().numpy() for a in
           hip.nm_refine(lcs, LO, HI, torch.tensor(x0, device="cuda"), cfg, reps=reps)]
    assert int(big[4].min()) > 0
    for k in (0, 1234, n_lc - 1):
        sl = slice(wl.off[k], wl.off[k + 1])
        one = hip.Lightcurves(torch.tensor([0, L], dtype=torch.int64, device="cuda"),
                              torch.tensor(wl.t[sl], device="cuda"),
                              torch.tensor(y[sl], device="cuda"),
                              torch.tensor(w[sl], device="cuda"))
        cols = slice(k * reps, (k + 1) * reps)
        small = [a.cpu().numpy() for a in
                 hip.nm_refine(one, LO, HI, torch.tensor(x0[:, cols].copy(), device="cuda"), cfg,
                               reps=reps)]
        for u, v in zip(big, small):
            ref = np.ascontiguousarray(u[:, cols] if u.ndim == 2 else u[cols])
            assert np.array_equal(ref.view(np.uint8), np.ascontiguousarray(v).view(np.uint8)), k
    j = 1234 * reps + 2
    sl = slice(wl.off[1234], wl.off[1235])
    xr, fr, steps, _, _ = NM.minimise(oracle_f(wl.t[sl], y[sl], w[sl]), x0[:, j],
                                      cfg.tol_x, cfg.tol_f, cfg.max_iter)
    assert big[4][j] == steps
    assert np.array_equal(big[0][:, j], xr)

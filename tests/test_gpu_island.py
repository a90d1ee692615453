"""Island form of the device EA (Sec. 5.3) against the island oracle: the
migration, island-keyed generations and restarts bit for bit, the graph's
migration timing, the best-island records and island-keyed seeding."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from oracle import island_oracle as IS
from oracle import mlp_oracle as M
from tests.helpers import csr_workload, oracle_lightcurves

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _cuda(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def _state(hip, wl, pop, seed, n_isl, every, m, **kw):
    y, w = oracle_lightcurves(wl)
    lcs = hip.Lightcurves(_cuda(wl.off, torch.int64), _cuda(wl.t), _cuda(y), _cuda(w))
    cfg = hip.ea_default_config()
    cfg.pop, cfg.n_islands, cfg.mig_every, cfg.n_migrants = pop, n_isl, every, m
    for k, v in kw.items():
        setattr(cfg, k, v)
    return hip.EAState(cfg, lcs, seed), y, w


def _compare(hip, st, isls, pop):
    """Population rows and every island record against the island oracle."""
    _, P, rec = hip.parse_snapshot(st.save())
    n_isl = isls[0].n_isl
    for k, isl in enumerate(isls):
        cols = slice(k * n_isl * pop, (k + 1) * n_isl * pop)
        assert np.array_equal(P[:, cols].T, isl.rows()), k
        for i, ea in enumerate(isl.eas):
            s, r = ea.summary(), rec[k * n_isl + i]
            assert (r["gen"], r["gen_restart"], r["n_restarts"], r["stag_count"]) == \
                (s["gen"], s["gen_restart"], s["n_restarts"], s["stag_count"]), (k, i)
            assert r["p_mut"] == s["p_mut"] and r["best_chi2"] == s["best_chi2"]
            assert r["best_gen"] == s["best_gen"]
            if np.isfinite(s["best_chi2"]):
                assert np.array_equal(r["best_p"], s["best_p"])
    return rec


@pytest.mark.parametrize("n_isl,pop,m", [(3, 32, 4), (2, 17, 8), (5, 24, 1)])
def test_island_generations_bit_exact(hip, n_isl, pop, m):
    # given fitness with NaN and ties, then constant fitness (stagnation,
    # restarts); migration forced through ea_migrate when the oracle's rule
    # says it is due
    wl = csr_workload(8, [50, 70, 90])
    every = 4
    kw = dict(stag_window=3, restart_after=2)  # restarts come early and often
    st, _, _ = _state(hip, wl, pop, 555, n_isl, every, m, **kw)
    isls = [IS.IslandEA(n_isl, pop, 555, k, every, m, **kw) for k in range(3)]
    _compare(hip, st, isls, pop)
    rng = np.random.default_rng(11)
    n = 3 * n_isl * pop
    for g in range(30):
        if g < 18:
            chi2 = rng.uniform(10, 1000, n)
            chi2[rng.integers(0, n, 6)] = np.nan
            chi2[rng.integers(0, n, 3)] = np.inf
            chi2[1::11] = chi2[::11][: chi2[1::11].size]
        else:
            chi2 = np.full(n, 5.0)
        Fs, Fb = rng.uniform(0.5, 1.5, n), rng.uniform(0, 0.5, n)
        c, f, b = _cuda(chi2), _cuda(Fs), _cuda(Fb)
        if g > 0 and g % every == 0:
            st.migrate(c, f, b)
        st.generation(c, f, b)
        cc, ff, bb = c.cpu().numpy(), f.cpu().numpy(), b.cpu().numpy()
        for k, isl in enumerate(isls):
            sl = slice(k * n_isl * pop, (k + 1) * n_isl * pop)
            rc, rf, rb = isl.generation(chi2[sl], Fs[sl], Fb[sl])
            # the migrated fitness arrays agree as well
            assert np.array_equal(cc[sl], rc, equal_nan=True), (g, k)
            assert np.array_equal(ff[sl], rf) and np.array_equal(bb[sl], rb), (g, k)
        _compare(hip, st, isls, pop)
    assert all(ea.summary()["n_restarts"] >= 1 for isl in isls for ea in isl.eas)


def test_fit_graph_migrates_on_schedule(hip):
    # ea_fit replays evaluate + migration (when due) + generation; it must
    # equal stepping with an explicit migration on the oracle's schedule, and
    # the oracle island EA driven by the same fitness
    wl = csr_workload(9, [150, 333, 80])
    pop, n_isl, every, m = 24, 3, 3, 4
    st_a, y, w = _state(hip, wl, pop, 91, n_isl, every, m)
    st_b, _, _ = _state(hip, wl, pop, 91, n_isl, every, m)
    isls = [IS.IslandEA(n_isl, pop, 91, k, every, m) for k in range(3)]
    ngen = 11
    for g in range(ngen):
        st_b.evaluate()
        c = st_b.view("chi2").cpu().numpy().copy()
        f = st_b.view("Fs").cpu().numpy().copy()
        b = st_b.view("Fb").cpu().numpy().copy()
        if g > 0 and g % every == 0:
            st_b.migrate()
        st_b.generation(st_b.view("chi2"), st_b.view("Fs"), st_b.view("Fb"))
        for k, isl in enumerate(isls):
            sl = slice(k * n_isl * pop, (k + 1) * n_isl * pop)
            isl.generation(c[sl], f[sl], b[sl])
    st_a.fit(ngen)
    torch.cuda.synchronize()
    assert st_a.save() == st_b.save()
    rec = _compare(hip, st_b, isls, pop)
    # the per-lightcurve summary and ea_best take the best island's record
    summ = st_a.summary()
    x, c = st_a.best()
    x, c = x.cpu().numpy(), c.cpu().numpy()
    for k, isl in enumerate(isls):
        i, s = isl.best()
        assert summ[k].best_chi2 == s["best_chi2"] and summ[k].gen == ngen
        assert summ[k].n_restarts == rec[k * n_isl + i]["n_restarts"]
        assert c[k] == s["best_chi2"] and np.array_equal(x[:, k], s["best_p"])
        th = np.array(summ[k].best_theta[:])[:, None]
        sl = slice(wl.off[k], wl.off[k + 1])
        A, _ = O.magnify(th, wl.t[sl])
        co, _, _ = O.lsq_chi2(A[0], y[sl], w[sl])
        assert abs(co - summ[k].best_chi2) <= 1e-8 * co


def test_refine_every_island_record(hip):
    # ea_refine runs a simplex from every island's record; a record is
    # replaced exactly when its simplex ends fitter; ea_records reads them
    from oracle import nm_oracle as NM
    wl = csr_workload(10, [200, 260])
    pop, n_isl = 16, 4
    st, y, w = _state(hip, wl, pop, 3, n_isl, 2, 2)
    st.fit(12)
    _, _, rec0 = hip.parse_snapshot(st.save())
    xr0, cr0 = (a.cpu().numpy() for a in st.records())
    assert np.array_equal(xr0.T, rec0["best_p"]) and np.array_equal(cr0, rec0["best_chi2"])
    lo, hi = np.array(st.cfg.lo[:]), np.array(st.cfg.hi[:])
    cfg = hip.nm_default_config()
    cfg.max_iter = 100
    it = st.refine(cfg).cpu().numpy()
    torch.cuda.synchronize()
    _, _, rec1 = hip.parse_snapshot(st.save())
    for k in range(2):
        sl = slice(wl.off[k], wl.off[k + 1])
        off = np.array([0, sl.stop - sl.start], np.int64)
        f = lambda x: O.chi2(off, wl.t[sl], y[sl], w[sl],
                             O.decode(np.asarray(x, float)[:, None], lo, hi), 1,
                             nthreads=1)[0][0]
        for i in range(n_isl):
            v = k * n_isl + i
            xr, fr, steps, _, _ = NM.minimise(f, rec0["best_p"][v], cfg.tol_x, cfg.tol_f,
                                              cfg.max_iter)
            assert it[v] == steps, (k, i)
            if rec1["best_chi2"][v] < rec0["best_chi2"][v]:
                assert np.array_equal(rec1["best_p"][v], xr), (k, i)
                assert abs(rec1["best_chi2"][v] - fr) <= 1e-8 * fr
            else:
                assert rec1[v].tobytes() == rec0[v].tobytes()
                assert fr >= rec0["best_chi2"][v] * (1 - 1e-8)
    x1, c1 = st.best()
    assert np.array_equal(c1.cpu().numpy(),
                          rec1["best_chi2"].reshape(2, n_isl).min(axis=1))
    st.close()


def test_seeding_uses_island_keys(hip):
    wl = csr_workload(12, [80, 0, 300])
    pop, n_isl, n_seed = 16, 3, 5
    st, _, _ = _state(hip, wl, pop, 77, n_isl, 0, 0)
    P0 = st.view("P").cpu().numpy().copy()
    rng = np.random.default_rng(5)
    out = np.zeros((3, 128), np.float32)
    out[:, :8] = rng.normal(size=(3, 8))
    out[:, 8:64] = rng.uniform(-0.2, 1.2, (3, 56))
    out[:, 64:120] = rng.uniform(-4, -0.5, (3, 56))
    st.seed(torch.tensor(out, device=DEV), n_seed)
    torch.cuda.synchronize()
    P = st.view("P").cpu().numpy()
    lo, hi = np.array(st.cfg.lo[:]), np.array(st.cfg.hi[:])
    for k in range(3):
        for i in range(n_isl):
            cols = (k * n_isl + i) * pop + np.arange(pop)
            if wl.off[k + 1] == wl.off[k]:
                assert np.array_equal(P[:, cols], P0[:, cols])
                continue
            tf = wl.t[wl.off[k]]
            span = wl.t[wl.off[k + 1] - 1] - tf
            ref = M.seed_rows(out[k].astype(np.float64), tf, span, lo, hi, 77,
                              k * n_isl + i, n_seed)
            assert np.allclose(P[:, cols[:n_seed]].T, ref, rtol=0, atol=1e-12), (k, i)
            assert np.array_equal(P[:, cols[n_seed:]], P0[:, cols[n_seed:]])
    st.close()


def test_island_config_errors(hip):
    wl = csr_workload(13, [40])
    with pytest.raises(hip.SblmError):
        _state(hip, wl, 16, 1, 2, 1, 9)  # 2 m > pop
    with pytest.raises(hip.SblmError):
        _state(hip, wl, 16, 1, 0, 1, 1)  # no island
    st, _, _ = _state(hip, wl, 16, 1, 1, 1, 1)  # one island: nothing to migrate
    with pytest.raises(hip.SblmError):
        st.migrate()
    st.close()
    st, _, _ = _state(hip, wl, 16, 1, 2, 1, 1)
    lib = hip.load()
    c = st.view("chi2")
    rc = lib.ea_migrate(st.h, ctypes.c_void_p(c.data_ptr()), None, None, None)
    assert rc != 0  # some but not all fitness pointers
    st.close()


def test_islands_full_size_sampled(hip):
    # the batched set (256 lightcurves x 1000 epochs) with the islands of the
    # bench's comparison (8 x 32 rows, 2 migrants), migrating every
    # generation, in the bench's schedule; sampled lightcurves follow the
    # island oracle driven by the device fitness through a migration
    from paper_1208_4830_amd import inputs
    wl = inputs.uniform_workload(2, 256, 1000)
    pop, n_isl, m = 32, 8, 2
    st, _, _ = _state(hip, wl, pop, 7, n_isl, 1, m)
    st.set_schedule(16, 4, 1, 0)
    sample = [0, 97, 255]
    isls = {k: IS.IslandEA(n_isl, pop, 7, k, 1, m) for k in sample}
    for g in range(2):
        st.evaluate()
        c, f, b = (st.view(n).cpu().numpy().copy() for n in ("chi2", "Fs", "Fb"))
        st.fit(1)  # evaluates the same rows again, migrates when due, steps
        for k in sample:
            sl = slice(k * n_isl * pop, (k + 1) * n_isl * pop)
            isls[k].generation(c[sl], f[sl], b[sl])
    torch.cuda.synchronize()
    _, P, rec = hip.parse_snapshot(st.save())
    for k in sample:
        cols = slice(k * n_isl * pop, (k + 1) * n_isl * pop)
        assert np.array_equal(P[:, cols].T, isls[k].rows()), k
        i, s = isls[k].best()
        assert rec["best_chi2"][k * n_isl + i] == s["best_chi2"]
    st.close()


def test_island_save_load_resume_bit_exact(hip):
    # a snapshot taken between migrations restores a state whose continued
    # run (migrations included) is bit-identical to the uninterrupted one
    wl = csr_workload(14, [90, 150])
    st_a, _, _ = _state(hip, wl, 16, 21, 3, 2, 2)
    st_a.fit(5)
    blob = st_a.save()
    st_a.fit(6)
    st_b, _, _ = _state(hip, wl, 16, 21, 3, 2, 2)
    st_b.load(blob)
    st_b.fit(6)
    torch.cuda.synchronize()
    assert st_a.save() == st_b.save()
    # a snapshot of another island configuration is refused
    st_c, _, _ = _state(hip, wl, 16, 21, 3, 3, 2)
    with pytest.raises(hip.SblmError):
        st_c.load(blob)
    for st in (st_a, st_b, st_c):
        st.close()

"""Bit-exact parity of the device EA (Appendix A) with the oracle EA, given
identical fitness, and of graph-replayed fits with stepped ones."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1208_4830_amd import inputs
from tests.helpers import csr_workload, oracle_lightcurves, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _cuda(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def test_philox_draws_bit_exact(hip):
    rng = np.random.default_rng(0)
    for _ in range(12):
        seed, lc, gen, purpose, row = (int(x) for x in rng.integers(0, 2 ** 40, 5))
        j0 = int(rng.integers(0, 64))
        got = hip.ea_draws(seed, lc, gen, purpose, row, j0, 37).cpu().numpy().view(np.uint64)
        ref = np.array([O.draw(seed, lc, gen, purpose, row, j0 + k) for k in range(37)],
                       dtype=np.uint64)
        assert np.array_equal(got, ref)
    # and against numpy's Philox4x64-10 (counter pre-incremented by numpy)
    key = np.array([99, 3], dtype=np.uint64)
    bg = np.random.Philox(key=key, counter=np.array([4, 2, 7, 0], dtype=np.uint64))
    ref = bg.random_raw(4)
    got = hip.ea_draws(99, 3, 5, 2, 7, 0, 4).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, ref)


def _make_state(hip, wl, pop, seed, mode=0, **kw):
    y, w = oracle_lightcurves(wl)
    lcs = hip.Lightcurves(_cuda(wl.off, torch.int64), _cuda(wl.t), _cuda(y), _cuda(w))
    cfg = hip.ea_default_config()
    cfg.pop = pop
    cfg.mode = mode
    for k, v in kw.items():
        setattr(cfg, k, v)
    return hip.EAState(cfg, lcs, seed), y, w


def _oracle_eas(n_lc, pop, seed, **kw):
    return [O.EA(pop, seed, lc, **kw) for lc in range(n_lc)]


def _population_rows(P, lc, pop):
    """[pop][6] rows of lightcurve lc from the device layout [6][n_lc*pop]."""
    return P[:, lc * pop:(lc + 1) * pop].T


def _compare(hip, st, eas, pop):
    _, P, rec = hip.parse_snapshot(st.save())
    for lc, ea in enumerate(eas):
        assert np.array_equal(_population_rows(P, lc, pop), ea.P), lc
        s = ea.summary()
        r = rec[lc]
        assert r["gen"] == s["gen"] and r["gen_restart"] == s["gen_restart"]
        assert r["p_mut"] == s["p_mut"] and r["stag_count"] == s["stag_count"]
        assert r["n_restarts"] == s["n_restarts"]
        assert r["best_chi2"] == s["best_chi2"] and r["best_gen"] == s["best_gen"]
        if np.isfinite(s["best_chi2"]):
            assert np.array_equal(r["best_p"], s["best_p"])
    return P


@pytest.mark.parametrize("pop", [48, 49, 128])
def test_init_and_generations_bit_exact(hip, pop):
    wl = csr_workload(5, [50, 70, 90])
    st, _, _ = _make_state(hip, wl, pop, seed=1234)
    eas = _oracle_eas(3, pop, 1234)
    _compare(hip, st, eas, pop)
    rng = np.random.default_rng(9)
    npair = pop // 2
    for g in range(40):
        if g < 15:  # random fitness with ties, NaN and inf
            chi2 = rng.uniform(10, 1000, 3 * pop)
            chi2[rng.integers(0, 3 * pop, 5)] = np.nan
            chi2[rng.integers(0, 3 * pop, 3)] = np.inf
            chi2[::7] = chi2[1::7][: chi2[::7].size] if pop > 7 else chi2[::7]
        else:  # constant fitness: stagnation flags, p_mut boosts, a restart
            chi2 = np.full(3 * pop, 5.0)
        Fs, Fb = rng.uniform(0.5, 1.5, 3 * pop), rng.uniform(0, 0.5, 3 * pop)
        parents = torch.zeros(3 * 2 * npair, dtype=torch.int32, device=DEV)
        st.generation_traced(_cuda(chi2), _cuda(Fs), _cuda(Fb), parents)
        par = parents.cpu().numpy().reshape(3, 2 * npair)
        for lc, ea in enumerate(eas):
            sl = slice(lc * pop, (lc + 1) * pop)
            ref = ea.generation(chi2[sl], Fs[sl], Fb[sl])
            if ea.summary()["gen_restart"] != g + 1:  # restarts skip reproduction
                assert np.array_equal(par[lc], ref), (g, lc)
        _compare(hip, st, eas, pop)
    assert all(ea.summary()["n_restarts"] >= 1 for ea in eas)


def test_fit_graph_equals_stepping_and_oracle(hip):
    # ea_fit (graph replay of evaluate + generation) must equal stepping
    # generation by generation with sblm_chi2 on the decoded population, and
    # the population must equal the oracle EA driven by the same fitness
    wl = csr_workload(6, [120, 333, 400])
    pop = 48
    st_a, y, w = _make_state(hip, wl, pop, seed=77)
    st_b, _, _ = _make_state(hip, wl, pop, seed=77)
    cfg = st_a.cfg
    lo = np.array(cfg.lo[:])
    hi = np.array(cfg.hi[:])
    eas = _oracle_eas(3, pop, 77)
    ngen = 12
    for g in range(ngen):
        _, P, _ = hip.parse_snapshot(st_b.save())
        theta = O.decode(P, lo, hi)
        c, fs, fb = hip.sblm_chi2(st_b.lcs, _cuda(theta), pop)
        if g == 0:  # GPU fitness of the stepped population vs the oracle's
            co, _, _ = O.chi2(wl.off, wl.t, y, w, theta, pop)
            assert np.all(rel_err(c.cpu().numpy(), co) < 1e-8)
        st_b.generation(c, fs, fb)
        cc, ff, bb = c.cpu().numpy(), fs.cpu().numpy(), fb.cpu().numpy()
        for lc, ea in enumerate(eas):
            sl = slice(lc * pop, (lc + 1) * pop)
            ea.generation(cc[sl], ff[sl], bb[sl])
    st_a.fit(ngen)
    torch.cuda.synchronize()
    blob_a, blob_b = st_a.save(), st_b.save()
    assert blob_a == blob_b
    _compare(hip, st_b, eas, pop)
    summ = st_a.summary()
    for lc in range(3):
        assert summ[lc].gen == ngen
        # best chi2 re-evaluated by the oracle at the decoded best parameters
        th = np.array(summ[lc].best_theta[:])[:, None]
        sl = slice(wl.off[lc], wl.off[lc + 1])
        A, _ = O.magnify(th, wl.t[sl])
        co, fso, fbo = O.lsq_chi2(A[0], y[sl], w[sl])
        assert rel_err(summ[lc].best_chi2, co) < 1e-8


def test_save_load_resume_bit_exact(hip):
    wl = csr_workload(8, [200, 250])
    pop = 64
    st, _, _ = _make_state(hip, wl, pop, seed=5)
    st.fit(7)
    snap = st.save()
    st.fit(9)
    final = st.save()
    st2, _, _ = _make_state(hip, wl, pop, seed=5)
    st2.load(snap)
    st2.fit(9)
    assert st2.save() == final
    # a snapshot does not load into a state with another seed
    st3, _, _ = _make_state(hip, wl, pop, seed=6)
    with pytest.raises(hip.SblmError):
        st3.load(snap)


@pytest.mark.parametrize("n_isl", [1, 2])
def test_freeze_skips_only_the_frozen_lightcurves(hip, n_isl):
    # two lightcurves frozen after 6 generations (with islands: migration
    # every 3 generations), one of them resumed after 12: the others evolve
    # bit for bit as in a fit without the freeze; a frozen lightcurve's
    # population and records stay as they were; the resumed one continues as
    # the unfrozen fit did from the same point
    wl = csr_workload(10, [150, 300, 0, 220, 180, 260])
    pop, n = 32, 6
    kw = dict(n_islands=2, mig_every=3, n_migrants=2) if n_isl > 1 else {}
    a, _, _ = _make_state(hip, wl, pop, seed=3, **kw)
    b, _, _ = _make_state(hip, wl, pop, seed=3, **kw)
    rows, recs = pop * n_isl, n_isl

    def snap(st):
        _, P, rec = hip.parse_snapshot(st.save())
        return P, rec

    def part(P, rec, k):
        return P[:, k * rows:(k + 1) * rows].copy(), rec[k * recs:(k + 1) * recs].tobytes()

    a.fit(6)
    b.fit(6)
    P6, r6 = snap(b)
    frozen = [0, 1, 0, 0, 1, 0]
    b.freeze(frozen)
    a.fit(6)
    b.fit(6)
    Pa, ra = snap(a)
    Pb, rb = snap(b)
    x_b, c_b = (t.cpu().numpy() for t in b.best())
    for k in range(n):
        pb, qb = part(Pb, rb, k)
        pr, qr = part(P6, r6, k) if frozen[k] else part(Pa, ra, k)
        assert np.array_equal(pb, pr) and qb == qr, k
    # ea_best of a frozen lightcurve: its record from before the freeze
    for k in (1, 4):
        best6 = min(r6[k * recs:(k + 1) * recs]["best_chi2"])
        assert c_b[k] == best6
    # resume lightcurve 1 for 6 generations: as the unfrozen fit's 6 to 12
    b.freeze([0, 0, 0, 0, 1, 0])
    b.fit(6)
    Pb2, rb2 = snap(b)
    p1, q1 = part(Pb2, rb2, 1)
    pa1, qa1 = part(Pa, ra, 1)
    assert np.array_equal(p1, pa1) and q1 == qa1
    pb4, qb4 = part(Pb2, rb2, 4)
    p64, q64 = part(P6, r6, 4)
    assert np.array_equal(pb4, p64) and qb4 == q64
    with pytest.raises(hip.SblmError):  # a mask of another length
        b.freeze([0, 1])
    # everything frozen: generations change nothing
    b.freeze([1] * n)
    before = b.save()
    b.fit(3)
    assert b.save() == before


@pytest.mark.parametrize("mode", [0, 1])
def test_fit_improves_and_best_is_monotone(hip, mode):
    # one paper-shaped lightcurve: 400 uniform epochs over t0 +- 2 tE,
    # sigma = 1% of the flux, population 48
    wl = inputs.uniform_workload(1, 1, 400)
    st, y, w = _make_state(hip, wl, 48, seed=1, mode=mode)
    best = []
    for _ in range(10):
        st.fit(10)
        best.append(st.summary()[0].best_chi2)
    assert all(b2 <= b1 for b1, b2 in zip(best, best[1:]))
    A, _ = O.magnify(wl.theta[:, :1], wl.t)
    chi2_true, _, _ = O.lsq_chi2(A[0], y, w)
    assert best[-1] < best[0] and np.isfinite(best[-1]) and chi2_true > 0


# every schedule ea_set_schedule accepts, by lanes per individual
_SCHEDULES = {g: [(g, wpb, pers, asy) for wpb in (1, 2, 4) for pers in (1, 0) for asy in (0, 1)]
              for g in (8, 16, 32, 64)}
_SCHEDULES[128] = [(128, 2, 0, 0), (128, 4, 0, 0)]
_SCHEDULES[256] = [(256, 4, 0, 0)]


@pytest.mark.parametrize("mode", [0, 1])
def test_schedules_agree_and_autotune(hip, mode):
    # The knobs the autotuner turns -- epoch stepping (lockstep or
    # asynchronous), waves per block, persistent or one-shot grid -- do not
    # change a result bit, in either precision form: a fit is the same under
    # every schedule with the same lanes per individual (those set where each
    # lane's chain of warm starts begins, so they are part of the fit).
    wl = csr_workload(9, [0, 5, 64, 201, 777, 1500, 3000])
    pop = 32
    lanes_all = (8, 16, 32, 64, 128, 256) if mode == 0 else (16, 128)
    blobs = {}
    for g in lanes_all:
        for sched in _SCHEDULES[g]:
            if mode == 1 and g == 16 and sched[1] == 2:
                continue  # (bounded run time; every stepping and grid form is still covered)
            st, y, w = _make_state(hip, wl, pop, seed=21, mode=mode)
            st.set_schedule(*sched)
            assert st.schedule() == sched
            st.fit(6)
            blobs[sched] = st.save()
            if sched == _SCHEDULES[g][0]:
                # one schedule per lanes value against the oracle's chi^2
                st.evaluate()
                c = st.view("chi2").cpu().numpy().copy()
                P = st.view("P").cpu().numpy()
                theta = O.decode(P, np.array(st.cfg.lo[:]), np.array(st.cfg.hi[:]))
                co, _, _ = O.chi2(wl.off, wl.t, y, w, theta, pop)
                scale = np.array([np.sum(w[wl.off[k]:wl.off[k + 1]] * y[wl.off[k]:wl.off[k + 1]] ** 2)
                                  for k in range(wl.n_lc)]).repeat(pop)
                tol = 1e-8 if mode == 0 else 1e-6
                assert np.all(np.abs(c - co) <= tol * co + 1e-14 * scale), sched
            st.close()
        ref = blobs[_SCHEDULES[g][0]]
        for sched in _SCHEDULES[g]:
            if sched in blobs:
                assert blobs[sched] == ref, (sched, _SCHEDULES[g][0])
    # the autotuner keeps the lanes and lands on a schedule of the same bits
    st, _, _ = _make_state(hip, wl, pop, seed=21, mode=mode)
    assert st.schedule() == (256, 4, 0, 0)  # a small state starts wide
    st.set_schedule(16, 4, 1, 0)
    rep = st.autotune()
    lanes, wpb, pers, asy = st.schedule()
    # the start, stepping (2), waves per block (3), launch form (2), chosen
    assert "chosen:" in rep and len(rep.splitlines()) == 9
    assert lanes == 16 and wpb in (1, 2, 4) and pers in (0, 1) and asy in (0, 1)
    st.fit(6)
    assert st.save() == blobs[(16, 4, 1, 0)]
    st.close()
    st, _, _ = _make_state(hip, wl, pop, seed=21, mode=mode)
    rep = st.autotune()  # wide: waves per block 4 only (one-shot, lockstep)
    assert st.schedule() == (256, 4, 0, 0) and len(rep.splitlines()) == 5
    with pytest.raises(hip.SblmError):  # blocks beyond the kernels' bound
        st.set_schedule(16, 8, 1)
    for bad in ((256, 2, 0, 0), (256, 4, 1, 0), (128, 4, 0, 1)):
        with pytest.raises(hip.SblmError):  # wide lanes: whole individuals, one-shot, lockstep
            st.set_schedule(*bad)
    st.close()


def test_autotune_keeps_its_choice(hip, tmp_path):
    # ea_autotune_cached: the first state of a workload is tuned and its
    # choice kept in the file; a second state of the same workload installs
    # it without timing, and the fit is the same bits either way
    wl = csr_workload(9, [0, 5, 64, 201, 777, 1500, 3000])
    path = tmp_path / "schedules.txt"
    st1, _, _ = _make_state(hip, wl, 32, seed=21)
    st1.set_schedule(16, 4, 1, 0)
    rep1 = st1.autotune(cache=path)
    assert "chosen:" in rep1
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split()[1:5] == [str(v) for v in st1.schedule()]
    st1.fit(6)
    st2, _, _ = _make_state(hip, wl, 32, seed=21)
    st2.set_schedule(16, 1, 0, 1)  # what the kept choice replaces
    assert st2.autotune(cache=path).startswith("kept:")
    assert st2.schedule() == st1.schedule() and len(path.read_text().splitlines()) == 1
    st2.fit(6)
    assert st2.save() == st1.save()
    # another workload (population) is another key: tuned and appended
    st3, _, _ = _make_state(hip, wl, 48, seed=21)
    assert "chosen:" in st3.autotune(cache=path)
    assert len(path.read_text().splitlines()) == 2
    # a kept entry whose lanes differ from the state's is refused (the lanes
    # are part of the fit, not of the schedule); the first matching line wins
    key = lines[0].split()[0]
    path.write_text(f"{key} 64 4 1 0 edited\n" + path.read_text())
    st4, _, _ = _make_state(hip, wl, 32, seed=21)
    st4.set_schedule(16, 4, 1, 0)  # (the key covers the state's lanes)
    with pytest.raises(hip.SblmError, match="lanes"):
        st4.autotune(cache=path)
    for st in (st1, st2, st3, st4):
        st.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_ragged_full_size_sampled(hip, mode):
    # 4096 lightcurves of 200-5000 epochs with survey-like cadence and
    # 0.5-3% errors, population 128: the persistent longest-first schedule
    # of ea_evaluate on the full batch, sampled individuals vs the oracle
    wl = inputs.ragged_workload(4, 4096)
    rng = np.random.default_rng(8)
    pick = rng.choice(4096, 24, replace=False)
    # observations of the sampled lightcurves from the oracle; the rest are
    # filled with the same recipe so the batch has its full shape
    y = np.ones_like(wl.t)
    w = np.ones_like(wl.t)
    for k in pick:
        sl = slice(wl.off[k], wl.off[k + 1])
        A, _ = O.magnify(wl.theta[:, k:k + 1], wl.t[sl])
        F = wl.Fs[k] * A[0] + wl.Fb[k]
        y[sl] = F + wl.sfrac[sl] * F * wl.noise[sl]
        w[sl] = 1 / (wl.sfrac[sl] * F) ** 2
    lcs = hip.Lightcurves(_cuda(wl.off, torch.int64), _cuda(wl.t), _cuda(y), _cuda(w))
    cfg = hip.ea_default_config()
    cfg.pop = 128
    cfg.mode = mode
    st = hip.EAState(cfg, lcs, 3)
    assert st.schedule()[2] == 1
    st.evaluate()
    c = st.view("chi2").cpu().numpy()
    P = st.view("P").cpu().numpy()
    lo, hi = np.array(cfg.lo[:]), np.array(cfg.hi[:])
    for k in pick:
        for i in rng.choice(128, 2, replace=False):
            col = k * 128 + i
            th = O.decode(P[:, col:col + 1], lo, hi)
            sl = slice(wl.off[k], wl.off[k + 1])
            A, _ = O.magnify(th, wl.t[sl])
            co, _, _ = O.lsq_chi2(A[0], y[sl], w[sl])
            assert rel_err(c[col], co) < 1e-8, (k, i, c[col], co)
    # the stateless call on the decoded population takes the state's lanes
    # per individual (8 here) and gives its chi^2 bit for bit
    assert st.schedule()[0] == 8
    theta = O.decode(P, lo, hi)
    c_api, _, _ = hip.sblm_chi2(lcs, _cuda(theta), 128, mode)
    assert np.array_equal(c_api.cpu().numpy(), c)
    st.close()


def test_fitness_timer_leaves_the_fit_unchanged(hip):
    # the device-clock stamps around the fitness kernel (ea_time_fitness)
    # count every replayed launch, give a duration near the event-timed one
    # of the same kernel, and change nothing in the fit
    wl = csr_workload(16, [300, 0, 511, 1200, 64])
    pop = 64
    st_a, _, _ = _make_state(hip, wl, pop, seed=5)
    st_b, _, _ = _make_state(hip, wl, pop, seed=5)
    st_a.time_fitness(True)
    stats = hip.new_stats()
    st_a.fit(0, stats=stats)  # captures only
    assert st_a.fitness_time() == (0.0, 0)
    st_a.fit(20, stats=stats)
    st_b.fit(20)
    torch.cuda.synchronize()
    assert st_a.save() == st_b.save()
    ms, n = st_a.fitness_time()
    assert n == 20 and ms > 0.0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    for _ in range(20):
        st_b.evaluate(stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ev_ms = e0.elapsed_time(e1) / 20
    print(f"fitness kernel: stamped {ms / n:.4f} ms, events {ev_ms:.4f} ms")
    assert 0.3 * ev_ms < ms / n < 3.0 * ev_ms
    # switching the stamps off clears the sums and stops counting
    st_a.time_fitness(False)
    st_a.fit(3)
    assert st_a.fitness_time() == (0.0, 0)
    assert hip.stats_dict(stats)["n_solves"] > 0
    st_a.close()
    st_b.close()

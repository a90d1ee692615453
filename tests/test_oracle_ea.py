"""Pins of the oracle's random numbers and evolutionary operators (Appendix A)
against independent implementations and the stated properties."""
import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest
from scipy import stats

import oracle as O
from oracle import oracle as OO

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def fma(a, b, c):
    """a*b + c rounded once (exact rational arithmetic, then nearest double)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def test_philox_matches_numpy():
    # numpy's Philox is Philox4x64-10; it increments the counter before
    # producing a block, so its first block for counter c is Philox(c + 1)
    rng = np.random.default_rng(0)
    for _ in range(20):
        key = rng.integers(0, 2 ** 63, 2, dtype=np.uint64)
        ctr = rng.integers(0, 2 ** 62, 4, dtype=np.uint64)
        bg = np.random.Philox(key=key, counter=ctr)
        ref = bg.random_raw(4)
        c1 = ctr.copy()
        c1[0] += np.uint64(1)
        assert np.array_equal(O.philox4x64_10(c1, key), ref)


def test_draw_layout():
    # word j%4 of the block at counter (gen, purpose, row, j//4), key (seed, lc)
    seed, lc, gen, purpose, row = 12345, 7, 33, 3, 19
    for j in range(10):
        blk = O.philox4x64_10([gen, purpose, row, j // 4], [seed, lc])
        assert O.draw(seed, lc, gen, purpose, row, j) == int(blk[j % 4])


def test_uniform_and_integer_maps():
    assert O.u01(0) == 0.5 * 2.0 ** -52
    assert O.u01(2 ** 64 - 1) == 1.0 - 0.5 * 2.0 ** -52
    assert 0.0 < O.u01(2 ** 64 - 1) < 1.0
    for n in (1, 2, 3, 48, 1000):
        assert O.below(0, n) == 0 and O.below(2 ** 64 - 1, n) == n - 1


def _coeff_table(path, name):
    src = open(path).read()
    body = src[src.index(name):]
    body = body[body.index("{") + 1: body.index("}")]
    return [float.fromhex(x.strip()) for x in body.split(",") if x.strip()]


def test_exp2_coefficients_are_rounded_taylor_terms():
    # coefficient n is (-ln 2)^n / n! rounded to the nearest double
    mpmath.mp.prec = 200
    table = _coeff_table(os.path.join(ROOT, "oracle", "ea_oracle.c"), "EXP2_NEG_TAYLOR")
    assert len(table) == 17
    for n, c in enumerate(table):
        exact = (-mpmath.log(2)) ** n / mpmath.factorial(n)
        assert abs(mpmath.mpf(c) - exact) <= mpmath.mpf(math.ulp(c)) / 2


def test_exp2_neg_accuracy():
    mpmath.mp.prec = 120
    rng = np.random.default_rng(1)
    for v in np.concatenate([rng.uniform(0, 52, 2000), [0.0, 1.0, 51.999, 0.5]]):
        x = O.exp2_neg(float(v))
        exact = mpmath.power(2, -mpmath.mpf(float(v)))
        assert abs(mpmath.mpf(x) / exact - 1) < 4 * 2.0 ** -53


def test_initial_population_is_antithetic():
    for pop in (48, 49, 256):
        ea = O.EA(pop, seed=5, lc=2)
        P = ea.P
        h = pop // 2
        assert np.all((P > 0) & (P < 1))
        assert np.array_equal(P[h:2 * h], 1.0 - P[:h])
        if pop % 2 == 0:
            assert np.allclose(P.mean(0), 0.5, rtol=0, atol=1e-14)
        # first row is draw (gen 0, purpose 1, row 0, gene g)
        for g in range(6):
            assert P[0, g] == O.u01(O.draw(5, 2, 0, 1, 0, g))


def test_elitism_clone_and_bounds():
    rng = np.random.default_rng(2)
    ea = O.EA(48, seed=9, lc=0)
    best_prev = np.inf
    for gen in range(30):
        chi2 = rng.uniform(10, 100, 48)
        P_old = ea.P.copy()
        parents = ea.generation(chi2)
        best = np.argmin(chi2)
        # row 0 of the next population is the fittest row, untouched
        assert np.array_equal(ea.P[0], P_old[best])
        assert np.all((ea.P >= 0) & (ea.P <= 1))
        assert np.all((parents >= 0) & (parents < 48))
        best_prev = min(best_prev, chi2.min())
        assert ea.summary()["best_chi2"] == best_prev


def test_nan_ranks_last():
    ea = O.EA(8, seed=1, lc=0)
    P0 = ea.P.copy()
    chi2 = np.array([np.nan, 5.0, np.nan, 3.0, 3.0, 9.0, np.inf, 4.0])
    ea.generation(chi2)
    # elite = first of the tied minimum (row 3), never a NaN row
    assert np.array_equal(ea.P[0], P0[3])
    assert ea.summary()["best_chi2"] == 3.0


def test_monotone_transform_invariance():
    # selection is rank based: any order-preserving transform of the fitness
    # gives the same trajectory while no stagnation test has fired (the
    # first `window` generations)
    rng = np.random.default_rng(3)
    a, b = O.EA(64, seed=4, lc=1), O.EA(64, seed=4, lc=1)
    for _ in range(9):
        chi2 = rng.uniform(1, 1000, 64)
        pa = a.generation(chi2)
        pb = b.generation(np.sqrt(chi2) * 3 - 7)
        assert np.array_equal(pa, pb) and np.array_equal(a.P, b.P)


def test_tournament_rank_distribution():
    # parent rank = min of N_tourn uniform draws from {0..N-1}:
    # P(rank >= r) = ((N - r)/N)^N_tourn
    N, nt = 100, 4  # N_tourn = ceil(100/25)
    ea = O.EA(N, seed=11, lc=3, p_mut0=0.0, p_mut_min=0.0)
    counts = np.zeros(N)
    rng = np.random.default_rng(4)
    for _ in range(200):
        parents = ea.generation(rng.uniform(1, 2, N))
        counts += np.bincount(parents, minlength=N)
    r = np.arange(N + 1)
    cdf_ge = ((N - r) / N) ** nt
    p = cdf_ge[:-1] - cdf_ge[1:]
    # pool the tail to keep expected counts >= 5
    exp = p * counts.sum()
    k = np.searchsorted(-exp, -5.0)
    obs = np.concatenate([counts[:k], [counts[k:].sum()]])
    ex = np.concatenate([exp[:k], [exp[k:].sum()]])
    assert stats.chisquare(obs, ex).pvalue > 1e-4


def test_creep_step_is_log_uniform():
    # ln X ~ U(ln eps, 0): -log2(X)/52 is uniform on (0,1)
    rng = np.random.default_rng(5)
    v = np.array([O.u01(int(x)) for x in rng.integers(0, 2 ** 64, 4000, dtype=np.uint64)])
    X = np.array([O.exp2_neg(52.0 * u) for u in v])
    assert np.all((X > 2.0 ** -52) & (X < 1.0))
    assert stats.kstest(-np.log2(X) / 52.0, "uniform").pvalue > 1e-4


def test_jump_rate():
    # with clone-free inputs, a gene equal to a fresh uniform draw of the
    # jump stream marks a jump; its frequency is p_mut
    pop, pm = 64, 0.2
    ea = O.EA(pop, seed=6, lc=0, p_mut0=pm, p_mut_min=pm, p_mut_max=pm)
    n_jump = n_tot = 0
    rng = np.random.default_rng(7)
    for g in range(20):
        ea.generation(rng.uniform(1, 2, pop))
        for i in range(1, pop):
            for j in range(6):
                jv = O.u01(O.draw(6, 0, g, 5, i, 2 * j + 1))
                n_jump += ea.P[i, j] == jv
                n_tot += 1
    frac = n_jump / n_tot
    assert abs(frac - pm) < 4 * math.sqrt(pm * (1 - pm) / n_tot)


def test_forced_stagnation_restarts():
    # constant fitness never improves: flags start `window` generations into
    # a sequence and a restart follows `restart_after` consecutive flags,
    # i.e. every 20 generations with the defaults
    pop = 16
    ea = O.EA(pop, seed=3, lc=5)
    restarts = []
    for g in range(65):
        ea.generation(np.full(pop, 7.0))
        s = ea.summary()
        if s["gen_restart"] == g + 1:
            restarts.append(g + 1)
            # the fresh population is the initialisation keyed by generation g+1
            for gene in range(6):
                assert ea.P[0, gene] == O.u01(O.draw(3, 5, g + 1, 1, 0, gene))
            assert s["p_mut"] == 0.01 and s["stag_count"] == 0
    assert restarts == [20, 40, 60]
    assert ea.summary()["n_restarts"] == 3


def test_p_mut_boost_and_throttle():
    pop = 16
    ea = O.EA(pop, seed=3, lc=5)
    for g in range(10):  # steady 5% improvement per generation
        ea.generation(np.full(pop, 100.0 * 0.95 ** g))
    assert ea.summary()["p_mut"] == 0.01  # no test before the window is full
    ea.generation(np.full(pop, 100.0 * 0.95 ** 10))
    assert ea.summary()["p_mut"] == 0.005  # improved > 1% over 10 generations
    ea.generation(np.full(pop, 100.0 * 0.95 ** 10))  # b(11) vs b(1): improved
    assert ea.summary()["p_mut"] == 0.0025


def test_clone_mode_copies_parents_bit_exactly():
    # mode 2 (all ones) copies the parents; creep is then the only change,
    # and creep with X -> 0 is the identity: check via the draw stream
    pop = 32
    ea = O.EA(pop, seed=21, lc=4, p_mut0=0.0, p_mut_min=0.0)
    P_old = ea.P.copy()
    chi2 = np.arange(pop, dtype=float)  # identity ranking
    parents = ea.generation(chi2)
    nt = math.ceil(pop / 25)
    for k in range(pop // 2):
        mode = O.below(O.draw(21, 4, 0, 3, k, 0), 3)
        if mode != 2:
            continue
        ra, rb = parents[2 * k], parents[2 * k + 1]
        for slot, src in ((2 * k + 1, ra), (2 * k + 2, rb)):
            if slot >= pop:
                continue
            for g in range(6):
                p = P_old[src, g]
                xs = O.draw(21, 4, 0, 4, slot, 2 * g)
                X = O.exp2_neg(52.0 * O.u01(O.draw(21, 4, 0, 4, slot, 2 * g + 1)))
                exp = fma(1.0 - p, X, p) if xs >> 63 else fma(-p, X, p)
                assert ea.P[slot, g] == min(max(exp, 0.0), 1.0)
    assert nt == 2


def _creep_inputs(seed, lc, slot, g):
    """Sign bit and factor X of the creep of gene g of row `slot` (App. A.6)."""
    xs = O.draw(seed, lc, 0, 4, slot, 2 * g)
    X = O.exp2_neg(52.0 * O.u01(O.draw(seed, lc, 0, 4, slot, 2 * g + 1)))
    return xs >> 63, X


def _uncreep(p_out, plus, X):
    """The gene before a creep with factor X (None where the creep lost it:
    X close to 1, or the result clamped)."""
    if X > 0.5 or p_out in (0.0, 1.0):
        return None
    return (p_out - X) / (1.0 - X) if plus else p_out / (1.0 - X)


def _crossover_generation(pop, seed, lc):
    ea = O.EA(pop, seed=seed, lc=lc, p_mut0=0.0, p_mut_min=0.0)  # no jumps
    P_old = ea.P.copy()
    parents = ea.generation(np.arange(pop, dtype=float))  # identity ranking
    return P_old, ea.P, parents


def test_crossover_binary_mode_swaps_whole_genes():
    # Bin(1, 1/2) mode (App. A.5): every gene of child 1 is the gene of one
    # parent, child 2 takes the other parent's, chosen per gene by its own
    # draw; after the creep the children are the creeps of those genes.
    seen = {0: 0, 1: 0}
    n_mode = 0
    for seed in (21, 22, 23):
        pop = 64
        P_old, P, parents = _crossover_generation(pop, seed, 4)
        for k in range(pop // 2):
            if O.below(O.draw(seed, 4, 0, 3, k, 0), 3) != 1:
                continue
            n_mode += 1
            pa, pb = P_old[parents[2 * k]], P_old[parents[2 * k + 1]]
            for g in range(6):
                f = O.draw(seed, 4, 0, 3, k, 1 + g) >> 63
                seen[f] += 1
                src = ((2 * k + 1, pa[g] if f else pb[g]), (2 * k + 2, pb[g] if f else pa[g]))
                for slot, p in src:
                    if slot >= pop:
                        continue
                    plus, X = _creep_inputs(seed, 4, slot, g)
                    exp = fma(1.0 - p, X, p) if plus else fma(-p, X, p)
                    assert P[slot, g] == min(max(exp, 0.0), 1.0)
    assert n_mode >= 10 and seen[0] > 20 and seen[1] > 20


def test_crossover_blend_mode_per_gene_weights():
    # U(0,1) mode (App. A.5): child 1 = f pa + (1-f) pb, child 2 = f pb +
    # (1-f) pa, with its own f ~ U(0,1) for every gene.  Checked on the
    # children recovered from the crept offspring: the sum of the two children
    # is the sum of the parents, and the weight implied by child 1 is that
    # gene's own draw.
    n_checked = 0
    for seed in (31, 32, 33):
        pop = 64
        P_old, P, parents = _crossover_generation(pop, seed, 6)
        for k in range(pop // 2):
            if O.below(O.draw(seed, 6, 0, 3, k, 0), 3) != 0:
                continue
            s1, s2 = 2 * k + 1, 2 * k + 2
            if s2 >= pop:
                continue
            pa, pb = P_old[parents[2 * k]], P_old[parents[2 * k + 1]]
            fs = []
            for g in range(6):
                c1 = _uncreep(P[s1, g], *_creep_inputs(seed, 6, s1, g))
                c2 = _uncreep(P[s2, g], *_creep_inputs(seed, 6, s2, g))
                if c1 is None or c2 is None or abs(pa[g] - pb[g]) < 1e-3:
                    continue
                assert abs((c1 + c2) - (pa[g] + pb[g])) < 1e-9
                lo, hi = min(pa[g], pb[g]), max(pa[g], pb[g])
                assert lo - 1e-9 <= c1 <= hi + 1e-9
                f_implied = (c1 - pb[g]) / (pa[g] - pb[g])
                f_draw = O.u01(O.draw(seed, 6, 0, 3, k, 1 + g))
                assert abs(f_implied - f_draw) < 1e-6
                fs.append(f_draw)
                n_checked += 1
            # one weight per gene, not one per child
            if len(fs) >= 2:
                assert len(set(fs)) == len(fs)
    assert n_checked >= 30


def test_crossover_mode_frequencies():
    # the mode is uniform over the three forms of App. A.5
    counts = np.zeros(3)
    for k in range(3000):
        counts[O.below(O.draw(5, 1, 0, 3, k, 0), 3)] += 1
    assert stats.chisquare(counts).pvalue > 1e-3


def test_generation_rejects_configurations_beyond_its_arrays():
    # the C oracle checks its own limits (fixed arrays of 1024 rows), so a
    # direct caller cannot overflow them
    import ctypes
    lib = OO._load()
    P = np.zeros((1025, 6))
    chi2 = np.zeros(1025)
    st = OO.EALCState()
    for pop, window in ((1025, 10), (1, 10), (16, 64), (16, 0)):
        cfg = OO.EAConfig(pop, 0, 0.01, 1e-4, 0.5, 0.01, window, 10)
        assert lib.orc_ea_init(ctypes.byref(cfg), 1, 0, OO._p(P), ctypes.byref(st)) == -1
        assert lib.orc_ea_generation(ctypes.byref(cfg), 1, 0, OO._p(P), OO._p(chi2), OO._p(chi2),
                                     OO._p(chi2), ctypes.byref(st), None) == -1
    cfg = OO.EAConfig(1024, 0, 0.01, 1e-4, 0.5, 0.01, 10, 10)
    assert lib.orc_ea_init(ctypes.byref(cfg), 1, 0, OO._p(P), ctypes.byref(st)) == 0
    assert lib.orc_ea_generation(ctypes.byref(cfg), 1, 0, OO._p(P), OO._p(chi2), OO._p(chi2),
                                 OO._p(chi2), ctypes.byref(st), None) == 0
    with pytest.raises(ValueError):
        O.EA(1025, seed=1, lc=0)

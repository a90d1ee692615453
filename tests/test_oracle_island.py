"""Pins of the island-EA oracle (Sec. 5.3, readings I1-I4 in its header)."""
import numpy as np
import pytest

from oracle import island_oracle as IS
from oracle import oracle as O


def _fitness(rng, n):
    c = rng.uniform(1, 100, n)
    c[rng.integers(0, n, 3)] = np.nan
    c[1::9] = c[::9][: c[1::9].size]  # ties
    return c, rng.uniform(0.5, 2, n), rng.uniform(0, 1, n)


@pytest.mark.parametrize("n_isl,m", [(1, 0), (3, 0)])
def test_without_migration_islands_are_plain_eas(n_isl, m):
    # I1: island i of lightcurve k is the Appendix-A EA keyed by k*n_isl + i
    pop, seed, lc = 24, 17, 2
    isl = IS.IslandEA(n_isl, pop, seed, lc, every=3, m=m)
    ref = [O.EA(pop, seed, lc * n_isl + i) for i in range(n_isl)]
    rng = np.random.default_rng(1)
    for g in range(25):
        c, f, b = _fitness(rng, n_isl * pop)
        isl.generation(c, f, b)
        for i, ea in enumerate(ref):
            ea.generation(c[i * pop:(i + 1) * pop], f[i * pop:(i + 1) * pop],
                          b[i * pop:(i + 1) * pop])
        assert np.array_equal(isl.rows(), np.concatenate([ea.P for ea in ref]))


def test_worked_example_by_hand():
    # three islands of four rows; rankings worked out by hand:
    #   island 0  chi2 [5, 1, 3, 9]      fittest rows 1, 2   least fit rows 3, 0
    #   island 1  chi2 [2, 8, 8, 4]      fittest rows 0, 3   least fit rows 2, 1 (tie: row 2 last)
    #   island 2  chi2 [nan, 7, 0.5, 6]  fittest rows 2, 3   least fit rows 0 (NaN), 1
    c0 = [np.array([5.0, 1, 3, 9]), np.array([2.0, 8, 8, 4]), np.array([np.nan, 7, 0.5, 6])]
    P0 = [np.arange(24, dtype=float).reshape(4, 6) + 100 * i for i in range(3)]
    for m, want_c, want_rows in [
        # m = 1: 0 <- row 2 of island 2 at row 3; 1 <- row 1 of 0 at row 2; 2 <- row 0 of 1 at row 0
        (1, [[5, 1, 3, 0.5], [2, 8, 1, 4], [2, 7, 0.5, 6]],
         [[(0, 0), (0, 1), (0, 2), (2, 2)], [(1, 0), (1, 1), (0, 1), (1, 3)],
          [(1, 0), (2, 1), (2, 2), (2, 3)]]),
        # m = 2: the fittest emigrant over the least fit row, the second over the next
        (2, [[6, 1, 3, 0.5], [2, 3, 1, 4], [2, 4, 0.5, 6]],
         [[(2, 3), (0, 1), (0, 2), (2, 2)], [(1, 0), (0, 2), (0, 1), (1, 3)],
          [(1, 0), (1, 3), (2, 2), (2, 3)]]),
    ]:
        c = [a.copy() for a in c0]
        P = [a.copy() for a in P0]
        f = [a * 10 for a in c0]
        b = [a * 100 for a in c0]
        IS.migrate(P, c, f, b, m)
        for j in range(3):
            assert np.array_equal(c[j], np.array(want_c[j], dtype=float), equal_nan=True)
            for row, (si, sr) in enumerate(want_rows[j]):
                assert np.array_equal(P[j][row], P0[si][sr])
                assert f[j][row] == c0[si][sr] * 10 and b[j][row] == c0[si][sr] * 100


@pytest.mark.parametrize("seed", range(6))
def test_migration_against_stable_argsort(seed):
    # the receiver keeps its pop - m fittest rows in place and takes the
    # sender's m fittest, found here with numpy's stable argsort instead
    rng = np.random.default_rng(seed)
    n, pop = int(rng.integers(2, 6)), int(rng.integers(4, 40))
    m = int(rng.integers(1, pop // 2 + 1))
    c = [_fitness(rng, pop)[0] for _ in range(n)]
    P = [rng.uniform(size=(pop, 6)) for _ in range(n)]
    f = [rng.uniform(size=pop) for _ in range(n)]
    b = [rng.uniform(size=pop) for _ in range(n)]
    c1, P1, f1, b1 = ([a.copy() for a in x] for x in (c, P, f, b))
    IS.migrate(P1, c1, f1, b1, m)
    key = lambda a: np.where(np.isnan(a), np.inf, a)
    for j in range(n):
        s = (j - 1) % n
        order_j = np.argsort(key(c[j]), kind="stable")
        order_s = np.argsort(key(c[s]), kind="stable")
        kept, out = order_j[:pop - m], order_j[pop - m:][::-1]
        assert np.array_equal(P1[j][kept], P[j][kept])
        assert np.array_equal(c1[j][kept], c[j][kept], equal_nan=True)
        for r in range(m):
            assert np.array_equal(P1[j][out[r]], P[s][order_s[r]])
            assert (c1[j][out[r]], f1[j][out[r]], b1[j][out[r]]) == \
                (c[s][order_s[r]], f[s][order_s[r]], b[s][order_s[r]]) or \
                np.isnan(c[s][order_s[r]])
        best = lambda a: np.min(key(a))
        assert best(c1[j]) == min(best(c[j]), best(c[s]))


def test_migration_timing():
    # I2: the islands evolve as independent EAs until generation `every`,
    # where the first migration makes them differ
    pop, every = 16, 4
    isl = IS.IslandEA(3, pop, 5, 0, every=every, m=3)
    ref = [O.EA(pop, 5, i) for i in range(3)]
    rng = np.random.default_rng(2)
    for g in range(every + 1):
        c, f, b = _fitness(rng, 3 * pop)
        c = c.copy()
        c[np.isnan(c)] = 50.0
        isl.generation(c, f, b)
        for i, ea in enumerate(ref):
            ea.generation(c[i * pop:(i + 1) * pop], f[i * pop:(i + 1) * pop],
                          b[i * pop:(i + 1) * pop])
        same = np.array_equal(isl.rows(), np.concatenate([ea.P for ea in ref]))
        assert same == (g < every), g


def test_best_record_over_islands():
    # I4 and the monotone record: the best island record never worsens
    isl = IS.IslandEA(4, 12, 3, 1, every=2, m=2)
    rng = np.random.default_rng(3)
    last = np.inf
    for g in range(20):
        c, f, b = _fitness(rng, 4 * 12)
        isl.generation(c, f, b)
        i, s = isl.best()
        assert s["best_chi2"] <= last
        assert s["best_chi2"] == min(ea.summary()["best_chi2"] for ea in isl.eas)
        last = s["best_chi2"]

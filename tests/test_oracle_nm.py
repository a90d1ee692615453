"""Pins of the simplex oracle: step-for-step agreement with scipy's
independent Nelder-Mead (same conventions) and known minima."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import nm_oracle as NM


def rosen(x):
    # weighted Rosenbrock (distinct weights keep simplex values free of ties;
    # scipy orders equal values differently), optimum at x = 0.75
    z = 4.0 * np.asarray(x) - 2.0
    a = 1.0 + 0.13 * np.arange(5)
    b = 1.0 + 0.07 * np.arange(5)
    return float(np.sum(a * 100.0 * (z[1:] - z[:-1] ** 2) ** 2 + b * (1 - z[:-1]) ** 2))


def bowl_outside(x):
    c = np.array([1.3, -0.2, 0.5, 0.9, 0.1, 1.05])  # two coordinates beyond [0, 1]
    w = np.arange(1, 7)
    return float(np.sum(w * (np.asarray(x) - c) ** 2))


def scipy_nm(f, x0, tol, max_iter):
    return minimize(f, x0, method="Nelder-Mead", bounds=[(0.0, 1.0)] * 6,
                    options=dict(maxiter=max_iter + 1, xatol=tol, fatol=tol))


@pytest.mark.parametrize("f,x0,tol,max_iter", [
    (rosen, np.full(6, 0.3), 1e-12, 600),
    (rosen, np.array([0.1, 0.9, 0.5, 0.0, 0.99, 0.6]), 1e-12, 900),
    (bowl_outside, np.array([0.98, 0.5, 0.0, 0.2, 1.0, 0.7]), 1e-6, 2000),
    (bowl_outside, np.full(6, 0.5), 1e-4, 1200),
])
def test_matches_scipy_step_for_step(f, x0, tol, max_iter):
    x, fx, steps, sim, fs = NM.minimise(f, x0, tol_x=tol, tol_f=tol, max_iter=max_iter)
    ref = scipy_nm(f, x0, tol, max_iter)
    assert steps == ref.nit - 1
    assert np.array_equal(x, ref.x) and fx == ref.fun


def test_initial_simplex_reflects_inside_the_box():
    sim = NM.initial_simplex([0.0, 1.0, 0.99, 0.5, -0.3, 2.0])
    assert sim[1, 0] == 0.00025             # zero coordinate: absolute step
    assert sim[2, 1] == 2.0 - 1.05          # 1.05 reflected to 0.95
    assert abs(sim[3, 2] - (2.0 - 1.05 * 0.99)) < 1e-15
    assert sim[4, 3] == 1.05 * 0.5
    assert np.all((sim >= 0) & (sim <= 1))
    assert sim[0, 4] == 0.0 and sim[0, 5] == 1.0   # x0 clipped


def test_finds_known_minima():
    x, fx, steps, _, _ = NM.minimise(rosen, np.full(6, 0.3), 1e-10, 1e-12, 5000)
    assert np.max(np.abs(x - 0.75)) < 1e-6 and fx < 1e-10
    c = np.array([0.2, 0.35, 0.5, 0.65, 0.8, 0.9])
    x, fx, _, _, _ = NM.minimise(lambda v: float(np.sum(np.arange(1, 7) * (v - c) ** 2)),
                                 np.full(6, 0.5), 1e-10, 1e-14, 5000)
    assert np.allclose(x, c, atol=1e-8)


def test_nan_counts_as_worst():
    # NaN outside a ball: the simplex stays where the function is defined
    f = lambda x: float(np.sum((np.asarray(x) - 0.6) ** 2)) if np.max(np.abs(np.asarray(x) - 0.5)) < 0.3 else np.nan
    x, fx, _, _, _ = NM.minimise(f, np.full(6, 0.5), 1e-9, 1e-14, 3000)
    assert np.allclose(x, 0.6, atol=1e-5) and np.isfinite(fx)


# ---------------------------------------------------------------- iterated simplex

def test_start_points_are_numpy_philox_words():
    # T1: start s of lightcurve lc is the block (0, 7, s, g // 4) of Philox
    # keyed (seed, lc); numpy's generator increments its counter before it
    # produces a block, so it is set one block back
    seed, lc, s = 99, 5, 12
    words = []
    for blk in range(2):
        bg = np.random.Philox(key=np.array([seed, lc], dtype=np.uint64),
                              counter=np.array([2**64 - 1, 6, s, blk], dtype=np.uint64))
        words += list(bg.random_raw(4))
    want = np.array([((int(x) >> 12) + 0.5) * 2.0**-52 for x in words[:6]])
    assert np.array_equal(NM.start_point(seed, lc, s), want)


def test_iterated_ties_go_to_the_first_start():
    # T3 on a constant function: every run ties, the first start wins
    x, fx, total, s = NM.iterated(lambda x: 1.0, 3, 1, 4, max_iter=200)
    assert s == 0 and fx == 1.0 and total > 0
    assert np.max(np.abs(x - NM.start_point(3, 1, 0))) < 0.06


def test_iterated_finds_the_global_basin():
    # two bowls; the lower one at a: the best of several starts sits at a
    a = np.full(6, 0.25)
    b = np.full(6, 0.75)
    f = lambda x: min(np.sum((x - a) ** 2), np.sum((x - b) ** 2) + 0.1)
    x, fx, total, s = NM.iterated(f, 21, 0, 8, tol_x=1e-7, tol_f=1e-12, max_iter=4000)
    assert fx < 1e-10 and np.max(np.abs(x - a)) < 1e-5
    # a single start in the other basin ends at b's value instead
    for k in range(8):
        p = NM.start_point(21, 0, k)
        if np.sum((p - b) ** 2) + 0.1 < np.sum((p - a) ** 2) - 0.3:
            _, fk, _, _, _ = NM.minimise(f, p, 1e-7, 1e-12, 4000)
            assert abs(fk - 0.1) < 1e-9

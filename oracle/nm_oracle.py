"""Downhill simplex (Nelder & Mead 1965) in the form of Lagarias, Reeds,
Wright & Wright (1998) -- TEST INFRASTRUCTURE, the reference of the GPU
simplex refinement.

The paper fine-tunes the fittest solution of the EA with the amoeba method
(its Sec. 4.1, "EA with amoeba" in Tables 2 and 3), using the Lagarias et
al. algorithm, without stating its settings.  Here it runs in the EA's
encoded domain [0, 1]^6 (Eq. EMMA-encoding) with the customary settings of
that algorithm:

* coefficients: reflection 1, expansion 2, contraction 1/2, shrink 1/2;
* initial simplex: x0 and x0 with coordinate k scaled by 1.05 (set to
  0.00025 where it is 0); a coordinate pushed above 1 is reflected to 2 - y,
  and every vertex is clipped to [0, 1];
* every trial point (reflection, expansion, outside and inside contraction,
  shrunk vertex) is clipped to [0, 1];
* order: ascending function value, ties kept in their previous order (the
  replaced worst vertex goes after vertices of equal value); NaN counts as
  +infinity;
* stop before a step when max |v_i - v_0| <= tol_x (every coordinate of
  every vertex) and max |f_i - f_0| <= tol_f, or after max_iter steps
  (a shrink is one step).
"""
import numpy as np

N = 6
RHO, CHI, PSI, SIGMA = 1.0, 2.0, 0.5, 0.5


def _val(f, x):
    v = float(f(x))
    return np.inf if np.isnan(v) else v


def initial_simplex(x0):
    x0 = np.clip(np.asarray(x0, dtype=float), 0.0, 1.0)
    sim = np.empty((N + 1, N))
    sim[0] = x0
    for k in range(N):
        y = x0.copy()
        y[k] = (1.0 + 0.05) * y[k] if y[k] != 0 else 0.00025
        sim[k + 1] = y
    sim = np.where(sim > 1.0, 2.0 * 1.0 - sim, sim)
    return np.clip(sim, 0.0, 1.0)


def _order(sim, fs):
    ind = np.argsort(fs, kind="stable")
    return sim[ind], fs[ind]


def minimise(f, x0, tol_x=1e-4, tol_f=1e-4, max_iter=1200):
    """(best vertex, best value, steps, simplex, values)."""
    sim = initial_simplex(x0)
    fs = np.array([_val(f, v) for v in sim])
    sim, fs = _order(sim, fs)
    steps = 0
    while steps < max_iter:
        if np.max(np.abs(sim[1:] - sim[0])) <= tol_x and np.max(np.abs(fs[0] - fs[1:])) <= tol_f:
            break
        xbar = np.add.reduce(sim[:-1], 0) / N
        xr = np.clip((1 + RHO) * xbar - RHO * sim[-1], 0.0, 1.0)
        fr = _val(f, xr)
        if fr < fs[0]:
            xe = np.clip((1 + RHO * CHI) * xbar - RHO * CHI * sim[-1], 0.0, 1.0)
            fe = _val(f, xe)
            sim[-1], fs[-1] = (xe, fe) if fe < fr else (xr, fr)
        elif fr < fs[-2]:
            sim[-1], fs[-1] = xr, fr
        else:
            shrink = False
            if fr < fs[-1]:
                xc = np.clip((1 + PSI * RHO) * xbar - PSI * RHO * sim[-1], 0.0, 1.0)
                fc = _val(f, xc)
                if fc <= fr:
                    sim[-1], fs[-1] = xc, fc
                else:
                    shrink = True
            else:
                xcc = np.clip((1 - PSI) * xbar + PSI * sim[-1], 0.0, 1.0)
                fcc = _val(f, xcc)
                if fcc < fs[-1]:
                    sim[-1], fs[-1] = xcc, fcc
                else:
                    shrink = True
            if shrink:
                for j in range(1, N + 1):
                    sim[j] = np.clip(sim[0] + SIGMA * (sim[j] - sim[0]), 0.0, 1.0)
                    fs[j] = _val(f, sim[j])
        steps += 1
        sim, fs = _order(sim, fs)
    return sim[0].copy(), fs[0], steps, sim, fs


# ------------------------------------------------------------ iterated simplex
#
# The paper's iterated simplex (Sec. 4.1, the second of the compared
# algorithms) deploys a fresh downhill simplex at each of a number of random
# starting points in the search space, stops each run at convergence or
# after 10^4 iterations, and keeps the best.  Readings taken here:
#   T1  start points are uniform over the encoded domain [0, 1]^6 (the
#       prior box); start s of lightcurve lc, coordinate g, is the Philox
#       word of key (seed, lc), counter (0, PURPOSE_START, s, g // 4), word
#       g % 4, mapped to the open unit interval;
#   T2  each run is `minimise` above (S1-S2) with its own max_iter;
#   T3  the result is the lowest value over all runs, the first start in
#       index order among equal values; the work is the sum of the steps.

PURPOSE_START = 7


def start_point(seed, lc, s):
    from . import oracle as O
    return np.array([O.u01(O.draw(seed, lc, 0, PURPOSE_START, s, g)) for g in range(N)])


def iterated(f, seed, lc, n_starts, tol_x=1e-4, tol_f=1e-4, max_iter=10000):
    """(best x, best f, total steps, index of the best start) over starts
    0 .. n_starts - 1 (T1-T3)."""
    best = (None, np.inf, 0, -1)
    total = 0
    for s in range(n_starts):
        x, fx, steps, _, _ = minimise(f, start_point(seed, lc, s), tol_x, tol_f, max_iter)
        total += steps
        if fx < best[1] or best[3] < 0:
            best = (x, fx, 0, s)
    return best[0], best[1], total, best[3]

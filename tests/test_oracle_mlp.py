"""Pins of the FP64 proposal-network oracle against closed forms, finite
differences and library routines."""
import numpy as np
from scipy import stats

from oracle import mlp_oracle as M
from oracle import oracle as O


def test_resample_closed_forms():
    t = np.linspace(0, 10, 2561)
    # a linear ramp normalises to (b - median)/(max - median) of bin means
    b = M.resample(t, 3 * t + 1, np.ones_like(t))
    assert b.shape == (256,) and abs(b.max() - 1) < 1e-12 and abs(np.median(b)) < 1e-12
    assert np.all(np.diff(b) > 0)
    # constant flux: all zero (divisor floor)
    assert np.all(M.resample(t, np.full_like(t, 2.0), np.ones_like(t)) == 0)
    # weighted mean inside a bin
    tt = np.array([0.0, 0.01, 0.02, 10.0])
    yy = np.array([1.0, 2.0, 4.0, 8.0])
    ww = np.array([1.0, 1.0, 2.0, 1.0])
    bb = M.resample(tt, yy, ww)
    raw0 = (1 + 2 + 8) / 4.0
    # empty interior bins interpolate linearly between bin 0 and bin 255
    raw = raw0 + (8 - raw0) * np.arange(256) / 255
    ref = (raw - np.median(raw)) / (raw.max() - np.median(raw))
    assert np.allclose(bb, ref, atol=1e-13)


def test_nll_single_component_is_gaussian_logpdf():
    rng = np.random.default_rng(0)
    B = 16
    O = np.zeros((B, 120))
    O[:, 0] = 50.0  # component 0 carries all the weight
    O[:, 1:8] = -50.0
    mu = rng.uniform(0.2, 0.8, (B, 7))
    ls = rng.uniform(-2, 0, (B, 7))
    O[:, 8:15] = mu
    O[:, 64:71] = ls
    Y = mu + rng.normal(size=(B, 7)) * 0.05
    L, _ = M.nll(O, Y)
    ref = -np.mean(np.sum(stats.norm.logpdf(Y, mu, np.exp(ls)), 1))
    assert abs(L - ref) < 1e-9


def test_nll_periodic_dimension_wraps():
    O = np.zeros((1, 120))
    O[0, 0] = 50.0
    O[0, 8 + 3] = 0.98  # mean of the angle target of component 0
    Y = np.full((1, 7), 0.0)
    Y[0, 3] = 0.01
    Y2 = Y.copy()
    Y2[0, 3] = 0.95  # residual -0.03 vs wrapped +0.03: same likelihood
    assert abs(M.nll(O, Y)[0] - M.nll(O, Y2)[0]) < 1e-12


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    p = M.init_params(rng, scale_out=0.3)
    X = rng.normal(size=(6, 256))
    Y = rng.uniform(0, 1, (6, 7))
    L, g = M.loss_and_grad(p, X, Y)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in p[name].shape)
            h = 1e-6
            p[name][idx] += h
            Lp, _ = M.loss_and_grad(p, X, Y)
            p[name][idx] -= 2 * h
            Lm, _ = M.loss_and_grad(p, X, Y)
            p[name][idx] += h
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-5 * max(1.0, abs(fd)), (name, idx, fd, g[name][idx])


def test_adam_first_step_moves_by_lr_times_sign():
    # with zero moments, the bias-corrected first step is lr * g/(|g| + eps')
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    M.adam_step(p, g, {}, lr=0.1, t=1)
    assert np.allclose(p["w"], [1.0 - 0.1, -2.0 + 0.1, 3.0 - 0.1], atol=1e-6)


def test_training_reduces_loss():
    rng = np.random.default_rng(2)
    p = M.init_params(rng)
    X = rng.normal(size=(64, 256))
    Y = np.clip(0.5 + 0.1 * X[:, :7], 0, 1)
    st = {}
    L0, _ = M.loss_and_grad(p, X, Y)
    for t in range(1, 31):
        L, g = M.loss_and_grad(p, X, Y)
        M.adam_step(p, g, st, lr=1e-3, t=t)
    assert L < L0 - 1.0


# ------------------------------------------------- training-sample pins

def test_poisson_count_is_the_poisson_quantile_function():
    rng = np.random.default_rng(3)
    n_checked = 0
    for _ in range(400):
        c = rng.uniform(0.01, 64.0)
        u = rng.uniform()
        k = M.poisson_count(c, u, 0.0)
        # skip draws that sit on a CDF step to rounding precision
        if min(abs(stats.poisson.cdf(k, c) - u), abs(stats.poisson.cdf(k - 1, c) - u)) < 1e-12:
            continue
        assert k == stats.poisson.ppf(u, c), (c, u)
        n_checked += 1
    assert n_checked > 390
    # large means: the rounded normal approximation, never negative
    assert M.poisson_count(100.0, 0.5, 1.5) == np.floor(100 + 10 * 1.5 + 0.5)
    assert M.poisson_count(100.0, 0.5, -50.0) == 0.0


def test_data_window_lies_in_nights_and_in_the_event_window():
    rng = np.random.default_rng(4)
    for _ in range(500):
        t0, tE = rng.uniform(-10, 10), rng.uniform(10, 100)
        a, b = rng.uniform(-3, -2), rng.uniform(2, 3)
        tf, tl = M.data_window(t0, tE, a, b)
        ta, tb = t0 + a * tE, t0 + b * tE
        assert ta <= tf < ta + 1.0 and tb - 1.0 < tl <= tb
        for x in (tf, tl):
            ph = x - np.floor(x)
            assert 0.1 - 1e-9 <= ph <= 0.1 + 1 / 3 + 1e-9
        # an endpoint already inside a night is kept
        pa = ta - np.floor(ta)
        if 0.1 <= pa <= 0.1 + 1 / 3:
            assert tf == ta


def test_expected_counts_add_up_to_the_epoch_count():
    for s in range(6):
        th, Fb, sn, L, win = M.sample_params(11, s)
        c, tf, span = M.expected_counts(th, L, win)
        assert np.all(c >= 0)
        assert -3 < win[0] < -2 and 2 < win[1] < 3
        # the dense window t0 +- 0.1 tE lies inside the observed span
        assert abs(c.sum() - L) <= 1e-9 * L
        assert 200 <= L <= 5000 and 0 <= Fb <= 0.5 and 0.005 <= sn <= 0.03


def test_observed_bins_are_the_forward_model_at_the_bin_centres():
    # noise-free limit: bin j holds Fs*A + Fb with A evaluated on the
    # physical time of its centre, t_first + span (j + 1/2)/256 (days); this
    # checks the window and the rescaled t0, tE that the sampler feeds the
    # forward model
    th = np.array([-1.3, 1.1, 0.15, 2.2, 35.0, -4.0])
    vals, filled, y, tf, span = M.observe(5, 0, th, 0.2, 1e-13, 3000, (-2.4, 2.7))
    j = np.flatnonzero(filled)
    assert j.size > 50
    t = tf + span * (j + 0.5) / 256
    A = O.magnify(th[:, None], t)[0][0]
    assert np.allclose(vals[j], A + 0.2, rtol=1e-9)
    assert np.allclose(y, [1.7 / 3, 0.6 / 1.5, 0.3, 2.2 / (2 * np.pi), (-4.0 - tf) / span,
                           35.0 / span, 1 / 1.2], rtol=1e-14)


def test_make_sample_is_normalised():
    t0_rel, tE_rel = [], []
    for s in range(40):
        x, y = M.make_sample(2, s)
        assert abs(np.median(x)) < 1e-12 and abs(x.max() - 1) < 1e-12
        assert np.all((y >= 0) & (y <= 1))
        # with the window from t0 + a tE to t0 + b tE, a ~ U(-3, -2), b ~
        # U(2, 3): t0 lies at -a/(b - a) of the span, tE is 1/(b - a) of it
        # (up to the trimming to nights)
        assert 0.38 < y[4] < 0.62 and 0.16 < y[5] < 0.26
        t0_rel.append(y[4])
        tE_rel.append(y[5])
    # the window no longer gives t0 and tE away: the targets spread out
    assert np.std(t0_rel) > 0.03 and np.std(tE_rel) > 0.01


# ------------------------------------------------------ seeding pins

def _mixture(logits, mu, ls):
    o = np.zeros(128)
    o[:8] = logits
    o[8:64] = np.asarray(mu, float).ravel()
    o[64:120] = np.asarray(ls, float).ravel()
    return o


LO = np.array([-3.0, 0.5, 0.0, 0.0, 10.0, -10.0])
HI = np.array([0.0, 2.0, 0.5, 2 * np.pi, 100.0, 10.0])


def test_seed_rows_point_mass_decodes_the_mean():
    mu = np.tile([0.2, 0.4, 0.6, 1.3, 0.5, 0.1, 0.7], (8, 1))
    o = _mixture([50] + [-50] * 7, mu, np.full((8, 7), -40.0))
    rows = M.seed_rows(o, 2.0, 200.0, LO, HI, seed=9, lc=4, n_seed=5)
    th = np.array([-3 + 0.6, 0.5 + 0.6, 0.3, 2 * np.pi * 0.3, 20.0, 2.0 + 100.0])
    ref = np.clip((th - LO) / (HI - LO), 0, 1)   # t0 = 102 clamps to 1
    assert np.allclose(rows, ref[None, :], atol=1e-12)
    assert rows[0, 5] == 1.0


def test_seed_rows_component_frequencies_and_gaussian_draws():
    pi = np.array([0.05, 0.1, 0.15, 0.2, 0.25, 0.1, 0.1, 0.05])
    mu = np.zeros((8, 7)) + 0.5
    mu[:, 1] = np.arange(8) / 10 + 0.1       # component k puts d at 0.1 k + 0.1
    ls = np.full((8, 7), -40.0)
    ls[:, 0] = np.log(0.05)                  # log10 q dimension ~ N(0.5, 0.05^2)
    o = _mixture(np.log(pi) + 3.0, mu, ls)
    n = 3000
    rows = M.seed_rows(o, 0.0, 100.0, LO, HI, seed=1, lc=0, n_seed=n)
    x1 = (rows[:, 1] * (HI[1] - LO[1]) + LO[1] - 0.5) / 1.5
    comp = np.rint((x1 - 0.1) * 10).astype(int)
    counts = np.bincount(comp, minlength=8)
    chi = ((counts - n * pi) ** 2 / (n * pi)).sum()
    assert chi < stats.chi2.ppf(0.999, 7)
    z = ((rows[:, 0] * 3 - 3 + 3) / 3 - 0.5) / 0.05
    assert stats.kstest(z, "norm").pvalue > 1e-3

"""Pins of the FP64 proposal-network oracle against closed forms, finite
differences and library routines."""
import numpy as np
from scipy import stats

from oracle import mlp_oracle as M


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

"""FP64 numpy reference of the learned proposal network (TEST INFRASTRUCTURE).

Not part of the paper's method: the proposal network seeds part of the EA's
initial population, and the plain EA's chi^2 still decides, and the EA is the
fallback.  This module is the oracle of the GPU implementation:

* resampling of a lightcurve to 256 bins over its observed span: the bin
  value is the weighted mean flux of the epochs in the bin, empty bins take
  the linear interpolation of their nearest filled neighbours (the nearest
  filled value at the ends), then the bins are normalised as
  (b - median) / (max - median) (divisor floored at 1e-12);
* the network 256 -> 512 (ReLU) -> 512 (ReLU) -> 120, the output read as a
  K = 8 mixture of diagonal Gaussians over D = 7 targets: 8 logits, 8x7 means,
  8x7 log standard deviations;
* the negative log-likelihood of the targets averaged over the batch, with
  target 3 (the encoded trajectory angle) periodic on [0, 1): its residual is
  wrapped to [-1/2, 1/2);
* the gradient of that loss by backpropagation, and one Adam step
  (Kingma & Ba 2015, bias-corrected).

Targets, in order: encoded log10 q, d, u0, alpha (Eq. EMMA-encoding with the
EA's domains), (t0 - t_first)/span, tE/span, and f = Fs / (Fs + Fb).

Also the definitions of the two random processes around the network (the
Philox words come from the EA oracle's generator):
* make_sample: one training lightcurve at bin level (parameters uniform
  over the default domain, nightly observing windows over t0 +- 2 tE, a
  Poisson epoch count and Gaussian noise per bin, the forward model of
  Sec. 2.2 at the bin centres), then the same filling and normalisation as
  resample;
* seed_rows: draws from the proposal mixture decoded into the EA's domain.
"""
import math

import numpy as np

from oracle import oracle as O

DIMS = (256, 512, 512, 120)
K, D = 8, 7
PERIODIC = 3


def resample(t, y, w, nbins=256):
    """Normalised 256-bin lightcurve (see the module docstring)."""
    t, y, w = np.asarray(t, float), np.asarray(y, float), np.asarray(w, float)
    out = np.zeros(nbins)
    if t.size == 0:
        return out
    t_a, t_b = t[0], t[-1]
    span = t_b - t_a
    idx = np.zeros(t.size, int) if span <= 0 else \
        np.minimum(((t - t_a) / span * nbins).astype(int), nbins - 1)
    sw = np.bincount(idx, weights=w, minlength=nbins)
    swy = np.bincount(idx, weights=w * y, minlength=nbins)
    filled = sw > 0
    vals = np.zeros(nbins)
    vals[filled] = swy[filled] / sw[filled]
    return fill_and_normalise(vals, filled)


def fill_and_normalise(vals, filled):
    """Empty bins by linear interpolation of the nearest filled ones (the
    nearest filled value beyond either end), then (v - median)/(max -
    median) with the divisor floored at 1e-12; zeros if nothing is filled."""
    vals = np.array(vals, dtype=float)
    nbins = vals.size
    fi = np.flatnonzero(filled)
    if fi.size == 0:
        return np.zeros(nbins)
    for b in range(nbins):
        if filled[b]:
            continue
        lo = fi[fi < b]
        hi = fi[fi > b]
        if lo.size and hi.size:
            l, h = lo[-1], hi[0]
            vals[b] = vals[l] + (vals[h] - vals[l]) * (b - l) / (h - l)
        else:
            vals[b] = vals[lo[-1]] if lo.size else vals[hi[0]]
    med = np.median(vals)
    return (vals - med) / max(vals.max() - med, 1e-12)


def init_params(rng, scale_out=0.01):
    """He-normal hidden layers, small output layer, zero biases."""
    p = {}
    for i, (a, b) in enumerate(zip(DIMS[:-1], DIMS[1:]), start=1):
        std = np.sqrt(2.0 / a) if i < 3 else scale_out
        p[f"W{i}"] = rng.standard_normal((a, b)) * std
        p[f"b{i}"] = np.zeros(b)
    return p


def forward(p, X):
    Z1 = X @ p["W1"] + p["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ p["W2"] + p["b2"]
    H2 = np.maximum(Z2, 0.0)
    O = H2 @ p["W3"] + p["b3"]
    return O, (X, H1, H2)


def split(O):
    B = O.shape[0]
    return O[:, :K], O[:, K:K + K * D].reshape(B, K, D), O[:, K + K * D:].reshape(B, K, D)


def _residual(Y, mu):
    r = Y[:, None, :] - mu
    r[:, :, PERIODIC] -= np.floor(r[:, :, PERIODIC] + 0.5)
    return r


def nll(O, Y):
    """Mean negative log-likelihood and its gradient dL/dO."""
    B = O.shape[0]
    logit, mu, ls = split(O)
    r = _residual(Y, mu)
    sig2 = np.exp(2 * ls)
    comp = -0.5 * r * r / sig2 - ls - 0.5 * np.log(2 * np.pi)     # [B,K,D]
    lognorm = comp.sum(2)                                          # [B,K]
    m = logit.max(1, keepdims=True)
    logpi = logit - m - np.log(np.exp(logit - m).sum(1, keepdims=True))
    a = logpi + lognorm
    am = a.max(1, keepdims=True)
    lp = am[:, 0] + np.log(np.exp(a - am).sum(1))
    gamma = np.exp(a - lp[:, None])                                # posterior
    pi = np.exp(logpi)
    g_logit = (pi - gamma) / B
    g_mu = -gamma[:, :, None] * r / sig2 / B
    g_ls = -gamma[:, :, None] * (r * r / sig2 - 1.0) / B
    dO = np.concatenate([g_logit, g_mu.reshape(B, -1), g_ls.reshape(B, -1)], 1)
    return -lp.mean(), dO


def backward(p, cache, dO):
    X, H1, H2 = cache
    g = {"W3": H2.T @ dO, "b3": dO.sum(0)}
    dZ2 = (dO @ p["W3"].T) * (H2 > 0)
    g["W2"], g["b2"] = H1.T @ dZ2, dZ2.sum(0)
    dZ1 = (dZ2 @ p["W2"].T) * (H1 > 0)
    g["W1"], g["b1"] = X.T @ dZ1, dZ1.sum(0)
    return g


def loss_and_grad(p, X, Y):
    O, cache = forward(p, X)
    L, dO = nll(O, Y)
    return L, backward(p, cache, dO)


def adam_step(p, g, state, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step at step number t >= 1 (in place)."""
    for k in p:
        m = state.setdefault("m" + k, np.zeros_like(p[k]))
        v = state.setdefault("v" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p


# ------------------------------------------------------- training samples

DATA_LO = np.array([-3.0, 0.5, 0.0, 0.0, 10.0, -10.0])
DATA_HI = np.array([0.0, 2.0, 0.5, 2.0 * np.pi, 100.0, 10.0])
NIGHT0, NIGHT_LEN = 0.1, 1.0 / 3.0
P_DATA = 33
P_SEED = 6


def data_window(t0, tE, a, b):
    """First and last instants of the observing window [t0 + a tE, t0 + b tE]
    inside a nightly window [n + 0.1, n + 0.1 + 1/3] (days)."""
    ta, tb = t0 + a * tE, t0 + b * tE
    na = math.floor(ta - NIGHT0)
    t_first = ta if ta <= na + NIGHT0 + NIGHT_LEN else na + 1.0 + NIGHT0
    nb = math.floor(tb - NIGHT0)
    t_last = tb if tb <= nb + NIGHT0 + NIGHT_LEN else nb + NIGHT0 + NIGHT_LEN
    return t_first, t_last


def _overlap(a0, a1, b0, b1):
    return max(0.0, min(a1, b1) - max(a0, b0))


def night_overlap(b0, b1):
    """Length of [b0, b1] covered by nightly windows."""
    o = 0.0
    nt = math.floor(b0) - 1.0
    while nt <= math.floor(b1):
        o += _overlap(b0, b1, nt + NIGHT0, nt + NIGHT0 + NIGHT_LEN)
        nt += 1.0
    return o


def poisson_count(c, u, z):
    """Poisson(c) by inversion of its CDF at u (c <= 64), else the rounded
    normal approximation c + sqrt(c) z."""
    if c <= 64.0:
        p = math.exp(-c)
        F, k = p, 0.0
        while u > F and k < 1000.0:
            k += 1.0
            p = p * c / k
            F += p
        return k
    return max(0.0, math.floor(c + math.sqrt(c) * z + 0.5))


def sample_params(seed, s):
    """(theta[6], Fb, noise fraction, L, (a, b)) of training sample s: the
    observing window runs from t0 + a tE to t0 + b tE, a ~ U(-3, -2) and
    b ~ U(2, 3), the random start and end of the paper's test lightcurves
    (Sec. 4.2)."""
    w = [O.draw(seed, s, 0, P_DATA, 0, j) for j in range(11)]
    th = np.array([DATA_LO[g] + (DATA_HI[g] - DATA_LO[g]) * O.u01(w[g]) for g in range(6)])
    win = (-3.0 + O.u01(w[9]), 2.0 + O.u01(w[10]))
    return (th, 0.5 * O.u01(w[6]), 0.005 + 0.025 * O.u01(w[7]), 200.0 + O.below(w[8], 4801),
            win)


def expected_counts(th, L, win, nbins=256):
    """Expected epoch count per bin and the window (t_first, span)."""
    tE, t0 = th[4], th[5]
    t_first, t_last = data_window(t0, tE, *win)
    span = t_last - t_first
    o = np.zeros(nbins)
    dj = np.zeros(nbins)
    for j in range(nbins):
        b0 = t_first + span * j / nbins
        b1 = t_first + span * (j + 1) / nbins
        o[j] = night_overlap(b0, b1)
        dj[j] = _overlap(b0, b1, t0 - 0.1 * tE, t0 + 0.1 * tE)
    osum = float(np.sum(o))
    n_dense = math.floor(0.1 * L + 0.5)
    n_sched = L - n_dense
    c = np.array([(n_sched * o[j] / osum if osum > 0 else 0.0) + n_dense * dj[j] / (0.2 * tE)
                  for j in range(nbins)])
    return c, t_first, span


def observe(seed, s, th, Fb, sn, L, win, nbins=256):
    """Bin-level observation of parameters th (Fs = 1) through the window
    win = (a, b): raw bin values, their filled flags, the targets y[7] and
    the window (t_first, span)."""
    c, t_first, span = expected_counts(th, L, win, nbins)
    thp = np.array(th, dtype=float)
    thp[4] = th[4] / span
    thp[5] = (th[5] - t_first) / span
    u = (np.arange(nbins) + 0.5) / nbins
    A = O.magnify(thp[:, None], u, nthreads=1)[0][0]
    vals = np.zeros(nbins)
    filled = np.zeros(nbins, bool)
    for j in range(nbins):
        w = [O.draw(seed, s, 0, P_DATA, 1 + j, k) for k in range(3)]
        r1, r2 = O.u01(w[1]), O.u01(w[2])
        rad = math.sqrt(-2.0 * math.log(r1))
        z1, z2 = rad * math.cos(2.0 * math.pi * r2), rad * math.sin(2.0 * math.pi * r2)
        cnt = poisson_count(c[j], O.u01(w[0]), z2)
        if cnt > 0:
            flux = 1.0 * A[j] + Fb
            vals[j] = flux + sn * flux / math.sqrt(cnt) * z1
            filled[j] = True
    y = np.array([(th[0] + 3.0) / 3.0, (th[1] - 0.5) / 1.5, th[2] / 0.5, th[3] / (2.0 * np.pi),
                  (th[5] - t_first) / span, th[4] / span, 1.0 / (1.0 + Fb)])
    return vals, filled, y, t_first, span


def make_sample(seed, s, nbins=256):
    """(x[256] normalised bins, y[7] targets) of training sample s."""
    th, Fb, sn, L, win = sample_params(seed, s)
    vals, filled, y, _, _ = observe(seed, s, th, Fb, sn, L, win, nbins)
    return fill_and_normalise(vals, filled), y


# --------------------------------------------------------------- seeding

def seed_rows(o, t_first, span, lo, hi, seed, lc, n_seed, gen=0, window_only=False):
    """Encoded population rows [n_seed][6] drawn from the mixture o[>=120]
    with the counters of generation `gen`; with window_only (o unused) t0 at
    the middle of the observed span, tE a quarter of it and the other four
    parameters uniform over their ranges (the ablation of the learned form)."""
    o = np.zeros(2 * K * D + K) if window_only else np.asarray(o, dtype=float)
    lmax = max(o[:K])
    e = [math.exp(o[k] - lmax) for k in range(K)]
    S = 0.0
    for k in range(K):
        S += e[k]
    mu = o[K:K + K * D].reshape(K, D)
    ls = o[K + K * D:K + 2 * K * D].reshape(K, D)
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    rows = np.zeros((n_seed, 6))
    for r in range(n_seed):
        if window_only:
            # the learned form's ablation: the observation window alone
            x = np.array([O.u01(O.draw(seed, lc, gen, P_SEED, r, 1 + d)) for d in range(4)]
                         + [0.5, 0.25])
            th = np.array([-3.0 + 3.0 * x[0], 0.5 + 1.5 * x[1], 0.5 * x[2], 2.0 * np.pi * x[3],
                           span * x[5], t_first + span * x[4]])
            rows[r] = np.minimum(np.maximum((th - lo) / (hi - lo), 0.0), 1.0)
            continue
        u = O.u01(O.draw(seed, lc, gen, P_SEED, r, 0))
        comp, acc = K - 1, 0.0
        for k in range(K):
            acc += e[k]
            if u * S < acc:
                comp = k
                break
        z = []
        for i in range(4):
            u1 = O.u01(O.draw(seed, lc, gen, P_SEED, r, 1 + 2 * i))
            u2 = O.u01(O.draw(seed, lc, gen, P_SEED, r, 2 + 2 * i))
            rad = math.sqrt(-2.0 * math.log(u1))
            z += [rad * math.cos(2.0 * math.pi * u2), rad * math.sin(2.0 * math.pi * u2)]
        x = np.array([mu[comp, d] + math.exp(ls[comp, d]) * z[d] for d in range(D)])
        x[PERIODIC] -= math.floor(x[PERIODIC])
        th = np.array([-3.0 + 3.0 * x[0], 0.5 + 1.5 * x[1], 0.5 * x[2], 2.0 * np.pi * x[3],
                       span * x[5], t_first + span * x[4]])
        rows[r] = np.minimum(np.maximum((th - lo) / (hi - lo), 0.0), 1.0)
    return rows

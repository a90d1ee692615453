"""FP64 numpy reference of the learned proposal network (TEST INFRASTRUCTURE).

Not part of the paper's method: the proposal network seeds part of the EA's
initial population, and the plain EA remains the judge (chi^2) and the
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
"""
import numpy as np

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
    fi = np.flatnonzero(filled)
    if fi.size == 0:
        return out
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

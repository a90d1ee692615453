"""Shared helpers of the test-suite: synthetic lightcurves assembled with the
oracle's magnifications, and the floating-point conditioning of A."""
import numpy as np

import oracle as O
from paper_1208_4830_amd import inputs

EPS = 2.0 ** -53


def observe(A, Fs, Fb, sfrac, noise):
    """Observed flux y and weights w = 1/sigma^2 from true magnifications."""
    F = Fs * A + Fb
    sigma = sfrac * F
    return F + sigma * noise, 1.0 / (sigma * sigma)


def oracle_lightcurves(wl, nthreads=None):
    """y, w for a Workload using the oracle's magnification of the true theta."""
    y = np.empty_like(wl.t)
    w = np.empty_like(wl.t)
    for k in range(wl.n_lc):
        sl = slice(wl.off[k], wl.off[k + 1])
        if wl.off[k + 1] == wl.off[k]:
            continue
        A, _ = O.magnify(wl.theta[:, k:k + 1], wl.t[sl], nthreads=nthreads)
        y[sl], w[sl] = observe(A[0], wl.Fs[k], wl.Fb[k], wl.sfrac[sl], wl.noise[sl])
    return y, w


def source_positions(theta, t):
    """zeta[n][n_t] (Eq. sourcePos) for theta[6][n], shared epochs t."""
    u0, al, tE, t0 = theta[2][:, None], theta[3][:, None], theta[4][:, None], theta[5][:, None]
    tau = (t[None, :] - t0) / tE
    return tau * np.sin(al) + u0 * np.cos(al) + 1j * (-tau * np.cos(al) + u0 * np.sin(al))


def magnification_condition(zeta, d, q, tau=0.0, u0=0.0):
    """First-order bound on the relative error of A that rounding alone can
    cause in a correct FP64 evaluation, for a comparison of two of them.

    Two sources, per accepted image z_i with g = 1/conj(z)^2 + q/(d-conj(z))^2,
    h = dg/dconj(z) = -2/conj(z)^3 + 2q/(d-conj(z))^3, det J = 1 - |g|^2:
    (a) coefficient rounding: a root moves by |dp(z_i)|/|p'(z_i)| with
        |dp| <= e sum_j |c_j| |z_i|^j, e = 128 eps (each coefficient is formed
        by ~20 rounded operations, some with cancellation, on each side);
    (b) input rounding: the source position (tau, sin, cos) and 10^log10q are
        each good to a few ulps; from d zeta = dz + g d conj(z), an image moves
        by |dz| <= (1 + |g|) |d zeta| / |det J| with
        |d zeta| = 16 eps (|tau| + u0 + 1) + 4 eps q / |d - conj(z)|.
    det J then moves by 2 |g| |h| |dz| and A_i = 1/|det J_i| by A_i^2 times
    that.  Returns sum_i dA_i / A."""
    imgs, dj, _ = O.images(zeta, d, q)
    c = O.lens_poly(zeta, d, q)
    dc = c[1:] * np.arange(1, 6)
    A = np.sum(1.0 / np.abs(dj))
    tot = 0.0
    for z, det in zip(imgs, dj):
        mag = np.sum(np.abs(c) * np.abs(z) ** np.arange(6))
        dp = abs(np.polyval(dc[::-1], z))
        zb = np.conj(z)
        g = 1 / zb ** 2 + q / (d - zb) ** 2
        h = -2 / zb ** 3 + 2 * q / (d - zb) ** 3
        dz_coef = 128 * EPS * mag / max(dp, 1e-300)
        dzeta = 16 * EPS * (abs(tau) + u0 + 1) + 4 * EPS * q / abs(d - zb)
        dz_in = (1 + abs(g)) * dzeta / abs(det)
        tot += (1.0 / det) ** 2 * 2 * abs(g) * abs(h) * (dz_coef + dz_in)
    return tot / A


def ambiguous_count(zeta, d, q, lo=1e-9, hi=1e-3):
    """True where the image count is decided by a residual close to the 1e-6
    threshold (the source is within ~1e-8 of a caustic)."""
    _, _, rs = O.images(zeta, d, q)
    return lo < rs[3] < hi


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def csr_workload(seed, lengths, sigma_frac=0.01):
    """Uniform-cadence lightcurves with the given (ragged) lengths."""
    rng = np.random.default_rng(seed)
    n = len(lengths)
    theta = inputs.draw_theta(rng, n)
    Fs, Fb = inputs.draw_blend(rng, n)
    ts = [inputs.uniform_epochs(theta[:, k:k + 1], L)[0] for k, L in enumerate(lengths)]
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(lengths)
    t = np.concatenate(ts) if sum(lengths) else np.zeros(0)
    return inputs.Workload(theta, Fs, Fb, off, t, np.full(t.size, sigma_frac),
                           rng.standard_normal(t.size))

"""Shared helpers of the test-suite: synthetic lightcurves assembled with the
oracle's magnifications, and the floating-point conditioning of A."""
import os

import mpmath
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

    Both implementations refine accepted images on the lens equation (the
    oracle every one, the kernel every one whose residual could move A by
    more than 1e-12 relative, and every one with |det J| < 0.01), so an image
    is determined by the lens equation, not by the quintic.  Per accepted
    image z_i, with g = 1/conj(z)^2 + q/(d-conj(z))^2,
    h = dg/dconj(z) = -2/conj(z)^3 + 2q/(d-conj(z))^3, det J = 1 - |g|^2 and
    s = |zeta| + |z| + 1/|z| + q/|d-z|, the image moves by at most
    (1 + |g|) (|d zeta| + 16 eps s) / |det J|: |d zeta| = 16 eps (|tau| + u0
    + 1) + 4 eps q / |d - conj(z)| is the rounding of the source position
    (tau, sin, cos) and of 10^log10q, 16 eps s that of the lens-equation
    residual the refinement drives to zero (from d zeta = dz + g d conj(z)).
    det J then moves by 2 |g| |h| |dz| and A_i = 1/|det J_i| by A_i^2 times
    that.  Returns sum_i dA_i / A + 5e-12 (the kernel's unrefined images)."""
    imgs, dj, _ = O.images(zeta, d, q)
    A = np.sum(1.0 / np.abs(dj))
    tot = 0.0
    for z, det in zip(imgs, dj):
        zb = np.conj(z)
        g = 1 / zb ** 2 + q / (d - zb) ** 2
        h = -2 / zb ** 3 + 2 * q / (d - zb) ** 3
        dzeta = 16 * EPS * (abs(tau) + u0 + 1) + 4 * EPS * q / abs(d - zb)
        s = abs(zeta) + abs(z) + 1 / abs(z) + q / abs(d - z)
        dz = (1 + abs(g)) * (dzeta + 16 * EPS * s) / abs(det)
        tot += (1.0 / det) ** 2 * 2 * abs(g) * abs(h) * dz
    return tot / A + 5e-12


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


def near_caustic_pairs(rng, n, r_max=0.01):
    """n (theta, t) pairs whose source lies within r_max theta_E of a caustic.

    Per pair: (log10 q, d) from the priors; a point of the critical curve from
    the quartic e^{i phi} z^2 (z-d)^2 - (z-d)^2 - q z^2 = 0 (phi uniform, one of
    its four roots at random, via batched companion-matrix eigenvalues),
    mapped through the lens equation to the caustic; an offset r e^{i psi}
    with r ~ U(0, r_max]; then a trajectory through that source position:
    alpha ~ U[0, 2 pi), u0 = Re(zeta e^{-i alpha}) (alpha += pi if negative),
    tau = -Im(zeta e^{-i alpha}), tE, t0 from the priors, t = t0 + tau tE."""
    lq = rng.uniform(-3, 0, n)
    d = rng.uniform(0.5, 2, n)
    q = 10 ** lq
    e = np.exp(1j * rng.uniform(0, 2 * np.pi, n))
    # monic quartic z^4 + a3 z^3 + a2 z^2 + a1 z + a0 (divide by e)
    a3 = -2 * d + 0j
    a2 = (e * d * d - 1 - q) / e
    a1 = 2 * d / e
    a0 = -d * d / e
    comp = np.zeros((n, 4, 4), dtype=complex)
    comp[:, 0, :] = -np.stack([a3, a2, a1, a0], 1)
    comp[:, 1, 0] = comp[:, 2, 1] = comp[:, 3, 2] = 1
    roots = np.linalg.eigvals(comp)
    z = roots[np.arange(n), rng.integers(0, 4, n)]
    zb = np.conj(z)
    zc = z - 1 / zb + q / (d - zb)
    zeta = zc + rng.uniform(0, r_max, n) * np.exp(1j * rng.uniform(0, 2 * np.pi, n))
    al = rng.uniform(0, 2 * np.pi, n)
    rot = zeta * np.exp(-1j * al)
    flip = rot.real < 0
    al = np.where(flip, al + np.pi, al)
    rot = np.where(flip, -rot, rot)
    u0, tau = rot.real, -rot.imag
    tE, t0 = rng.uniform(10, 100, n), rng.uniform(-10, 10, n)
    theta = np.stack([lq, d, u0, al, tE, t0])
    return theta, t0 + tau * tE


def generic_pairs(rng, n):
    """n (theta, t) pairs from the priors with tau ~ U[-2, 2]."""
    theta = inputs.draw_theta(rng, n)
    return theta, theta[5] + rng.uniform(-2, 2, n) * theta[4]


def exact_magnification(zeta, d, q, dps=50):
    """A and the image count at a source position from dps-digit roots of the
    quintic, formed by exact polynomial products as in the paper's
    derivation; zeta, d, q may be floats or mpmath numbers (taken exactly)."""
    mpmath.mp.dps = dps
    zeta = mpmath.mpc(zeta)
    d, q = mpmath.mpf(d), mpmath.mpf(q)
    w = mpmath.conj(zeta)
    N = [-d, 1 + q - d * w, w]
    D = [0, -d, 1]
    M = [N[k] - d * D[k] for k in range(3)]

    def mul(a, b):
        o = [0] * (len(a) + len(b) - 1)
        for i, x in enumerate(a):
            for j, y in enumerate(b):
                o[i + j] += x * y
        return o
    c = [0] * 6
    for k, v in enumerate(mul([zeta, -1], mul(N, M))):
        c[k] += v
    for k, v in enumerate(mul(M, D)):
        c[k] += v
    for k, v in enumerate(mul(N, D)):
        c[k] += q * v
    roots = mpmath.polyroots(c[::-1], maxsteps=400, extraprec=400)
    res = [abs(zeta - z + 1 / mpmath.conj(z) - q / (d - mpmath.conj(z))) for z in roots]
    order = sorted(range(5), key=lambda k: res[k])
    n5 = sum(r < mpmath.mpf("1e-6") for r in res) >= 4
    A = 0
    for k in (order if n5 else order[:3]):
        zb = mpmath.conj(roots[k])
        g = 1 / zb ** 2 + q / (d - zb) ** 2
        A += 1 / abs(1 - abs(g) ** 2)
    return float(A), (5 if n5 else 3)


def exact_magnification_theta(theta, t, dps=50):
    """A of the FP64 parameters theta[6] at epoch t with every step after
    the inputs in dps-digit arithmetic: the source position of Eq. sourcePos
    from the exact values of log10 q, u0, alpha, tE, t0 and t, so that it is
    the answer to the FP64 problem, free of any implementation's rounding."""
    mpmath.mp.dps = dps
    lq, d, u0, al, tE, t0 = (mpmath.mpf(float(v)) for v in theta)
    tau = (mpmath.mpf(float(t)) - t0) / tE
    sa, ca = mpmath.sin(al), mpmath.cos(al)
    zeta = mpmath.mpc(tau * sa + u0 * ca, -tau * ca + u0 * sa)
    return exact_magnification(zeta, d, mpmath.power(10, lq), dps)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden_rows(name):
    """Rows of a fixture under tests/golden/ (whitespace-separated fields,
    '#' comment lines skipped)."""
    with open(os.path.join(GOLDEN, name)) as f:
        return [line.split() for line in f if line.strip() and not line.startswith("#")]

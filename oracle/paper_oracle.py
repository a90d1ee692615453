"""The paper's fitting experiments (Sec. 2.4, 4.2-4.4): observations in
magnitudes, the photometric noise model, and the success criterion -- TEST
INFRASTRUCTURE, the reference of the measurement harness.

Readings taken where the text is silent:
  P3  experiment 1: noise-free, sigma = 0.01 mag for the statistic;
      experiment 2: sigma from Eq. noiseModel at the true magnitude,
      Gaussian in magnitude.
  P4  fitting in flux: F = 10^(-0.4 (m - 20)), sigma_F = 0.4 ln(10) F sigma
      (F observed); the profiled fluxes give m0 = 20 - 2.5 log10(Fs + Fb)
      and f = Fs / (Fs + Fb) (Eq. A_s with Eq. blend).
  P5  Delta chi^2 = chi^2 of the fit - chi^2 of the true model, both in
      magnitudes on the observed points; nu = N - 7 (experiment 1) or N - 8
      (experiment 2, with f).  Weak success: Delta chi^2 / nu < 1.  Strict:
      also every parameter within 10%: |error| / |true| for q, a (= d),
      b (= u0), tE, m0 and f; |error| / tE for tm; the wrapped angle error
      / 2 pi for theta.  A fitted model with non-positive flux somewhere is
      a failure.
  P6  peaks: local maxima of the source magnification on a uniform grid of
      4000 points over [t_start, t_end] whose prominence (2.5 log10 of the
      peak over the higher of the lowest points separating it from higher
      ground or the ends) is at least 0.01 mag; classes 1, 2, 3 and 4 (four
      or more; a curve without an interior maximum is class 1).
"""
import math

import numpy as np

ZP = 20.0
NOISE_SLOPE, NOISE_ICPT = 0.3416, -7.7095
SIGMA_EXP1 = 0.01
GRID = 4000
PROMINENCE = 0.01


def noise_sigma(m):
    """Eq. noiseModel: log10 sigma = 0.3416 m - 7.7095 (magnitudes)."""
    return 10.0 ** (NOISE_SLOPE * np.asarray(m, float) + NOISE_ICPT)


def magnitude(A, m0, f):
    """Eq. A_s with Eq. blend: m = m0 - 2.5 log10(f A + 1 - f)."""
    return m0 - 2.5 * np.log10(f * np.asarray(A, float) + (1.0 - f))


def observe(experiment, A, m0, f, noise):
    """(m_true, m_obs, sigma) for one lightcurve (P3)."""
    m_true = magnitude(A, m0, f)
    if experiment == 1:
        return m_true, m_true.copy(), np.full(m_true.shape, SIGMA_EXP1)
    sigma = noise_sigma(m_true)
    return m_true, m_true + sigma * np.asarray(noise, float), sigma


def to_flux(m_obs, sigma):
    """(y, w) in flux units with zero point 20 mag (P4)."""
    y = 10.0 ** (-0.4 * (np.asarray(m_obs, float) - ZP))
    s = 0.4 * math.log(10.0) * y * np.asarray(sigma, float)
    return y, 1.0 / s ** 2


def fitted_m0_f(Fs, Fb):
    """(m0, f) from profiled fluxes (P4); None when Fs + Fb <= 0."""
    tot = Fs + Fb
    if not tot > 0:
        return None
    return ZP - 2.5 * math.log10(tot), Fs / tot


def chi2_mag(m_obs, sigma, m_model):
    r = (np.asarray(m_obs, float) - m_model) / sigma
    return float(np.sum(r * r))


def success(experiment, theta_fit, Fs, Fb, A_fit, m_obs, sigma, m_true, theta_true, m0, f,
            lens_only=False):
    """(weak, strict, Delta chi^2 / nu) of one fitted model (P5).  With
    lens_only the strict test leaves out the photometric parameters m0 and f
    (which the fit profiles instead of searching) and checks the six lens and
    trajectory parameters only."""
    N = len(m_obs)
    nu = N - (7 if experiment == 1 else 8)
    mf = fitted_m0_f(Fs, Fb)
    if mf is None:
        return False, False, math.inf
    m0_fit, f_fit = mf
    flux = f_fit * np.asarray(A_fit, float) + (1.0 - f_fit)
    if not np.all(flux > 0):
        return False, False, math.inf
    m_model = m0_fit - 2.5 * np.log10(flux)
    dchi = (chi2_mag(m_obs, sigma, m_model) - chi2_mag(m_obs, sigma, m_true)) / nu
    weak = bool(dchi < 1.0)
    q_fit, q_true = 10.0 ** theta_fit[0], 10.0 ** theta_true[0]
    errs = [abs(q_fit - q_true) / q_true]
    for j in (1, 2, 4):  # d, u0, tE
        errs.append(abs(theta_fit[j] - theta_true[j]) / abs(theta_true[j]))
    if not lens_only:
        errs.append(abs(m0_fit - m0) / abs(m0))
        if experiment == 2:
            errs.append(abs(f_fit - f) / abs(f))
    errs.append(abs(theta_fit[5] - theta_true[5]) / theta_true[4])
    da = (theta_fit[3] - theta_true[3]) % (2.0 * math.pi)
    errs.append(min(da, 2.0 * math.pi - da) / (2.0 * math.pi))
    strict = bool(weak and max(errs) < 0.1)
    return weak, strict, float(dchi)


def peak_count(A):
    """Peaks of a sampled magnification curve with prominence >= 0.01 mag (P6).

    A maximum is a rise into a run of equal values that is followed by a
    fall; on each side the lowest value before higher ground (or the end of
    the curve) is found, and the higher of the two is the reference."""
    A = np.asarray(A, float)
    n = len(A)
    count = 0
    i = 1
    while i < n - 1:
        if not A[i] > A[i - 1]:
            i += 1
            continue
        j = i
        while j + 1 < n and A[j + 1] == A[i]:
            j += 1
        if j + 1 < n and A[j + 1] < A[i]:
            lo_l, k = A[i], i - 1
            while k >= 0 and A[k] <= A[i]:
                lo_l = min(lo_l, A[k])
                k -= 1
            lo_r, k = A[i], j + 1
            while k < n and A[k] <= A[i]:
                lo_r = min(lo_r, A[k])
                k += 1
            if 2.5 * math.log10(A[i] / max(lo_l, lo_r)) >= PROMINENCE:
                count += 1
        i = j + 1
    return count


def peak_class(count):
    return min(max(count, 1), 4)


def grid(t_start, t_end):
    return np.linspace(t_start, t_end, GRID)

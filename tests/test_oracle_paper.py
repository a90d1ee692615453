"""Pins of the experiment oracle (readings P3-P6 in its header): the noise
model's worked value, magnitudes and fluxes, the success criterion, peak
counting against scipy's topographic prominence."""
import math

import numpy as np
import pytest
from scipy.signal import find_peaks

from oracle import paper_oracle as P
from paper_1208_4830_amd import inputs
from tests.helpers import golden_rows


def test_noise_model_worked_value():
    g = {r[0]: float(r[1]) for r in golden_rows("noise_model.txt")}
    # the paper's remark: an error of the order of 0.1% at m_I ~ 14
    s = float(P.noise_sigma(g["example_m_I"]))
    assert 0.5 * g["example_sigma_order"] < s < 2.0 * g["example_sigma_order"]
    # the printed coefficients: 10^(0.3416 * 14 - 7.7095) = 1.18e-3 mag, and
    # one magnitude fainter multiplies sigma by 10^0.3416
    assert 1.17e-3 < s < 1.19e-3
    assert math.isclose(s, 10 ** (g["slope"] * 14.0 + g["intercept"]), rel_tol=1e-12)
    assert math.isclose(float(P.noise_sigma(19.0) / P.noise_sigma(18.0)), 10 ** g["slope"],
                        rel_tol=1e-12)


def test_paper_workload_draws_within_table1():
    # the paper-shaped inputs use Table 1's ranges (q searched as log10 q)
    rows = {r[1]: (float(r[3]), float(r[4])) for r in golden_rows("table1_parameter_ranges.txt")}
    names = ["q", "d", "u0", "alpha", "tE", "t0"]
    for j, nm in enumerate(names):
        lo, hi = rows[nm]
        if nm == "q":
            lo, hi = math.log10(lo), math.log10(hi)
        assert math.isclose(inputs.PAPER_LO[j], lo, abs_tol=1e-15), nm
        assert math.isclose(inputs.PAPER_HI[j], hi, rel_tol=1e-15, abs_tol=1e-15), nm
    assert inputs.PAPER_M0 == rows["m0"]
    wl = inputs.paper_workload(3, 500, 2)
    th = wl.theta
    for j, nm in enumerate(names):
        lo, hi = rows[nm]
        v = 10 ** th[j] if nm == "q" else th[j]
        tol = 1e-12 * max(abs(lo), abs(hi))
        assert np.all(v >= lo - tol) and np.all(v <= hi + tol), nm


def test_magnitudes_and_fluxes():
    # Pogson: 5 mag is a factor 100 in flux; the zero point maps to flux 1
    y, _ = P.to_flux(np.array([20.0, 25.0]), np.array([0.01, 0.01]))
    assert math.isclose(y[0], 1.0) and math.isclose(y[0] / y[1], 100.0, rel_tol=1e-12)
    # no magnification or no source light: the baseline magnitude
    assert np.allclose(P.magnitude(np.array([1.0, 7.3]), 19.0, np.array([0.4, 0.0])), 19.0)
    # unblended: m = m0 - 2.5 log10 A
    assert math.isclose(float(P.magnitude(10.0, 20.0, 1.0)), 17.5, rel_tol=1e-15)
    # fluxes of (m0, f) give back (m0, f)
    m0, f = 21.3, 0.27
    F0 = 10 ** (-0.4 * (m0 - 20.0))
    m0b, fb = P.fitted_m0_f(f * F0, (1 - f) * F0)
    assert math.isclose(m0b, m0, rel_tol=1e-14) and math.isclose(fb, f, rel_tol=1e-14)
    assert P.fitted_m0_f(-1.0, 0.5) is None


def test_flux_weights_match_magnitude_chi2_to_first_order():
    rng = np.random.default_rng(1)
    m = rng.uniform(18, 22, 200)
    sigma = P.noise_sigma(m)
    dm = 1e-5 * rng.standard_normal(200)
    y, w = P.to_flux(m, sigma)
    y2, _ = P.to_flux(m + dm, sigma)
    chi_f = np.sum(w * (y2 - y) ** 2)
    chi_m = np.sum((dm / sigma) ** 2)
    assert abs(chi_f / chi_m - 1) < 1e-4


def _case(experiment):
    theta = np.array([math.log10(0.5), 1.2, 0.3, 2.0, 20.0, 3.0])
    m0, f = 19.5, (1.0 if experiment == 1 else 0.6)
    A = np.linspace(1.0, 8.0, 100)
    m_true = P.magnitude(A, m0, f)
    sigma = np.full(100, 0.01)
    F0 = 10 ** (-0.4 * (m0 - 20.0))
    return theta, m0, f, A, m_true, sigma, f * F0, (1 - f) * F0


@pytest.mark.parametrize("experiment", [1, 2])
def test_success_criterion(experiment):
    theta, m0, f, A, m_true, sigma, Fs, Fb = _case(experiment)
    nu = 100 - (7 if experiment == 1 else 8)
    # the truth itself
    assert P.success(experiment, theta, Fs, Fb, A, m_true, sigma, m_true, theta, m0, f) == \
        (True, True, 0.0)
    # identical curve but one parameter 11% off: weak only; 9% off: strict
    for j, scale in ((1, 1.11), (2, 1.11), (4, 1.11)):
        th = theta.copy()
        th[j] *= scale
        assert P.success(experiment, th, Fs, Fb, A, m_true, sigma, m_true, theta, m0, f)[:2] \
            == (True, False)
        th[j] = theta[j] * 1.09
        assert P.success(experiment, th, Fs, Fb, A, m_true, sigma, m_true, theta, m0, f)[:2] \
            == (True, True)
    th = theta.copy()
    th[0] = math.log10(0.5 * 1.11)  # q 11% off
    assert P.success(experiment, th, Fs, Fb, A, m_true, sigma, m_true, theta, m0, f)[1] is False
    th = theta.copy()
    th[5] = theta[5] + 0.11 * theta[4]  # tm off by 0.11 tE
    assert P.success(experiment, th, Fs, Fb, A, m_true, sigma, m_true, theta, m0, f)[1] is False
    th = theta.copy()
    th[3] = theta[3] + 2 * math.pi - 0.05  # wrapped angle error 0.05 rad
    assert P.success(experiment, th, Fs, Fb, A, m_true, sigma, m_true, theta, m0, f)[1] is True
    # a fitted model offset by d magnitudes everywhere (through m0):
    # Delta chi^2 / nu = 100 (d / sigma)^2 / nu, just above and just below 1
    for factor, weak in ((1.01, False), (0.99, True)):
        d = 0.01 * math.sqrt(nu / 100.0) * factor
        g = 10 ** (-0.4 * d)
        w, s, dchi = P.success(experiment, theta, Fs * g, Fb * g, A, m_true, sigma, m_true,
                               theta, m0, f)
        assert w == weak and math.isclose(dchi, 100 * (d / 0.01) ** 2 / nu, rel_tol=1e-9)
    # a model with negative flux somewhere fails
    assert P.success(experiment, theta, -Fs, Fb, A, m_true, sigma, m_true, theta, m0, f)[:2] \
        == (False, False)
    # the lens-only strict test: the true lens with a blend fraction 20% off
    # (same m0; errors so large that the weak test passes) passes it and,
    # with blending, fails the full strict test
    tot, f2, big = Fs + Fb, f * 0.8, np.full(100, 10.0)
    r = P.success(experiment, theta, f2 * tot, (1 - f2) * tot, A, m_true, big, m_true,
                  theta, m0, f, lens_only=True)
    full = P.success(experiment, theta, f2 * tot, (1 - f2) * tot, A, m_true, big, m_true,
                     theta, m0, f)
    assert r[:2] == (True, True) and full[:2] == (True, experiment == 1)
    # a lens parameter 11% off fails the lens-only test, 9% off passes it
    th = theta.copy()
    th[2] *= 1.11
    assert P.success(experiment, th, Fs, Fb, A, m_true, sigma, m_true, theta, m0, f,
                     lens_only=True)[:2] == (True, False)
    th[2] = theta[2] * 1.09
    assert P.success(experiment, th, Fs, Fb, A, m_true, sigma, m_true, theta, m0, f,
                     lens_only=True)[:2] == (True, True)


def test_peak_count_against_scipy_prominence():
    rng = np.random.default_rng(2)
    t = np.linspace(-3, 3, P.GRID)
    for _ in range(40):
        k = int(rng.integers(1, 6))
        centres = rng.uniform(-2.5, 2.5, k)
        widths = rng.uniform(0.02, 0.5, k)
        heights = rng.uniform(0.001, 3.0, k)
        A = 1.0 + 1.0 / np.sqrt(t ** 2 + 0.3 ** 2)
        for c, wd, h in zip(centres, widths, heights):
            A = A + h * np.exp(-0.5 * ((t - c) / wd) ** 2)
        M = 2.5 * np.log10(A)
        peaks, props = find_peaks(M, prominence=0.0)
        prom = props["prominences"]
        if np.any(np.abs(prom - P.PROMINENCE) < 1e-6):
            continue  # too close to the threshold to compare
        assert P.peak_count(A) == int(np.sum(prom >= P.PROMINENCE))


def test_peak_count_simple_curves():
    t = np.linspace(-3, 3, P.GRID)
    u = np.sqrt(t ** 2 + 0.1 ** 2)
    A = (u ** 2 + 2) / (u * np.sqrt(u ** 2 + 4))  # a point lens: one peak
    assert P.peak_count(A) == 1
    assert P.peak_count(np.ones(50)) == 0 and P.peak_class(0) == 1
    assert P.peak_count(np.linspace(1, 2, 50)) == 0  # monotone: no interior maximum
    # a flat top counts once
    assert P.peak_count(np.array([1.0, 2.0, 3.0, 3.0, 3.0, 2.0, 1.0])) == 1
    # two bumps 0.5 mag apart from the saddle
    B = np.concatenate([np.linspace(1, 2, 10), np.linspace(2, 1.2, 10), np.linspace(1.2, 2.5, 10),
                        np.linspace(2.5, 1, 10)])
    assert P.peak_count(B) == 2
    assert [P.peak_class(c) for c in (1, 2, 3, 4, 7)] == [1, 2, 3, 4, 4]

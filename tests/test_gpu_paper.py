"""The experiment harness (lightcurves, noise, fluxes, peak classes, the
paper's success criterion) against the experiment oracle on the same draws;
the harness takes its magnifications from the library, the oracle from the
CPU oracle."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from oracle import paper_oracle as P
from paper_1208_4830_amd import experiments as E
from paper_1208_4830_amd import inputs

pytestmark = pytest.mark.gpu


def _oracle_obs(wl, k):
    sl = slice(wl.off[k], wl.off[k + 1])
    A, _ = O.magnify(wl.theta[:, k:k + 1], wl.t[sl])
    return P.observe(wl.experiment, A[0], wl.m0[k], wl.f[k], wl.noise[sl])


@pytest.mark.parametrize("experiment", [1, 2])
def test_harness_matches_oracle(hip, experiment):
    wl = inputs.paper_workload(5, 24, experiment)
    obs = E.observations(hip, torch, wl)
    y_dev, w_dev = obs["lcs"].y.cpu().numpy(), obs["lcs"].w.cpu().numpy()
    for k in range(wl.n_lc):
        sl = slice(wl.off[k], wl.off[k + 1])
        m_true, m_obs, sigma = _oracle_obs(wl, k)
        assert np.max(np.abs(obs["m_obs"][sl] - m_obs)) < 1e-9
        assert np.max(np.abs(obs["sigma"][sl] / sigma - 1)) < 1e-9
        y, w = P.to_flux(m_obs, sigma)
        assert np.max(np.abs(y_dev[sl] / y - 1)) < 1e-9
        assert np.max(np.abs(w_dev[sl] / w - 1)) < 1e-8
    # peak classes from the library's magnification on the grid
    classes = E.peak_classes(hip, torch, wl)
    for k in range(wl.n_lc):
        A, _ = O.magnify(wl.theta[:, k:k + 1], P.grid(wl.t_start[k], wl.t_end[k]))
        assert classes[k] == P.peak_class(P.peak_count(A[0])), k
    # the truth passes both criteria with Delta chi^2 = 0
    F0 = 10 ** (-0.4 * (wl.m0 - 20.0))
    weak, strict, dchi = E.evaluate(hip, torch, wl, obs, wl.theta, wl.f * F0, (1 - wl.f) * F0)
    assert weak.all() and strict.all() and np.all(np.abs(dchi) < 1e-9)
    # perturbed fits with fluxes profiled by the library: the same Delta
    # chi^2 / nu and decisions as the oracle's evaluation
    rng = np.random.default_rng(6)
    lo, hi = inputs.PAPER_LO, inputs.PAPER_HI
    for scale in (1e-4, 3e-3, 3e-2):
        x = (wl.theta - lo[:, None]) / (hi - lo)[:, None]
        x = np.clip(x + scale * rng.standard_normal(x.shape), 0, 1)
        th = lo[:, None] + (hi - lo)[:, None] * x
        _, fs, fb = hip.sblm_chi2(obs["lcs"], torch.as_tensor(th, device="cuda"), 1)
        fs, fb = fs.cpu().numpy(), fb.cpu().numpy()
        weak, strict, dchi = E.evaluate(hip, torch, wl, obs, th, fs, fb)
        _, strict_l, _ = E.evaluate(hip, torch, wl, obs, th, fs, fb, lens_only=True)
        for k in range(wl.n_lc):
            sl = slice(wl.off[k], wl.off[k + 1])
            m_true, m_obs, sigma = _oracle_obs(wl, k)
            A, _ = O.magnify(th[:, k:k + 1], wl.t[sl])
            w_o, s_o, d_o = P.success(experiment, th[:, k], fs[k], fb[k], A[0], m_obs, sigma,
                                      m_true, wl.theta[:, k], wl.m0[k], wl.f[k])
            if math.isinf(d_o):
                assert math.isinf(dchi[k]) and not weak[k]
                continue
            assert abs(dchi[k] - d_o) <= 1e-7 * abs(d_o) + 1e-9, (scale, k)
            if abs(d_o - 1.0) > 1e-6:
                assert (weak[k], strict[k]) == (w_o, s_o), (scale, k)
                l_o = P.success(experiment, th[:, k], fs[k], fb[k], A[0], m_obs, sigma, m_true,
                                wl.theta[:, k], wl.m0[k], wl.f[k], lens_only=True)[1]
                assert strict_l[k] == l_o, (scale, k)


def test_experiment_runs_end_to_end(hip):
    out = E.run_experiment(hip, torch, 2, n_lc=12, pop=32, checkpoints=(10, 20), passes=1,
                           iterated=(2, 1, 50), seed=3)
    assert out["experiment"] == 2 and sum(out["classes"].values()) == 12
    assert [r["gen"] for r in out["checkpoints"]] == [10, 20]
    for r in out["checkpoints"]:
        for form in ("ea", "ea_amoeba"):
            s, w = r[form]["strict"]["all"], r[form]["weak"]["all"]
            sl = r[form]["strict_lens"]["all"]
            assert 0.0 <= s <= sl <= w <= 1.0
    assert 0.0 <= out["iterated_simplex"]["weak"]["all"] <= 1.0

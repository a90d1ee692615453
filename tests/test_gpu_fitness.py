"""Parity of the HIP fitness path (sblm_magnify, sblm_chi2) with the FP64 CPU
oracle on identical seeded inputs."""
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_1208_4830_amd import inputs
from tests.helpers import (ambiguous_count, csr_workload, magnification_condition,
                           oracle_lightcurves, rel_err, source_positions)

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _cuda(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def _check_magnify(hip, theta, t, mode, floor):
    n_img = torch.zeros((theta.shape[1], t.size), dtype=torch.int8, device=DEV)
    st = hip.new_stats()
    A = hip.sblm_magnify(_cuda(theta), _cuda(t), mode=mode, n_img=n_img, stats=st)
    torch.cuda.synchronize()
    A, n_img = A.cpu().numpy(), n_img.cpu().numpy()
    Ao, no = O.magnify(theta, t)
    err = rel_err(A, Ao)
    zeta = source_positions(theta, t)
    bad = np.argwhere(err > floor)
    tau = (t[None, :] - theta[5][:, None]) / theta[4][:, None]
    for i, k in bad:  # beyond the floor only where the problem is ill-conditioned
        q, d = 10 ** theta[0, i], theta[1, i]
        kappa = magnification_condition(zeta[i, k], d, q, tau[i, k], theta[2, i])
        assert err[i, k] <= max(floor, kappa), (i, k, err[i, k], kappa, A[i, k])
    mism = np.argwhere(n_img != no)
    for i, k in mism:
        q, d = 10 ** theta[0, i], theta[1, i]
        assert ambiguous_count(zeta[i, k], d, q), (i, k, n_img[i, k], no[i, k])
    s = hip.stats_dict(st)
    assert s["n_solves"] == theta.shape[1] * t.size and s["n_capped"] == 0
    return err, s


@pytest.mark.parametrize("mode,floor", [(0, 1e-10), (1, 1e-6)])
def test_magnify_parity(hip, mode, floor):
    rng = np.random.default_rng(100)
    theta = inputs.draw_theta(rng, 24)
    # ragged tail: 1237 = 19 chunks of 64 + 21; epochs cover t0 +- 2 tE of all
    t = np.linspace(-210.0, 210.0, 1237)
    err, s = _check_magnify(hip, theta, t, mode, floor)
    print(f"mode {mode}: max rel err {err.max():.3e}, median {np.median(err):.3e}, "
          f"sweeps/solve {s['n_iter'] / s['n_solves']:.2f}, fallback {s['n_fallback']}")


@pytest.mark.parametrize("mode", [0, 1])
def test_magnify_small_and_tail_shapes(hip, mode):
    rng = np.random.default_rng(101)
    for n, n_t in [(1, 1), (1, 2), (3, 63), (2, 64), (2, 65), (5, 17)]:
        theta = inputs.draw_theta(rng, n)
        t = np.sort(rng.uniform(-150, 150, n_t))
        _check_magnify(hip, theta, t, mode, 1e-10 if mode == 0 else 1e-6)
    # n_t = 0 is a no-op
    A = torch.zeros((2, 0), dtype=torch.float64, device=DEV)
    hip.sblm_magnify(_cuda(inputs.draw_theta(rng, 2)), torch.zeros(0, dtype=torch.float64,
                                                                     device=DEV), A=A)


def test_magnify_source_on_primary(hip):
    # u0 = 0 and t = t0: zeta = 0, the leading coefficient vanishes (degree 4)
    theta = np.array([[-1.0], [1.2], [0.0], [0.3], [20.0], [1.5]])
    t = np.array([1.5 - 0.2, 1.5, 1.5 + 0.2])
    st = hip.new_stats()
    for mode in (0, 1):
        A = hip.sblm_magnify(_cuda(theta), _cuda(t), mode=mode, stats=st).cpu().numpy()
        Ao, _ = O.magnify(theta, t)
        assert np.all(rel_err(A, Ao) < 1e-9), (A, Ao)
    assert hip.stats_dict(st)["n_degree4"] == 2


def test_magnify_source_near_a_lens(hip):
    # sources 1e-3 ... 1e-11 theta_E from the primary or the secondary (one
    # epoch each, every solve cold): the spurious fifth root lies near
    # -c4/c5, out to ~1/|zeta|; every solve converges, and A agrees with the
    # oracle
    thetas, ts = [], []
    rng = np.random.default_rng(103)
    for lq, d in ((0.0, 1.0), (-3.0, 0.5), (-1.0, 2.0)):
        for r in (1e-3, 1e-5, 1e-7, 1e-9, 1e-11):
            for lens in (0.0, d):
                zeta = lens + r * np.exp(1j * rng.uniform(0, 2 * np.pi))
                al = rng.uniform(0, 2 * np.pi)
                rot = zeta * np.exp(-1j * al)
                u0, tau = rot.real, -rot.imag
                if u0 < 0:
                    al += np.pi
                    u0, tau = -u0, -tau
                tE, t0 = rng.uniform(10, 100), rng.uniform(-10, 10)
                thetas.append([lq, d, u0, al, tE, t0])
                ts.append(t0 + tau * tE)
    theta = np.array(thetas).T
    for mode in (0, 1):
        st = hip.new_stats()
        for i in range(theta.shape[1]):
            A = hip.sblm_magnify(_cuda(theta[:, i:i + 1]), _cuda([ts[i]]), mode=mode,
                                 stats=st).cpu().numpy()[0, 0]
            Ao, _ = O.magnify(theta[:, i:i + 1], np.array([ts[i]]), nthreads=1)
            assert rel_err(A, Ao[0, 0]) < 1e-9, (i, A, Ao[0, 0])
        s = hip.stats_dict(st)
        assert s["n_capped"] == 0 and s["n_unsettled"] == 0, s
        # the fifth root starts where it lies: no solve needs the 50-80
        # sweeps that walking it out from the circle start would take
        assert s["n_iter"] <= 40 * s["n_solves"], s


def test_magnify_near_caustics(hip):
    # sources placed within 0.01 theta_E of caustics: agreement to the
    # conditioning of the problem; image counts agree off the ambiguous zone
    rng = np.random.default_rng(102)
    thetas, ts = [], []
    for _ in range(6):
        lq, d = rng.uniform(-3, 0), rng.uniform(0.5, 2)
        zc, _ = O.caustic_points(d, 10 ** lq, 40, rng)
        zeta = zc + rng.uniform(0, 0.01, zc.size) * np.exp(1j * rng.uniform(0, 2 * np.pi, zc.size))
        for z in zeta:
            al = rng.uniform(0, 2 * np.pi)
            rot = z * np.exp(-1j * al)
            u0, tau = rot.real, -rot.imag
            if u0 < 0:
                al += np.pi
                u0, tau = -u0, -tau
            tE, t0 = rng.uniform(10, 100), rng.uniform(-10, 10)
            thetas.append([lq, d, u0, al, tE, t0])
            ts.append(t0 + tau * tE)
    theta = np.array(thetas).T
    for mode, floor in [(0, 1e-10), (1, 1e-6)]:
        # one epoch per individual: evaluate each on its own epoch
        A = np.zeros(theta.shape[1])
        for i in range(theta.shape[1]):
            A[i] = hip.sblm_magnify(_cuda(theta[:, i:i + 1]), _cuda([ts[i]]),
                                    mode=mode).cpu().numpy()[0, 0]
        for i in range(theta.shape[1]):
            Ao, _ = O.magnify(theta[:, i:i + 1], np.array([ts[i]]), nthreads=1)
            e = rel_err(A[i], Ao[0, 0])
            if e > floor:
                z = source_positions(theta[:, i:i + 1], np.array([ts[i]]))[0, 0]
                tau = (ts[i] - theta[5, i]) / theta[4, i]
                kappa = magnification_condition(z, theta[1, i], 10 ** theta[0, i], tau,
                                                theta[2, i])
                assert e <= kappa, (i, e, kappa)


def _chi2_case(hip, wl, pop, mode, seed=7):
    y, w = oracle_lightcurves(wl)
    rng = np.random.default_rng(seed)
    n = wl.n_lc * pop
    th = inputs.draw_theta(rng, n)
    th[:, ::pop] = wl.theta  # first individual of every lightcurve = truth
    lcs = hip.Lightcurves(_cuda(wl.off, torch.int64), _cuda(wl.t), _cuda(y), _cuda(w))
    st = hip.new_stats()
    c, fs, fb = hip.sblm_chi2(lcs, _cuda(th), pop, mode=mode, stats=st)
    torch.cuda.synchronize()
    co, fso, fbo = O.chi2(wl.off, wl.t, y, w, th, pop)
    return (c.cpu().numpy(), fs.cpu().numpy(), fb.cpu().numpy()), (co, fso, fbo), st


@pytest.mark.parametrize("mode", [0, 1])
def test_chi2_parity_ragged(hip, mode):
    lengths = [0, 1, 2, 3, 63, 64, 65, 127, 400, 1000, 1537]
    wl = csr_workload(11, lengths)
    (c, fs, fb), (co, fso, fbo), st = _chi2_case(hip, wl, pop=5, mode=mode)
    # relative 1e-8, with an absolute floor at the rounding level of sum w y^2
    # (lightcurves of <= 2 points are fitted exactly: chi2 is rounding noise)
    y, w = oracle_lightcurves(wl)
    scale = np.array([np.sum(w[wl.off[k]:wl.off[k + 1]] * y[wl.off[k]:wl.off[k + 1]] ** 2)
                      for k in range(wl.n_lc)]).repeat(5)
    assert np.all(np.abs(c - co) <= 1e-8 * co + 1e-14 * scale), rel_err(c, co).max()
    assert np.all(np.abs(fs - fso) <= 1e-7 * np.maximum(np.abs(fso), 1e-3))
    assert np.all(np.abs(fb - fbo) <= 1e-7 * np.maximum(np.abs(fbo), 1e-3))
    # empty / single-point lightcurves: degenerate 2x2 system
    assert np.all(c[:5] == 0) and np.all(fs[:10] == 0) and np.all(fb[:5] == 0)
    assert hip.stats_dict(st)["n_capped"] == 0


def test_chi2_deterministic_and_schedule_independent(hip):
    wl = csr_workload(12, [300, 700, 1000])
    outs = []
    for lanes, asy in (("64", "0"), ("64", "0"), ("32", "0"), ("16", "0"), ("16", "1"),
                       ("32", "1"), ("256", "0"), ("128", "0")):
        os.environ["SBLM_LANES"], os.environ["SBLM_ASYNC"] = lanes, asy
        try:
            (c, fs, fb), (co, _, _), _ = _chi2_case(hip, wl, pop=8, mode=0)
        finally:
            del os.environ["SBLM_LANES"], os.environ["SBLM_ASYNC"]
        outs.append(c)
        assert np.all(rel_err(c, co) < 1e-8)
    assert np.array_equal(outs[0], outs[1])  # bitwise repeatable


@pytest.mark.parametrize("mode", [0, 1])
def test_chi2_full_size_sampled(hip, mode):
    # 256 lightcurves x 1000 uniform epochs, population 256 (the batched
    # FP64 workload), in the default launch configuration; sampled
    # individuals checked against the oracle one by one
    wl = inputs.uniform_workload(2, 256, 1000)
    rng = np.random.default_rng(3)
    y, w = oracle_lightcurves(wl)
    pop = 256
    th = inputs.draw_theta(rng, wl.n_lc * pop)
    th[:, ::pop] = wl.theta
    lcs = hip.Lightcurves(_cuda(wl.off, torch.int64), _cuda(wl.t), _cuda(y), _cuda(w))
    c, fs, fb = hip.sblm_chi2(lcs, _cuda(th), pop, mode=mode)
    c = c.cpu().numpy()
    sample = np.concatenate([np.arange(0, wl.n_lc * pop, pop)[:16],
                             rng.choice(wl.n_lc * pop, 48, replace=False)])
    for i in sample:
        lc = i // pop
        sl = slice(wl.off[lc], wl.off[lc + 1])
        Ao, _ = O.magnify(th[:, i:i + 1], wl.t[sl])
        co, _, _ = O.lsq_chi2(Ao[0], y[sl], w[sl])
        assert rel_err(c[i], co) < 1e-8, (i, c[i], co)

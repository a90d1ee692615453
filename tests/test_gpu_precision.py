"""Magnification error of the FP64 and mixed paths against the FP64 oracle on
10^7 (parameters, epoch) pairs, 20% of them within 0.01 theta_E of a caustic."""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
from tests.helpers import (generic_pairs, magnification_condition, near_caustic_pairs,
                           rel_err)

pytestmark = pytest.mark.gpu

N_PAIRS = int(os.environ.get("SBLM_PRECISION_PAIRS", "10000000"))


def _gpu_A(hip, theta_shift, mode, chunk=2_000_000):
    """A of pairs given as individuals evaluated at the shared epoch t = 0."""
    out = np.empty(theta_shift.shape[1])
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    for a in range(0, theta_shift.shape[1], chunk):
        th = torch.as_tensor(np.ascontiguousarray(theta_shift[:, a:a + chunk]), device="cuda")
        out[a:a + chunk] = hip.sblm_magnify(th, t, mode=mode).cpu().numpy()[:, 0]
    return out


def test_precision_report(hip):
    rng = np.random.default_rng(2024)
    n_c = N_PAIRS // 5
    th_g, t_g = generic_pairs(rng, N_PAIRS - n_c)
    th_c, t_c = near_caustic_pairs(rng, n_c)
    theta = np.concatenate([th_g, th_c], axis=1)
    t = np.concatenate([t_g, t_c])
    near = np.zeros(theta.shape[1], bool)
    near[N_PAIRS - n_c:] = True
    # every pair as its own individual at epoch 0: shift t0 by the epoch
    sh = theta.copy()
    sh[5] = theta[5] - t
    Ao, _ = O.magnify(sh, np.zeros(1))
    Ao = Ao[:, 0]
    report = {"pairs": int(theta.shape[1]), "near_caustic": int(n_c)}
    for mode, floor in ((0, 1e-10), (1, 1e-6)):
        A = _gpu_A(hip, sh, mode)
        err = rel_err(A, Ao)
        r = {}
        for name, m in (("all", np.ones_like(near)), ("generic", ~near), ("near_caustic", near)):
            e = err[m]
            r[name] = dict(max=float(e.max()), p999=float(np.quantile(e, 0.999)),
                           median=float(np.median(e)), beyond_floor=int(np.sum(e > floor)))
        # every point beyond the floor must lie within the rounding bound of
        # the problem at that point (checked on up to 3000 of them)
        bad = np.flatnonzero(err > floor)
        checked = bad if bad.size <= 3000 else rng.choice(bad, 3000, replace=False)
        unexplained = 0
        for i in checked:
            zeta = (sh[5, i] * -1 / sh[4, i]) * np.sin(sh[3, i]) + sh[2, i] * np.cos(sh[3, i]) + \
                1j * ((sh[5, i] / sh[4, i]) * np.cos(sh[3, i]) + sh[2, i] * np.sin(sh[3, i]))
            tau = -sh[5, i] / sh[4, i]
            kappa = magnification_condition(zeta, sh[1, i], 10 ** sh[0, i], tau, sh[2, i])
            unexplained += err[i] > max(floor, kappa)
        r["beyond_floor_checked"] = int(checked.size)
        r["beyond_floor_unexplained"] = int(unexplained)
        report["fp64" if mode == 0 else "mixed"] = r
        assert unexplained == 0, r
    print("PRECISION_REPORT " + json.dumps(report))

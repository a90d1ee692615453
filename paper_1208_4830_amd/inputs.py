"""Seeded synthetic workloads shaped like the paper's fitting experiments.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no magnification, no chi^2), so both the HIP library's
tests and the CPU oracle can take their inputs from it.  Observed fluxes are
assembled by the caller from its own magnifications as
    F_true = Fs * A + Fb,   sigma = s * F_true,   y = F_true + sigma * noise.

Parameter priors (planes in the library's order):
    log10 q ~ U[-3, 0], d ~ U[0.5, 2], u0 ~ U[0, 0.5], alpha ~ U[0, 2 pi),
    tE ~ U[10, 100] d, t0 ~ U[-10, 10] d;  Fs = 1, Fb ~ U[0, 0.5].
"""
from dataclasses import dataclass

import numpy as np

PRIOR_LO = np.array([-3.0, 0.5, 0.0, 0.0, 10.0, -10.0])
PRIOR_HI = np.array([0.0, 2.0, 0.5, 2.0 * np.pi, 100.0, 10.0])
PARAM_NAMES = ("log10q", "d", "u0", "alpha", "tE", "t0")


def draw_theta(rng, n):
    """theta[6][n] from the priors above (alpha in [0, 2 pi))."""
    u = rng.random((6, n))
    return PRIOR_LO[:, None] + (PRIOR_HI - PRIOR_LO)[:, None] * u


def draw_blend(rng, n):
    """(Fs, Fb): Fs = 1, Fb ~ U[0, 0.5]."""
    return np.ones(n), rng.uniform(0.0, 0.5, n)


def uniform_epochs(theta, L):
    """L epochs uniform over [t0 - 2 tE, t0 + 2 tE] for every column of theta."""
    tE, t0 = theta[4], theta[5]
    k = np.arange(L) / max(L - 1, 1)
    return t0[:, None] - 2.0 * tE[:, None] + 4.0 * tE[:, None] * k[None, :]


def irregular_epochs(rng, tE, t0, L, window=(-2.0, 2.0)):
    """Survey-like cadence for one lightcurve, sorted, length L.

    Nightly 8-hour windows over [t0 + a tE, t0 + b tE] ((a, b) = window),
    consecutive points 5-30 min apart within a night; 0.9 L points drawn
    without replacement from that schedule (its spacing is scaled down if it
    holds fewer points) plus 0.1 L points uniform in [t0 - 0.1 tE, t0 + 0.1 tE].
    """
    n_dense = int(round(0.1 * L))
    n_sched = L - n_dense
    t_a, t_b = t0 + window[0] * tE, t0 + window[1] * tE
    night0 = np.floor(t_a)
    nights = np.arange(night0, np.ceil(t_b) + 1.0)
    expect = len(nights) * (8 * 60) / 17.5
    scale = min(1.0, expect / max(1.5 * n_sched, 1))
    sched = []
    for nt in nights:
        start, end = nt + 0.1, nt + 0.1 + 8.0 / 24.0
        gaps = rng.uniform(5.0, 30.0, int(8 * 60 / (5.0 * scale)) + 2) * scale / 1440.0
        ts = start + np.cumsum(gaps)
        ts = ts[(ts < end) & (ts >= t_a) & (ts <= t_b)]
        sched.append(ts)
    sched = np.concatenate(sched)
    if sched.size < n_sched:  # extremely short events: top up uniformly
        sched = np.concatenate([sched, rng.uniform(t_a, t_b, n_sched - sched.size)])
    pick = rng.choice(sched.size, n_sched, replace=False)
    dense = rng.uniform(t0 - 0.1 * tE, t0 + 0.1 * tE, n_dense)
    return np.sort(np.concatenate([sched[pick], dense]))


@dataclass
class Workload:
    """A batch of synthetic lightcurves before fluxes are assembled."""
    theta: np.ndarray     # [6][n_lc] true parameters
    Fs: np.ndarray        # [n_lc]
    Fb: np.ndarray        # [n_lc]
    off: np.ndarray       # [n_lc+1] CSR offsets (int64)
    t: np.ndarray         # [off[-1]] epochs
    sfrac: np.ndarray     # [off[-1]] sigma / F_true per point
    noise: np.ndarray     # [off[-1]] standard normal draws

    @property
    def n_lc(self):
        return self.off.shape[0] - 1


def uniform_workload(seed, n_lc, L, sigma_frac=0.01):
    """n_lc lightcurves, L uniform epochs over t0 +- 2 tE, sigma = 1% of flux."""
    rng = np.random.default_rng(seed)
    theta = draw_theta(rng, n_lc)
    Fs, Fb = draw_blend(rng, n_lc)
    t = uniform_epochs(theta, L).ravel()
    off = np.arange(n_lc + 1, dtype=np.int64) * L
    return Workload(theta, Fs, Fb, off, t, np.full(t.size, sigma_frac),
                    rng.standard_normal(t.size))


def ragged_workload(seed, n_lc, L_min=200, L_max=5000):
    """Ragged batch: L ~ U{L_min..L_max}, irregular cadence, s ~ U[0.5%, 3%];
    each lightcurve observed from t0 + a tE to t0 + b tE with a ~ U(-3, -2),
    b ~ U(2, 3), the random start and end of the paper's test lightcurves
    (Sec. 4.2)."""
    rng = np.random.default_rng(seed)
    theta = draw_theta(rng, n_lc)
    Fs, Fb = draw_blend(rng, n_lc)
    lens = rng.integers(L_min, L_max + 1, n_lc)
    wins = np.stack([rng.uniform(-3.0, -2.0, n_lc), rng.uniform(2.0, 3.0, n_lc)], 1)
    ts = [irregular_epochs(rng, theta[4, k], theta[5, k], int(lens[k]), tuple(wins[k]))
          for k in range(n_lc)]
    off = np.zeros(n_lc + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    t = np.concatenate(ts)
    return Workload(theta, Fs, Fb, off, t, rng.uniform(0.005, 0.03, t.size),
                    rng.standard_normal(t.size))


def population(rng, n_lc, pop):
    """Random encoded population P[6][n_lc*pop], entries in (0,1)."""
    return rng.random((6, n_lc * pop))


# ------------------------------------------------ the paper's own experiments
#
# Table 1 ranges (the paper's a, b, m0, q, theta, tE, tm are the library's
# d, u0, m0, q, alpha, tE, t0), 100 points per lightcurve between a start in
# tm + tE (-3, -2) and an end in tm + tE (2, 3) (Sec. 4.2).  Experiment 1
# (Table 2): uniform sampling, no noise, no blending.  Experiment 2 (Table
# 3): times uniform at random in (t_start, t_end), Gaussian magnitude noise
# and a blend fraction f.  Only draws here; magnitudes, the noise model and
# fluxes are assembled by the caller.

PAPER_LO = np.array([-1.0, 0.6, 0.001, 0.0, 5.0, -20.0])  # log10 q for q in [0.1, 1]
PAPER_HI = np.array([0.0, 1.7, 1.0, 2.0 * np.pi, 50.0, 20.0])
PAPER_M0 = (18.0, 22.0)


@dataclass
class PaperWorkload:
    """Lightcurves of the paper's experiments before magnitudes are made."""
    experiment: int       # 1 (Table 2) or 2 (Table 3)
    theta: np.ndarray     # [6][n_lc] true parameters, library order
    m0: np.ndarray        # [n_lc] baseline magnitude
    f: np.ndarray         # [n_lc] blend fraction (1 in experiment 1)
    t_start: np.ndarray   # [n_lc]
    t_end: np.ndarray     # [n_lc]
    off: np.ndarray       # [n_lc+1] CSR offsets (int64)
    t: np.ndarray         # [off[-1]] epochs
    noise: np.ndarray     # [off[-1]] standard normal draws (experiment 2)

    @property
    def n_lc(self):
        return self.off.shape[0] - 1


def paper_workload(seed, n_lc, experiment, L=100):
    """n_lc lightcurves of experiment 1 or 2, L points each.  q is drawn
    uniformly in [0.1, 1] (the table's range), the others uniformly in
    theirs; f ~ U(0, 1] in experiment 2."""
    if experiment not in (1, 2):
        raise ValueError("experiment is 1 or 2")
    rng = np.random.default_rng(seed)
    theta = np.empty((6, n_lc))
    theta[0] = np.log10(rng.uniform(0.1, 1.0, n_lc))
    for j in range(1, 6):
        theta[j] = rng.uniform(PAPER_LO[j], PAPER_HI[j], n_lc)
    m0 = rng.uniform(PAPER_M0[0], PAPER_M0[1], n_lc)
    f = np.ones(n_lc) if experiment == 1 else 1.0 - rng.random(n_lc)
    tE, tm = theta[4], theta[5]
    t_start = tm + tE * rng.uniform(-3.0, -2.0, n_lc)
    t_end = tm + tE * rng.uniform(2.0, 3.0, n_lc)
    if experiment == 1:
        k = np.arange(L) / (L - 1)
        t = t_start[:, None] + (t_end - t_start)[:, None] * k[None, :]
    else:
        t = np.sort(t_start[:, None] + (t_end - t_start)[:, None] * rng.random((n_lc, L)),
                    axis=1)
    off = np.arange(n_lc + 1, dtype=np.int64) * L
    return PaperWorkload(experiment, theta, m0, f, t_start, t_end, off, t.ravel(),
                         rng.standard_normal(n_lc * L))

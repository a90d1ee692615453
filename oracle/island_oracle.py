"""Island (coarse-grained) form of the evolutionary algorithm: several
populations per lightcurve that evolve independently by the rules of
Appendix A and exchange their fittest members now and then (Sec. 5.3, the
second of the parallelisation schemes discussed there).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain Python around
the C oracle EA (`oracle.EA`), one island at a time, migration written out
rank by rank.

The paper names the scheme but fixes none of its settings; the readings
taken here:
  I1  Lightcurve k has n_isl islands of pop rows each.  Island i is an
      Appendix-A EA of its own whose random draws are keyed by
      lc = k * n_isl + i, so that a one-island run is the plain EA.
  I2  Migration happens before the generation step of generation g (g =
      generations completed, the same on every island) when g > 0 and
      g % every == 0, on the fitness just evaluated for that generation.
      All islands send at once, from the state before any of them receives.
  I3  Ring topology: island i sends to island (i + 1) % n_isl.  The m
      fittest rows of the sender (stable ascending chi^2, NaN counted as
      +inf, ties in row order) are copied, with their chi^2, Fs and Fb,
      over the m least fit rows of the receiver ranked the same way: the
      r-th fittest emigrant replaces the row of rank pop - 1 - r.
      Requires 2 m <= pop.
  I4  A lightcurve's result is the best record over its islands (lowest
      island index on equal chi^2).
"""
import math

import numpy as np

from . import oracle as O


def _key(c):
    return math.inf if math.isnan(c) else c


def ranking(chi2):
    """Row indices from fittest to least fit (stable, NaN as +inf)."""
    return sorted(range(len(chi2)), key=lambda i: (_key(chi2[i]), i))


def migrate(P, chi2, Fs, Fb, m):
    """Ring migration (I3) among the islands of one lightcurve, in place.

    P: list of [pop][6] arrays; chi2, Fs, Fb: lists of [pop] arrays, one
    entry per island.
    """
    n = len(P)
    pop = len(chi2[0])
    assert 2 * m <= pop
    send = []
    for i in range(n):
        r = ranking(chi2[i])[:m]
        send.append([(P[i][row].copy(), chi2[i][row], Fs[i][row], Fb[i][row]) for row in r])
    for j in range(n):
        src = send[(j - 1) % n]
        worst = ranking(chi2[j])[::-1][:m]
        for r, row in enumerate(worst):
            p, c, s, b = src[r]
            P[j][row] = p
            chi2[j][row], Fs[j][row], Fb[j][row] = c, s, b


class IslandEA:
    """The n_isl islands of lightcurve lc (I1); P of island i is eas[i].P."""

    def __init__(self, n_isl, pop, seed, lc, every, m, **kw):
        self.n_isl, self.pop, self.every, self.m = n_isl, pop, every, m
        self.eas = [O.EA(pop, seed, lc * n_isl + i, **kw) for i in range(n_isl)]
        self.gen = 0

    def generation(self, chi2, Fs, Fb, force=False):
        """One step from the fitness [n_isl * pop] of the current rows
        (island-major): migrate when due (I2), then every island's
        Appendix-A generation.  Returns the fitness after migration."""
        pop = self.pop
        chi2, Fs, Fb = (np.array(a, dtype=np.float64) for a in (chi2, Fs, Fb))
        parts = [slice(i * pop, (i + 1) * pop) for i in range(self.n_isl)]
        c = [chi2[s] for s in parts]
        f = [Fs[s] for s in parts]
        b = [Fb[s] for s in parts]
        due = self.m > 0 and self.n_isl > 1 and self.every > 0 and \
            self.gen > 0 and self.gen % self.every == 0
        if due or force:
            migrate([ea.P for ea in self.eas], c, f, b, self.m)
        for i, ea in enumerate(self.eas):
            ea.generation(c[i], f[i], b[i])
        self.gen += 1
        return np.concatenate(c), np.concatenate(f), np.concatenate(b)

    def rows(self):
        """[n_isl * pop][6], island-major."""
        return np.concatenate([ea.P for ea in self.eas])

    def best(self):
        """(island index, summary) of the best record (I4)."""
        sums = [ea.summary() for ea in self.eas]
        i = min(range(self.n_isl), key=lambda k: (_key(sums[k]["best_chi2"]), k))
        return i, sums[i]

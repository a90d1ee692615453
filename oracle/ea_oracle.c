/*
 * ea_oracle.c -- plain CPU reference of the evolutionary algorithm of
 * Rajpaul (2012), Appendix A.  TEST INFRASTRUCTURE ONLY (see
 * sblm_oracle.c).  One lightcurve at a time, population matrix stored
 * row-major as P[i*6 + j] (row i = individual, column j = gene), entries
 * encoded in [0,1] (Sec. A.2).
 *
 * The paper draws its random numbers from MATLAB's generator; here every
 * draw is a word of Philox4x64-10 (Salmon, Moraes, Dror & Shaw 2011,
 * "Parallel random numbers: as easy as 1, 2, 3") so that any implementation
 * can reproduce the exact sequence.  Stream layout: key = (seed, lc),
 * counter = (generation, purpose, row, j/4), word j%4.
 *
 * Readings of Appendix A adopted here, where the text is silent:
 *   E1 (A.1)  "another random element gets 1 - X": row i + pop/2 is the
 *             complement of row i; an odd last row is drawn fresh.
 *   E2 (A.3)  ranking is a stable ascending sort on chi^2 (lower chi^2 =
 *             fitter), NaN counted as +inf, ties kept in row order.
 *   E3 (A.4)  the N_tourn tournament draws are with replacement; a pairing
 *             may select the same parent twice.
 *   E4 (A.5)  rows 1..pop-1 are filled pairing by pairing (pairing k gives
 *             rows 2k+1 and 2k+2); when pop-1 is odd the second child of the
 *             last pairing is discarded.  Mode chosen uniformly from
 *             {U(0,1), Bin(1,1/2), all ones}; the two children are
 *             fma(f, p_i, (1-f) p_j) and fma(f, p_j, (1-f) p_i), clamped.
 *   E5 (A.6)  creep acts on every gene of every offspring (never on row 0),
 *             X = 2^(-52 u) with u uniform (so ln X ~ U(ln eps, 0) with eps
 *             = 2^-52), p- = p - p X, p+ = p + (1-p) X, each computed with
 *             one fused multiply-add, sign from the top bit of a draw; jump
 *             follows creep, gene by gene, with probability p_mut.
 *   E6 (A.7)  stagnation test on b(g) = best chi^2 of generation g, once g
 *             is at least `window` generations into the current sequence:
 *             stagnated unless b(g - window) - b(g) > frac * b(g - window)
 *             (b(g - window) = +inf counts as improved when b(g) is finite).
 *             Stagnated: p_mut = min(1.5 p_mut, p_max), flags += 1; else
 *             p_mut = max(0.5 p_mut, p_min), flags = 0.  At `restart_after`
 *             consecutive flags the population is re-initialised as at the
 *             start (draws keyed by the next generation), p_mut reset, and
 *             the best-ever record kept.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "sblm_oracle.h"

/* Philox4x64 round multipliers and key increments (Salmon et al. 2011). */
#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2],
                       uint64_t out[4]) {
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

uint64_t orc_draw(uint64_t seed, uint64_t lc, uint64_t gen, uint64_t purpose,
                  uint64_t row, uint64_t j) {
  uint64_t ctr[4] = {gen, purpose, row, j >> 2}, key[2] = {seed, lc}, out[4];
  orc_philox4x64_10(ctr, key, out);
  return out[j & 3];
}

/* open unit interval, 52-bit grid: ((x >> 12) + 1/2) 2^-52 */
double orc_u01(uint64_t x) { return ((double)(x >> 12) + 0.5) * 0x1p-52; }

/* integer in {0..n-1} from the top 32 bits */
uint32_t orc_below(uint64_t x, uint32_t n) {
  return (uint32_t)(((x >> 32) * (uint64_t)n) >> 32);
}

/*
 * 2^(-v) for 0 <= v < 64: v = k + f with integer k and f in [0,1);
 * 2^(-f) = exp(-f ln 2) from its Taylor series truncated after the f^16 term
 * (truncation error below 6e-18), evaluated by Horner's rule with fused
 * multiply-adds in a fixed order, then scaled by 2^-k exactly.
 * Coefficient n is (-ln 2)^n / n! rounded to the nearest double.
 */
static const double EXP2_NEG_TAYLOR[17] = {
    0x1.0000000000000p+0,   -0x1.62e42fefa39efp-1, 0x1.ebfbdff82c58fp-3,
    -0x1.c6b08d704a0c0p-5,  0x1.3b2ab6fba4e77p-7,  -0x1.5d87fe78a6731p-10,
    0x1.430912f86c787p-13,  -0x1.ffcbfc588b0c7p-17, 0x1.62c0223a5c824p-20,
    -0x1.b5253d395e7c4p-24, 0x1.e4cf5158b8ecap-28, -0x1.e8cac7351bb25p-32,
    0x1.c3bd650fc2986p-36,  -0x1.816193166d0f9p-40, 0x1.314964d5878a9p-44,
    -0x1.c36e843b04022p-49, 0x1.38e89ae79f8b4p-53};

double orc_exp2_neg(double v) {
  double k = floor(v);
  double f = v - k;
  double s = EXP2_NEG_TAYLOR[16];
  for (int n = 15; n >= 0; --n) s = fma(s, f, EXP2_NEG_TAYLOR[n]);
  return ldexp(s, -(int)k);
}

static double clamp01(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

#define PURPOSE_INIT 1
#define PURPOSE_TOURN 2
#define PURPOSE_MODE 3
#define PURPOSE_CREEP 4
#define PURPOSE_JUMP 5

/* Sec. A.1, reading E1; draws keyed by generation `gen`. */
static void init_population(const orc_ea_config* cfg, uint64_t seed,
                            int64_t lc, int64_t gen, double* P) {
  int half = cfg->pop / 2;
  for (int i = 0; i < half; ++i)
    for (int g = 0; g < 6; ++g) {
      double x = orc_u01(orc_draw(seed, (uint64_t)lc, (uint64_t)gen,
                                  PURPOSE_INIT, (uint64_t)i, (uint64_t)g));
      P[i * 6 + g] = x;
      P[(i + half) * 6 + g] = 1.0 - x;
    }
  if (cfg->pop % 2)
    for (int g = 0; g < 6; ++g)
      P[(cfg->pop - 1) * 6 + g] =
          orc_u01(orc_draw(seed, (uint64_t)lc, (uint64_t)gen, PURPOSE_INIT,
                           (uint64_t)(cfg->pop - 1), (uint64_t)g));
}

/* The configuration limits of this oracle: the generation works in fixed
 * arrays of ORC_EA_POP_MAX rows and keeps a history of 64 generations. */
static int config_ok(const orc_ea_config* cfg) {
  return cfg && cfg->pop >= 2 && cfg->pop <= ORC_EA_POP_MAX &&
         cfg->stag_window >= 1 && cfg->stag_window <= 63 && cfg->n_tourn >= 0;
}

int orc_ea_init(const orc_ea_config* cfg, uint64_t seed, int64_t lc,
                double* P, orc_ea_lc* st) {
  if (!config_ok(cfg) || !P || !st) return -1;
  memset(st, 0, sizeof(*st));
  st->p_mut = cfg->p_mut0;
  st->best_chi2 = INFINITY;
  st->best_gen = -1;
  for (int k = 0; k < 64; ++k) st->hist[k] = INFINITY;
  init_population(cfg, seed, lc, 0, P);
  return 0;
}

static double rank_key(double c) { return isnan(c) ? INFINITY : c; }

int orc_ea_generation(const orc_ea_config* cfg, uint64_t seed, int64_t lc,
                      double* P, const double* chi2, const double* Fs,
                      const double* Fb, orc_ea_lc* st, int32_t* parents) {
  if (!config_ok(cfg) || !P || !chi2 || !Fs || !Fb || !st) return -1;
  const int N = cfg->pop;
  const int64_t gen = st->gen;
  const uint64_t L = (uint64_t)lc, G = (uint64_t)gen;
  int nt = cfg->n_tourn > 0 ? cfg->n_tourn : (N + 24) / 25;

  /* (A.3) rank: stable insertion sort of row indices by chi^2 */
  int perm[ORC_EA_POP_MAX];
  for (int i = 0; i < N; ++i) perm[i] = i;
  for (int i = 1; i < N; ++i) {
    int v = perm[i], j = i - 1;
    while (j >= 0 && rank_key(chi2[perm[j]]) > rank_key(chi2[v])) {
      perm[j + 1] = perm[j];
      --j;
    }
    perm[j + 1] = v;
  }
  double sorted[ORC_EA_POP_MAX * 6];
  for (int r = 0; r < N; ++r)
    for (int g = 0; g < 6; ++g) sorted[r * 6 + g] = P[perm[r] * 6 + g];
  double b = rank_key(chi2[perm[0]]);

  /* best-ever record (elitism keeps it monotone within a sequence) */
  if (b < st->best_chi2) {
    st->best_chi2 = b;
    st->best_Fs = Fs[perm[0]];
    st->best_Fb = Fb[perm[0]];
    for (int g = 0; g < 6; ++g) st->best_p[g] = sorted[g];
    st->best_gen = gen;
  }
  const int W = cfg->stag_window;
  st->hist[gen % (W + 1)] = b;

  /* (A.4, A.5) selection and reproduction; row 0 keeps the fittest */
  double next[ORC_EA_POP_MAX * 6];
  for (int g = 0; g < 6; ++g) next[g] = sorted[g];
  int npair = N / 2;
  for (int k = 0; k < npair; ++k) {
    int ra = N, rb = N;
    for (int m = 0; m < nt; ++m) {
      int x = (int)orc_below(orc_draw(seed, L, G, PURPOSE_TOURN, (uint64_t)k,
                                      (uint64_t)m),
                             (uint32_t)N);
      int y = (int)orc_below(orc_draw(seed, L, G, PURPOSE_TOURN, (uint64_t)k,
                                      (uint64_t)(nt + m)),
                             (uint32_t)N);
      if (x < ra) ra = x;
      if (y < rb) rb = y;
    }
    if (parents) {
      parents[2 * k] = ra;
      parents[2 * k + 1] = rb;
    }
    int mode = (int)orc_below(
        orc_draw(seed, L, G, PURPOSE_MODE, (uint64_t)k, 0), 3u);
    const double* pa = &sorted[ra * 6];
    const double* pb = &sorted[rb * 6];
    int s1 = 2 * k + 1, s2 = 2 * k + 2;
    for (int g = 0; g < 6; ++g) {
      double f;
      if (mode == 0)
        f = orc_u01(
            orc_draw(seed, L, G, PURPOSE_MODE, (uint64_t)k, (uint64_t)(1 + g)));
      else if (mode == 1)
        f = (orc_draw(seed, L, G, PURPOSE_MODE, (uint64_t)k,
                      (uint64_t)(1 + g)) >> 63)
                ? 1.0
                : 0.0;
      else
        f = 1.0;
      double omf = 1.0 - f;
      next[s1 * 6 + g] = clamp01(fma(f, pa[g], omf * pb[g]));
      if (s2 < N) next[s2 * 6 + g] = clamp01(fma(f, pb[g], omf * pa[g]));
    }
  }

  /* (A.6) creep then jump on every offspring gene */
  for (int i = 1; i < N; ++i)
    for (int g = 0; g < 6; ++g) {
      double p = next[i * 6 + g];
      uint64_t xs = orc_draw(seed, L, G, PURPOSE_CREEP, (uint64_t)i,
                             (uint64_t)(2 * g));
      uint64_t xu = orc_draw(seed, L, G, PURPOSE_CREEP, (uint64_t)i,
                             (uint64_t)(2 * g + 1));
      double X = orc_exp2_neg(52.0 * orc_u01(xu));
      if (xs >> 63)
        p = fma(1.0 - p, X, p);
      else
        p = fma(-p, X, p);
      p = clamp01(p);
      uint64_t j1 = orc_draw(seed, L, G, PURPOSE_JUMP, (uint64_t)i,
                             (uint64_t)(2 * g));
      if (orc_u01(j1) < st->p_mut)
        p = orc_u01(orc_draw(seed, L, G, PURPOSE_JUMP, (uint64_t)i,
                             (uint64_t)(2 * g + 1)));
      next[i * 6 + g] = p;
    }
  memcpy(P, next, sizeof(double) * 6 * (size_t)N);

  /* (A.7) stagnation test, p_mut boost / throttle, restart */
  if (gen - st->gen_restart >= W) {
    double old = st->hist[(gen - W) % (W + 1)];
    int improved;
    if (isinf(old))
      improved = (b < old);
    else
      improved = (old - b) > cfg->stag_frac * old;
    if (improved) {
      st->p_mut = fmax(0.5 * st->p_mut, cfg->p_mut_min);
      st->stag_count = 0;
    } else {
      st->p_mut = fmin(1.5 * st->p_mut, cfg->p_mut_max);
      st->stag_count += 1;
    }
    if (st->stag_count >= cfg->restart_after) {
      init_population(cfg, seed, lc, gen + 1, P);
      st->p_mut = cfg->p_mut0;
      st->stag_count = 0;
      st->gen_restart = gen + 1;
      st->n_restarts += 1;
    }
  }
  st->gen = gen + 1;
  return 0;
}

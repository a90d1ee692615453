/*
 * sanitize_check.c -- a driver that runs every entry point of the C oracle
 * once on small fixed inputs, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer.  TEST INFRASTRUCTURE ONLY (built and run by
 * the CPU test-suite; not part of the library).
 *
 * Inputs come from a fixed linear congruential sequence (no part of the
 * method); the driver prints every input and output as hexadecimal floats,
 * one "name index value" per line, so that the test can recompute the same
 * outputs through the ordinary build and compare them bit for bit.
 * Covered: magnification on a shared epoch grid (two threads), the source
 * on a lens (degree-4 polynomial), the image list, chi^2 on a CSR batch with
 * an empty and a one-epoch lightcurve, the EA initialisation and generations
 * with NaN and infinite fitness (odd and even populations, the largest one),
 * and the rejected configurations.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "sblm_oracle.h"

static uint64_t lcg_state = 0x853c49e6748fea9bULL;
static double lcg_u01(void) {
  lcg_state = lcg_state * 6364136223846793005ULL + 1442695040888963407ULL;
  return ((double)(lcg_state >> 11) + 0.5) * 0x1p-53;
}

static void put(const char* name, int64_t i, double v) { printf("%s %lld %a\n", name, (long long)i, v); }

/* theta plane by plane from the prior box of the workloads */
static void draw_theta(double* th, int64_t n) {
  const double lo[6] = {-3.0, 0.5, 0.0, 0.0, 10.0, -10.0};
  const double hi[6] = {0.0, 2.0, 0.5, 6.283185307179586, 100.0, 10.0};
  for (int j = 0; j < 6; ++j)
    for (int64_t i = 0; i < n; ++i) th[j * n + i] = lo[j] + (hi[j] - lo[j]) * lcg_u01();
}

int main(void) {
  int fails = 0;
  /* magnification: 5 parameter sets x 37 epochs, two threads */
  {
    const int64_t n = 5, nt = 37;
    double th[6 * 5], t[37], A[5 * 37];
    int8_t ni[5 * 37];
    draw_theta(th, n);
    for (int64_t k = 0; k < nt; ++k) t[k] = -150.0 + 300.0 * (double)k / (double)(nt - 1);
    orc_magnify(th, n, t, nt, A, ni, 2);
    for (int64_t i = 0; i < 6 * n; ++i) put("mag_theta", i, th[i]);
    for (int64_t k = 0; k < nt; ++k) put("mag_t", k, t[k]);
    for (int64_t i = 0; i < n * nt; ++i) {
      put("mag_A", i, A[i]);
      put("mag_nimg", i, (double)ni[i]);
    }
  }
  /* the source on either lens (leading coefficient zero) and a generic point */
  {
    const double pts[3][4] = {{0.0, 0.0, 1.1, 0.3}, {1.1, 0.0, 1.1, 0.3}, {0.2, 0.05, 0.9, 0.7}};
    for (int p = 0; p < 3; ++p) {
      double ir[5], ii[5], dj[5], rs[5];
      int nimg = orc_images(pts[p][0], pts[p][1], pts[p][2], pts[p][3], ir, ii, dj, rs);
      int nn;
      double a = orc_point_magnification(pts[p][0], pts[p][1], pts[p][2], pts[p][3], &nn);
      put("img_n", p, (double)nimg);
      put("img_A", p, a);
      for (int k = 0; k < nimg; ++k) put("img_detj", p * 5 + k, dj[k]);
    }
  }
  /* chi^2: lightcurves of 0, 1 and 23 epochs, population 3, two threads */
  {
    const int32_t n_lc = 3, pop = 3;
    const int64_t off[4] = {0, 0, 1, 24};
    double t[24], y[24], w[24], th[6 * 9], c2[9], fs[9], fb[9];
    for (int k = 0; k < 24; ++k) {
      t[k] = -60.0 + 120.0 * lcg_u01();
      y[k] = 1.0 + lcg_u01();
      w[k] = 1.0 / (0.01 + 0.02 * lcg_u01());
    }
    draw_theta(th, 9);
    orc_chi2(off, n_lc, t, y, w, th, pop, c2, fs, fb, 2);
    for (int k = 0; k < 24; ++k) {
      put("chi_t", k, t[k]);
      put("chi_y", k, y[k]);
      put("chi_w", k, w[k]);
    }
    for (int i = 0; i < 54; ++i) put("chi_theta", i, th[i]);
    for (int i = 0; i < 9; ++i) {
      put("chi_chi2", i, c2[i]);
      put("chi_Fs", i, fs[i]);
      put("chi_Fb", i, fb[i]);
    }
  }
  /* EA: populations 2, 3, 48 and 1024, 25 generations of drawn fitness with
   * NaN and infinite entries */
  {
    const int pops[4] = {2, 3, 48, ORC_EA_POP_MAX};
    for (int c = 0; c < 4; ++c) {
      const int pop = pops[c];
      orc_ea_config cfg = {pop, 0, 0.01, 1e-4, 0.5, 0.01, 10, 10};
      double* P = malloc(sizeof(double) * 6 * (size_t)pop);
      double* chi2 = malloc(sizeof(double) * (size_t)pop);
      double* fsb = calloc((size_t)pop, sizeof(double));
      int32_t* par = malloc(sizeof(int32_t) * (size_t)(pop / 2) * 2);
      orc_ea_lc st;
      if (orc_ea_init(&cfg, 77, c, P, &st) != 0) ++fails;
      for (int g = 0; g < 25; ++g) {
        for (int i = 0; i < pop; ++i) {
          const double u = lcg_u01();
          chi2[i] = u < 0.05 ? NAN : (u < 0.1 ? INFINITY : 100.0 * u);
        }
        if (orc_ea_generation(&cfg, 77, c, P, chi2, fsb, fsb, &st, par) != 0) ++fails;
      }
      double sum = 0.0;
      for (int i = 0; i < 6 * pop; ++i) sum += P[i] * (double)(i % 7 + 1);
      put("ea_sum", c, sum);
      put("ea_best", c, st.best_chi2);
      put("ea_pmut", c, st.p_mut);
      put("ea_restarts", c, (double)st.n_restarts);
      free(P);
      free(chi2);
      free(fsb);
      free(par);
    }
  }
  /* rejected configurations: nothing is written */
  {
    double P[6 * 4], chi2[4] = {1, 2, 3, 4};
    orc_ea_lc st;
    orc_ea_config bad[3] = {{ORC_EA_POP_MAX + 1, 0, 0.01, 1e-4, 0.5, 0.01, 10, 10},
                            {1, 0, 0.01, 1e-4, 0.5, 0.01, 10, 10},
                            {4, 0, 0.01, 1e-4, 0.5, 0.01, 64, 10}};
    for (int c = 0; c < 3; ++c) {
      if (orc_ea_init(&bad[c], 1, 0, P, &st) != -1) ++fails;
      if (orc_ea_generation(&bad[c], 1, 0, P, chi2, chi2, chi2, &st, NULL) != -1) ++fails;
    }
    if (orc_ea_generation(NULL, 1, 0, P, chi2, chi2, chi2, &st, NULL) != -1) ++fails;
  }
  printf("fails %d\n", fails);
  return fails ? 1 : 0;
}

/*
 * sblm_oracle.h -- declarations of the FP64 CPU oracle (test infrastructure;
 * see sblm_oracle.c and ea_oracle.c).  Not part of the library ABI.
 */
#ifndef SBLM_ORACLE_H
#define SBLM_ORACLE_H
#include <stdint.h>

void orc_source_position(double t, double u0, double alpha, double tE,
                         double t0, double* zr, double* zi);
void orc_lens_poly(double zr, double zi, double d, double q, double* cr,
                   double* ci);
int orc_poly_roots(const double* cr, const double* ci, int deg, double* rr,
                   double* ri);
int orc_images(double zr, double zi, double d, double q, double* img_r,
               double* img_i, double* detj, double* resid_sorted);
double orc_point_magnification(double zr, double zi, double d, double q,
                               int* n_img);
void orc_magnify(const double* theta, int64_t n, const double* t, int64_t n_t,
                 double* A, int8_t* n_img, int nthreads);
void orc_lsq_chi2(const double* A, const double* y, const double* w,
                  int64_t n, double* chi2, double* Fs, double* Fb);
void orc_chi2(const int64_t* off, int32_t n_lc, const double* t,
              const double* y, const double* w, const double* theta,
              int32_t pop, double* chi2, double* Fs, double* Fb, int nthreads);
void orc_decode(const double* P, int64_t n, const double* lo, const double* hi,
                double* theta);

/* ea_oracle.c */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2],
                       uint64_t out[4]);
uint64_t orc_draw(uint64_t seed, uint64_t lc, uint64_t gen, uint64_t purpose,
                  uint64_t row, uint64_t j);
double orc_u01(uint64_t x);
uint32_t orc_below(uint64_t x, uint32_t n);
double orc_exp2_neg(double v);

typedef struct {
  int32_t pop, n_tourn;
  double p_mut0, p_mut_min, p_mut_max, stag_frac;
  int32_t stag_window, restart_after;
} orc_ea_config;

typedef struct {
  int64_t gen, gen_restart, best_gen;
  double p_mut;
  int32_t stag_count, n_restarts;
  double best_chi2, best_Fs, best_Fb;
  double best_p[6];
  double hist[64]; /* best chi^2 of generation g at hist[g % (window+1)] */
} orc_ea_lc;

/* Both return 0, or -1 (nothing written) for a null pointer or a
 * configuration outside 2 <= pop <= ORC_EA_POP_MAX, 1 <= stag_window <= 63,
 * n_tourn >= 0. */
#define ORC_EA_POP_MAX 1024
int orc_ea_init(const orc_ea_config* cfg, uint64_t seed, int64_t lc,
                double* P /* [pop][6] row-major */, orc_ea_lc* st);
int orc_ea_generation(const orc_ea_config* cfg, uint64_t seed, int64_t lc,
                      double* P, const double* chi2, const double* Fs,
                      const double* Fb, orc_ea_lc* st,
                      int32_t* parents /* nullable [2*floor(pop/2)] ranks */);
#endif

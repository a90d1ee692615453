/*
 * sblm_oracle.c -- plain, slow FP64 reference of the forward model and the
 * chi^2 fitness of Rajpaul (2012).  TEST INFRASTRUCTURE ONLY: it exists to
 * check the HIP implementation and is called by the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark; no product code path may
 * call it.  It shares no source with the HIP library.
 *
 * Everything is computed by the plain definition, in double precision:
 *   - the source position of Sec. 2.2 (Eq. sourcePos with tau = (t-t_m)/t_E);
 *   - the lens polynomial, formed by polynomial multiplication from the lens
 *     equation (Eq. lensing) -- the paper prints no coefficients, so the
 *     construction is derived below;
 *   - its roots, by Laguerre's method with deflation followed by polishing
 *     on the undeflated polynomial (the paper names Laguerre's method as one
 *     standard choice);
 *   - rejection of the spurious roots by substitution into the lens
 *     equation, and the magnification as the sum over accepted images of
 *     1/|det J| with det J = 1 - |1/conj(z)^2 + q/(d - conj(z))^2|^2;
 *   - the chi^2 of the blended flux model F = Fs*A + Fb (Sec. 4.4, Eq. blend,
 *     times the baseline flux) with Fs and Fb from the weighted linear
 *     least-squares problem, evaluated in three passes (means, centred
 *     sums, residuals).
 *
 * Readings of the paper adopted here (the paper is silent or garbled):
 *   R1  The per-image amplification is printed without the square on the
 *       inner modulus; with it missing the q -> 0 limit does not reproduce the
 *       single-lens magnification, so det J = 1 - |dzeta/dconj(z)|^2 is used.
 *   R2  Spurious-root test: residual r = |zeta - z + 1/conj(z) - q/(d - conj(z))|.
 *       Five images iff at least four roots have r < 1e-6 (and the
 *       polynomial has full degree); otherwise the three roots with the
 *       smallest residuals are the images.  Ties are broken by position in
 *       the root list after ordering the roots by (Re, Im).
 *   R3  If |c5| <= 1e-12 max_j |c_j| (source on a lens position) the fifth
 *       root is at infinity; the degree-4 polynomial is solved instead.
 *   R4  chi^2 is written in flux with unconstrained Fs, Fb; a 2x2 system with
 *       sum w (A - Abar)^2 <= 1e-14 sum w A^2 is degenerate and falls back to
 *       Fs = 0, Fb = weighted mean of y.
 *   R5  The images are the solutions of the lens equation; the polynomial's
 *       roots only start them.  Each accepted root is refined by Newton's
 *       method on Eq. (lensing) itself (a step is kept only while it lowers
 *       the residual), because next to a caustic two roots of the quintic
 *       nearly coincide and its roots lose accuracy that the lens equation
 *       does not.
 */
#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "sblm_oracle.h"

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Polynomial arithmetic on coefficient arrays, index = power of z.          */
/* ------------------------------------------------------------------------ */

/* out[0..na+nb-2] = a * b */
static void poly_mul(const cplx* a, int na, const cplx* b, int nb, cplx* out) {
  for (int k = 0; k < na + nb - 1; ++k) out[k] = 0;
  for (int i = 0; i < na; ++i)
    for (int j = 0; j < nb; ++j) out[i + j] += a[i] * b[j];
}

/* out[0..n-1] += s * a[0..na-1] (na <= n) */
static void poly_axpy(cplx s, const cplx* a, int na, cplx* out) {
  for (int i = 0; i < na; ++i) out[i] += s * a[i];
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.2: trajectory, lens polynomial.                                    */
/* ------------------------------------------------------------------------ */

void orc_source_position(double t, double u0, double alpha, double tE,
                         double t0, double* zr, double* zi) {
  /* dimensionless time, then Eq. (sourcePos) */
  double tau = (t - t0) / tE;
  *zr = tau * sin(alpha) + u0 * cos(alpha);
  *zi = -tau * cos(alpha) + u0 * sin(alpha);
}

/*
 * Coefficients c[0..5] (c[j] multiplies z^j) of the lens polynomial for
 * source position zeta, lens separation d and mass ratio q.
 *
 * Derivation from Eq. (lensing), zeta = z - 1/conj(z) + q/(d - conj(z)):
 * conjugating it gives conj(z) = conj(zeta) + 1/z + q/(z - d), i.e.
 * conj(z) = N(z)/D(z) with D = z^2 - d z and
 * N = conj(zeta) z^2 + (1 + q - d conj(zeta)) z - d.  Writing w = conj(z)
 * in the lens equation as zeta - z + 1/w + q/(w - d) = 0, multiplying by
 * w (w - d) D^2 and using w - d = (N - d D)/D gives the quintic
 *     (zeta - z) N (N - d D) + (N - d D) D + q N D = 0.
 * No root is introduced by clearing denominators because N(0) = -d and
 * N(d) = q d are non-zero.
 */
void orc_lens_poly(double zr, double zi, double d, double q, double* cr,
                   double* ci) {
  cplx zeta = zr + I * zi;
  cplx zc = conj(zeta);
  cplx N[3] = {-d, 1.0 + q - d * zc, zc};
  cplx D[3] = {0.0, -d, 1.0};
  cplx M[3]; /* N - d D */
  for (int k = 0; k < 3; ++k) M[k] = N[k] - d * D[k];
  cplx NM[5], MD[5], ND[5], lin[2] = {zeta, -1.0}, t1[6];
  poly_mul(N, 3, M, 3, NM);
  poly_mul(M, 3, D, 3, MD);
  poly_mul(N, 3, D, 3, ND);
  poly_mul(lin, 2, NM, 5, t1); /* (zeta - z) N M, degree 5 */
  cplx c[6];
  for (int k = 0; k < 6; ++k) c[k] = t1[k];
  poly_axpy(1.0, MD, 5, c);
  poly_axpy(q, ND, 5, c);
  for (int k = 0; k < 6; ++k) {
    cr[k] = creal(c[k]);
    ci[k] = cimag(c[k]);
  }
}

/* ------------------------------------------------------------------------ */
/* Roots: Laguerre's method with deflation, then polishing.                  */
/* ------------------------------------------------------------------------ */

/* p, p', p'' at x (Horner); also the running bound sum |c_j| |x|^j. */
static void eval3(const cplx* c, int deg, cplx x, cplx* p, cplx* dp, cplx* d2p,
                  double* mag) {
  cplx b = c[deg], d1 = 0, d2 = 0;
  double m = cabs(c[deg]), ax = cabs(x);
  for (int j = deg - 1; j >= 0; --j) {
    d2 = d2 * x + d1;
    d1 = d1 * x + b;
    b = b * x + c[j];
    m = m * ax + cabs(c[j]);
  }
  *p = b;
  *dp = d1;
  *d2p = 2.0 * d2;
  *mag = m;
}

/*
 * One root of the degree-`deg` polynomial c by Laguerre's iteration
 *   G = p'/p,  H = G^2 - p''/p,  a = n / (G +- sqrt((n-1)(n H - G^2))),
 *   x <- x - a,
 * with the sign that maximises |denominator|.  Stops when |p(x)| is at the
 * rounding level of its evaluation, when the step no longer changes x, or
 * after 400 iterations.  Every 20th step is shortened by a varying factor
 * to break the rare limit cycles of the plain iteration.
 */
static cplx laguerre(const cplx* c, int deg, cplx x) {
  static const double frac[4] = {0.5, 0.25, 0.75, 0.125};
  const double eps = 0x1p-52;
  for (int it = 1; it <= 400; ++it) {
    cplx p, dp, d2p;
    double mag;
    eval3(c, deg, x, &p, &dp, &d2p, &mag);
    if (cabs(p) <= 2.0 * eps * mag) return x;
    cplx G = dp / p;
    cplx H = G * G - d2p / p;
    cplx sq = csqrt((double)(deg - 1) * ((double)deg * H - G * G));
    cplx den = (cabs(G + sq) >= cabs(G - sq)) ? G + sq : G - sq;
    cplx a;
    if (cabs(den) > 0.0)
      a = (double)deg / den;
    else
      a = (1.0 + cabs(x)) * cexp(I * (double)it);
    cplx xn = (it % 20 == 0) ? x - frac[(it / 20) % 4] * a : x - a;
    if (xn == x) return x;
    x = xn;
  }
  return x;
}

/* Roots of sum_{j<=deg} c_j z^j (deg 1..5), written to roots[0..deg-1]. */
static void poly_roots(const cplx* c, int deg, cplx* roots) {
  cplx work[6];
  for (int k = 0; k <= deg; ++k) work[k] = c[k];
  for (int n = deg; n >= 1; --n) {
    cplx x = laguerre(work, n, 0.0);
    roots[deg - n] = x;
    /* deflate: divide work by (z - x) */
    cplx carry = work[n];
    for (int j = n - 1; j >= 0; --j) {
      cplx tmp = work[j];
      work[j] = carry;
      carry = tmp + carry * x;
    }
  }
  /* polish every root on the undeflated polynomial */
  for (int k = 0; k < deg; ++k) roots[k] = laguerre(c, deg, roots[k]);
}

int orc_poly_roots(const double* cr, const double* ci, int deg, double* rr,
                   double* ri) {
  if (deg < 1 || deg > 5) return -1;
  cplx c[6], r[5];
  for (int k = 0; k <= deg; ++k) c[k] = cr[k] + I * ci[k];
  poly_roots(c, deg, r);
  for (int k = 0; k < deg; ++k) {
    rr[k] = creal(r[k]);
    ri[k] = cimag(r[k]);
  }
  return deg;
}

/* ------------------------------------------------------------------------ */
/* Images and magnification.                                                 */
/* ------------------------------------------------------------------------ */

/* |zeta - (z - 1/conj(z) + q/(d - conj(z)))|: residual of Eq. (lensing). */
static double lens_residual(cplx zeta, cplx z, double d, double q) {
  cplx zb = conj(z);
  return cabs(zeta - (z - 1.0 / zb + q / (d - zb)));
}

/* det J of the lens mapping at image z: 1 - |1/conj(z)^2 + q/(d-conj(z))^2|^2 */
static double det_jacobian(cplx z, double d, double q) {
  cplx zb = conj(z);
  cplx g = 1.0 / (zb * zb) + q / ((d - zb) * (d - zb));
  double ag = cabs(g);
  return 1.0 - ag * ag;
}

static int cmp_root(const void* a, const void* b) {
  cplx x = *(const cplx*)a, y = *(const cplx*)b;
  if (creal(x) < creal(y)) return -1;
  if (creal(x) > creal(y)) return 1;
  if (cimag(x) < cimag(y)) return -1;
  if (cimag(x) > cimag(y)) return 1;
  return 0;
}

#define ORC_IMAGE_TOL 1e-6

/*
 * Newton's method on the lens equation at an image z: with
 * r = zeta - (z - 1/conj(z) + q/(d - conj(z))) and g = dzeta/dconj(z),
 * the step dz solves dz + g conj(dz) = r, i.e. dz = (r - g conj(r)) / (1 - |g|^2).
 * Steps are taken while they lower |r| and exceed 1e-16 |z|, at most 8.
 */
static cplx polish_image(cplx zeta, cplx z, double d, double q) {
  double rn = lens_residual(zeta, z, d, q);
  for (int it = 0; it < 8; ++it) {
    cplx zb = conj(z);
    cplx r = zeta - (z - 1.0 / zb + q / (d - zb));
    cplx g = 1.0 / (zb * zb) + q / ((d - zb) * (d - zb));
    double ag = cabs(g);
    cplx dz = (r - g * conj(r)) / (1.0 - ag * ag);
    cplx zn = z + dz;
    double rnn = lens_residual(zeta, zn, d, q);
    if (!(rnn < rn)) break;
    z = zn;
    rn = rnn;
    if (cabs(dz) <= 1e-16 * cabs(z)) break;
  }
  return z;
}

int orc_images(double zr, double zi, double d, double q, double* img_r,
               double* img_i, double* detj, double* resid_sorted) {
  cplx zeta = zr + I * zi;
  double cr[6], ci[6];
  orc_lens_poly(zr, zi, d, q, cr, ci);
  cplx c[6];
  double cmax = 0.0;
  for (int k = 0; k < 6; ++k) {
    c[k] = cr[k] + I * ci[k];
    if (cabs(c[k]) > cmax) cmax = cabs(c[k]);
  }
  int deg = (cabs(c[5]) <= 1e-12 * cmax) ? 4 : 5;
  cplx roots[5];
  poly_roots(c, deg, roots);
  qsort(roots, (size_t)deg, sizeof(cplx), cmp_root);

  double res[5];
  int order[5];
  for (int k = 0; k < deg; ++k) {
    res[k] = lens_residual(zeta, roots[k], d, q);
    order[k] = k;
  }
  /* stable insertion sort of root indices by residual */
  for (int i = 1; i < deg; ++i) {
    int v = order[i], j = i - 1;
    while (j >= 0 && res[order[j]] > res[v]) {
      order[j + 1] = order[j];
      --j;
    }
    order[j + 1] = v;
  }
  int below = 0;
  for (int k = 0; k < deg; ++k) below += (res[k] < ORC_IMAGE_TOL);
  int n = (deg == 5 && below >= 4) ? 5 : 3;
  for (int k = 0; k < n; ++k) {
    cplx z = polish_image(zeta, roots[order[k]], d, q);
    if (img_r) img_r[k] = creal(z);
    if (img_i) img_i[k] = cimag(z);
    if (detj) detj[k] = det_jacobian(z, d, q);
  }
  if (resid_sorted)
    for (int k = 0; k < 5; ++k)
      resid_sorted[k] = (k < deg) ? res[order[k]] : INFINITY;
  return n;
}

double orc_point_magnification(double zr, double zi, double d, double q,
                               int* n_img) {
  double dj[5];
  int n = orc_images(zr, zi, d, q, NULL, NULL, dj, NULL);
  double A = 0.0;
  for (int k = 0; k < n; ++k) A += 1.0 / fabs(dj[k]);
  if (n_img) *n_img = n;
  return A;
}

/* ------------------------------------------------------------------------ */
/* Batched forward model and chi^2, threaded over individuals.               */
/* ------------------------------------------------------------------------ */

typedef struct {
  const double* theta;
  int64_t n;
  const double* t;
  int64_t n_t;
  double* A;
  int8_t* n_img;
  int64_t begin, end;
} magnify_job;

static void magnify_range(const magnify_job* J) {
  for (int64_t i = J->begin; i < J->end; ++i) {
    double q = pow(10.0, J->theta[0 * J->n + i]);
    double d = J->theta[1 * J->n + i];
    double u0 = J->theta[2 * J->n + i];
    double al = J->theta[3 * J->n + i];
    double tE = J->theta[4 * J->n + i];
    double t0 = J->theta[5 * J->n + i];
    for (int64_t k = 0; k < J->n_t; ++k) {
      double zr, zi;
      int ni;
      orc_source_position(J->t[k], u0, al, tE, t0, &zr, &zi);
      J->A[i * J->n_t + k] = orc_point_magnification(zr, zi, d, q, &ni);
      if (J->n_img) J->n_img[i * J->n_t + k] = (int8_t)ni;
    }
  }
}

static void* magnify_thread(void* arg) {
  magnify_range((const magnify_job*)arg);
  return NULL;
}

void orc_magnify(const double* theta, int64_t n, const double* t, int64_t n_t,
                 double* A, int8_t* n_img, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > n) nthreads = (int)(n > 0 ? n : 1);
  magnify_job* jobs = calloc((size_t)nthreads, sizeof(magnify_job));
  pthread_t* th = calloc((size_t)nthreads, sizeof(pthread_t));
  for (int k = 0; k < nthreads; ++k) {
    magnify_job J = {theta, n, t, n_t, A, n_img, n * k / nthreads,
                     n * (k + 1) / nthreads};
    jobs[k] = J;
  }
  for (int k = 1; k < nthreads; ++k)
    pthread_create(&th[k], NULL, magnify_thread, &jobs[k]);
  magnify_range(&jobs[0]);
  for (int k = 1; k < nthreads; ++k) pthread_join(th[k], NULL);
  free(jobs);
  free(th);
}

void orc_lsq_chi2(const double* A, const double* y, const double* w,
                  int64_t n, double* chi2, double* Fs, double* Fb) {
  double S1 = 0.0, SA = 0.0, Sy = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    S1 += w[k];
    SA += w[k] * A[k];
    Sy += w[k] * y[k];
  }
  if (!(S1 > 0.0)) {
    *chi2 = 0.0;
    *Fs = 0.0;
    *Fb = 0.0;
    return;
  }
  double Abar = SA / S1, ybar = Sy / S1;
  double Saa = 0.0, Say = 0.0, SAA = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    double da = A[k] - Abar, dy = y[k] - ybar;
    Saa += w[k] * da * da;
    Say += w[k] * da * dy;
    SAA += w[k] * A[k] * A[k];
  }
  double fs, fb;
  if (Saa <= 1e-14 * SAA) {
    fs = 0.0;
    fb = ybar;
  } else {
    fs = Say / Saa;
    fb = ybar - fs * Abar;
  }
  double c2 = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    double r = y[k] - fs * A[k] - fb;
    c2 += w[k] * r * r;
  }
  *chi2 = c2;
  *Fs = fs;
  *Fb = fb;
}

typedef struct {
  const int64_t* off;
  const double *t, *y, *w, *theta;
  int32_t pop;
  int64_t n_ind;
  double *chi2, *Fs, *Fb;
  int64_t begin, end;
} chi2_job;

static void chi2_range(const chi2_job* J) {
  double* A = NULL;
  int64_t cap = 0;
  for (int64_t i = J->begin; i < J->end; ++i) {
    int64_t lc = i / J->pop;
    int64_t e0 = J->off[lc], e1 = J->off[lc + 1], L = e1 - e0;
    if (L > cap) {
      free(A);
      cap = L;
      A = malloc((size_t)cap * sizeof(double));
    }
    double th[6];
    for (int j = 0; j < 6; ++j) th[j] = J->theta[j * J->n_ind + i];
    double q = pow(10.0, th[0]);
    for (int64_t k = 0; k < L; ++k) {
      double zr, zi;
      orc_source_position(J->t[e0 + k], th[2], th[3], th[4], th[5], &zr, &zi);
      A[k] = orc_point_magnification(zr, zi, th[1], q, NULL);
    }
    orc_lsq_chi2(A, J->y + e0, J->w + e0, L, &J->chi2[i], &J->Fs[i],
                 &J->Fb[i]);
  }
  free(A);
}

static void* chi2_thread(void* arg) {
  chi2_range((const chi2_job*)arg);
  return NULL;
}

void orc_chi2(const int64_t* off, int32_t n_lc, const double* t,
              const double* y, const double* w, const double* theta,
              int32_t pop, double* chi2, double* Fs, double* Fb,
              int nthreads) {
  int64_t n_ind = (int64_t)n_lc * pop;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > n_ind) nthreads = (int)(n_ind > 0 ? n_ind : 1);
  chi2_job* jobs = calloc((size_t)nthreads, sizeof(chi2_job));
  pthread_t* th = calloc((size_t)nthreads, sizeof(pthread_t));
  for (int k = 0; k < nthreads; ++k) {
    chi2_job J = {off,  t,    y,  w,  theta,
                  pop,  n_ind, chi2, Fs, Fb,
                  n_ind * k / nthreads, n_ind * (k + 1) / nthreads};
    jobs[k] = J;
  }
  for (int k = 1; k < nthreads; ++k)
    pthread_create(&th[k], NULL, chi2_thread, &jobs[k]);
  chi2_range(&jobs[0]);
  for (int k = 1; k < nthreads; ++k) pthread_join(th[k], NULL);
  free(jobs);
  free(th);
}

/* Eq. (EMMA-encoding): a = alpha_j + (beta_j - alpha_j) p, plane by plane. */
void orc_decode(const double* P, int64_t n, const double* lo, const double* hi,
                double* theta) {
  for (int j = 0; j < 6; ++j)
    for (int64_t i = 0; i < n; ++i)
      theta[j * n + i] = lo[j] + (hi[j] - lo[j]) * P[j * n + i];
}

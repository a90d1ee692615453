// sblm_math.h -- the arithmetic of one magnification and one fit update
// (Rajpaul 2012, Sec. 2.2 and Sec. 4.4): source position, lens polynomial,
// Ehrlich-Aberth sweep, image evaluation and refinement on the lens
// equation, least-squares row update.
//
// Written once for any number type R and shared by two builds: the fitness
// kernel (device code, R = double or float) and the FLOP counting build
// (host code, R = a number type that counts its operations), so that the
// operation counts used for the roofline come from this very code.  Every R
// supplies, found by overload resolution: fma(a, b, c), rcp_hw(x) (the
// hardware reciprocal estimate), vmin / vmax (minimum / maximum), fabs and
// isfinite; is_single<R> says whether R stands for FP32 (its reciprocal
// steps take no refinement).
#pragma once

#ifdef __HIP__
#define SBLM_FN __host__ __device__ __forceinline__
#else
#define SBLM_FN inline
#endif

namespace sblm {

template <typename R>
struct is_single {
  static constexpr bool value = false;
};
template <>
struct is_single<float> {
  static constexpr bool value = true;
};

// ---------------------------------------------------------------- reciprocals

// Raw hardware reciprocal (relative error < 5e-8 in FP64): used only for the
// pairwise terms of the Aberth correction, whose error scales the size of a
// correction that is itself second order.
template <typename R>
SBLM_FN R rcp_raw(R x) {
  return rcp_hw(x);
}
// Approximate reciprocal for iteration steps (the fixed point of the
// iteration does not depend on its accuracy): FP64 one Newton step on the
// estimate, FP32 the estimate.
template <typename R>
SBLM_FN R rcp_fast(R x) {
  if constexpr (is_single<R>::value) {
    return rcp_hw(x);
  } else {
    const R r = rcp_hw(x);
    return fma(r, fma(-x, r, R(1.0)), r);
  }
}
// Reciprocal to about 1 ulp (two Newton steps), for det J, image positions
// and the fit.
template <typename R>
SBLM_FN R rcp_acc(R x) {
  R r = rcp_hw(x);
  r = fma(r, fma(-x, r, R(1.0)), r);
  return fma(r, fma(-x, r, R(1.0)), r);
}

// ---------------------------------------------------------------- complex

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
SBLM_FN cx<T> c_sub(cx<T> a, cx<T> b) {
  return {a.re - b.re, a.im - b.im};
}
// a*b + c
template <typename T>
SBLM_FN cx<T> c_fma(cx<T> a, cx<T> b, cx<T> c) {
  return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
template <typename T>
SBLM_FN cx<T> c_mul(cx<T> a, cx<T> b) {
  return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
template <typename T>
SBLM_FN T c_norm(cx<T> a) {
  return fma(a.re, a.re, a.im * a.im);
}

// ---------------------------------------------------------------- polynomial

// Source position of Eq. (sourcePos) at dimensionless time tau = (t - t0)/tE
// (itE = 1/tE), trajectory angle alpha (sa = sin, ca = cos), impact u0.
template <typename R>
SBLM_FN cx<R> source_position(R t, R t0, R itE, R sa, R ca, R u0) {
  const R tau = (t - t0) * itE;
  return {fma(tau, sa, u0 * ca), fma(-tau, ca, u0 * sa)};
}

// Coefficients c[0..5] of the lens polynomial for source zeta, separation d,
// mass ratio q.  From Eq. (lensing): conj(z) = N(z)/D(z) with
// N = w z^2 + (1+q-dw) z - d, D = z^2 - d z, w = conj(zeta); substituting
// back and clearing denominators gives (zeta - z) N M + M D + q N D = 0 with
// M = N - d D = (w-d) z^2 + (1+q+d^2-dw) z - d.  Expanded here by hand.
template <typename R>
SBLM_FN void lens_coeffs(cx<R> zeta, R d, R q, cx<R> c[6]) {
  const cx<R> w = {zeta.re, -zeta.im};
  const R opq = R(1.0) + q;
  const cx<R> n2 = w;
  const cx<R> n1 = {fma(-d, w.re, opq), -d * w.im};
  const cx<R> m2 = {w.re - d, w.im};
  const cx<R> m1 = {fma(-d, w.re, fma(d, d, opq)), -d * w.im};
  const R dd = d * d;
  // products of N and M, by power of z (n0 = m0 = -d)
  const cx<R> nm4 = c_mul(n2, m2);
  const cx<R> nm3 = c_fma(n2, m1, c_mul(n1, m2));
  const cx<R> s2 = {n2.re + m2.re, n2.im + m2.im};
  const cx<R> nm2 = c_fma(n1, m1, cx<R>{-d * s2.re, -d * s2.im});
  const cx<R> nm1 = {-d * (n1.re + m1.re), -d * (n1.im + m1.im)};
  // (zeta - z) N M + M D + q N D
  c[5] = {-nm4.re, -nm4.im};
  // z^4: zeta nm4 - nm3 + m2 + q n2
  c[4] = c_fma(zeta, nm4,
               cx<R>{m2.re + fma(q, n2.re, -nm3.re), m2.im + fma(q, n2.im, -nm3.im)});
  // z^3: zeta nm3 - nm2 + (m1 - d m2) + q (n1 - d n2)
  c[3] = c_fma(zeta, nm3,
               cx<R>{fma(-d, m2.re, m1.re) + fma(q, fma(-d, n2.re, n1.re), -nm2.re),
                     fma(-d, m2.im, m1.im) + fma(q, fma(-d, n2.im, n1.im), -nm2.im)});
  // z^2: zeta nm2 - nm1 + (m0 - d m1) + q (n0 - d n1)
  c[2] = c_fma(zeta, nm2,
               cx<R>{fma(-d, m1.re, -d) + fma(q, fma(-d, n1.re, -d), -nm1.re),
                     fma(-d, m1.im, R(0.0)) + fma(q, -d * n1.im, -nm1.im)});
  // z^1: zeta nm1 - nm0 - d m0 - q d n0 = zeta nm1 + q d^2
  c[1] = c_fma(zeta, nm1, cx<R>{q * dd, R(0.0)});
  // z^0: zeta nm0 = zeta d^2
  c[0] = {zeta.re * dd, zeta.im * dd};
}

// A negligible leading coefficient (the source on a lens): the polynomial is
// solved as one of degree 4 and c[5] is set to zero.
template <typename R>
SBLM_FN bool drop_to_degree4(cx<R> c[6]) {
  R cmax = R(0.0);
#pragma unroll
  for (int j = 0; j < 6; ++j) cmax = vmax(cmax, c_norm(c[j]));
  const bool deg4 = c_norm(c[5]) <= R(1e-24) * cmax;
  if (deg4) c[5] = {R(0.0), R(0.0)};
  return deg4;
}

// A source very close to a lens (within ~1e-3 theta_E of either) gives a
// small leading coefficient: one root -- always spurious -- lies far out, at
// about -c4/c5, the others near the lenses.  |c4| > 1e3 |c5| marks it.
template <typename R>
SBLM_FN bool far_root(const cx<R> c[6]) {
  return c_norm(c[4]) > R(1e6) * c_norm(c[5]);
}

// p(z) and p'(z) by Horner's rule.
template <typename T>
SBLM_FN void horner(const cx<T> c[6], cx<T> z, cx<T>& p, cx<T>& dp) {
  dp = c[5];
  p = c_fma(c[5], z, c[4]);
#pragma unroll
  for (int j = 3; j >= 0; --j) {
    dp = c_fma(dp, z, p);
    p = c_fma(p, z, c[j]);
  }
}

// One Ehrlich-Aberth sweep (Jacobi form) over the five roots:
//   S_i = sum_{j != i} 1/(z_i - z_j),
//   z_i <- z_i - p(z_i) / (p'(z_i) - p(z_i) S_i),
// (the usual w/(1 - w S) with w = p/p', written with one complex division).
// The iteration converges cubically: after a step of length e the error
// left in z_i is about e^3 / s_i^2, s_i the distance to the nearest other
// root.  Returns 1 when, for every root, e^3 / (s_i^2 max(1,|z_i|)) <= tau or
// e <= 1e-13 max(1,|z_i|) (a step at the rounding level, which also ends the
// slow approach of a double root).  With EM, *emax receives
// max_i e_i^2 / max(1,|z_i|^2) (a termination heuristic: the raw reciprocal,
// no division); without, emax is not touched.
template <bool EM = true, typename T>
SBLM_FN bool aberth_sweep(const cx<T> c[6], cx<T> z[5], bool deg4, T tau, T* emax) {
  // pairwise terms from the current roots first, so that each root's p, p'
  // is used as soon as it is computed (fewer live registers)
  cx<T> S[5];
  T dmin[5];  // (distance to the nearest other root)^2
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    S[i] = {T(0.0), T(0.0)};
    dmin[i] = T(INFINITY);
  }
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i + 1; j < 5; ++j) {
      const cx<T> dz = c_sub(z[i], z[j]);
      const T n = c_norm(dz);
      const T r = rcp_raw(n);
      const T ire = dz.re * r, iim = -dz.im * r;  // 1/(z_i - z_j)
      S[i].re += ire;
      S[i].im += iim;
      S[j].re -= ire;
      S[j].im -= iim;
      dmin[i] = vmin(n, dmin[i]);
      dmin[j] = vmin(n, dmin[j]);
    }
  bool conv = true;
  T em = T(0.0);
  const T tau2 = tau * tau;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    cx<T> p, dp;
    horner(c, z[i], p, dp);
    // den = p' - p S ; dz = p / den
    const cx<T> pS = c_mul(p, S[i]);
    const cx<T> den = c_sub(dp, pS);
    const T r = rcp_fast(c_norm(den));
    cx<T> dz = {fma(p.re, den.re, p.im * den.im) * r, fma(p.im, den.re, -p.re * den.im) * r};
    if (i == 4 && deg4) dz = {T(0.0), T(0.0)};
    z[i] = c_sub(z[i], dz);
    const T zn = c_norm(z[i]);
    const T sc = vmax(zn, T(1.0));
    const T e2 = c_norm(dz);
    // (e^2)^3 <= tau^2 |z|^2 (s^2)^2, or e^2 <= 1e-26 |z|^2
    const bool ok = (e2 * e2 * e2 <= tau2 * sc * (dmin[i] * dmin[i])) || (e2 <= T(1e-26) * sc);
    conv = conv && (ok || (i == 4 && deg4));
    if constexpr (EM) em = vmax(e2 * rcp_raw(sc), em);
  }
  if constexpr (EM) *emax = em;
  return conv;
}

// Squared distance from each root to its nearest other root.
template <typename T>
SBLM_FN void nearest2(const cx<T> z[5], T d2[5]) {
#pragma unroll
  for (int i = 0; i < 5; ++i) d2[i] = T(INFINITY);
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i + 1; j < 5; ++j) {
      const T n = c_norm(c_sub(z[i], z[j]));
      d2[i] = vmin(n, d2[i]);
      d2[j] = vmin(n, d2[j]);
    }
}

// One Newton step on every root, z_i <- z_i - p(z_i)/p'(z_i) (the polish of
// roots found in lower precision).  Newton's method converges
// quadratically: after a step of length e the error left is about e^2/s_i
// (s_i the distance to the nearest other root, from d2).  Returns 1 when,
// for every root, e^2/s_i <= tau max(1,|z_i|), i.e. e^4 <= tau^2 |z_i|^2
// s_i^2, or e <= 1e-13 max(1,|z_i|) (a step at the rounding level).
template <typename T>
SBLM_FN bool newton_pass(const cx<T> c[6], cx<T> z[5], const T d2[5], T tau) {
  bool conv = true;
  const T tau2 = tau * tau;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    cx<T> p, dp;
    horner(c, z[i], p, dp);
    const T r = rcp_fast(c_norm(dp));
    const cx<T> dz = {fma(p.re, dp.re, p.im * dp.im) * r, fma(p.im, dp.re, -p.re * dp.im) * r};
    z[i] = c_sub(z[i], dz);
    const T sc = vmax(c_norm(z[i]), T(1.0));
    const T e2 = c_norm(dz);
    conv = conv && ((e2 * e2 <= tau2 * sc * d2[i]) || (e2 <= T(1e-26) * sc));
  }
  return conv;
}

// ---------------------------------------------------------------- images

#define SBLM_IMAGE_TOL2 1e-12 /* residual threshold 1e-6, squared */
#define SBLM_POLISH_DETJ 0.01 /* images with |det J| below this are refined */
#define SBLM_POLISH_EST2 1e-24 /* ... and those whose residual could move A by \
                                  more than 1e-12 relative (squared) */

// Lens-equation quantities at a trial image z: the residual
// r = zeta - z + 1/conj(z) - q/(d - conj(z)) of Eq. (lensing) and
// g = dzeta/dconj(z) = 1/conj(z)^2 + q/(d - conj(z))^2; returns |r|^2.
// *iz2, *ie2 receive |1/z|^2 and |1/(d - z)|^2.
template <typename R>
SBLM_FN R image_eval(cx<R> z, cx<R> zeta, R d, R q, cx<R>& res, cx<R>& g, R* iz2, R* ie2) {
  const R x = z.re, y = z.im;
  // a = 1/conj(z) = z / |z|^2 ; b = 1/(d - conj(z))
  // one reciprocal for both: 1/|z|^2 = |d-z|^2 / P, 1/|d-z|^2 = |z|^2 / P with
  // P = |z|^2 |d-z|^2 (within range: |z| stays far from the FP64 limits)
  const R n2 = fma(x, x, y * y);
  const R ex = d - x;
  const R e2 = fma(ex, ex, y * y);
  const R ip = rcp_acc(n2 * e2);
  const R iz = e2 * ip;
  const cx<R> a = {x * iz, y * iz};
  const R ie = n2 * ip;
  const cx<R> b = {ex * ie, -y * ie};
  res = {fma(-q, b.re, (zeta.re - x) + a.re), fma(-q, b.im, (zeta.im - y) + a.im)};
  const cx<R> b2 = c_mul(b, b);
  g = c_fma(a, a, cx<R>{q * b2.re, q * b2.im});
  *iz2 = iz;
  *ie2 = ie;
  return c_norm(res);
}

// The image test of one root: its squared residual *r2 on the lens equation,
// |det J| (*adet), and whether the image needs refining: when it lies very
// close to a critical curve (|det J| < 0.01) or when its residual r could
// move A by more than 1e-12 relative -- the image moves by about
// (1 + |g|) |r| / |det J|, det J by 2 |g| |h| times that
// (h = dg/dconj(z), |h| <= 2|1/z|^3 + 2q|1/(d-z)|^3) and A_i by A_i^2 times
// that, with A >= 1.
template <typename R>
SBLM_FN bool image_score(cx<R> z, cx<R> zeta, R d, R q, R* r2, R* adet) {
  cx<R> res, g;
  R iz2, ie2;
  *r2 = image_eval(z, zeta, d, q, res, g, &iz2, &ie2);
  const R gn = c_norm(g);
  *adet = fabs(R(1.0) - gn);
  // (dA/A)^2 <= 64 |g|^2 (1 + |g|^2) (|1/z|^6 + q^2 |1/(d-z)|^6) |r|^2 / |det J|^6;
  // refine when that exceeds SBLM_POLISH_EST2 (compared without dividing)
  const R a3 = *adet * *adet * *adet;
  const R num = R(64.0) * gn * (R(1.0) + gn) * fma(q * q * ie2, ie2 * ie2, iz2 * iz2 * iz2) * *r2;
  return !(num <= R(SBLM_POLISH_EST2) * (a3 * a3)) || *adet < R(SBLM_POLISH_DETJ);
}

// One image refined by up to two Newton steps on the lens equation itself,
// dz = (r - g conj(r))/(1 - |g|^2), each kept only if it lowers the
// residual; returns its 1/|det J|.  Near a critical curve (near-coincident
// roots next to a caustic) or in the root cluster around the secondary lens
// at small q the quintic's roots lose accuracy, while the lens equation does
// not.
template <typename R>
SBLM_FN R refine_image(cx<R> zi, cx<R> zeta, R d, R q) {
  cx<R> res, g;
  R iz2, ie2;
  R rn = image_eval(zi, zeta, d, q, res, g, &iz2, &ie2);
  for (int step = 0; step < 2; ++step) {
    const R det = R(1.0) - c_norm(g);
    const R idet = rcp_acc(det);
    // dz = (r - g conj(r)) / det
    const cx<R> gr = c_mul(g, cx<R>{res.re, -res.im});
    const cx<R> dz = {(res.re - gr.re) * idet, (res.im - gr.im) * idet};
    const cx<R> zn = {zi.re + dz.re, zi.im + dz.im};
    cx<R> resn, gn2;
    const R rnn = image_eval(zn, zeta, d, q, resn, gn2, &iz2, &ie2);
    if (!(rnn < rn)) break;
    zi = zn;
    res = resn;
    g = gn2;
    rn = rnn;
    // Newton converges quadratically: after a step of 1e-10 |z| the next
    // one would be at the rounding level
    if (c_norm(dz) <= R(1e-20) * c_norm(zi)) break;
  }
  return rcp_acc(fabs(R(1.0) - c_norm(g)));
}

// ---------------------------------------------------------------- fit

// Square-root-free Givens state for columns (1, A | y): D = diag(d1, d2),
// unit upper-triangular factor with off-diagonal r12, transformed right-hand
// side (t1, t2) and the accumulated weighted residual sum of squares.
template <typename R>
struct LsqT {
  R d1, d2, r12, t1, t2, sse;
};

// Include the row (x1, x2 | y) with weight w (Gentleman's algorithm).
template <typename R>
SBLM_FN void lsq_include(LsqT<R>& s, R w, R x1, R x2, R y) {
  if (w == R(0.0)) return;
  if (x1 != R(0.0)) {
    const R wx = w * x1;
    const R dp = fma(wx, x1, s.d1);
    const R r = rcp_acc(dp);
    const R cb = s.d1 * r, sb = wx * r;
    w = cb * w;
    s.d1 = dp;
    const R xk = x2;
    x2 = fma(-x1, s.r12, xk);
    s.r12 = fma(cb, s.r12, sb * xk);
    const R yk = y;
    y = fma(-x1, s.t1, yk);
    s.t1 = fma(cb, s.t1, sb * yk);
  }
  if (w == R(0.0)) return;
  if (x2 != R(0.0)) {
    const R wx = w * x2;
    const R dp = fma(wx, x2, s.d2);
    const R r = rcp_acc(dp);
    const R cb = s.d2 * r, sb = wx * r;
    w = cb * w;
    s.d2 = dp;
    const R yk = y;
    y = fma(-x2, s.t2, yk);
    s.t2 = fma(cb, s.t2, sb * yk);
  }
  s.sse = fma(w * y, y, s.sse);
}

// ---------------------------------------------------------------- warm start

// Weights (w1, w2, w3) of the roots of the three previous epochs t1 > t2 >
// t3 for the start at epoch t: quadratic (Lagrange in t) extrapolation when
// all three are known (have3), however far t lies beyond them; else linear
// from two (have2), scaled by the ratio of epoch spacings clamped to [0, 4];
// else the previous roots themselves.  Across a gap in the cadence (a night
// between two runs of epochs minutes apart) the root paths are smooth, and
// the curvature the three close epochs give carries the start to within one
// sweep, where the linear start, clamped, left most such epochs two or three
// sweeps short; a poor start over a very long gap costs sweeps, or a cold
// retry, never a wrong root.
template <typename R>
SBLM_FN void warm_weights(R t, R t1, R t2, R t3, bool have2, bool have3, R& w1, R& w2, R& w3) {
  w1 = R(1.0);
  w2 = R(0.0);
  w3 = R(0.0);
  const R d12 = t1 - t2, d23 = t2 - t3, d13 = t1 - t3;
  if (have2 && have3 && d12 > R(0.0) && d23 > R(0.0)) {
    const R a1 = t - t1, a2 = t - t2, a3 = t - t3;
    const R r = rcp_fast(d12 * d13 * d23);
    w1 = a2 * a3 * (d23 * r);
    w2 = -a1 * a3 * (d13 * r);
    w3 = a1 * a2 * (d12 * r);
  } else if (have2 && d12 > R(0.0)) {
    const R r = vmin(vmax((t - t1) * rcp_fast(d12), R(0.0)), R(4.0));
    w1 = R(1.0) + r;
    w2 = -r;
  }
}

// The start of one root at the new epoch from its values at the three
// previous epochs, with the weights of warm_weights.
template <typename R>
SBLM_FN cx<R> extrapolate(cx<R> z1, cx<R> z2, cx<R> z3, R w1, R w2, R w3) {
  return {fma(w1, z1.re, fma(w2, z2.re, w3 * z3.re)), fma(w1, z1.im, fma(w2, z2.im, w3 * z3.im))};
}

}  // namespace sblm

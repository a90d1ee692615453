// sblm_fitness.hip -- batched binary-lens magnification and chi^2 fitness on
// gfx950 (MI355X).
//
// Method (Rajpaul 2012, Sec. 2.2 and Sec. 4): for every (individual, epoch)
// pair the source position follows Eq. (sourcePos) with tau = (t - t0)/tE;
// the images solve the lens equation Eq. (lensing), whose fifth-order
// polynomial form Eq. (lensingPoly) is solved here for all five roots; the
// two spurious roots are rejected by substitution into the lens equation;
// the magnification is sum_i 1/|det J_i| with
// det J = 1 - |1/conj(z)^2 + q/(d - conj(z))^2|^2.  The fitness is chi^2 of
// the blended flux Fs*A + Fb (Sec. 4.4, Eq. blend) with Fs, Fb profiled by
// weighted linear least squares.
//
// Mapping onto CDNA4:
//   * one group of G lanes (G = 64, 32 or 16) per individual, each lane
//     owning a contiguous chunk of C = ceil(L/G) epochs; the individual's
//     parameters are wave-uniform (scalar registers), epochs are read once;
//   * all five roots are found together by the Ehrlich-Aberth simultaneous
//     iteration -- branch-free and identical work per lane, so a wavefront
//     stays in lockstep.  The first epoch of a chunk starts from a circle
//     around the root centroid; every later epoch starts from the previous
//     epoch's roots (the source moves little between epochs), which cuts the
//     wave-level sweep count by ~2.5x.  The loop ends when every lane of the
//     wave has converged (wave vote);
//   * FP64 mode iterates in FP64.  MIXED mode iterates in FP32 to a loose
//     tolerance, then continues in FP64 (normally two sweeps) from there; the
//     image test, det J and the fit are FP64 in both modes;
//   * the weighted least-squares fit is accumulated on the fly with
//     square-root-free Givens rotations (Gentleman 1973, the row-update form
//     of a QR factorisation) over columns (1, A | y), so chi^2 comes out as
//     the accumulated residual, with no A stored and no cancellation of
//     large sums; lane results are merged by a fixed shuffle tree (bitwise
//     deterministic).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include "sblm_internal.h"

// Stopping tolerance of the FP64 root iteration: the estimated error left in
// every root after the last step, relative to max(1, |z|).  The roots only
// start the images: an accepted image whose residual on the lens equation
// could move A by more than 1e-12 relative is refined on the lens equation
// itself (see magnification), so this tolerance sets the work, not the
// accuracy of A: 1e-9 leaves the measured magnification errors as they are
// at 1e-16 (they first grow at 1e-8) while most warm-started solves end
// after one sweep.
#ifndef SBLM_ROOT_TAU
#define SBLM_ROOT_TAU 1e-9
#endif
// The FP32 iteration of the precision form only has to bring the roots
// within reach of two FP64 Newton steps (quadratic: an error e0 goes to
// about e0^2/s, then e0^4/s^3): an estimated error of 1e-5 relative.
#ifndef SBLM_ROOT_TAU32
#define SBLM_ROOT_TAU32 1e-5f
#endif

namespace sblm {

// The primitive operations the shared arithmetic (sblm_math.h) takes from
// its number type, for FP64 and FP32 on the device.
// Smaller / larger of two values, the non-NaN one if one is NaN (one v_min /
// v_max where the operands are results of arithmetic, which the compiler knows
// to be quiet).
__device__ __forceinline__ double vmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float vmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float vmax(float a, float b) { return fmaxf(a, b); }
// Hardware reciprocal estimate (relative error < 5e-8 in FP64).
__device__ __forceinline__ double rcp_hw(double x) { return __builtin_amdgcn_rcp(x); }
__device__ __forceinline__ float rcp_hw(float x) { return __builtin_amdgcn_rcpf(x); }

}  // namespace sblm

#include "sblm_math.h"

namespace sblm {

// Starting points for a cold solve: five points on a circle about the root
// centroid -c4/(5 c5) of radius (|c0|/|c5|)^(1/5) (geometric mean of the
// root moduli); for a degree-4 polynomial four points and one root parked
// far away, where it never moves; with a far root (far_root) the four near
// roots start as for the degree-4 polynomial and the fifth at -c4/c5, which
// it would otherwise take the iteration some 50-80 sweeps to walk out to.
template <typename T>
__device__ __forceinline__ void cold_start(const cx<T> c[6], bool deg4,
                                           cx<T> z[5], bool far = false) {
  // cos/sin of 2 pi k/5 + 0.4 and 2 pi k/4 + 0.4
  const float c5a[5] = {0.92106099f, 0.06083749f, -0.88523008f, -0.62472004f,
                        0.52805164f};
  const float s5a[5] = {0.38941834f, 0.99814771f, 0.46517413f, -0.78084257f,
                        -0.84920782f};
  const float c4a[4] = {0.92106099f, -0.38941834f, -0.92106099f, 0.38941834f};
  const float s4a[4] = {0.38941834f, 0.92106099f, -0.38941834f, -0.92106099f};
  const bool four = deg4 || far;
  const int lead = four ? 4 : 5;
  const float n_lead = (float)c_norm(c[lead]);
  const float n_0 = (float)c_norm(c[0]);
  float ratio = n_0 / n_lead;
  if (!(ratio > 1e-30f) || !(ratio < 1e30f)) ratio = 1.0f;
  const float R = powf(ratio, four ? 0.125f : 0.1f);
  // centroid = -c[lead-1] / (lead c[lead])
  const cx<float> a = {(float)c[lead - 1].re, (float)c[lead - 1].im};
  const cx<float> b = {(float)c[lead].re, (float)c[lead].im};
  const float ib = 1.0f / (fmaf(b.re, b.re, b.im * b.im) * (float)lead);
  const float cen_re = -(a.re * b.re + a.im * b.im) * ib;
  const float cen_im = -(a.im * b.re - a.re * b.im) * ib;
  if (four) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      z[k] = {(T)(cen_re + R * c4a[k]), (T)(cen_im + R * s4a[k])};
    z[4] = {(T)1e18, (T)1e18};
    if (far) {  // -c4/c5
      const T n5 = c_norm(c[5]);
      z[4] = {-(c[4].re * c[5].re + c[4].im * c[5].im) / n5,
              -(c[4].im * c[5].re - c[4].re * c[5].im) / n5};
    }
  } else {
#pragma unroll
    for (int k = 0; k < 5; ++k)
      z[k] = {(T)(cen_re + R * c5a[k]), (T)(cen_im + R * s5a[k])};
  }
}

// Images, det J and the magnification from five FP64 roots.  The image
// count and the choice of images use the roots' residuals (image_score); an
// accepted image that needs it is refined on the lens equation
// (refine_image).
__device__ __forceinline__ double magnification(const cx<double> z[5],
                                                cx<double> zeta, double d,
                                                double q, bool deg4,
                                                int& nimg, int& npolish) {
  double r2[5], adet[5];
  bool refine[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) refine[i] = image_score(z[i], zeta, d, q, &r2[i], &adet[i]);
  if (deg4) r2[4] = INFINITY;
  int below = 0;
#pragma unroll
  for (int i = 0; i < 5; ++i) below += (r2[i] < SBLM_IMAGE_TOL2) ? 1 : 0;
  const bool five = !deg4 && below >= 4;
  // accepted images: sum those that need no refinement, list the others
  double A = 0.0;
  unsigned int todo = 0u;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    int rank = 0;
#pragma unroll
    for (int j = 0; j < 5; ++j)
      rank += (r2[j] < r2[i] || (r2[j] == r2[i] && j < i)) ? 1 : 0;
    const bool acc = five || rank < 3;
    if (acc && refine[i])
      todo |= 1u << i;
    else if (acc)
      A += rcp_acc(adet[i]);
  }
  // refinement: one image per lane per pass, so the wavefront runs as many
  // passes as the lane with the most images to refine
  while (__any(todo != 0u)) {
    if (todo) {
      const int i = __builtin_ctz(todo);
      todo &= todo - 1u;
      cx<double> zi = z[0];
#pragma unroll
      for (int k = 1; k < 5; ++k)
        if (i == k) zi = z[k];
      ++npolish;
      A += refine_image(zi, zeta, d, q);
    }
  }
  nimg = five ? 5 : 3;
  return A;
}

// ---------------------------------------------------------------- fit

using Lsq = LsqT<double>;

// ---------------------------------------------------------------- kernel

template <int G>
__device__ __forceinline__ double grp_shfl_down(double v, int off) {
  return __shfl_down(v, off, G);
}

// Per-lane counters (32 bits: a lane's share of one launch stays far below
// 2^32 events), summed over the wave and added to sblm_stats at the end.
struct LaneStats {
  unsigned int solves, iters, capped, fallback, deg4, wave_iters, iters32, polished, retried,
      unsettled, newton;
};

// A solve that reaches the iteration cap has settled when its roots are
// finite and its last sweep moved them by less than this much relative
// (squared, i.e. 1e-4): the iteration has stalled at the rounding level next
// to a near-multiple root -- two images merging at a fold of the caustic,
// three at a cusp, where FP64 resolves the roots only to about eps^(1/2) and
// eps^(1/3) ~ 6e-6 relative and the steps jitter at that level; the
// accepted images are refined on the lens equation anyway.
#define SBLM_SETTLED_STEP2 1e-8

// Solve one polynomial from the roots in z (warm) or from a cold start;
// ok = converged to finite roots; settled = ok, or capped with finite roots
// that no longer move (see SBLM_SETTLED_STEP2).  `retry` marks a second,
// cold attempt at an epoch whose warm-started solve failed (not counted as
// another solve).
template <int MODE>
__device__ __forceinline__ void solve_roots(const cx<double> c[6], bool deg4,
                                            bool warm, bool active,
                                            cx<double> z[5], LaneStats& st,
                                            bool& ok, bool& settled, bool retry = false) {
  constexpr int MAXIT64 = 60, MAXIT32 = 30;
  // estimated relative error left after the last step
  const double tau64 = SBLM_ROOT_TAU;
  const float tau32 = SBLM_ROOT_TAU32;
  const bool far = !deg4 && far_root(c);
  if (!warm && active) cold_start<double>(c, deg4, z, far);
  unsigned int it_lane = 0, it32_lane = 0, it_wave = 0, newton_lane = 0;
  bool done = !active, fell_back = false;
  if (MODE == SBLM_MIXED) {
    // The precision form: the root iteration in FP32 to a loose tolerance,
    // then at most two FP64 Newton steps on every root, the image test, det J
    // and the fit in FP64.  A polish that has not converged after two steps
    // falls back to FP64 Aberth sweeps from the polished roots (counted).
    // A warm start (the previous epochs' roots, extrapolated) is already as
    // close as FP32 can resolve and goes straight to the polish; degree-4
    // polynomials (parked root out of FP32 range) and those with a far root
    // (its powers overflow FP32) straight to FP64 sweeps.  The FP32
    // iteration ends at its own convergence test, or, after its first few
    // sweeps (the global phase, where steps need not shrink), when its steps
    // stop shrinking (the FP32 rounding floor next to clustered roots).
    const bool use32 = !deg4 && !far;
    cx<float> cf[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) cf[j] = {(float)c[j].re, (float)c[j].im};
    cx<float> zf[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) zf[i] = {(float)z[i].re, (float)z[i].im};
    bool done32 = done || !use32 || warm;
    float prev = INFINITY;
    for (int it = 0; it < MAXIT32; ++it) {
      if (__all(done32)) break;
      ++it_wave;
      if (!done32) {
        float em;
        done32 = aberth_sweep<true>(cf, zf, false, tau32, &em);
        done32 = done32 || (it >= 4 && em > 0.25f * prev);  // shrank by < 2x
        prev = em;
        ++it32_lane;
      }
    }
    const bool polish = active && use32;
    if (polish && !warm) {
#pragma unroll
      for (int i = 0; i < 5; ++i) z[i] = {(double)zf[i].re, (double)zf[i].im};
    }
    double d2[5];
    nearest2(z, d2);
    bool pol_done = !polish;
    for (int k = 0; k < 2; ++k) {
      if (__all(pol_done)) break;
      ++it_wave;
      if (!pol_done) {
        pol_done = newton_pass(c, z, d2, tau64);
        ++newton_lane;
      }
    }
    if (polish) {
      // Newton steps that drew two roots together (a root taken over by its
      // neighbour's basin) leave the distinct FP32 roots behind: start the
      // FP64 iteration afresh
      double d2n[5];
      nearest2(z, d2n);
      bool apart = true;
#pragma unroll
      for (int i = 0; i < 5; ++i) apart = apart && (d2n[i] >= 0.25 * d2[i]);
      if (!apart) cold_start<double>(c, deg4, z, far);
      done = pol_done && apart;
      fell_back = !done;
    }
  }
  for (int it = 0; it < MAXIT64; ++it) {
    if (__all(done)) break;
    ++it_wave;
    if (!done) {
      done = aberth_sweep<false>(c, z, deg4, tau64, (double*)nullptr);
      ++it_lane;
    }
  }
  // a capped solve: one more sweep measures how far its roots still move
  double em_last = 0.0;
  if (__any(active && !done)) {
    if (active && !done) (void)aberth_sweep<true>(c, z, deg4, tau64, &em_last);
  }
  bool finite = true;
#pragma unroll
  for (int i = 0; i < 5; ++i)
    finite = finite && isfinite(z[i].re) && isfinite(z[i].im);
  ok = done && finite;
  settled = finite && (done || em_last <= SBLM_SETTLED_STEP2);
  if (active) {
    st.solves += retry ? 0 : 1;
    st.iters += it_lane + it32_lane;
    st.deg4 += (deg4 && !retry) ? 1 : 0;
    // MIXED: a polish that needed the FP64 iteration after its two steps
    if (MODE == SBLM_MIXED) st.fallback += fell_back ? 1 : 0;
    st.wave_iters += it_wave;
    st.iters32 += it32_lane;
    st.newton += newton_lane;
  }
}

// The cold second attempt at an epoch whose warm-started solve failed (a
// warm start from the roots of another epoch or, in the simplex rounds, of
// another point), called by the whole wave when any lane needs it; lanes
// with active = 0 only follow along.  Kept out of line: a second inlined
// copy of the iteration would cost the hot path registers.  Coefficients,
// roots (in and out) and the lane's counters travel through memory.
template <int MODE>
__device__ __noinline__ void cold_retry(const double* cr, double* zr, int deg4, int active,
                                        unsigned int* counts) {
  cx<double> c[6], z[5];
  for (int j = 0; j < 6; ++j) c[j] = {cr[2 * j], cr[2 * j + 1]};
  for (int i = 0; i < 5; ++i) z[i] = {zr[2 * i], zr[2 * i + 1]};
  LaneStats st = {};
  bool ok, settled;
  solve_roots<MODE>(c, deg4 != 0, false, active != 0, z, st, ok, settled, true);
  for (int i = 0; i < 5; ++i) {
    zr[2 * i] = z[i].re;
    zr[2 * i + 1] = z[i].im;
  }
  counts[0] = st.iters;
  counts[1] = st.wave_iters;
  counts[2] = st.iters32;
  counts[3] = st.newton;
  counts[4] = st.fallback;
  counts[5] = (ok ? 1u : 0u) | (settled ? 2u : 0u);
}

#ifndef SBLM_MIN_WAVES_PER_EU
#define SBLM_MIN_WAVES_PER_EU 1
#endif

// Per-lane context of one work item: the individual, its parameters and the
// lane's chunk [k0, k1) of the lightcurve's epochs.
struct Item {
  bool valid;
  int gl;  // lane within the group
  int64_t ind;
  double q, d, u0, sa, ca, t0, itE;
  int64_t e0, k0, k1, Cg, C;  // C: longest chunk in the wave
};

// The transcendental part of an individual's set-up: q = 10^(log10 q),
// sin and cos of alpha, 1/tE.  Out of line: inlined, the many constants of
// the exp10 and sincos expansions are hoisted out of the persistent grid's
// work loop into registers that then spill to scratch memory in every wave.
struct ItemTrig {
  double q, sa, ca, itE;
};
__device__ __noinline__ ItemTrig item_trig(double lq, double alpha, double tE) {
  ItemTrig r;
  r.q = exp10(lq);
  sincos(alpha, &r.sa, &r.ca);
  r.itE = 1.0 / tE;
  return r;
}

template <int G>
__device__ __forceinline__ Item item_setup(const FitArgs& a, int64_t wave_item) {
  Item x;
  const int lane = threadIdx.x & 63;
  int64_t item;
  if constexpr (G > 64) {  // G / 64 waves per individual: wave item = (individual, part)
    item = wave_item / (G / 64);
    x.gl = (int)(wave_item % (G / 64)) * 64 + lane;
  } else {
    x.gl = lane & (G - 1);
    item = wave_item * (64 / G) + (lane / G);
  }
  x.valid = item < a.n_ind;
  x.ind = x.valid ? (a.order ? (int64_t)a.order[item] : item) : 0;
  // parameters of this individual (uniform within the group)
  double th[SBLM_NPAR];
#pragma unroll
  for (int j = 0; j < SBLM_NPAR; ++j) {
    const double v = x.valid ? a.theta[j * a.n_ind + x.ind] : 0.5;
    th[j] = a.encoded ? a.lo[j] + a.span[j] * v : v;
  }
  const ItemTrig tr = item_trig(th[0], th[3], th[4]);
  x.q = tr.q;
  x.d = th[1];
  x.u0 = th[2];
  x.t0 = th[5];
  x.sa = tr.sa;
  x.ca = tr.ca;
  x.itE = tr.itE;
  int64_t e0 = 0, e1 = a.n_t;
  if (a.off) {
    const int64_t lc = x.ind / a.pop;
    e0 = x.valid ? a.off[lc] : 0;
    e1 = x.valid ? a.off[lc + 1] : 0;
    if (a.skip && x.valid && a.skip[x.ind / a.skip_per]) e1 = e0;
  }
  if (!x.valid) e1 = e0;
  x.e0 = e0;
  const int64_t L = e1 - e0;
  x.Cg = (L + G - 1) / G;
  x.C = x.Cg;
#pragma unroll
  for (int o = G; o < 64; o <<= 1) {
    const int64_t oc = __shfl_xor(x.C, o, 64);
    x.C = oc > x.C ? oc : x.C;
  }
  x.k0 = e0 + x.gl * x.Cg;
  x.k1 = (x.k0 + x.Cg < e1) ? x.k0 + x.Cg : e1;
  return x;
}

// Source position (Eq. sourcePos) and lens polynomial at epoch t.
__device__ __forceinline__ bool epoch_poly(const Item& x, double t, cx<double>& zeta,
                                           cx<double> c[6]) {
  zeta = source_position(t, x.t0, x.itE, x.sa, x.ca, x.u0);
  lens_coeffs(zeta, x.d, x.q, c);
  return drop_to_degree4(c);
}

// Per-lane history of the roots of the two epochs before the current one,
// kept in LDS (touched once per epoch, at the warm start; in registers it
// would hold 40 VGPRs through the whole solve).  Dynamic shared memory of
// ROOT_HIST_BYTES per thread; element [((slot*5 + i)*2 + part) * blockDim.x +
// thread] holds root i of epoch slot (0: previous but one, 1: the one
// before), real (part 0) or imaginary (part 1).
constexpr size_t ROOT_HIST_BYTES = 2 * 5 * 2 * sizeof(double);

// Dynamic shared memory: the root history, then (G > 64) one least-squares
// state per wave for the merge across the waves of an individual.
extern __shared__ double fit_dyn_smem[];

// Merge the lanes' least-squares states of each group (fixed tree) and write
// chi^2, Fs, Fb of the group's individual.  With G > 64 each wave merges its
// 64 lanes the same way, and the first wave of the individual then absorbs
// the states of the others in wave order (all waves of the block pass one
// barrier here).
template <int G>
__device__ __forceinline__ void finish_chi2(const FitArgs& a, const Item& x, Lsq ls) {
  constexpr int GW = G > 64 ? 64 : G;  // lanes merged by shuffles
  const int gl = x.gl;
  const bool valid = x.valid;
  const int64_t ind = x.ind;
  {
    // lane gl absorbs lane gl + off: fixed tree inside each group (wave)
#pragma unroll
    for (int off = GW / 2; off >= 1; off >>= 1) {
      Lsq o;
      o.d1 = grp_shfl_down<GW>(ls.d1, off);
      o.d2 = grp_shfl_down<GW>(ls.d2, off);
      o.r12 = grp_shfl_down<GW>(ls.r12, off);
      o.t1 = grp_shfl_down<GW>(ls.t1, off);
      o.t2 = grp_shfl_down<GW>(ls.t2, off);
      o.sse = grp_shfl_down<GW>(ls.sse, off);
      if ((gl & (GW - 1)) < off) {
        lsq_include(ls, o.d1, 1.0, o.r12, o.t1);
        lsq_include(ls, o.d2, 0.0, 1.0, o.t2);
        ls.sse += o.sse;
      }
    }
    if constexpr (G > 64) {
      double* part = fit_dyn_smem + (ROOT_HIST_BYTES / sizeof(double)) * blockDim.x;
      const int w = threadIdx.x >> 6;
      if ((threadIdx.x & 63) == 0) {
        part[w * 6 + 0] = ls.d1;
        part[w * 6 + 1] = ls.d2;
        part[w * 6 + 2] = ls.r12;
        part[w * 6 + 3] = ls.t1;
        part[w * 6 + 4] = ls.t2;
        part[w * 6 + 5] = ls.sse;
      }
      __syncthreads();
      if (gl == 0) {
        for (int p = 1; p < G / 64; ++p) {
          const double* o = part + (w + p) * 6;
          lsq_include(ls, o[0], 1.0, o[2], o[3]);
          lsq_include(ls, o[1], 0.0, 1.0, o[4]);
          ls.sse += o[5];
        }
      }
    }
    if (gl == 0 && valid) {
      const double saa = fma(ls.d1 * ls.r12, ls.r12, ls.d2);
      double fs, fb, c2;
      if (!(ls.d2 > 1e-14 * saa)) {  // singular 2x2 system
        fs = 0.0;
        fb = ls.t1;
        c2 = fma(ls.d2 * ls.t2, ls.t2, ls.sse);
      } else {
        fs = ls.t2;
        fb = fma(-ls.r12, fs, ls.t1);
        c2 = ls.sse;
      }
      a.chi2[ind] = c2;
      a.Fs[ind] = fs;
      a.Fb[ind] = fb;
      if (a.stats && !(ls.d2 > 1e-14 * saa))
        atomicAdd(&a.stats->n_degenerate, 1ull);
    }
  }

}

struct RootHist {
  double* h;
  __device__ __forceinline__ cx<double> get(int slot, int i) const {
    const int n = blockDim.x;
    return {h[((slot * 5 + i) * 2) * n + threadIdx.x],
            h[((slot * 5 + i) * 2 + 1) * n + threadIdx.x]};
  }
  __device__ __forceinline__ void set(int slot, int i, cx<double> v) const {
    const int n = blockDim.x;
    h[((slot * 5 + i) * 2) * n + threadIdx.x] = v.re;
    h[((slot * 5 + i) * 2 + 1) * n + threadIdx.x] = v.im;
  }
};

// One wave's share of the work, lockstep form: 64/G individuals (items
// wave_item*64/G ...); every lane solves its s-th epoch at the same time and
// the wave moves on when all of them have converged.
template <int MODE, bool CHI2, int G>
__device__ __forceinline__ void fit_wave(const FitArgs& a, int64_t wave_item,
                                         LaneStats& st) {
  Item x = item_setup<G>(a, wave_item);
  const int64_t C = x.C, Cg = x.Cg, k0 = x.k0, k1 = x.k1, e0 = x.e0, ind = x.ind;
  const double q = x.q, d = x.d, t0 = x.t0;
  Lsq ls = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  cx<double> z[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) z[i] = {0.0, 0.0};
  const RootHist hist = {fit_dyn_smem};  // zp (slot 0), zpp (slot 1)
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    hist.set(0, i, {0.0, 0.0});
    hist.set(1, i, {0.0, 0.0});
  }
  bool have_prev = false, prev_deg4 = false, have_prev2 = false, have_prev3 = false;
  double t1 = 0.0, t2 = 0.0, t3 = 0.0;  // epochs of z, zp and zpp

  // the epoch time one step ahead, the observation at the top of its step:
  // the loads are in flight during the solve
  double t_next = (0 < Cg && k0 < k1) ? a.t[k0] : t0;
  for (int64_t s = 0; s < C; ++s) {
    const int64_t k = k0 + s;
    const bool active = (s < Cg) && (k < k1);
    const double t = active ? t_next : t0;
    t_next = (s + 1 < Cg && k + 1 < k1) ? a.t[k + 1] : t0;
    double wk = 0.0, yk = 0.0;
    if (CHI2 && active) {
      wk = a.w[k];
      yk = a.y[k];
    }
    // the root history, read before the polynomial is formed (its latency
    // then overlaps the coefficients)
    cx<double> hp[5], hpp[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      hp[i] = hist.get(0, i);
      hpp[i] = hist.get(1, i);
    }
    cx<double> zeta, c[6];
    const bool deg4 = epoch_poly(x, t, zeta, c);
    bool warm = have_prev && !deg4 && !prev_deg4;
    bool cached = false;  // started from the root cache (not a solved epoch)
    if constexpr (G >= 64) {
      // simplex rounds: a lane's first epoch starts from the roots the lane
      // found there for the same trial slot in the previous round (the
      // simplex moves little between rounds), else cold -- always cold in
      // the first round of a run, so that a run does not depend on what ran
      // in its slot before
      if (s == 0 && a.root_cache && active && !deg4 &&
          !(a.cold && a.cold[x.ind / a.cold_per])) {
        const double* rc = a.root_cache + (x.ind * G + x.gl) * 10;
        cx<double> zc[5];
        bool fin = true;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          zc[i] = {rc[2 * i], rc[2 * i + 1]};
          fin = fin && isfinite(zc[i].re) && isfinite(zc[i].im);
        }
        if (fin) {
#pragma unroll
          for (int i = 0; i < 5; ++i) z[i] = zc[i];
          warm = true;
          cached = true;
        }
      }
    }
    // Warm start: quadratic (Lagrange in t) extrapolation of every root from
    // the three previous epochs, else linear from two (warm_weights); the
    // history shifts as it is used.
    {
      double w1, w2, w3;
      warm_weights(t, t1, t2, t3, warm && have_prev2, have_prev3, w1, w2, w3);
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        const cx<double> old = z[i], zp = hp[i], zpp = hpp[i];
        z[i] = extrapolate(old, zp, zpp, w1, w2, w3);
        hist.set(1, i, zp);
        hist.set(0, i, old);
      }
    }
    bool ok, settled;
    solve_roots<MODE>(c, deg4, warm, active, z, st, ok, settled);
    {
      // a warm start that did not converge: solve again from the cold
      // start; roots that still have not settled poison the result (A and
      // with it chi^2 become NaN, which ranks last)
      const bool again = active && !ok && warm;
      if (__any(again)) {
        double cr[12], zr[10];
        unsigned int cnt[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          cr[2 * j] = c[j].re;
          cr[2 * j + 1] = c[j].im;
        }
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          zr[2 * i] = z[i].re;
          zr[2 * i + 1] = z[i].im;
        }
        cold_retry<MODE>(cr, zr, deg4 ? 1 : 0, again ? 1 : 0, cnt);
        if (again) {
#pragma unroll
          for (int i = 0; i < 5; ++i) z[i] = {zr[2 * i], zr[2 * i + 1]};
          ok = (cnt[5] & 1u) != 0;
          settled = (cnt[5] & 2u) != 0;
          st.iters += cnt[0];
          st.iters32 += cnt[2];
          st.newton += cnt[3];
          st.fallback += cnt[4];
          st.retried += 1;
        }
        st.wave_iters += active ? cnt[1] : 0;
      }
      if (active && !ok) st.capped += 1;
      if (active && !settled) st.unsettled += 1;
    }
    if constexpr (G >= 64) {
      if (s == 0 && a.root_cache && active) {
        double* rc = a.root_cache + (x.ind * G + x.gl) * 10;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          rc[2 * i] = ok ? z[i].re : NAN;
          rc[2 * i + 1] = ok ? z[i].im : NAN;
        }
      }
    }
    // (roots started from the cache follow no solved epoch: the next epoch
    // extrapolates from this one alone)
    have_prev3 = have_prev2 && warm && ok;
    have_prev2 = warm && !cached && ok;
    t3 = t2;
    t2 = t1;
    t1 = t;
    have_prev = ok;
    prev_deg4 = deg4;
    if (active) {
      int nimg, npol = 0;
      double A = magnification(z, zeta, d, q, deg4, nimg, npol);
      if (!settled) {
        A = NAN;
        nimg = 0;
      }
      st.polished += npol;
      if (CHI2) {
        lsq_include(ls, wk, 1.0, A, yk);
      } else {
        const int64_t o = ind * a.n_t + (k - e0);
        a.A[o] = A;
        if (a.n_img) a.n_img[o] = (int8_t)nimg;
      }
    }
  }

  if (CHI2) finish_chi2<G>(a, x, ls);
}

// One wave's share of the work, asynchronous form: every lane moves on to
// its next epoch as soon as its own solve has converged, so a wavefront pays
// for the lanes' own sweeps (plus the epoch set-up and image work of the
// lanes finishing in a pass) instead of the slowest lane of every epoch.
// The warm start is that of the lockstep form (warm_weights), and so is
// every lane's arithmetic: the two forms give the same results bit for bit.
template <int MODE, bool CHI2, int G>
__device__ __forceinline__ void fit_wave_async(const FitArgs& a, int64_t wave_item,
                                               LaneStats& st) {
  constexpr int MAXIT64 = 60, MAXIT32 = 30;
  const double tau64 = SBLM_ROOT_TAU;
  const float tau32 = SBLM_ROOT_TAU32;
  const Item x = item_setup<G>(a, wave_item);
  Lsq ls = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  cx<double> z[5];  // iterate; the roots of the two epochs before are in LDS
  const RootHist hist = {fit_dyn_smem};  // zp (slot 0), zpp (slot 1)
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    z[i] = {0.0, 0.0};
    hist.set(0, i, {0.0, 0.0});
    hist.set(1, i, {0.0, 0.0});
  }
  int nhist = 0;  // solved epochs held in z (after convergence), zp, zpp
  double t1 = 0.0, t2 = 0.0, t3 = 0.0;
  bool prev_deg4 = false;
  int64_t k = x.k0;
  bool busy = k < x.k1, need_setup = busy;
  cx<double> zeta = {0.0, 0.0}, c[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) c[j] = {0.0, 0.0};
  // phase of the current solve: 0 FP32 iteration, 1 FP64 Newton polish
  // (MIXED), 2 FP64 iteration
  bool deg4 = false, warm = false, fell_back = false;
  int phase = 2;
  double t = 0.0;
  int it64 = 0, it32 = 0, it_prior = 0, nw = 0;
  double d2[5];  // squared nearest-root distances at the start of the polish
#pragma unroll
  for (int i = 0; i < 5; ++i) d2[i] = 0.0;
  bool retried = false;
  double em64 = INFINITY;
  float prev32 = INFINITY;
  unsigned long long passes = 0;
  while (__any(busy)) {
    ++passes;
    if (busy) {
      if (need_setup) {
        t = a.t[k];
        deg4 = epoch_poly(x, t, zeta, c);
        warm = nhist >= 1 && !deg4 && !prev_deg4;
        if (warm) {
          // weights of z (epoch t1), zp (t2), zpp (t3)
          double w1, w2, w3;
          warm_weights(t, t1, t2, t3, nhist >= 2, nhist >= 3, w1, w2, w3);
#pragma unroll
          for (int i = 0; i < 5; ++i) {
            const cx<double> zp = hist.get(0, i), zpp = hist.get(1, i);
            const cx<double> p = extrapolate(z[i], zp, zpp, w1, w2, w3);
            hist.set(1, i, zp);
            hist.set(0, i, z[i]);
            z[i] = p;
          }
          t3 = t2;
          t2 = t1;
        } else {
          cold_start<double>(c, deg4, z, !deg4 && far_root(c));
        }
        phase = (MODE == SBLM_MIXED) && !deg4 && !far_root(c) ? (warm ? 1 : 0) : 2;
        if (phase == 1) nearest2(z, d2);
        it64 = 0;
        it32 = 0;
        nw = 0;
        fell_back = false;
        it_prior = 0;
        retried = false;
        em64 = INFINITY;
        prev32 = INFINITY;
        need_setup = false;
      }
      bool finished = false, conv = false;
      if (MODE == SBLM_MIXED && phase == 0) {
        // FP32 sweep on the rounded iterate (exactly representable back in FP64)
        cx<float> cf[6], zf[5];
#pragma unroll
        for (int j = 0; j < 6; ++j) cf[j] = {(float)c[j].re, (float)c[j].im};
#pragma unroll
        for (int i = 0; i < 5; ++i) zf[i] = {(float)z[i].re, (float)z[i].im};
        float em;
        bool d32 = aberth_sweep<true>(cf, zf, false, tau32, &em);
        d32 = d32 || (it32 >= 4 && em > 0.25f * prev32);
        prev32 = em;
#pragma unroll
        for (int i = 0; i < 5; ++i) z[i] = {(double)zf[i].re, (double)zf[i].im};
        ++it32;
        if (d32 || it32 >= MAXIT32) {
          phase = 1;
          nearest2(z, d2);
        }
      } else if (MODE == SBLM_MIXED && phase == 1) {
        // at most two FP64 Newton steps on every root (see solve_roots)
        const bool pol = newton_pass(c, z, d2, tau64);
        ++nw;
        if (pol || nw >= 2) {
          double d2n[5];
          nearest2(z, d2n);
          bool apart = true;
#pragma unroll
          for (int i = 0; i < 5; ++i) apart = apart && (d2n[i] >= 0.25 * d2[i]);
          if (!apart) cold_start<double>(c, deg4, z, false);
          if (pol && apart) {
            conv = true;
            finished = true;
          } else {
            phase = 2;
            fell_back = true;
          }
        }
      } else {
        conv = aberth_sweep<false>(c, z, deg4, tau64, (double*)nullptr);
        ++it64;
        finished = conv || it64 >= MAXIT64;
        // a capped solve: one more sweep measures how far its roots still move
        if (finished && !conv) (void)aberth_sweep<true>(c, z, deg4, tau64, &em64);
      }
      bool finite = true;
      if (finished) {
#pragma unroll
        for (int i = 0; i < 5; ++i)
          finite = finite && isfinite(z[i].re) && isfinite(z[i].im);
        if (!(conv && finite) && warm && !retried) {
          // the warm-started solve failed: again from the cold start (see
          // the lockstep form)
          cold_start<double>(c, deg4, z, !deg4 && far_root(c));
          warm = false;
          retried = true;
          phase = (MODE == SBLM_MIXED) && !deg4 && !far_root(c) ? 0 : 2;
          it_prior += it64 + it32;
          st.iters32 += it32;
          st.newton += nw;
          it64 = 0;
          it32 = 0;
          nw = 0;
          fell_back = false;
          em64 = INFINITY;
          prev32 = INFINITY;
          st.retried += 1;
          finished = false;
        }
      }
      if (finished) {
        const bool ok = conv && finite;
        const bool settled = finite && (conv || em64 <= SBLM_SETTLED_STEP2);
        int nimg, npol = 0;
        double A = magnification(z, zeta, x.d, x.q, deg4, nimg, npol);
        if (!settled) {
          A = NAN;
          nimg = 0;
        }
        if (CHI2) {
          lsq_include(ls, a.w[k], 1.0, A, a.y[k]);
        } else {
          const int64_t o = x.ind * a.n_t + (k - x.e0);
          a.A[o] = A;
          if (a.n_img) a.n_img[o] = (int8_t)nimg;
        }
        st.solves += 1;
        st.iters += it_prior + it64 + it32;
        st.iters32 += it32;
        st.capped += ok ? 0 : 1;
        st.unsettled += settled ? 0 : 1;
        st.deg4 += deg4 ? 1 : 0;
        st.polished += npol;
        if (MODE == SBLM_MIXED) {
          st.fallback += fell_back ? 1 : 0;
          st.newton += nw;
        }
        // z now holds the roots of epoch t
        nhist = ok ? (warm ? (nhist < 3 ? nhist + 1 : 3) : 1) : 0;
        t1 = t;
        prev_deg4 = deg4;
        ++k;
        busy = k < x.k1;
        need_setup = busy;
      }
    }
  }
  if (x.k1 > x.k0) st.wave_iters += passes;
  if (CHI2) finish_chi2<G>(a, x, ls);
}

// PERSIST = 0: one-shot grid.  PERSIST = 1: persistent grid fed by a work
// counter; its loop keeps the kernel arguments live, so it is compiled for
// two waves per SIMD (a few bytes of spill) instead of letting scalar-register
// spills push it to one.
template <int MODE, bool CHI2, int G, int PERSIST, int ASYNC>
__global__ __launch_bounds__(256, PERSIST ? 2 : SBLM_MIN_WAVES_PER_EU) void fitness_kernel(
    FitArgs a) {
  // (blocks of at most 256 threads: launch_gg refuses larger ones)
  constexpr int GPW = G > 64 ? 1 : 64 / G;  // individuals per wave
  const int lane = threadIdx.x & 63;
  LaneStats st = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  // One-shot grid: wave w takes wave item w (blocks remapped so that
  // consecutive logical blocks sit on one XCD, unless a work order is
  // given).  Persistent grid: waves take items from a shared counter until
  // it runs past the last one, so every wave reaches the exit.  One call
  // site keeps one inlined copy of the body.
  const int64_t n_wave_items = G > 64 ? a.n_ind * (G / 64) : (a.n_ind + GPW - 1) / GPW;
  if constexpr (PERSIST) {
    if (a.xcd_start) {
      // per-XCD queues: first the items of the lightcurves this block's XCD
      // owns (their epochs stay in its L2; workgroups are dealt to the XCDs
      // round-robin), then what is left in the other XCDs' queues.  Each
      // queue is visited until it runs past its last item, so every wave
      // reaches the exit.
      const int x0 = blockIdx.x & 7;
      for (int k = 0; k < 8; ++k) {
        const int x = (x0 + k) & 7;
        const int64_t w0 = (a.xcd_start[x] + GPW - 1) / GPW;
        const int64_t w1 = (a.xcd_start[x + 1] + GPW - 1) / GPW;
        for (;;) {
          unsigned int v = 0;
          if (lane == 0) v = atomicAdd(a.queue + x, 1u);
          const int64_t wi = w0 + (int64_t)__shfl(v, 0, 64);
          if (wi >= w1) break;
          if constexpr (ASYNC)
            fit_wave_async<MODE, CHI2, G>(a, wi, st);
          else
            fit_wave<MODE, CHI2, G>(a, wi, st);
        }
      }
    } else {
      for (;;) {
        unsigned int v = 0;
        if (lane == 0) v = atomicAdd(a.queue, 1u);
        const int64_t wi = (int64_t)__shfl(v, 0, 64);
        if (wi >= n_wave_items) break;
        if constexpr (ASYNC)
          fit_wave_async<MODE, CHI2, G>(a, wi, st);
        else
          fit_wave<MODE, CHI2, G>(a, wi, st);
      }
    }
  } else {
    // (with a work order, longest first, blocks keep the hardware order:
    // consecutive items, of similar length, go to different XCDs, where the
    // remap would put the longest eighth of the work on one of them)
    const int nb = gridDim.x, b = blockIdx.x;
    const int per = nb / 8, rem = nb % 8, xcd = b % 8, idx = b / 8;
    const int lb = a.order ? b
                   : (xcd < rem) ? xcd * (per + 1) + idx
                                 : rem * (per + 1) + (xcd - rem) * per + idx;
    const int64_t wi = (int64_t)lb * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if constexpr (ASYNC)
      fit_wave_async<MODE, CHI2, G>(a, wi, st);
    else
      fit_wave<MODE, CHI2, G>(a, wi, st);
  }
  if (a.stats) {
    // wave sums in 64 bits
    unsigned long long v[11] = {st.solves,  st.iters,     st.capped,   st.fallback,
                                st.deg4,    st.wave_iters, st.iters32, st.polished,
                                st.retried, st.unsettled, st.newton};
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
      for (int k = 0; k < 11; ++k) v[k] += __shfl_down(v[k], off, 64);
    if (lane == 0 && v[0]) {
      unsigned long long* dst[11] = {&a.stats->n_solves,    &a.stats->n_iter,
                                     &a.stats->n_capped,    &a.stats->n_fallback,
                                     &a.stats->n_degree4,   &a.stats->n_wave_iter,
                                     &a.stats->n_iter_fp32, &a.stats->n_polished,
                                     &a.stats->n_retried,   &a.stats->n_unsettled,
                                     &a.stats->n_newton};
#pragma unroll
      for (int k = 0; k < 11; ++k)
        if (v[k]) atomicAdd(dst[k], v[k]);
    }
  }
}

// The kernels are compiled for blocks of at most this many threads.
#define SBLM_FIT_MAX_THREADS 256

template <int MODE, bool CHI2, int G>
static hipError_t launch_gg(const FitArgs& a, hipStream_t s, int wpb) {
  if (wpb < 1 || 64 * wpb > SBLM_FIT_MAX_THREADS) return hipErrorInvalidConfiguration;
  if constexpr (G > 64) {
    // several waves per individual: one-shot grid, lockstep, whole
    // individuals in every block (for chi^2 their waves meet at the merge)
    constexpr int P = G / 64;
    if (a.queue || a.async || wpb % P != 0) return hipErrorInvalidConfiguration;
    const size_t smem = ROOT_HIST_BYTES * 64 * wpb + 6 * sizeof(double) * wpb;
    const int64_t nblk = (a.n_ind * P + wpb - 1) / wpb;
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL((fitness_kernel<MODE, CHI2, G, 0, 0>), dim3((unsigned)nblk),
                       dim3(64 * wpb), smem, s, a);
    return hipGetLastError();
  } else {
    const size_t smem = ROOT_HIST_BYTES * 64 * wpb;
    const int64_t groups_per_block = (int64_t)wpb * (64 / G);
    int64_t nblk = (a.n_ind + groups_per_block - 1) / groups_per_block;
    if (nblk <= 0) return hipSuccess;
    auto kern = a.async ? (a.queue ? fitness_kernel<MODE, CHI2, G, 1, 1>
                                   : fitness_kernel<MODE, CHI2, G, 0, 1>)
                        : (a.queue ? fitness_kernel<MODE, CHI2, G, 1, 0>
                                   : fitness_kernel<MODE, CHI2, G, 0, 0>);
    if (a.queue) {  // persistent grid: as many blocks as can be resident
      int dev = 0, ncu = 0, per_cu = 0;
      hipError_t e = hipGetDevice(&dev);
      if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
      if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * wpb, smem);
      if (e != hipSuccess) return e;
      const int64_t resident = (int64_t)(per_cu > 0 ? per_cu : 1) * ncu;
      nblk = nblk < resident ? nblk : resident;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(64 * wpb), smem, s, a);
    return hipGetLastError();
  }
}

template <int MODE, bool CHI2>
static hipError_t launch_g(const FitArgs& a, hipStream_t s, int wpb) {
  if (a.lanes_per_ind == 256) return launch_gg<MODE, CHI2, 256>(a, s, wpb);
  if (a.lanes_per_ind == 128) return launch_gg<MODE, CHI2, 128>(a, s, wpb);
  if (a.lanes_per_ind == 64) return launch_gg<MODE, CHI2, 64>(a, s, wpb);
  if (a.lanes_per_ind == 32) return launch_gg<MODE, CHI2, 32>(a, s, wpb);
  if (a.lanes_per_ind == 8) return launch_gg<MODE, CHI2, 8>(a, s, wpb);
  return launch_gg<MODE, CHI2, 16>(a, s, wpb);
}

hipError_t launch_fitness(const FitArgs& a, int mode, bool chi2,
                          hipStream_t s, int wpb) {
  if (mode == SBLM_MIXED)
    return chi2 ? launch_g<SBLM_MIXED, true>(a, s, wpb)
                : launch_g<SBLM_MIXED, false>(a, s, wpb);
  return chi2 ? launch_g<SBLM_FP64, true>(a, s, wpb)
              : launch_g<SBLM_FP64, false>(a, s, wpb);
}

}  // namespace sblm

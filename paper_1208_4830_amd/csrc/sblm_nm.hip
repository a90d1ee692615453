// sblm_nm.hip -- batched downhill-simplex refinement, one or several
// simplices per lightcurve (the amoeba fine-tuning of the EA's fittest
// solution, Sec. 4.1 and the "EA with amoeba" rows of Tables 2-3, and the
// iterated simplex compared there; method of Nelder & Mead 1965 in the form
// of Lagarias, Reeds, Wright & Wright 1998).
//
// The simplex lives in the EA's encoded domain [0, 1]^6 (Eq. EMMA-encoding):
// reflection 1, expansion 2, contraction 1/2, shrink 1/2; the initial
// simplex is x0 plus x0 with coordinate k scaled by 1.05 (0.00025 where it
// is 0), reflected below 1 and clipped; every trial point is clipped to the
// domain; vertices stay in ascending chi^2 order with ties kept in their
// previous order (NaN counts as +inf); the run stops before a step once
// every vertex is within tol_x of the best in every coordinate and within
// tol_f in chi^2, or after max_iter steps.
//
// Device form: a round is one launch of the fitness kernel over the trial
// points that the running simplices need, in one of two forms chosen per
// round by the number of running simplices.  While many run, a round is
// bound by its work: a step evaluates the reflection alone and, in the next
// round, the one other point that the reflection's value asks for (the
// expansion, or the outside or the inside contraction), if any -- about 1.6
// points per step.  While few run, a round is bound by the latency of its
// longest lightcurve: a step evaluates the reflection and, speculatively,
// the expansion and both contractions in one round, since all four depend
// only on the current simplex.  The six vertices of a shrink are evaluated
// over the next two rounds, and the seven initial vertices over the first
// two.  Only the needed trial points are launched in full (the others are
// evaluated as empty), packed to the front of the launch in the work order.
// Either way the sequence of simplices is that of the sequential algorithm.
//
// Iterated simplex (the comparison algorithm of Sec. 4.1): every slot of a
// lightcurve runs simplices from random start points one after another; a
// run that ends records its best vertex and the slot begins the next start
// in the same round, so no slot waits for the others between runs.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include <algorithm>

#include "sblm_internal.h"
#include "sblm_rng.h"

namespace sblm {
namespace {

constexpr int NP = SBLM_NPAR;  // 6 coordinates
constexpr int NV = NP + 1;     // 7 vertices
constexpr int NS = 4;          // trial slots per lightcurve and round
constexpr int NM_ITER_REPS_MAX = 1024;  // slots per lightcurve of nm_iterated

// A step in the two-round form waits in PH_WAIT_E, _OC or _IC for its second
// point, which goes in trial slot 1, 2 or 3 (the slot the speculative form
// gives the same point, so a slot's root cache holds roots of like points).
enum : int32_t {
  PH_INIT1 = 0,
  PH_INIT2,
  PH_STEP,
  PH_SHRINK1,
  PH_SHRINK2,
  PH_WAIT_E,
  PH_WAIT_OC,
  PH_WAIT_IC,
  PH_DONE
};
constexpr int COMPACT_CHUNK = 4096;  // trial points per block of the work-order packing
constexpr int COMPACT_ONE = 16384;   // at most this many: one block packs them all

struct NmWork {
  int32_t n;       // lightcurves
  double* V;       // [NV][NP][n] vertices
  double* F;       // [NV][n] chi^2 of the vertices
  double* FsV;     // [NV][n]
  double* FbV;     // [NV][n]
  double* T;       // [NP][n * NS] trial points, individual lc * NS + slot
  double* cT;      // [n * NS] trial chi^2
  double* fsT;
  double* fbT;
  double* rF;      // [3][n] chi^2, Fs, Fb of the reflection of a waiting step
  int32_t* phase;  // [n]
  int32_t* steps;  // [n]
  int32_t* skipT;  // [n * NS] 1: the trial slot is not needed in this round
                   // (evaluated as empty)
  int32_t spec;    // this round's form of a step: 1 four points at once
  int32_t* fresh;  // [n] 1 in the first round of a run: its trial points start
                   // their root solves cold, not from the slot's root cache
  unsigned int* active;
  // iterated mode: slot j = k * reps + i of lightcurve k begins with start
  // i; a slot whose run ends takes the lightcurve's next unstarted start (the
  // slots ending in one round in slot order), until reps * runs starts have
  // been taken.  Each start's run and the best-of rule do not depend on
  // which slot runs it.
  int32_t iter, reps, runs;
  uint64_t seed;
  int32_t* run;         // [n] the start the slot runs
  int32_t* ending;      // [n] the slot's run ended in this round's test
  int32_t* next_start;  // [n / reps] the lightcurve's next unstarted start
  int64_t* total;  // [n] steps over the completed runs
  double* bX;      // [NP][n] best result of the completed runs
  double* bF;      // [n]
  double* bFs;
  double* bFb;
  int32_t* bS;     // [n] its start index, -1 before the first
};

__device__ __forceinline__ double clip01(double x) { return fmin(fmax(x, 0.0), 1.0); }
__device__ __forceinline__ double finite_or_inf(double x) { return isnan(x) ? INFINITY : x; }

__device__ __forceinline__ double& vtx(const NmWork& w, int v, int g, int lc) {
  return w.V[((int64_t)v * NP + g) * w.n + lc];
}
__device__ __forceinline__ void put_trial(const NmWork& w, int lc, int slot, const double* x) {
  for (int g = 0; g < NP; ++g) w.T[(int64_t)g * w.n * NS + (int64_t)lc * NS + slot] = x[g];
}
__device__ __forceinline__ void get_trial(const NmWork& w, int lc, int slot, double* x) {
  for (int g = 0; g < NP; ++g) x[g] = w.T[(int64_t)g * w.n * NS + (int64_t)lc * NS + slot];
}

// The initial simplex around x (clipped) and a fresh run.
__device__ void begin_run(const NmWork& w, int lc, const double* x0) {
  double x[NP];
  for (int g = 0; g < NP; ++g) x[g] = clip01(x0[g]);
  for (int v = 0; v < NV; ++v)
    for (int g = 0; g < NP; ++g) {
      double y = x[g];
      if (v == g + 1) y = (y != 0.0) ? (1.0 + 0.05) * y : 0.00025;
      if (y > 1.0) y = 2.0 * 1.0 - y;
      vtx(w, v, g, lc) = clip01(y);
    }
  w.phase[lc] = PH_INIT1;
  w.steps[lc] = 0;
  w.fresh[lc] = 1;
}

// Start s of the lightcurve of slot lc (iterated mode): coordinate g = the
// open-interval map of the Philox word of key (seed, k), counter
// (0, NM_PURPOSE_START, s, g / 4), word g % 4.
__device__ void start_point(const NmWork& w, int lc, int s, double* x) {
  const int k = lc / w.reps;
  const Stream rs = {w.seed, (uint64_t)k, 0};
  for (int g = 0; g < NP; ++g) x[g] = u01(rs.draw(NM_PURPOSE_START, (uint64_t)s, (uint64_t)g));
}

// A run of slot lc ends (iterated mode): its best vertex becomes the slot's
// best when strictly lower (a slot takes its starts in increasing order, so
// earlier starts win ties within a slot).
__device__ void end_run(const NmWork& w, int lc) {
  const double f = w.F[lc];
  if (w.bS[lc] < 0 || f < w.bF[lc]) {
    for (int g = 0; g < NP; ++g) w.bX[(int64_t)g * w.n + lc] = vtx(w, 0, g, lc);
    w.bF[lc] = f;
    w.bFs[lc] = w.FsV[lc];
    w.bFb[lc] = w.FbV[lc];
    w.bS[lc] = w.run[lc];
  }
  w.total[lc] += w.steps[lc];
}

__global__ void nm_start_kernel(NmWork w, const double* x0) {
  const int lc = blockIdx.x * blockDim.x + threadIdx.x;
  if (lc >= w.n) return;
  double x[NP];
  if (w.iter) {
    const int i = lc % w.reps;
    w.run[lc] = i;
    w.ending[lc] = 0;
    if (i == 0) w.next_start[lc / w.reps] = w.reps;
    w.total[lc] = 0;
    w.bS[lc] = -1;
    w.bF[lc] = INFINITY;
    start_point(w, lc, i, x);
  } else {
    for (int g = 0; g < NP; ++g) x[g] = x0[(int64_t)g * w.n + lc];
  }
  begin_run(w, lc, x);
}

// NaN marks an empty root cache entry (the lane starts cold).
__global__ void nm_nan_fill_kernel(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = NAN;
}

// The stopping test of this round (and the round's active count reset: the
// update kernel that counts runs after this one on the same stream).  In
// iterated mode a run that stops is recorded and its slot marked as ending;
// the next kernel gives it its next start.
__global__ void nm_test_kernel(NmWork w, double tol_x, double tol_f, int32_t max_iter) {
  const int lc = blockIdx.x * blockDim.x + threadIdx.x;
  if (lc == 0) *w.active = 0u;
  if (lc >= w.n) return;
  if (w.iter) w.ending[lc] = 0;
  if (w.phase[lc] != PH_STEP) return;
  double dx = 0.0, df = 0.0;
  bool undefined = false;  // inf - inf: never converged
  const double f0 = w.F[lc];
  for (int v = 1; v < NV; ++v) {
    const double d = fabs(f0 - w.F[(int64_t)v * w.n + lc]);
    undefined |= isnan(d);
    df = fmax(df, d);
    for (int g = 0; g < NP; ++g) dx = fmax(dx, fabs(vtx(w, v, g, lc) - vtx(w, 0, g, lc)));
  }
  if ((!undefined && dx <= tol_x && df <= tol_f) || w.steps[lc] >= max_iter) {
    w.phase[lc] = PH_DONE;
    if (w.iter) {
      end_run(w, lc);
      w.ending[lc] = 1;
    }
  }
}

// The centroid of the best six vertices and the worst vertex.
__device__ __forceinline__ void centroid(const NmWork& w, int lc, double* xbar, double* xw) {
  for (int g = 0; g < NP; ++g) {
    double sum = vtx(w, 0, g, lc);
    for (int v = 1; v < NV - 1; ++v) sum += vtx(w, v, g, lc);
    xbar[g] = sum / NP;
    xw[g] = vtx(w, NV - 1, g, lc);
  }
}

// Point k of a step: 0 reflection, 1 expansion, 2 outside and 3 inside
// contraction (coefficients 1, 2 and 1/2), clipped to the domain.
__device__ __forceinline__ void step_point(const double* xbar, const double* xw, int k,
                                           double* x) {
  const double rho = 1.0, chi = 2.0, psi = 0.5;
  for (int g = 0; g < NP; ++g) {
    double y;
    if (k == 0)
      y = (1 + rho) * xbar[g] - rho * xw[g];
    else if (k == 1)
      y = (1 + rho * chi) * xbar[g] - rho * chi * xw[g];
    else if (k == 2)
      y = (1 + psi * rho) * xbar[g] - psi * rho * xw[g];
    else
      y = (1 - psi) * xbar[g] + psi * xw[g];
    x[g] = clip01(y);
  }
}

// Trial points of this round, and which slots it evaluates.  In iterated
// mode an ending slot first takes its lightcurve's next unstarted start: the
// slots of a lightcurve that end in this round take them in slot order (the
// update kernel then advances the lightcurve's counter), and a slot with
// none left stays done.
__global__ void nm_propose_kernel(NmWork w) {
  const int lc = blockIdx.x * blockDim.x + threadIdx.x;
  if (lc >= w.n) return;
  int ph = w.phase[lc];
  double x[NP];
  if (w.iter && w.ending[lc]) {
    const int k = lc / w.reps, i = lc - k * w.reps;
    int rank = 0;
    for (int j = 0; j < i; ++j) rank += w.ending[k * w.reps + j];
    const int64_t s = (int64_t)w.next_start[k] + rank;
    if (s < (int64_t)w.reps * w.runs) {
      w.run[lc] = (int32_t)s;
      start_point(w, lc, (int)s, x);
      begin_run(w, lc, x);
      ph = PH_INIT1;
    }
  }
  int need = 0;  // bit s: slot s is evaluated
  switch (ph) {
    case PH_INIT1:
    case PH_SHRINK1:
      for (int s = 0; s < NS; ++s) {
        const int v = (ph == PH_INIT1) ? s : 1 + s;
        for (int g = 0; g < NP; ++g) x[g] = vtx(w, v, g, lc);
        put_trial(w, lc, s, x);
      }
      need = 0xF;
      break;
    case PH_INIT2:
    case PH_SHRINK2:
      // vertices 4..6 (initial) or 5..6 (shrink)
      for (int s = 0; s < NS; ++s) {
        const int v = (ph == PH_INIT2) ? (s < 3 ? 4 + s : 6) : (s < 2 ? 5 + s : 6);
        for (int g = 0; g < NP; ++g) x[g] = vtx(w, v, g, lc);
        put_trial(w, lc, s, x);
      }
      need = (ph == PH_INIT2) ? 0x7 : 0x3;
      break;
    case PH_STEP: {
      double xbar[NP], xw[NP];
      centroid(w, lc, xbar, xw);
      const int kn = w.spec ? NS : 1;
      for (int k = 0; k < kn; ++k) {
        step_point(xbar, xw, k, x);
        put_trial(w, lc, k, x);
      }
      need = w.spec ? 0xF : 0x1;
      break;
    }
    case PH_WAIT_E:
    case PH_WAIT_OC:
    case PH_WAIT_IC: {
      // the step's second point (the reflection stays in slot 0)
      double xbar[NP], xw[NP];
      centroid(w, lc, xbar, xw);
      const int k = 1 + (ph - PH_WAIT_E);
      step_point(xbar, xw, k, x);
      put_trial(w, lc, k, x);
      need = 1 << k;
      break;
    }
    default:  // done: the best vertex, so that the slots stay valid inputs
      for (int g = 0; g < NP; ++g) x[g] = vtx(w, 0, g, lc);
      for (int s = 0; s < NS; ++s) put_trial(w, lc, s, x);
      break;
  }
  for (int s = 0; s < NS; ++s) w.skipT[(int64_t)lc * NS + s] = ((need >> s) & 1) ? 0 : 1;
}

// Work order of a round: the entries of the fixed order (longest lightcurve
// first) whose trial slot is needed, in that order, then the others, in
// that order.  Every wave takes PACK_ROWS rows of 64 consecutive entries
// (coalesced loads, held in registers); a ballot per row gives each lane the
// needed entries before it.  Up to COMPACT_ONE entries one block of 16 waves
// does it; beyond, two launches of 4-wave blocks: the needed entries per
// block of COMPACT_CHUNK, then each block places its entries after those of
// the blocks before it.
constexpr int PACK_ROWS = 16;  // 1024 entries per wave

__device__ __forceinline__ int pack_load(const int32_t* __restrict__ skip,
                                         const int32_t* __restrict__ ord0, int64_t n,
                                         int64_t wbase, int32_t* e, bool* need) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < PACK_ROWS; ++i) {
    const int64_t j = wbase + i * 64 + lane;
    e[i] = (j < n) ? ord0[j] : -1;
  }
  int c = 0;
#pragma unroll
  for (int i = 0; i < PACK_ROWS; ++i) {
    need[i] = e[i] >= 0 && !skip[e[i]];
    c += __popcll(__ballot(need[i]));
  }
  return c;  // the wave's needed entries (the same in every lane)
}

// The wave's entries to their places: k needed entries precede the wave's
// first entry, total in all.
__device__ __forceinline__ void pack_store(int32_t* __restrict__ ord, int64_t wbase, int64_t k,
                                           int64_t total, const int32_t* e, const bool* need) {
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int i = 0; i < PACK_ROWS; ++i) {
    const unsigned long long m = __ballot(need[i]);
    const int64_t kb = k + __popcll(m & below);  // needed entries before entry j
    const int64_t j = wbase + i * 64 + lane;
    if (e[i] >= 0) {
      if (need[i])
        ord[kb] = e[i];
      else
        ord[total + (j - kb)] = e[i];  // j - kb: the skipped entries before j
    }
    k += __popcll(m);
  }
}

// Needed entries before this wave within the block (exclusive), and the
// block's total, from every wave's count.
template <int NW>
__device__ __forceinline__ int wave_prefix(int c, int32_t* sh, int& block_total) {
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[wv] = c;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int v = 0; v < NW; ++v) {
    before += (v < wv) ? sh[v] : 0;
    all += sh[v];
  }
  block_total = all;
  return before;
}

__global__ __launch_bounds__(1024) void nm_pack_kernel(const int32_t* __restrict__ skip,
                                                       const int32_t* __restrict__ ord0,
                                                       int64_t n, int32_t* __restrict__ ord) {
  __shared__ int32_t sh[16];
  const int64_t wbase = (int64_t)(threadIdx.x >> 6) * (PACK_ROWS * 64);
  int32_t e[PACK_ROWS];
  bool need[PACK_ROWS];
  const int c = pack_load(skip, ord0, n, wbase, e, need);
  int total = 0;
  const int before = wave_prefix<16>(c, sh, total);
  pack_store(ord, wbase, before, total, e, need);
}

__global__ __launch_bounds__(256) void nm_count_kernel(const int32_t* __restrict__ skip,
                                                       const int32_t* __restrict__ ord0,
                                                       int64_t n, int32_t* counts) {
  __shared__ int32_t sh[4];
  const int64_t wbase =
      (int64_t)blockIdx.x * COMPACT_CHUNK + (int64_t)(threadIdx.x >> 6) * (PACK_ROWS * 64);
  int32_t e[PACK_ROWS];
  bool need[PACK_ROWS];
  const int c = pack_load(skip, ord0, n, wbase, e, need);
  int total = 0;
  wave_prefix<4>(c, sh, total);
  if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void nm_place_kernel(const int32_t* __restrict__ skip,
                                                       const int32_t* __restrict__ ord0,
                                                       int64_t n, const int32_t* counts,
                                                       int32_t* __restrict__ ord) {
  __shared__ int64_t red[2][256];
  __shared__ int32_t sh[4];
  const int nb = gridDim.x, b = blockIdx.x, t = threadIdx.x;
  const int64_t wbase = (int64_t)b * COMPACT_CHUNK + (int64_t)(t >> 6) * (PACK_ROWS * 64);
  int32_t e[PACK_ROWS];
  bool need[PACK_ROWS];
  const int c = pack_load(skip, ord0, n, wbase, e, need);
  // needed entries before this block, and in all
  int64_t before = 0, total = 0;
  for (int i = t; i < nb; i += 256) {
    total += counts[i];
    if (i < b) before += counts[i];
  }
  red[0][t] = before;
  red[1][t] = total;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      red[0][t] += red[0][t + o];
      red[1][t] += red[1][t + o];
    }
    __syncthreads();
  }
  before = red[0][0];
  total = red[1][0];
  int block_total = 0;
  const int in_block = wave_prefix<4>(c, sh, block_total);
  pack_store(ord, wbase, before + in_block, total, e, need);
}

struct Vertex {
  double x[NP];
  double f, fs, fb;
};

// The simplex lives in registers: every index into Vertex arrays below is a
// compile-time constant after unrolling (a runtime index would put the
// array in scratch memory).
__device__ __forceinline__ void load_simplex(const NmWork& w, int lc, Vertex* s) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
#pragma unroll
    for (int g = 0; g < NP; ++g) s[v].x[g] = vtx(w, v, g, lc);
    s[v].f = w.F[(int64_t)v * w.n + lc];
    s[v].fs = w.FsV[(int64_t)v * w.n + lc];
    s[v].fb = w.FbV[(int64_t)v * w.n + lc];
  }
}

// Stores vertex v at place rank[v] (a memory index, so it may be a runtime
// value).
__device__ __forceinline__ void store_simplex(const NmWork& w, int lc, const Vertex* s,
                                              const int* rank) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int r = rank[v];
#pragma unroll
    for (int g = 0; g < NP; ++g) vtx(w, r, g, lc) = s[v].x[g];
    w.F[(int64_t)r * w.n + lc] = s[v].f;
    w.FsV[(int64_t)r * w.n + lc] = s[v].fs;
    w.FbV[(int64_t)r * w.n + lc] = s[v].fb;
  }
}

// Stable sort by f (equal values keep their order): the place of vertex i
// is the number of vertices with a lower f, or an equal f and a lower index
// -- the permutation of a stable insertion sort.  The vertices stay where
// they are; store_simplex writes each to its place.
__device__ __forceinline__ void rank_simplex(const Vertex* s, int* rank) {
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    int r = 0;
#pragma unroll
    for (int j = 0; j < NV; ++j) r += (s[j].f < s[i].f || (s[j].f == s[i].f && j < i)) ? 1 : 0;
    rank[i] = r;
  }
}

__device__ __forceinline__ void take_trial(const NmWork& w, int lc, int slot, Vertex& v) {
  const int64_t i = (int64_t)lc * NS + slot;
  get_trial(w, lc, slot, v.x);
  v.f = finite_or_inf(w.cT[i]);
  v.fs = w.fsT[i];
  v.fb = w.fbT[i];
}

// A point that coincides with one evaluated before gets that point's value.
// Clipping to the domain can map a trial point onto a vertex or onto another
// trial point; evaluated again, its chi^2 would differ at the rounding level
// (each evaluation starts its root solves from its own cached roots), and an
// exact tie, which a function decides the same way every time, could go
// either way.
__device__ __forceinline__ bool same_point(const double* a, const double* b) {
  bool eq = true;
#pragma unroll
  for (int g = 0; g < NP; ++g) eq = eq & (a[g] == b[g]);
  return eq;
}

// Vertices LO..HI-1 (just evaluated) take the value of the first earlier
// vertex at the same point.
template <int LO, int HI>
__device__ __forceinline__ void share_values(Vertex* s) {
#pragma unroll
  for (int v = LO; v < HI; ++v) {
    bool found = false;
#pragma unroll
    for (int u = 0; u < v; ++u) {
      const bool m = !found && same_point(s[v].x, s[u].x);
      if (m) {
        s[v].f = s[u].f;
        s[v].fs = s[u].fs;
        s[v].fb = s[u].fb;
      }
      found = found | m;
    }
  }
}

__device__ __forceinline__ void copy_value(Vertex& d, const Vertex& src) {
  d.f = src.f;
  d.fs = src.fs;
  d.fb = src.fb;
}

// A trial point at a vertex takes the first such vertex's value.
__device__ __forceinline__ bool at_vertex(Vertex& t, const Vertex* s) {
  bool found = false;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const bool m = !found && same_point(t.x, s[v].x);
    if (m) copy_value(t, s[v]);
    found = found | m;
  }
  return found;
}

// Shrink towards the best vertex (coefficient 1/2); the moved vertices are
// evaluated in the next two rounds.
__device__ __forceinline__ void shrink(Vertex* s) {
  const double sigma = 0.5;
#pragma unroll
  for (int v = 1; v < NV; ++v)
#pragma unroll
    for (int g = 0; g < NP; ++g) s[v].x[g] = clip01(s[0].x[g] + sigma * (s[v].x[g] - s[0].x[g]));
}

__global__ __launch_bounds__(256) void nm_update_kernel(NmWork w) {
  const int lc = blockIdx.x * blockDim.x + threadIdx.x;
  if (lc >= w.n) return;
  if (w.iter && lc % w.reps == 0) {  // starts taken by this round's ending slots
    const int k = lc / w.reps;
    int taken = 0;
    for (int j = 0; j < w.reps; ++j) taken += w.ending[k * w.reps + j];
    // at most reps * runs (< 2^31): the counter never passes the last start
    const int64_t nx = (int64_t)w.next_start[k] + taken, all = (int64_t)w.reps * w.runs;
    w.next_start[k] = (int32_t)(nx < all ? nx : all);
  }
  w.fresh[lc] = 0;
  const int ph = w.phase[lc];
  if (ph == PH_DONE) return;
  Vertex s[NV];
  load_simplex(w, lc, s);
  int rank[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) rank[v] = v;
  int next = ph;
  switch (ph) {
    case PH_INIT1:
#pragma unroll
      for (int k = 0; k < NS; ++k) take_trial(w, lc, k, s[k]);
      share_values<1, NS>(s);
      next = PH_INIT2;
      break;
    case PH_INIT2:
#pragma unroll
      for (int k = 0; k < 3; ++k) take_trial(w, lc, k, s[4 + k]);
      share_values<4, NV>(s);
      rank_simplex(s, rank);
      next = PH_STEP;
      break;
    case PH_SHRINK1:
#pragma unroll
      for (int k = 0; k < NS; ++k) take_trial(w, lc, k, s[1 + k]);
      share_values<1, 1 + NS>(s);
      next = PH_SHRINK2;
      break;
    case PH_SHRINK2:
#pragma unroll
      for (int k = 0; k < 2; ++k) take_trial(w, lc, k, s[5 + k]);
      share_values<5, NV>(s);
      rank_simplex(s, rank);
      next = PH_STEP;
      break;
    case PH_STEP:
      if (w.spec) {
        // the decision needs only the four values (each trial point at a
        // vertex or at an earlier trial point takes that point's value);
        // then the accepted point
        Vertex t[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          take_trial(w, lc, k, t[k]);
          bool found = false;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const bool m = !found && same_point(t[k].x, s[v].x);
            if (m) copy_value(t[k], s[v]);
            found = found | m;
          }
#pragma unroll
          for (int j = 0; j < k; ++j) {
            const bool m = !found && same_point(t[k].x, t[j].x);
            if (m) copy_value(t[k], t[j]);
            found = found | m;
          }
        }
        const double fr = t[0].f;
        int accept = -1;  // 0 r, 1 e, 2 oc, 3 ic; -1 shrink
        if (fr < s[0].f) accept = (t[1].f < fr) ? 1 : 0;
        else if (fr < s[NV - 2].f) accept = 0;
        else if (fr < s[NV - 1].f) accept = (t[2].f <= fr) ? 2 : -1;
        else accept = (t[3].f < s[NV - 1].f) ? 3 : -1;
        if (accept >= 0) {
#pragma unroll
          for (int k = 0; k < NS; ++k)
            if (accept == k) s[NV - 1] = t[k];
          rank_simplex(s, rank);
          next = PH_STEP;
        } else {
          shrink(s);
          next = PH_SHRINK1;
        }
        w.steps[lc] += 1;
      } else {
        // the reflection alone (at a vertex: that vertex's value); it
        // decides the step or which point the step needs next
        Vertex r;
        take_trial(w, lc, 0, r);
        at_vertex(r, s);
        if (r.f < s[0].f) {
          next = PH_WAIT_E;
        } else if (r.f < s[NV - 2].f) {
          s[NV - 1] = r;
          rank_simplex(s, rank);
          w.steps[lc] += 1;
          next = PH_STEP;
        } else {
          next = (r.f < s[NV - 1].f) ? PH_WAIT_OC : PH_WAIT_IC;
        }
        if (next != PH_STEP) {
          w.rF[lc] = r.f;
          w.rF[(int64_t)w.n + lc] = r.fs;
          w.rF[2 * (int64_t)w.n + lc] = r.fb;
        }
      }
      break;
    case PH_WAIT_E:
    case PH_WAIT_OC:
    case PH_WAIT_IC: {
      // the second point of a step (at a vertex or at the reflection: that
      // point's value), then the step's outcome as in the four-point form
      Vertex r, t;
      get_trial(w, lc, 0, r.x);
      r.f = w.rF[lc];
      r.fs = w.rF[(int64_t)w.n + lc];
      r.fb = w.rF[2 * (int64_t)w.n + lc];
      const int k = 1 + (ph - PH_WAIT_E);
      take_trial(w, lc, k, t);
      if (!at_vertex(t, s) && same_point(t.x, r.x)) copy_value(t, r);
      bool take_t, take_r = false;
      if (ph == PH_WAIT_E) {
        take_t = t.f < r.f;
        take_r = !take_t;
      } else if (ph == PH_WAIT_OC) {
        take_t = t.f <= r.f;
      } else {
        take_t = t.f < s[NV - 1].f;
      }
      if (take_t || take_r) {
        s[NV - 1] = take_t ? t : r;
        rank_simplex(s, rank);
        next = PH_STEP;
      } else {
        shrink(s);
        next = PH_SHRINK1;
      }
      w.steps[lc] += 1;
      break;
    }
  }
  store_simplex(w, lc, s, rank);
  w.phase[lc] = next;
  atomicAdd(w.active, 1u);
}

__global__ void nm_finish_kernel(NmWork w, double* x, double* chi2, double* Fs, double* Fb,
                                 int32_t* n_iter) {
  const int lc = blockIdx.x * blockDim.x + threadIdx.x;
  if (lc >= w.n) return;
  for (int g = 0; g < NP; ++g) x[(int64_t)g * w.n + lc] = vtx(w, 0, g, lc);
  if (chi2) chi2[lc] = w.F[lc];
  if (Fs) Fs[lc] = w.FsV[lc];
  if (Fb) Fb[lc] = w.FbV[lc];
  if (n_iter) n_iter[lc] = w.steps[lc];
}

// Iterated mode: per lightcurve, the best over its slots (lowest chi^2, then
// lowest start index) and the steps of all its runs.
__global__ void nm_best_kernel(NmWork w, double* x, double* chi2, double* Fs, double* Fb,
                               int64_t* n_iter) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int n_lc = w.n / w.reps;
  if (k >= n_lc) return;
  int b = k * w.reps;
  int64_t total = w.total[b];
  for (int i = 1; i < w.reps; ++i) {
    const int j = k * w.reps + i;
    total += w.total[j];
    if (w.bF[j] < w.bF[b] || (w.bF[j] == w.bF[b] && w.bS[j] < w.bS[b])) b = j;
  }
  for (int g = 0; g < NP; ++g) x[(int64_t)g * n_lc + k] = w.bX[(int64_t)g * w.n + b];
  if (chi2) chi2[k] = w.bF[b];
  if (Fs) Fs[k] = w.bFs[b];
  if (Fb) Fb[k] = w.bFb[b];
  if (n_iter) n_iter[k] = total;
}

}  // namespace

int nm_check(const nm_config* cfg, const char* who) {
  if (!cfg) return set_error(SBLM_EINVAL, "%s: null config", who);
  if (!(cfg->tol_x >= 0.0) || !(cfg->tol_f >= 0.0))
    return set_error(SBLM_EINVAL, "%s: negative tolerance", who);
  if (cfg->max_iter < 0 || cfg->max_iter > 1000000)
    return set_error(SBLM_EINVAL, "%s: max_iter = %d outside [0, 10^6]", who, cfg->max_iter);
  if (cfg->mode != SBLM_FP64 && cfg->mode != SBLM_MIXED)
    return set_error(SBLM_EINVAL, "%s: unknown mode %d", who, cfg->mode);
  return SBLM_OK;
}

// The arrays of NmWork for n simplices, carved one after another (each
// aligned to 256 bytes) from one block at `base`; returns the block's size
// (with base == nullptr only the size).
static size_t nm_carve(NmWork& w, char* base, size_t n, bool iter) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  w.V = (double*)take(n * NV * NP * 8);
  w.F = (double*)take(n * NV * 8);
  w.FsV = (double*)take(n * NV * 8);
  w.FbV = (double*)take(n * NV * 8);
  w.T = (double*)take(n * NS * NP * 8);
  w.cT = (double*)take(n * NS * 8);
  w.fsT = (double*)take(n * NS * 8);
  w.fbT = (double*)take(n * NS * 8);
  w.rF = (double*)take(n * 3 * 8);
  w.phase = (int32_t*)take(n * 4);
  w.steps = (int32_t*)take(n * 4);
  w.skipT = (int32_t*)take(n * NS * 4);
  w.fresh = (int32_t*)take(n * 4);
  w.active = (unsigned int*)take(4);
  if (iter) {
    w.run = (int32_t*)take(n * 4);
    w.total = (int64_t*)take(n * 8);
    w.bX = (double*)take(n * NP * 8);
    w.bF = (double*)take(n * 8);
    w.bFs = (double*)take(n * 8);
    w.bFb = (double*)take(n * 8);
    w.bS = (int32_t*)take(n * 4);
    w.ending = (int32_t*)take(n * 4);
    w.next_start = (int32_t*)take(n * 4);  // n / reps used
  }
  return off;
}

size_t nm_work_bytes(int64_t n_simplices) {
  NmWork w;
  return nm_carve(w, nullptr, (size_t)n_simplices, false);
}

int nm_run(const sblm_lcs& lcs, int32_t reps, const double* lo, const double* span,
           const double* x0, const nm_config& cfg, double* x, double* chi2, double* Fs,
           double* Fb, int32_t* n_iter, sblm_stats* stats, hipStream_t st,
           const NmIterated* iter, void* workspace) {
  // simplex j = k * reps + i works on lightcurve k: its trial points are
  // individuals j * NS + slot, that is NS * reps individuals per lightcurve
  const int n = lcs.n_lc * reps;
  NmWork w;
  memset(&w, 0, sizeof(w));
  w.n = n;
  w.reps = reps;
  w.iter = iter != nullptr;
  w.runs = iter ? iter->runs : 1;
  w.seed = iter ? iter->seed : 0;
  const size_t nn = (size_t)n;
  // the workspace: the caller's (nm_refine_noalloc), else one allocation
  // freed before returning
  void* block = workspace;
  bool ok = true;
  if (!block) ok = hipMalloc(&block, nm_carve(w, nullptr, nn, w.iter)) == hipSuccess;
  if (ok)
    nm_carve(w, (char*)block, nn, w.iter);
  else
    block = nullptr;
  int rc = SBLM_OK;
  if (!ok) {
    (void)hipGetLastError();
    rc = set_error(SBLM_ENOMEM, "nm_refine: device allocation");
  }
  FitArgs a;
  memset(&a, 0, sizeof(a));
  double* root_cache = nullptr;
  a.theta = w.T;
  a.n_ind = (int64_t)n * NS;
  a.encoded = 1;
  for (int g = 0; g < NP; ++g) {
    a.lo[g] = lo[g];
    a.span[g] = span[g];
  }
  a.off = lcs.off;
  a.pop = NS * reps;
  a.t = lcs.t;
  a.y = lcs.y;
  a.w = lcs.w;
  a.chi2 = w.cT;
  a.Fs = w.fsT;
  a.Fb = w.fbT;
  a.stats = stats;
  a.skip = w.skipT;  // trial slots this round does not need
  a.skip_per = 1;
  a.cold_per = NS;
  // Lanes per trial point.  While most simplices are still running a
  // round is bound by its work, and 64 lanes (long chains of warm-started
  // epochs per lane, one wave per trial point) do it fastest; later rounds
  // hold few unfinished simplices and are bound by the chain of epochs of
  // their longest lightcurve, which 128 or 256 lanes (several waves per
  // trial point) shorten.  So the lanes follow the number of simplices that
  // ran in the last round (read every 16 rounds): the fewest of 64, 128, 256
  // that give the round's trial points 2^19 lanes, else 256.  Every width
  // keeps the roots of each lane's first epoch (80 B per lane and trial
  // slot) and starts there in its next round (the simplex moves little
  // between rounds; a cache of a width not used for a while is only a
  // poorer start).  The choice depends on the simplices alone, so results
  // are deterministic.  Without room for the three caches (1 GiB) a fixed
  // width: 256 lanes, else 128, else 64 without a cache; the
  // allocation-free entry point and SBLM_NM_LANES fix it too (a cache only
  // above 64 lanes).
  const int64_t n_trial = (int64_t)n * NS;
  const int64_t cache_max = (int64_t)1 << 30;
  int fixed_g = 0;
  if (workspace) {
    fixed_g = 64;
  } else if (const char* env = getenv("SBLM_NM_LANES")) {
    const int g = atoi(env);
    if (g == 64 || g == 128 || g == 256) fixed_g = g;
  }
  if (!fixed_g && n_trial * (64 + 128 + 256) * 80 > cache_max)
    fixed_g = n_trial * 256 * 80 <= cache_max ? 256 : n_trial * 128 * 80 <= cache_max ? 128 : 64;
  // The offsets on the host, for the work order below.
  const int nl = lcs.n_lc;
  int64_t* off_h = nullptr;
  if (rc == SBLM_OK && !workspace) {
    off_h = (int64_t*)malloc((size_t)(nl + 1) * sizeof(int64_t));
    if (!off_h) {
      rc = set_error(SBLM_ENOMEM, "nm_refine: host allocation");
    } else {
      rc = check_hip(hipMemcpyAsync(off_h, lcs.off, (size_t)(nl + 1) * sizeof(int64_t),
                                    hipMemcpyDeviceToHost, st),
                     "nm_refine: offsets");
      if (rc == SBLM_OK) rc = check_hip(hipStreamSynchronize(st), "nm_refine: offsets");
    }
  }
  // cache of width 64 << i at root_cache + cache_off[i] (-1: none)
  int64_t cache_off[3] = {-1, -1, -1}, n_cache = 0;
  for (int i = 0; i < 3; ++i) {
    const int g = 64 << i;
    if (fixed_g ? (g == fixed_g && g > 64) : true) {
      cache_off[i] = n_cache;
      n_cache += n_trial * g * 10;
    }
  }
  if (rc == SBLM_OK && n_cache > 0) {
    if (hipMalloc(&root_cache, (size_t)n_cache * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      root_cache = nullptr;
      rc = set_error(SBLM_ENOMEM, "nm_refine: device allocation");
    } else {
      hipLaunchKernelGGL(nm_nan_fill_kernel, dim3((unsigned)((n_cache + 255) / 256)), dim3(256),
                         0, st, root_cache, n_cache);
      rc = check_hip(hipGetLastError(), "nm_refine: cache");
    }
  }
  // Work order of the trial points, longest lightcurve first (stable), a
  // simplex's four trial points together: one round launches every trial
  // point at once, over lightcurves of very different lengths, and a long
  // one dispatched last would hold the round up.  Each round packs the
  // slots it needs to the front of this order (`ord`), so that the blocks
  // of the launch hold needed trial points only and the others end at once.
  // (Not with a caller's workspace: the order changes no result, only the
  // balance.)
  int32_t* order = nullptr;  // [n_trial] fixed order, then [n_trial] packed, then counts
  int32_t* ord = nullptr;
  int32_t* counts = nullptr;
  const int64_t n_blk = (n_trial + COMPACT_CHUNK - 1) / COMPACT_CHUNK;
  if (rc == SBLM_OK && !workspace) {
    int32_t* lc_h = (int32_t*)malloc((size_t)nl * sizeof(int32_t));
    int32_t* ord_h = (int32_t*)malloc((size_t)n_trial * sizeof(int32_t));
    if (!lc_h || !ord_h) rc = set_error(SBLM_ENOMEM, "nm_refine: host allocation");
    if (rc == SBLM_OK) {
      for (int k = 0; k < nl; ++k) lc_h[k] = k;
      std::stable_sort(lc_h, lc_h + nl, [&](int32_t i, int32_t j) {
        return off_h[i + 1] - off_h[i] > off_h[j + 1] - off_h[j];
      });
      int64_t o = 0;
      for (int r = 0; r < nl; ++r)
        for (int64_t j = (int64_t)lc_h[r] * reps; j < (int64_t)(lc_h[r] + 1) * reps; ++j)
          for (int slot = 0; slot < NS; ++slot) ord_h[o++] = (int32_t)(j * NS + slot);
      if (hipMalloc(&order, (size_t)(2 * n_trial + n_blk) * sizeof(int32_t)) != hipSuccess) {
        (void)hipGetLastError();
        order = nullptr;
        rc = set_error(SBLM_ENOMEM, "nm_refine: device allocation");
      } else {
        ord = order + n_trial;
        counts = ord + n_trial;
        rc = check_hip(hipMemcpyAsync(order, ord_h, (size_t)n_trial * sizeof(int32_t),
                                      hipMemcpyHostToDevice, st),
                       "nm_refine: order");
        if (rc == SBLM_OK) rc = check_hip(hipStreamSynchronize(st), "nm_refine: order");
      }
    }
    free(lc_h);
    free(ord_h);
  }
  free(off_h);
  a.order = ord;
  auto set_lanes = [&](int g) {
    a.lanes_per_ind = g;
    const int i = g == 64 ? 0 : g == 128 ? 1 : 2;
    a.root_cache = (root_cache && cache_off[i] >= 0) ? root_cache + cache_off[i] : nullptr;
  };
  set_lanes(fixed_g ? fixed_g : 64);
  a.cold = w.fresh;
  const dim3 grid((n + 255) / 256), blk(256);
  if (rc == SBLM_OK) {
    hipLaunchKernelGGL(nm_start_kernel, grid, blk, 0, st, w, x0);
    rc = check_hip(hipGetLastError(), "nm_refine: start");
  }
  // The form of a step, per 16 rounds: one point at a time while more than
  // spec_max simplices ran in the last block of rounds (bound by work), all
  // four at once below (bound by latency).  SBLM_NM_SPEC_MAX overrides the
  // threshold (0: always one at a time; large: always all four); results do
  // not depend on it.
  int64_t spec_max = 256;
  if (const char* env = getenv("SBLM_NM_SPEC_MAX")) spec_max = atoll(env);
  // rounds per run: 2 for the initial simplex, at most 2 per step, 2 more per
  // shrink (one slot may run every start of its lightcurve)
  const int64_t max_rounds =
      (4 + 4 * (int64_t)cfg.max_iter) * (iter ? (int64_t)w.reps * w.runs : 1);
  const int chunk = 16;
  unsigned int active = (unsigned int)n;  // simplices that ran in the last round
  for (int64_t r = 0; rc == SBLM_OK && r < max_rounds; r += chunk) {
    w.spec = (int64_t)active <= spec_max ? 1 : 0;
    if (!fixed_g) {
      // trial points of a round: four per simplex, or about one
      const int64_t want = (int64_t)1 << 19;
      const int64_t tp = (int64_t)active * (w.spec ? NS : 1);
      set_lanes(tp * 64 >= want ? 64 : tp * 128 >= want ? 128 : 256);
    }
    for (int k = 0; k < chunk && rc == SBLM_OK; ++k) {
      hipLaunchKernelGGL(nm_test_kernel, grid, blk, 0, st, w, cfg.tol_x, cfg.tol_f,
                         cfg.max_iter);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess) {
        hipLaunchKernelGGL(nm_propose_kernel, grid, blk, 0, st, w);
        e = hipGetLastError();
      }
      if (e == hipSuccess && ord && n_trial <= COMPACT_ONE) {
        hipLaunchKernelGGL(nm_pack_kernel, dim3(1), dim3(1024), 0, st, w.skipT, order, n_trial,
                           ord);
        e = hipGetLastError();
      } else if (e == hipSuccess && ord) {
        hipLaunchKernelGGL(nm_count_kernel, dim3((unsigned)n_blk), dim3(256), 0, st, w.skipT,
                           order, n_trial, counts);
        e = hipGetLastError();
        if (e == hipSuccess) {
          hipLaunchKernelGGL(nm_place_kernel, dim3((unsigned)n_blk), dim3(256), 0, st, w.skipT,
                             order, n_trial, counts, ord);
          e = hipGetLastError();
        }
      }
      if (e == hipSuccess) e = launch_fitness(a, cfg.mode, true, st, 4);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(nm_update_kernel, grid, blk, 0, st, w);
        e = hipGetLastError();
      }
      rc = check_hip(e, "nm_refine: round");
    }
    if (rc == SBLM_OK)
      rc = check_hip(hipMemcpyAsync(&active, w.active, 4, hipMemcpyDeviceToHost, st),
                     "nm_refine: copy");
    if (rc == SBLM_OK) rc = check_hip(hipStreamSynchronize(st), "nm_refine: synchronise");
    if (active == 0) break;
  }
  if (rc == SBLM_OK && !iter) {
    hipLaunchKernelGGL(nm_finish_kernel, grid, blk, 0, st, w, x, chi2, Fs, Fb, n_iter);
    rc = check_hip(hipGetLastError(), "nm_refine: finish");
  }
  if (rc == SBLM_OK && iter) {
    hipLaunchKernelGGL(nm_best_kernel, dim3((lcs.n_lc + 255) / 256), blk, 0, st, w, iter->x,
                       iter->chi2, iter->Fs, iter->Fb, iter->n_iter);
    rc = check_hip(hipGetLastError(), "nm_iterated: finish");
  }
  if (hipStreamSynchronize(st) != hipSuccess && rc == SBLM_OK)
    rc = check_hip(hipGetLastError(), "nm_refine: synchronise");
  if (block && !workspace) (void)hipFree(block);
  if (root_cache) (void)hipFree(root_cache);
  if (order) (void)hipFree(order);
  return rc;
}

}  // namespace sblm

using namespace sblm;

extern "C" void nm_default_config(nm_config* cfg) {
  if (!cfg) return;
  cfg->tol_x = 1e-4;
  cfg->tol_f = 1e-4;
  cfg->max_iter = 200 * SBLM_NPAR;
  cfg->mode = SBLM_FP64;
}

extern "C" int nm_refine_multi(const sblm_lcs* lcs, int32_t reps, const double* lo,
                               const double* hi, const double* x0, const nm_config* cfg,
                               double* x, double* chi2, double* Fs, double* Fb,
                               int32_t* n_iter, sblm_stats* stats, void* stream) {
  int rc = nm_check(cfg, "nm_refine");
  if (rc) return rc;
  if (!lcs || !lcs->off || !lcs->t || !lcs->y || !lcs->w)
    return set_error(SBLM_EINVAL, "nm_refine: null lightcurve descriptor or array");
  if (lcs->n_lc < 1) return set_error(SBLM_EINVAL, "nm_refine: n_lc < 1");
  if (reps < 1) return set_error(SBLM_EINVAL, "nm_refine: reps = %d < 1", reps);
  if ((int64_t)lcs->n_lc * reps > (1 << 24))
    return set_error(SBLM_ERANGE, "nm_refine: n_lc * reps beyond 2^24");
  if (!lo || !hi || !x0 || !x) return set_error(SBLM_EINVAL, "nm_refine: null lo, hi, x0 or x");
  double span[SBLM_NPAR];
  for (int g = 0; g < SBLM_NPAR; ++g) {
    if (!(hi[g] > lo[g])) return set_error(SBLM_EINVAL, "nm_refine: hi[%d] <= lo[%d]", g, g);
    span[g] = hi[g] - lo[g];
  }
  return nm_run(*lcs, reps, lo, span, x0, *cfg, x, chi2, Fs, Fb, n_iter, stats,
                (hipStream_t)stream);
}

extern "C" int nm_iterated(const sblm_lcs* lcs, int32_t reps, int32_t runs, uint64_t seed,
                           const double* lo, const double* hi, const nm_config* cfg, double* x,
                           double* chi2, double* Fs, double* Fb, int64_t* n_iter,
                           sblm_stats* stats, void* stream) {
  int rc = nm_check(cfg, "nm_iterated");
  if (rc) return rc;
  if (!lcs || !lcs->off || !lcs->t || !lcs->y || !lcs->w)
    return set_error(SBLM_EINVAL, "nm_iterated: null lightcurve descriptor or array");
  if (lcs->n_lc < 1) return set_error(SBLM_EINVAL, "nm_iterated: n_lc < 1");
  if (reps < 1 || runs < 1)
    return set_error(SBLM_EINVAL, "nm_iterated: reps = %d, runs = %d", reps, runs);
  // the slots of a lightcurve that end in one round rank themselves by a
  // loop over the lightcurve's earlier slots (O(reps) per slot and round)
  if (reps > NM_ITER_REPS_MAX)
    return set_error(SBLM_ERANGE, "nm_iterated: reps = %d beyond %d", reps, NM_ITER_REPS_MAX);
  if ((int64_t)lcs->n_lc * reps > (1 << 24))
    return set_error(SBLM_ERANGE, "nm_iterated: n_lc * reps beyond 2^24");
  if ((int64_t)reps * runs > (1LL << 31) - 1 ||
      (int64_t)runs * (cfg->max_iter + 1) > (1LL << 31) - 1)
    return set_error(SBLM_ERANGE, "nm_iterated: too many starts or steps per slot");
  if (!lo || !hi || !x) return set_error(SBLM_EINVAL, "nm_iterated: null lo, hi or x");
  double span[SBLM_NPAR];
  for (int g = 0; g < SBLM_NPAR; ++g) {
    if (!(hi[g] > lo[g])) return set_error(SBLM_EINVAL, "nm_iterated: hi[%d] <= lo[%d]", g, g);
    span[g] = hi[g] - lo[g];
  }
  NmIterated it = {seed, runs, x, chi2, Fs, Fb, n_iter};
  return nm_run(*lcs, reps, lo, span, nullptr, *cfg, nullptr, nullptr, nullptr, nullptr, nullptr,
                stats, (hipStream_t)stream, &it);
}

extern "C" int nm_refine(const sblm_lcs* lcs, const double* lo, const double* hi,
                         const double* x0, const nm_config* cfg, double* x, double* chi2,
                         double* Fs, double* Fb, int32_t* n_iter, sblm_stats* stats,
                         void* stream) {
  return nm_refine_multi(lcs, 1, lo, hi, x0, cfg, x, chi2, Fs, Fb, n_iter, stats, stream);
}

// ---------------------------------------------------------------------------
// nm_refine_noalloc: nm_refine without any device allocation.  The simplices'
// state lives in `scratch`, a static device array of SBLM_NM_SCRATCH_BYTES
// that every GPU the library runs on holds until the process ends.  In host
// code `scratch` names a host-side stand-in, not device memory: its device
// address is taken once per device with hipGetSymbolAddress (with that
// device current) and only that address is passed to kernels.
#define SBLM_NM_SCRATCH_BYTES (8u << 20)
#define SBLM_MAX_DEVICES 64

static __device__ __align__(256) unsigned char scratch[SBLM_NM_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[SBLM_MAX_DEVICES];

// Device address of this device's copy of `scratch` (looked up on the first
// call on the device).
int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return check_hip(e, "nm_refine_noalloc: hipGetDevice");
  if (dev < 0 || dev >= SBLM_MAX_DEVICES)
    return set_error(SBLM_EDEVICE, "nm_refine_noalloc: device %d beyond %d", dev,
                     SBLM_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return check_hip(e, "nm_refine_noalloc: hipGetSymbolAddress");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SBLM_OK;
}

// The most lightcurves whose simplices fit the scratch array.
int nm_noalloc_max_lc() {
  int lo = 0, hi = 1 << 24;
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    if (nm_work_bytes(mid) <= SBLM_NM_SCRATCH_BYTES)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}
}  // namespace

extern "C" int nm_refine_noalloc(const sblm_lcs* lcs, const double* lo, const double* hi,
                                 const double* x0, const nm_config* cfg, double* x,
                                 double* chi2, double* Fs, double* Fb, int32_t* n_iter,
                                 sblm_stats* stats, void* stream) {
  int rc = nm_check(cfg, "nm_refine_noalloc");
  if (rc) return rc;
  if (!lcs || !lcs->off || !lcs->t || !lcs->y || !lcs->w)
    return set_error(SBLM_EINVAL, "nm_refine_noalloc: null lightcurve descriptor or array");
  if (lcs->n_lc < 1) return set_error(SBLM_EINVAL, "nm_refine_noalloc: n_lc < 1");
  const size_t need = nm_work_bytes(lcs->n_lc);
  if (need > SBLM_NM_SCRATCH_BYTES)
    return set_error(SBLM_ERANGE,
                     "nm_refine_noalloc: %d lightcurves need %zu bytes of scratch, beyond its "
                     "%u bytes (at most %d lightcurves)",
                     lcs->n_lc, need, SBLM_NM_SCRATCH_BYTES, nm_noalloc_max_lc());
  if (!lo || !hi || !x0 || !x)
    return set_error(SBLM_EINVAL, "nm_refine_noalloc: null lo, hi, x0 or x");
  double span[SBLM_NPAR];
  for (int g = 0; g < SBLM_NPAR; ++g) {
    if (!(hi[g] > lo[g]))
      return set_error(SBLM_EINVAL, "nm_refine_noalloc: hi[%d] <= lo[%d]", g, g);
    span[g] = hi[g] - lo[g];
  }
  void* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  return nm_run(*lcs, 1, lo, span, x0, *cfg, x, chi2, Fs, Fb, n_iter, stats,
                (hipStream_t)stream, nullptr, ws);
}

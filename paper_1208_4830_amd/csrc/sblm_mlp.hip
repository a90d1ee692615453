// sblm_mlp.hip -- learned proposal network for seeding the EA population.
//
// Not part of the paper's method (its neural network is a competing fitter,
// Sec. 4.1); the network only proposes starting points, and the EA's chi^2
// (Sec. 4.1, 4.4) still decides.  Contents:
//   * sblm_resample: a lightcurve -> 256 normalised bins;
//   * mlp_make_data: training lightcurves drawn from the EA's parameter
//     domain and observed at bin level through the forward model (Sec. 2.2);
//   * the network 256 -> 512 -> 512 -> 120 (ReLU hidden layers) whose output
//     is a K = 8 mixture of diagonal Gaussians over 7 targets, trained by its
//     own BF16 MFMA forward and backward GEMMs, an FP64 mixture-likelihood
//     kernel, deterministic column sums and Adam on FP32 master weights.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "sblm_internal.h"
#include "sblm_rng.h"

namespace sblm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int NB = MLP_NBINS;      // 256 input bins
constexpr int NH = MLP_HIDDEN;     // 512 hidden units
constexpr int NO = MLP_NOUT;       // 120 outputs
constexpr int NOP = MLP_NOUT_PAD;  // 128 (padded output width)
constexpr int KM = MLP_K, DM = MLP_D;

// Device parameter layout (FP32 master copy, BF16 shadow and Adam moments):
// W1 [256][512], b1 [512], W2 [512][512], b2 [512], W3 [512][128], b3 [128];
// the 8 pad columns of W3 and b3 hold zeros and receive zero gradient.
constexpr int64_t OFF_W1 = 0;
constexpr int64_t OFF_B1 = OFF_W1 + (int64_t)NB * NH;
constexpr int64_t OFF_W2 = OFF_B1 + NH;
constexpr int64_t OFF_B2 = OFF_W2 + (int64_t)NH * NH;
constexpr int64_t OFF_W3 = OFF_B2 + NH;
constexpr int64_t OFF_B3 = OFF_W3 + (int64_t)NH * NOP;
constexpr int64_t NP_DEV = OFF_B3 + NOP;

constexpr uint64_t P_MLP_INIT = 32;  // Philox purposes of this file (key
constexpr uint64_t P_DATA = 33;      // word 1 = sample index or 0)

// ------------------------------------------------------------------ BF16

__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)0x7fc0;  // NaN
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);      // RNE
}

// ------------------------------------------------------------------ GEMM
//
// C[M][N] = A[M][K] * B[K][N] on BF16 operands with FP32 accumulation in
// the 32x32x16 matrix-core instruction.  A workgroup of four waves owns a
// 64x64 tile of C (2x2 waves of 32x32); K advances through LDS
// (double-buffered, one barrier per stage) in stages of TKS = 128 (32 when
// K per range is not a multiple of 128), TKS/16 MFMA per wave and stage.
// Operands are read from either layout:
//   AK: A[m*lda + k] (k contiguous)   else A[k*lda + m]
//   BK: B[n*ldb + k] (k contiguous)   else B[k*ldb + n]
// LDS holds both tiles as [row = m or n][TKS k] so every lane fetches its 8
// consecutive k values with one 16-byte read (row stride padded by 8).
// Epilogue: + bias[n], then * (mask[m][n] > 0), then ReLU, written as FP32
// and/or BF16.  Requires M % 64 == 0, N % 64 == 0, K % (32 * ksplit) == 0.
// With ksplit > 1 (the weight gradients, a contraction over the batch) each
// K range writes its own FP32 partial (no bias, mask or ReLU) and
// splitk_reduce_kernel adds them in order.
struct GemmArgs {
  const uint16_t* A;
  int64_t lda;
  const uint16_t* B;
  int64_t ldb;
  int M, N, K;
  const float* bias;     // [N] or null
  const uint16_t* mask;  // [M][ldm] BF16 or null
  int64_t ldm;
  float* Cf;             // [M][ldc] or null (with ksplit > 1: [ksplit][M][ldc])
  uint16_t* Cb;          // [M][ldc] or null
  int64_t ldc;
  int relu;
  int ksplit;            // K is cut into ksplit equal ranges (blockIdx.z), 0/1: none
};

constexpr int TM = 64;

// One K stage of a 64-row operand tile: TKS k values per row, TKS/32 chunks
// of 8 BF16 (16 bytes) per thread, all loads issued before any is used.
template <bool KC, int TKS>
__device__ __forceinline__ void load_tile(const uint16_t* X, int64_t ld, int r0, int k0,
                                          uint4* v) {
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < TKS / 32; ++j) {
    const int q = t + 256 * j;  // chunk index
    if (KC) {  // row q / (TKS/8), k chunk q % (TKS/8)
      v[j] = *(const uint4*)(X + (int64_t)(r0 + q / (TKS / 8)) * ld + k0 + (q % (TKS / 8)) * 8);
    } else {   // k row q / 8, 8 consecutive rows from (q % 8) * 8
      v[j] = *(const uint4*)(X + (int64_t)(k0 + q / 8) * ld + r0 + (q % 8) * 8);
    }
  }
}

template <bool KC, int TKS>
__device__ __forceinline__ void store_tile(uint16_t* S, const uint4* v) {
  constexpr int STRIDE = TKS + 8;
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < TKS / 32; ++j) {
    const int q = t + 256 * j;
    if (KC) {
      *(uint4*)(S + (q / (TKS / 8)) * STRIDE + (q % (TKS / 8)) * 8) = v[j];
    } else {
      const int k = q / 8, r = (q % 8) * 8;
      const uint16_t* e = (const uint16_t*)&v[j];
#pragma unroll
      for (int i = 0; i < 8; ++i) S[(r + i) * STRIDE + k] = e[i];
    }
  }
}

// TKS: k values per LDS stage (32 or 128); deeper stages keep more loads in
// flight per round trip, which is what bounds these small GEMMs.
// Up to three independent products of one shape class in one launch (the
// three weight gradients of a step): blockIdx.x runs over the output tiles
// of problem 0, then 1, then 2 (first[p] = its first block), blockIdx.z over
// the K ranges, which all problems share.
struct GemmGroup {
  GemmArgs g[3];
  int first[4];
  int nprob;
};

template <bool AK, bool BK, int TKS>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmGroup gg) {
  constexpr int STRIDE = TKS + 8;  // padded LDS row (elements)
  __shared__ __attribute__((aligned(16))) uint16_t sA[2][TM * STRIDE];
  __shared__ __attribute__((aligned(16))) uint16_t sB[2][TM * STRIDE];
  int prob = 0;
  while (prob + 1 < gg.nprob && (int)blockIdx.x >= gg.first[prob + 1]) ++prob;
  const GemmArgs& g = gg.g[prob];
  const int tile = (int)blockIdx.x - gg.first[prob], ntn = g.N / TM;
  const int m0 = (tile / ntn) * TM, n0 = (tile % ntn) * TM;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int nst = g.K / TKS / gridDim.z;  // stages of this K range
  const int kb = blockIdx.z * nst * TKS;  // its first k

  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;

  // the MFMAs of the stage in LDS buffer `buf`
  auto mfma_stage = [&](int buf) {
    const uint16_t* pa = sA[buf] + (wm + (lane & 31)) * STRIDE + 8 * (lane >> 5);
    const uint16_t* pb = sB[buf] + (wn + (lane & 31)) * STRIDE + 8 * (lane >> 5);
#pragma unroll
    for (int kk = 0; kk < TKS; kk += 16) {
      const bf16x8 a = *(const bf16x8*)(pa + kk);
      const bf16x8 b = *(const bf16x8*)(pb + kk);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
  };
  uint4 ra[TKS / 32], rb[TKS / 32];
  load_tile<AK, TKS>(g.A, g.lda, m0, kb, ra);
  load_tile<BK, TKS>(g.B, g.ldb, n0, kb, rb);
  store_tile<AK, TKS>(sA[0], ra);
  store_tile<BK, TKS>(sB[0], rb);
  __syncthreads();
  // software pipeline: the next stage's loads are in flight during this
  // stage's MFMAs; the last stage is peeled off, so the staging registers
  // are written on every pass of the loop (a conditional load kept them in
  // scratch memory, and the loads were waited for at once)
  for (int s = 0; s + 1 < nst; ++s) {
    const int cur = s & 1;
    load_tile<AK, TKS>(g.A, g.lda, m0, kb + (s + 1) * TKS, ra);
    load_tile<BK, TKS>(g.B, g.ldb, n0, kb + (s + 1) * TKS, rb);
    mfma_stage(cur);
    store_tile<AK, TKS>(sA[cur ^ 1], ra);
    store_tile<BK, TKS>(sB[cur ^ 1], rb);
    __syncthreads();
  }
  mfma_stage((nst - 1) & 1);

  // lane l, register r holds C[(r%4) + 8(r/4) + 4(l/32)][l%32] of the wave
  const int n = n0 + wn + (lane & 31);
  const float bias = g.bias ? g.bias[n] : 0.0f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + wm + (r & 3) + 8 * (r >> 2) + 4 * (lane >> 5);
    float v = acc[r] + bias;
    if (g.mask) {
      const uint16_t h = g.mask[(int64_t)m * g.ldm + n];
      if (h == 0 || (h & 0x8000u)) v = 0.0f;
    }
    if (g.relu) v = fmaxf(v, 0.0f);
    if (g.Cf) g.Cf[(int64_t)blockIdx.z * g.M * g.ldc + (int64_t)m * g.ldc + n] = v;
    if (g.Cb) g.Cb[(int64_t)m * g.ldc + n] = f2bf(v);
  }
}

template <int TKS>
hipError_t gemm_t(const GemmGroup& gg, bool ak, bool bk, hipStream_t st) {
  const int ks = gg.g[0].ksplit > 1 ? gg.g[0].ksplit : 1;
  const dim3 grid(gg.first[gg.nprob], 1, ks);
  if (ak && !bk)
    hipLaunchKernelGGL((gemm_bf16_kernel<true, false, TKS>), grid, dim3(256), 0, st, gg);
  else if (ak && bk)
    hipLaunchKernelGGL((gemm_bf16_kernel<true, true, TKS>), grid, dim3(256), 0, st, gg);
  else if (!ak && !bk)
    hipLaunchKernelGGL((gemm_bf16_kernel<false, false, TKS>), grid, dim3(256), 0, st, gg);
  else
    hipLaunchKernelGGL((gemm_bf16_kernel<false, true, TKS>), grid, dim3(256), 0, st, gg);
  return hipGetLastError();
}

// C = A B for n (1..3) problems with the same operand layouts, K and K split.
hipError_t gemm_group(const GemmArgs* gs, int n, bool ak, bool bk, hipStream_t st) {
  GemmGroup gg;
  memset(&gg, 0, sizeof(gg));
  gg.nprob = n;
  gg.first[0] = 0;
  for (int i = 0; i < n; ++i) {
    gg.g[i] = gs[i];
    gg.first[i + 1] = gg.first[i] + (gs[i].N / TM) * (gs[i].M / TM);
  }
  const int ks = gs[0].ksplit > 1 ? gs[0].ksplit : 1;
  return (gs[0].K / ks) % 128 == 0 ? gemm_t<128>(gg, ak, bk, st) : gemm_t<32>(gg, ak, bk, st);
}

hipError_t gemm(const GemmArgs& g, bool ak, bool bk, hipStream_t st) {
  return gemm_group(&g, 1, ak, bk, st);
}

// --------------------------------------------------- mixture likelihood
//
// Eight threads per sample, thread k owning mixture component k.  Output row
// O = (8 logits, 8x7 means, 8x7 log standard deviations, 8 pad); target row
// y[7], target 3 periodic on [0, 1).  loss_row = -log p(y)/n and dO = d loss
// / dO (pad entries 0), in FP64:
//   log pi_k = logit_k - logsumexp(logit),  r_kd = y_d - mu_kd (wrapped),
//   a_k = log pi_k + sum_d [-r^2/(2 s^2) - log s - log(2 pi)/2],
//   gamma_k = exp(a_k - logsumexp(a)),
//   dlogit_k = (pi_k - gamma_k)/n, dmu = -gamma r/s^2/n,
//   dlog s = -gamma (r^2/s^2 - 1)/n.
// The maxima and sums over the eight components are butterflies inside each
// group of eight lanes (a fixed order, so the result is deterministic).
__device__ __forceinline__ double grp8_max(double v) {
#pragma unroll
  for (int m = 1; m < 8; m <<= 1) v = fmax(v, __shfl_xor(v, m, 8));
  return v;
}
__device__ __forceinline__ double grp8_sum(double v) {
#pragma unroll
  for (int m = 1; m < 8; m <<= 1) v += __shfl_xor(v, m, 8);
  return v;
}

__global__ __launch_bounds__(256) void mlp_nll_kernel(const float* O, const float* y, int n,
                                                      float* dOf, uint16_t* dOb,
                                                      float* loss_row) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = gid >> 3, k = gid & 7;  // n * 8 threads, a multiple of 64
  const bool valid = b < n;
  const int bb = valid ? b : 0;
  const float* o = O + (int64_t)bb * NOP;
  const double inv_n = 1.0 / (double)n;
  const double HALF_LOG_2PI = 0.91893853320467274178;
  const double logit = (double)o[k];
  const double lse_l = [&] {
    const double m = grp8_max(logit);
    return m + log(grp8_sum(exp(logit - m)));
  }();
  double r[DM], is2[DM];
  double a = logit - lse_l;
#pragma unroll
  for (int d = 0; d < DM; ++d) {
    double rr = (double)y[(int64_t)bb * DM + d] - (double)o[KM + k * DM + d];
    if (d == MLP_PERIODIC) rr -= floor(rr + 0.5);
    const double ls = (double)o[KM + KM * DM + k * DM + d];
    is2[d] = exp(-2.0 * ls);
    r[d] = rr;
    a += -0.5 * rr * rr * is2[d] - ls - HALF_LOG_2PI;
  }
  const double amax = grp8_max(a);
  const double lp = amax + log(grp8_sum(exp(a - amax)));
  const double gam = exp(a - lp);
  const double pi = exp(logit - lse_l);
  if (!valid) return;
  if (k == 0) loss_row[b] = (float)(-lp * inv_n);
  float* gf = dOf + (int64_t)b * NOP;
  uint16_t* gb = dOb + (int64_t)b * NOP;
  const float gl = (float)((pi - gam) * inv_n);
  gf[k] = gl;
  gb[k] = f2bf(gl);
#pragma unroll
  for (int d = 0; d < DM; ++d) {
    const float gm = (float)(-gam * r[d] * is2[d] * inv_n);
    const float gs = (float)(-gam * (r[d] * r[d] * is2[d] - 1.0) * inv_n);
    gf[KM + k * DM + d] = gm;
    gb[KM + k * DM + d] = f2bf(gm);
    gf[KM + KM * DM + k * DM + d] = gs;
    gb[KM + KM * DM + k * DM + d] = f2bf(gs);
  }
  gf[NO + k] = 0.0f;  // the eight pad columns
  gb[NO + k] = 0;
}

// Column sums out[c] = sum_r X[r][c] of up to four matrices in one pair of
// launches (bias gradients and the loss).  Stage 1: block (column tile of
// 64, row chunk rc) sums its rows in four interleaved groups combined in a
// fixed order into part[rc][column]; stage 2 adds the RC chunks in order.
// Deterministic.
constexpr int CS_RC = 16;
struct ColSeg {
  const float* X;
  int64_t ld;
  int ncol;
  float* out;
};
struct ColSegs {
  ColSeg s[4];
  int nseg;
  int tile0[5];  // first 64-column tile of each segment
  int col0[5];   // first column of each segment in the partial array
  int nrow;
};

__global__ __launch_bounds__(256) void colsum_stage1(ColSegs cs, float* part, int ncol_all) {
  __shared__ float red[4][64];
  int sg = 0;
  while (sg + 1 < cs.nseg && (int)blockIdx.x >= cs.tile0[sg + 1]) ++sg;
  const ColSeg& g = cs.s[sg];
  const int c = ((int)blockIdx.x - cs.tile0[sg]) * 64 + (threadIdx.x & 63);
  const int grp = threadIdx.x >> 6;
  const int per = (cs.nrow + CS_RC - 1) / CS_RC;
  const int r0 = blockIdx.y * per, r1 = min(cs.nrow, r0 + per);
  float acc = 0.0f;
  if (c < g.ncol)
    for (int r = r0 + grp; r < r1; r += 4) acc += g.X[(int64_t)r * g.ld + c];
  red[grp][threadIdx.x & 63] = acc;
  __syncthreads();
  if (grp == 0 && c < g.ncol) {
    const int j = threadIdx.x;
    part[(int64_t)blockIdx.y * ncol_all + cs.col0[sg] + c] =
        ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
  }
}

__global__ void colsum_stage2(ColSegs cs, const float* part, int ncol_all) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol_all) return;
  int sg = 0;
  while (sg + 1 < cs.nseg && c >= cs.col0[sg + 1]) ++sg;
  float t = part[c];
  for (int rc = 1; rc < CS_RC; ++rc) t += part[(int64_t)rc * ncol_all + c];
  cs.s[sg].out[c - cs.col0[sg]] = t;
}

// part must hold CS_RC x (total columns) floats.  stage2 = false leaves the
// partials for the captured training step's Adam kernel to add.
hipError_t colsums(ColSegs cs, float* part, hipStream_t st, bool stage2 = true) {
  cs.tile0[0] = 0;
  cs.col0[0] = 0;
  for (int i = 0; i < cs.nseg; ++i) {
    cs.tile0[i + 1] = cs.tile0[i] + (cs.s[i].ncol + 63) / 64;
    cs.col0[i + 1] = cs.col0[i] + cs.s[i].ncol;
  }
  const int ncol_all = cs.col0[cs.nseg];
  hipLaunchKernelGGL(colsum_stage1, dim3(cs.tile0[cs.nseg], CS_RC), dim3(256), 0, st, cs, part,
                     ncol_all);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !stage2) return e;
  hipLaunchKernelGGL(colsum_stage2, dim3((ncol_all + 255) / 256), dim3(256), 0, st, cs, part,
                     ncol_all);
  return hipGetLastError();
}

// Sum of ks partial matrices part[z][i], z in order (split-K reduction).
__global__ void splitk_reduce_kernel(const float* part, int ks, int64_t n, float* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    float t = part[i];
    for (int z = 1; z < ks; ++z) t += part[(int64_t)z * n + i];
    out[i] = t;
  }
}

// Adam (Kingma & Ba 2015) with bias correction factors c1 = 1/(1 - b1^t),
// c2 = 1/(1 - b2^t):  p -= lr * (m c1) / (sqrt(v c2) + eps); also refreshes
// the BF16 shadow of the weights.  1 - b1 and 1 - b2 come from the host in
// double (1.0f - 0.999f would carry a 1e-5 relative error into v).
__global__ void adam_kernel(float* p, const float* g, float* m, float* v,
                            uint16_t* pb, int64_t n, float lr, float b1, float b2,
                            float omb1, float omb2, float eps, float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    p[i] = pi;
    pb[i] = f2bf(pi);
  }
}

// The split-K partials of the three weight gradients of one step (a buffer
// each), for the graph form of training: the Adam kernel sums them.
struct KParts {
  const float* part[3];
  int64_t off[3];  // first parameter of the tensor
  int64_t mn[3];   // its elements
  int ks;          // partials per tensor (1: none, the GEMM wrote the gradient)
};

// The column-sum partials of one step (colsum_stage1 without its second
// stage): the three bias gradients and the loss.
struct CParts {
  const float* part;  // [CS_RC][ncol_all]
  int ncol_all;
  int64_t off[3];     // first parameter of b3, b2, b1
  int ncol[3];
  int col0[3];        // their first columns in part
  int loss_col;
};

// adam_kernel for a step of the captured training graph: the step's learning
// rate and bias-correction factors are read from sched[3k .. 3k+2] (k = the
// device step counter); a weight tensor's gradient is first summed over its
// split-K partials, in range order (as splitk_reduce sums them), a bias
// gradient over its column-sum partials, in row-chunk order (as
// colsum_stage2 sums them), and stored to g.
__global__ void adam_graph_kernel(float* p, float* g, float* m, float* v, uint16_t* pb,
                                  int64_t n, const float* sched, const int64_t* dstep,
                                  KParts kp, CParts cp, float b1, float b2, float omb1,
                                  float omb2, float eps) {
  const int64_t k = *dstep;
  const float lr = sched[3 * k], c1 = sched[3 * k + 1], c2 = sched[3 * k + 2];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    float gi = 0.0f;
    bool summed = false;
    if (kp.ks > 1) {
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int64_t j = i - kp.off[t];
        if (j >= 0 && j < kp.mn[t]) {
          float sum = kp.part[t][j];
          for (int z = 1; z < kp.ks; ++z) sum += kp.part[t][(int64_t)z * kp.mn[t] + j];
          g[i] = sum;
          gi = sum;
          summed = true;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int64_t j = i - cp.off[t];
      if (j >= 0 && j < cp.ncol[t]) {
        const int c = cp.col0[t] + (int)j;
        float sum = cp.part[c];
        for (int rc = 1; rc < CS_RC; ++rc) sum += cp.part[(int64_t)rc * cp.ncol_all + c];
        g[i] = sum;
        gi = sum;
        summed = true;
      }
    }
    if (!summed) gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    p[i] = pi;
    pb[i] = f2bf(pi);
  }
}

// Last node of a training step: the step's loss (its column-sum partials
// added in row-chunk order, as colsum_stage2 adds them) to losses[k], and
// k + 1 to the counter.
__global__ void step_advance_kernel(int64_t* dstep, CParts cp, float* losses) {
  const int64_t k = *dstep;
  float t = cp.part[cp.loss_col];
  for (int rc = 1; rc < CS_RC; ++rc) t += cp.part[(int64_t)rc * cp.ncol_all + cp.loss_col];
  losses[k] = t;
  *dstep = k + 1;
}

// First node of a training step: batch k mod per of (x, y) into the net's
// own buffers, k = the device step counter.
__global__ void batch_gather_kernel(const uint16_t* x, const float* y, int64_t per, int batch,
                                    const int64_t* dstep, uint16_t* xb, float* yb) {
  const int64_t r0 = (*dstep % per) * batch;
  const uint4* xs = (const uint4*)(x + r0 * NB);
  uint4* xd = (uint4*)xb;
  const int64_t nx = (int64_t)batch * NB / 8, ny = (int64_t)batch * DM;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nx + ny;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < nx)
      xd[i] = xs[i];
    else
      yb[i - nx] = y[r0 * DM + (i - nx)];
  }
}

__global__ void to_bf16_kernel(const float* p, uint16_t* pb, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    pb[i] = f2bf(p[i]);
}

__global__ void fill_u16_kernel(uint16_t* x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0;
}

// He-normal weights (std sqrt(2/fan_in); output layer std 0.01), zero
// biases.  Normal deviates by the Box-Muller transform of two Philox words.
__global__ void mlp_init_kernel(float* p, uint16_t* pb, uint64_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < NP_DEV;
       i += (int64_t)gridDim.x * blockDim.x) {
    float val = 0.0f;
    double sd = 0.0;
    if (i < OFF_B1) sd = sqrt(2.0 / NB);
    else if (i >= OFF_W2 && i < OFF_B2) sd = sqrt(2.0 / NH);
    else if (i >= OFF_W3 && i < OFF_B3 && (i - OFF_W3) % NOP < NO) sd = 0.01;
    if (sd > 0.0) {
      const u64x4 w = philox4x64_10(0, P_MLP_INIT, (uint64_t)i, 0, seed, 0);
      const double u1 = u01(w.v[0]), u2 = u01(w.v[1]);
      val = (float)(sd * sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2));
    }
    p[i] = val;
    pb[i] = f2bf(val);
  }
}

// ------------------------------------------------------------ resampling
//
// Shared by sblm_resample and mlp_make_data; 256 threads, thread j owns
// bin j.  On entry val[j] holds the bin value and filled[j] its flag.
// Empty bins take the linear interpolation of the nearest filled bins on
// either side, evaluated as v_l + (v_h - v_l)(j - l)/(h - l) (the nearest
// filled value beyond the last filled bin at either end); then the bins are
// normalised as (v - median)/max(max - median, 1e-12), the median of 256
// values being the mean of the two central order statistics.
__device__ void finish_bins(double* val, int* filled, double* srt, int any_filled,
                            float* xf, uint16_t* xb) {
  const int j = threadIdx.x;
  if (!any_filled) {
    if (xf) xf[j] = 0.0f;
    if (xb) xb[j] = 0;
    return;
  }
  double v = val[j];
  if (!filled[j]) {
    int l = j - 1, h = j + 1;
    while (l >= 0 && !filled[l]) --l;
    while (h < NB && !filled[h]) ++h;
    if (l >= 0 && h < NB)
      v = val[l] + (val[h] - val[l]) * (double)(j - l) / (double)(h - l);
    else
      v = (l >= 0) ? val[l] : val[h];
  }
  srt[j] = v;
  __syncthreads();
  // bitonic sort of srt[0..255], ascending
  for (int k = 2; k <= NB; k <<= 1) {
    for (int s = k >> 1; s > 0; s >>= 1) {
      const int p = j ^ s;
      if (p > j) {
        const double x = srt[j], y = srt[p];
        const bool up = (j & k) == 0;
        if ((x > y) == up) {
          srt[j] = y;
          srt[p] = x;
        }
      }
      __syncthreads();
    }
  }
  const double med = (srt[NB / 2 - 1] + srt[NB / 2]) / 2.0;
  const double div = fmax(srt[NB - 1] - med, 1e-12);
  const double r = (v - med) / div;
  if (xf) xf[j] = (float)r;
  if (xb) xb[j] = f2bf((float)r);
}

__device__ __forceinline__ int bin_of(double t, double t_a, double span) {
  if (span <= 0.0) return 0;
  const double u = (t - t_a) / span * (double)NB;
  return (int)fmin(u, (double)(NB - 1));
}

// One block of 256 threads per lightcurve (t ascending within each).
__global__ __launch_bounds__(256) void resample_kernel(const int64_t* off,
                                                       const double* t,
                                                       const double* y,
                                                       const double* w, float* xf,
                                                       uint16_t* xb) {
  __shared__ double val[NB], srt[NB];
  __shared__ int filled[NB];
  __shared__ int any;
  const int lc = blockIdx.x, j = threadIdx.x;
  const int64_t o0 = off[lc], o1 = off[lc + 1];
  float* xfl = xf ? xf + (int64_t)lc * NB : nullptr;
  uint16_t* xbl = xb ? xb + (int64_t)lc * NB : nullptr;
  if (j == 0) any = 0;
  __syncthreads();
  double sw = 0.0, swy = 0.0;
  if (o1 > o0) {
    const double t_a = t[o0], span = t[o1 - 1] - t_a;
    // first epoch of bin >= j and of bin >= j + 1 (bins non-decreasing)
    int64_t lo = o0, hi = o1;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (bin_of(t[mid], t_a, span) < j) lo = mid + 1; else hi = mid;
    }
    int64_t e1 = lo, hi2 = o1;
    while (e1 < hi2) {
      const int64_t mid = e1 + (hi2 - e1) / 2;
      if (bin_of(t[mid], t_a, span) <= j) e1 = mid + 1; else hi2 = mid;
    }
    for (int64_t e = lo; e < e1; ++e) {
      const double we = w[e];
      sw += we;
      swy += we * y[e];
    }
  }
  filled[j] = sw > 0.0;
  val[j] = sw > 0.0 ? swy / sw : 0.0;
  if (sw > 0.0) any = 1;
  __syncthreads();
  finish_bins(val, filled, srt, any, xfl, xbl);
}

// ------------------------------------------------------- training data
//
// Sample s uses Philox key (seed, s), counter (0, P_DATA, row, j / 4):
//   row 0: words 0..5 the parameters (uniform over the domain below, in the
//          library's plane order), word 6 Fb ~ U[0, 0.5] (Fs = 1), word 7
//          the noise fraction s ~ U[0.005, 0.03], word 8 the epoch count
//          L ~ U{200..5000}, words 9, 10 the start and the end of the
//          observing window, t0 + a tE and t0 + b tE with a ~ U(-3, -2) and
//          b ~ U(2, 3) (the random start and end of Sec. 4.2);
//   row 1 + j: words 0..3 for bin j (Poisson count, two normal deviates).
// The observing window is seen through nightly windows
// [n + 0.1, n + 0.1 + 1/3] days; t_first, t_last are its first and last
// observable instants and span = t_last - t_first.  Bin j covers
// [t_first + span j/256, t_first + span (j+1)/256]; its expected epoch count
// is c_j = n_sched o_j / sum(o) + n_dense d_j / (0.2 tE), with o_j its
// overlap with the nightly windows, d_j its overlap with t0 +- 0.1 tE,
// n_dense = round(L/10), n_sched = L - n_dense; the count is Poisson(c_j)
// (inversion for c_j <= 64, else the rounded normal approximation).  A
// counted bin holds F = Fs A(t_j) + Fb plus N(0, (s F)^2 / count) noise, A
// from the forward model at the bin centre; then empty bins and
// normalisation as for sblm_resample.
//
// Targets: (log10 q + 3)/3, (d - 0.5)/1.5, u0/0.5, alpha/(2 pi),
// (t0 - t_first)/span, tE/span, Fs/(Fs + Fb).
constexpr double NIGHT0 = 0.1, NIGHT_LEN = 1.0 / 3.0;

__device__ void data_window(double t0, double tE, double a, double b, double& t_first,
                            double& t_last) {
  const double ta = t0 + a * tE, tb = t0 + b * tE;
  const double na = floor(ta - NIGHT0);
  t_first = (ta <= na + NIGHT0 + NIGHT_LEN) ? ta : na + 1.0 + NIGHT0;
  const double nb = floor(tb - NIGHT0);
  t_last = (tb <= nb + NIGHT0 + NIGHT_LEN) ? tb : nb + NIGHT0 + NIGHT_LEN;
}

// aux row per sample: t_first, span, t0, tE, Fb, s, L
constexpr int NAUX = 8;

__global__ void data_draw_kernel(uint64_t seed, int64_t first, int n, double* theta,
                                 double* aux, float* y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double DLO[6] = {-3.0, 0.5, 0.0, 0.0, 10.0, -10.0};
  const double DHI[6] = {0.0, 2.0, 0.5, 2.0 * M_PI, 100.0, 10.0};
  const uint64_t s = (uint64_t)(first + i);
  const u64x4 w0 = philox4x64_10(0, P_DATA, 0, 0, seed, s);
  const u64x4 w1 = philox4x64_10(0, P_DATA, 0, 1, seed, s);
  const u64x4 w2 = philox4x64_10(0, P_DATA, 0, 2, seed, s);
  const uint64_t wd[9] = {w0.v[0], w0.v[1], w0.v[2], w0.v[3], w1.v[0],
                          w1.v[1], w1.v[2], w1.v[3], w2.v[0]};
  double th[6];
  for (int g = 0; g < 6; ++g) th[g] = DLO[g] + (DHI[g] - DLO[g]) * u01(wd[g]);
  const double Fb = 0.5 * u01(wd[6]);
  const double sn = 0.005 + 0.025 * u01(wd[7]);
  const double L = (double)(200u + below(wd[8], 4801u));
  const double wa = -3.0 + u01(w2.v[1]), wb = 2.0 + u01(w2.v[2]);
  double t_first, t_last;
  data_window(th[5], th[4], wa, wb, t_first, t_last);
  const double span = t_last - t_first;
  for (int g = 0; g < 4; ++g) theta[(int64_t)g * n + i] = th[g];
  theta[(int64_t)4 * n + i] = th[4] / span;
  theta[(int64_t)5 * n + i] = (th[5] - t_first) / span;
  double* a = aux + (int64_t)i * NAUX;
  a[0] = t_first;
  a[1] = span;
  a[2] = th[5];
  a[3] = th[4];
  a[4] = Fb;
  a[5] = sn;
  a[6] = L;
  a[7] = 0.0;
  float* yy = y + (int64_t)i * DM;
  yy[0] = (float)((th[0] + 3.0) / 3.0);
  yy[1] = (float)((th[1] - 0.5) / 1.5);
  yy[2] = (float)(th[2] / 0.5);
  yy[3] = (float)(th[3] / (2.0 * M_PI));
  yy[4] = (float)((th[5] - t_first) / span);
  yy[5] = (float)(th[4] / span);
  yy[6] = (float)(1.0 / (1.0 + Fb));
}

__device__ __forceinline__ double overlap(double a0, double a1, double b0, double b1) {
  return fmax(0.0, fmin(a1, b1) - fmax(a0, b0));
}

__global__ __launch_bounds__(256) void data_finish_kernel(uint64_t seed, int64_t first,
                                                          const double* aux,
                                                          const double* A, float* xf,
                                                          uint16_t* xb) {
  __shared__ double val[NB], srt[NB], red[NB];
  __shared__ int filled[NB];
  __shared__ int any;
  const int i = blockIdx.x, j = threadIdx.x;
  const uint64_t s = (uint64_t)(first + i);
  const double* a = aux + (int64_t)i * NAUX;
  const double t_first = a[0], span = a[1], t0 = a[2], tE = a[3], Fb = a[4],
               sn = a[5], L = a[6];
  const double b0 = t_first + span * (double)j / NB;
  const double b1 = t_first + span * (double)(j + 1) / NB;
  double o = 0.0;
  for (double nt = floor(b0) - 1.0; nt <= floor(b1); nt += 1.0)
    o += overlap(b0, b1, nt + NIGHT0, nt + NIGHT0 + NIGHT_LEN);
  const double dj = overlap(b0, b1, t0 - 0.1 * tE, t0 + 0.1 * tE);
  red[j] = o;
  if (j == 0) any = 0;
  __syncthreads();
  for (int h = NB / 2; h > 0; h >>= 1) {  // fixed-order tree sum
    if (j < h) red[j] += red[j + h];
    __syncthreads();
  }
  const double osum = red[0];
  const double n_dense = floor(0.1 * L + 0.5), n_sched = L - n_dense;
  const double c = (osum > 0.0 ? n_sched * o / osum : 0.0) + n_dense * dj / (0.2 * tE);
  const u64x4 wb = philox4x64_10(0, P_DATA, 1 + (uint64_t)j, 0, seed, s);
  const double r1 = u01(wb.v[1]), r2 = u01(wb.v[2]);
  const double rad = sqrt(-2.0 * log(r1));
  const double z1 = rad * cos(2.0 * M_PI * r2), z2 = rad * sin(2.0 * M_PI * r2);
  double cnt;
  if (c <= 64.0) {
    const double u = u01(wb.v[0]);
    double p = exp(-c), F = p;
    cnt = 0.0;
    while (u > F && cnt < 1000.0) {
      cnt += 1.0;
      p = p * c / cnt;
      F += p;
    }
  } else {
    cnt = fmax(0.0, floor(c + sqrt(c) * z2 + 0.5));
  }
  const double flux = A[(int64_t)i * NB + j] + Fb;
  filled[j] = cnt > 0.0;
  val[j] = cnt > 0.0 ? flux + sn * flux / sqrt(cnt) * z1 : 0.0;
  if (cnt > 0.0) any = 1;
  __syncthreads();
  finish_bins(val, filled, srt, any, xf ? xf + (int64_t)i * NB : nullptr,
              xb ? xb + (int64_t)i * NB : nullptr);
}

__global__ void bin_centres_kernel(double* u) {
  u[threadIdx.x] = ((double)threadIdx.x + 0.5) / NB;
}

}  // namespace
}  // namespace sblm

using namespace sblm;

// ------------------------------------------------------------- network

struct mlp_net {
  int device = 0;
  int batch_max = 0;
  int64_t step = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  uint16_t* pb = nullptr;
  uint16_t* xbuf = nullptr;   // [batch_max][256]
  uint16_t *h1 = nullptr, *h2 = nullptr;  // [batch_max][512] post-ReLU
  float* o = nullptr;         // [batch_max][128]
  float* dof = nullptr;       // [batch_max][128]
  uint16_t* dob = nullptr;
  float *dz2f = nullptr, *dz1f = nullptr;  // [batch_max][512]
  uint16_t *dz2b = nullptr, *dz1b = nullptr;
  float* lrow = nullptr;      // [batch_max]
  float* kpart = nullptr;     // split-K partials: [KSPLIT_MAX][512 * 512], the
                              // first of three buffers (W2, then W3, W1)
  float* cpart = nullptr;     // column-sum partials, [CS_RC][COLS_ALL] + a loss slot
  // the training graph (mlp_train) and what it reads
  float* ybuf = nullptr;      // [batch_max][7]
  int64_t* dstep = nullptr;   // device step counter of the graph
  float* sched = nullptr;     // [sched_cap][3]: learning rate, c1, c2 per step
  float* losses = nullptr;    // [sched_cap]
  int64_t sched_cap = 0;
  hipStream_t work = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t train_exec = nullptr;
  int64_t train_key[4] = {0, 0, 0, 0};  // batch, split, rows per epoch, sched buffer
};

constexpr int KSPLIT_MAX = 8;
constexpr int COLS_ALL = NOP + NH + NH + 1;  // b3, b2, b1 gradients and the loss

// Split-K partial buffers of the three weight gradients (one block).
constexpr int64_t KPART_W2 = 0;
constexpr int64_t KPART_W3 = KPART_W2 + (int64_t)KSPLIT_MAX * NH * NH;
constexpr int64_t KPART_W1 = KPART_W3 + (int64_t)KSPLIT_MAX * NH * NOP;
constexpr int64_t KPART_ALL = KPART_W1 + (int64_t)KSPLIT_MAX * NB * NH;

static void net_free(mlp_net* n) {
  if (n->train_exec) (void)hipGraphExecDestroy(n->train_exec);
  void* ptrs[] = {n->p,    n->g,    n->m,    n->v,     n->pb,    n->xbuf,  n->h1,
                  n->h2,   n->o,    n->dof,  n->dob,   n->dz2f,  n->dz1f,  n->dz2b,
                  n->dz1b, n->lrow, n->kpart, n->cpart, n->ybuf, n->dstep, n->sched,
                  n->losses};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (n->ev_in) (void)hipEventDestroy(n->ev_in);
  if (n->ev_out) (void)hipEventDestroy(n->ev_out);
  if (n->work) (void)hipStreamDestroy(n->work);
}

static int grid_for(int64_t n) {
  return (int)std::min<int64_t>((n + 255) / 256, 4096);
}

extern "C" int mlp_create(int32_t batch_max, uint64_t seed, mlp_net** out) {
  if (!out) return set_error(SBLM_EINVAL, "mlp_create: null out");
  *out = nullptr;
  if (batch_max < 64 || batch_max % 64 != 0)
    return set_error(SBLM_EINVAL, "mlp_create: batch_max = %d is not a positive multiple of 64",
                     batch_max);
  if (batch_max > (1 << 20))
    return set_error(SBLM_ERANGE, "mlp_create: batch_max = %d beyond 2^20", batch_max);
  mlp_net* n = new (std::nothrow) mlp_net();
  if (!n) return set_error(SBLM_ENOMEM, "mlp_create: host allocation");
  n->batch_max = batch_max;
  if (hipGetDevice(&n->device) != hipSuccess) {
    delete n;
    return set_error(SBLM_EDEVICE, "mlp_create: hipGetDevice");
  }
  const size_t B = (size_t)batch_max;
  bool ok = hipMalloc(&n->p, NP_DEV * 4) == hipSuccess &&
            hipMalloc(&n->g, NP_DEV * 4) == hipSuccess &&
            hipMalloc(&n->m, NP_DEV * 4) == hipSuccess &&
            hipMalloc(&n->v, NP_DEV * 4) == hipSuccess &&
            hipMalloc(&n->pb, NP_DEV * 2) == hipSuccess &&
            hipMalloc(&n->xbuf, B * NB * 2) == hipSuccess &&
            hipMalloc(&n->h1, B * NH * 2) == hipSuccess &&
            hipMalloc(&n->h2, B * NH * 2) == hipSuccess &&
            hipMalloc(&n->o, B * NOP * 4) == hipSuccess &&
            hipMalloc(&n->dof, B * NOP * 4) == hipSuccess &&
            hipMalloc(&n->dob, B * NOP * 2) == hipSuccess &&
            hipMalloc(&n->dz2f, B * NH * 4) == hipSuccess &&
            hipMalloc(&n->dz1f, B * NH * 4) == hipSuccess &&
            hipMalloc(&n->dz2b, B * NH * 2) == hipSuccess &&
            hipMalloc(&n->dz1b, B * NH * 2) == hipSuccess &&
            hipMalloc(&n->lrow, B * 4) == hipSuccess &&
            hipMalloc(&n->kpart, (size_t)KPART_ALL * 4) == hipSuccess &&
            hipMalloc(&n->cpart, ((size_t)CS_RC * COLS_ALL + 1) * 4) == hipSuccess &&
            hipMalloc(&n->ybuf, B * DM * 4) == hipSuccess &&
            hipMalloc(&n->dstep, 8) == hipSuccess &&
            hipStreamCreateWithFlags(&n->work, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&n->ev_in, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&n->ev_out, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    net_free(n);
    delete n;
    return set_error(SBLM_ENOMEM, "mlp_create: device allocation");
  }
  hipLaunchKernelGGL(mlp_init_kernel, dim3(grid_for(NP_DEV)), dim3(256), 0, nullptr, n->p,
                     n->pb, seed);
  int rc = check_hip(hipGetLastError(), "mlp_create: init launch");
  if (rc == SBLM_OK)
    rc = check_hip(hipMemset(n->g, 0, NP_DEV * 4), "mlp_create: memset");
  if (rc == SBLM_OK)
    rc = check_hip(hipMemset(n->m, 0, NP_DEV * 4), "mlp_create: memset");
  if (rc == SBLM_OK)
    rc = check_hip(hipMemset(n->v, 0, NP_DEV * 4), "mlp_create: memset");
  if (rc == SBLM_OK) rc = check_hip(hipDeviceSynchronize(), "mlp_create: init");
  if (rc != SBLM_OK) {
    net_free(n);
    delete n;
    return rc;
  }
  *out = n;
  return SBLM_OK;
}

extern "C" void mlp_destroy(mlp_net* n) {
  if (!n) return;
  (void)hipDeviceSynchronize();
  net_free(n);
  delete n;
}

// canonical (host) order: W1 [256][512], b1, W2 [512][512], b2, W3 [512][120], b3 [120]
static void canon_map(int64_t* dst_of_src) {
  int64_t k = 0;
  for (int64_t i = 0; i < OFF_W3; ++i) dst_of_src[k++] = i;
  for (int r = 0; r < NH; ++r)
    for (int c = 0; c < NO; ++c) dst_of_src[k++] = OFF_W3 + (int64_t)r * NOP + c;
  for (int c = 0; c < NO; ++c) dst_of_src[k++] = OFF_B3 + c;
}

static int copy_canonical(mlp_net* n, float* dev, float* host, bool to_host,
                          const char* who) {
  float* tmp = (float*)calloc(NP_DEV, sizeof(float));
  int64_t* map = (int64_t*)malloc(MLP_NPARAMS * sizeof(int64_t));
  if (!tmp || !map) {
    free(tmp);
    free(map);
    return set_error(SBLM_ENOMEM, "%s: host allocation", who);
  }
  canon_map(map);
  int rc = SBLM_OK;
  if (to_host) {
    rc = check_hip(hipMemcpy(tmp, dev, NP_DEV * 4, hipMemcpyDeviceToHost), who);
    if (rc == SBLM_OK)
      for (int64_t i = 0; i < MLP_NPARAMS; ++i) host[i] = tmp[map[i]];
  } else {
    for (int64_t i = 0; i < MLP_NPARAMS; ++i) tmp[map[i]] = host[i];
    rc = check_hip(hipMemcpy(dev, tmp, NP_DEV * 4, hipMemcpyHostToDevice), who);
  }
  free(tmp);
  free(map);
  (void)n;
  return rc;
}

extern "C" int mlp_set_params(mlp_net* n, const float* params) {
  if (!n || !params) return set_error(SBLM_EINVAL, "mlp_set_params: null argument");
  int rc = copy_canonical(n, n->p, (float*)params, false, "mlp_set_params");
  if (rc != SBLM_OK) return rc;
  hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(NP_DEV)), dim3(256), 0, nullptr, n->p,
                     n->pb, NP_DEV);
  rc = check_hip(hipGetLastError(), "mlp_set_params: launch");
  if (rc == SBLM_OK) rc = check_hip(hipMemset(n->m, 0, NP_DEV * 4), "mlp_set_params");
  if (rc == SBLM_OK) rc = check_hip(hipMemset(n->v, 0, NP_DEV * 4), "mlp_set_params");
  if (rc == SBLM_OK) rc = check_hip(hipDeviceSynchronize(), "mlp_set_params");
  n->step = 0;
  return rc;
}

extern "C" int mlp_get_params(mlp_net* n, float* params) {
  if (!n || !params) return set_error(SBLM_EINVAL, "mlp_get_params: null argument");
  int rc = check_hip(hipDeviceSynchronize(), "mlp_get_params");
  if (rc != SBLM_OK) return rc;
  return copy_canonical(n, n->p, params, true, "mlp_get_params");
}

extern "C" int mlp_get_grad(mlp_net* n, float* grad) {
  if (!n || !grad) return set_error(SBLM_EINVAL, "mlp_get_grad: null argument");
  int rc = check_hip(hipDeviceSynchronize(), "mlp_get_grad");
  if (rc != SBLM_OK) return rc;
  return copy_canonical(n, n->g, grad, true, "mlp_get_grad");
}

extern "C" int mlp_set_grad(mlp_net* n, const float* grad) {
  if (!n || !grad) return set_error(SBLM_EINVAL, "mlp_set_grad: null argument");
  int rc = check_hip(hipDeviceSynchronize(), "mlp_set_grad");
  if (rc != SBLM_OK) return rc;
  return copy_canonical(n, n->g, (float*)grad, false, "mlp_set_grad");
}

// Forward pass of rows [0, nb) of X (nb % 64 == 0) into n->o.
static hipError_t forward_rows(mlp_net* n, const uint16_t* X, int nb, hipStream_t st) {
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.A = X; g.lda = NB; g.B = n->pb + OFF_W1; g.ldb = NH;
  g.M = nb; g.N = NH; g.K = NB; g.bias = n->p + OFF_B1; g.Cb = n->h1; g.ldc = NH;
  g.relu = 1;
  hipError_t e = gemm(g, true, false, st);
  if (e != hipSuccess) return e;
  g.A = n->h1; g.lda = NH; g.B = n->pb + OFF_W2; g.ldb = NH; g.K = NH;
  g.bias = n->p + OFF_B2; g.Cb = n->h2;
  e = gemm(g, true, false, st);
  if (e != hipSuccess) return e;
  g.A = n->h2; g.B = n->pb + OFF_W3; g.ldb = NOP; g.N = NOP; g.bias = n->p + OFF_B3;
  g.Cb = nullptr; g.Cf = n->o; g.ldc = NOP; g.relu = 0;
  return gemm(g, true, false, st);
}

extern "C" int mlp_forward(mlp_net* n, const uint16_t* x, int64_t rows, float* out,
                           void* stream) {
  if (!n) return set_error(SBLM_ESTATE, "mlp_forward: null network");
  if (rows < 0) return set_error(SBLM_EINVAL, "mlp_forward: rows < 0");
  if (rows == 0) return SBLM_OK;
  if (!x || !out) return set_error(SBLM_EINVAL, "mlp_forward: null x or out");
  hipStream_t st = (hipStream_t)stream;
  for (int64_t r0 = 0; r0 < rows; r0 += n->batch_max) {
    const int nr = (int)std::min<int64_t>(n->batch_max, rows - r0);
    const int nb = (nr + 63) / 64 * 64;
    hipError_t e = hipMemcpyAsync(n->xbuf, x + r0 * NB, (size_t)nr * NB * 2,
                                  hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && nb > nr) {
      hipLaunchKernelGGL(fill_u16_kernel, dim3(grid_for((int64_t)(nb - nr) * NB)), dim3(256),
                         0, st, n->xbuf + (int64_t)nr * NB, (int64_t)(nb - nr) * NB);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = forward_rows(n, n->xbuf, nb, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(out + r0 * NOP, n->o, (size_t)nr * NOP * 4,
                         hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return check_hip(e, "mlp_forward");
  }
  return SBLM_OK;
}

// K ranges of the weight-gradient products for a batch of `rows`: at least
// 128 rows each (more workgroups, shorter chains).
static int ksplit_for(int rows) {
  int ks = 1;
  while (ks < KSPLIT_MAX && rows % (64 * ks) == 0 && rows / (2 * ks) >= 128) ks *= 2;
  return ks;
}

// Loss and gradient of a batch.  fold: leave the weight gradients as split-K
// partials and the bias gradients and the loss as column-sum partials (all
// summed by adam_graph_kernel) instead of reducing them here.
static hipError_t loss_grad(mlp_net* n, const uint16_t* x, const float* y, int rows,
                            float* loss, hipStream_t st, bool fold = false) {
  hipError_t e = forward_rows(n, x, rows, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_nll_kernel, dim3((rows * 8 + 255) / 256), dim3(256), 0, st, n->o, y,
                     rows, n->dof, n->dob, n->lrow);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  // dZ2 = (dO W3^T) * [H2 > 0]
  g.A = n->dob; g.lda = NOP; g.B = n->pb + OFF_W3; g.ldb = NOP;
  g.M = rows; g.N = NH; g.K = NOP; g.mask = n->h2; g.ldm = NH;
  g.Cf = n->dz2f; g.Cb = n->dz2b; g.ldc = NH;
  if ((e = gemm(g, true, true, st)) != hipSuccess) return e;
  // dZ1 = (dZ2 W2^T) * [H1 > 0]
  g.A = n->dz2b; g.lda = NH; g.B = n->pb + OFF_W2; g.ldb = NH; g.K = NH;
  g.mask = n->h1; g.Cf = n->dz1f; g.Cb = n->dz1b;
  if ((e = gemm(g, true, true, st)) != hipSuccess) return e;
  // weight gradients: gW = (layer input)^T dZ, a contraction over the batch,
  // cut into K ranges of at least 128 rows (more workgroups, shorter chains)
  const int ks = ksplit_for(rows);
  struct { const uint16_t* A; int64_t lda; const uint16_t* B; int64_t ldb; int M, N;
           float* out; float* part; } wg[3] = {
      {n->h2, NH, n->dob, NOP, NH, NOP, n->g + OFF_W3, n->kpart + KPART_W3},
      {n->h1, NH, n->dz2b, NH, NH, NH, n->g + OFF_W2, n->kpart + KPART_W2},
      {x, NB, n->dz1b, NH, NB, NH, n->g + OFF_W1, n->kpart + KPART_W1}};
  // the three products in one launch (independent once dZ1 is known)
  GemmArgs gw[3];
  for (int i = 0; i < 3; ++i) {
    memset(&gw[i], 0, sizeof(gw[i]));
    gw[i].A = wg[i].A; gw[i].lda = wg[i].lda; gw[i].B = wg[i].B; gw[i].ldb = wg[i].ldb;
    gw[i].M = wg[i].M; gw[i].N = wg[i].N; gw[i].K = rows; gw[i].ldc = wg[i].N;
    gw[i].ksplit = ks;
    gw[i].Cf = ks > 1 ? wg[i].part : wg[i].out;
  }
  if ((e = gemm_group(gw, 3, false, false, st)) != hipSuccess) return e;
  for (int i = 0; i < 3; ++i) {
    const GemmArgs& g = gw[i];
    if (ks > 1 && !fold) {
      const int64_t mn = (int64_t)g.M * g.N;
      hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid_for(mn)), dim3(256), 0, st,
                         wg[i].part, ks, mn, wg[i].out);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  // bias gradients and the loss
  ColSegs cs;
  memset(&cs, 0, sizeof(cs));
  cs.s[0] = {n->dof, NOP, NOP, n->g + OFF_B3};
  cs.s[1] = {n->dz2f, NH, NH, n->g + OFF_B2};
  cs.s[2] = {n->dz1f, NH, NH, n->g + OFF_B1};
  cs.s[3] = {n->lrow, 1, 1, loss ? loss : n->cpart};  // unused slot when no loss
  cs.nseg = loss ? 4 : 3;
  cs.nrow = rows;
  return colsums(cs, n->cpart, st, !fold);
}

extern "C" int mlp_loss_grad(mlp_net* n, const uint16_t* x, const float* y, int32_t rows,
                             float* loss, void* stream) {
  if (!n) return set_error(SBLM_ESTATE, "mlp_loss_grad: null network");
  if (!x || !y) return set_error(SBLM_EINVAL, "mlp_loss_grad: null x or y");
  if (rows < 64 || rows % 64 != 0 || rows > n->batch_max)
    return set_error(SBLM_EINVAL,
                     "mlp_loss_grad: rows = %d must be a multiple of 64 in [64, %d]", rows,
                     n->batch_max);
  return check_hip(loss_grad(n, x, y, rows, loss, (hipStream_t)stream), "mlp_loss_grad");
}

static hipError_t adam(mlp_net* n, float lr, hipStream_t st) {
  const double b1 = 0.9, b2 = 0.999;
  n->step += 1;
  const double c1 = 1.0 / (1.0 - pow(b1, (double)n->step));
  const double c2 = 1.0 / (1.0 - pow(b2, (double)n->step));
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(NP_DEV)), dim3(256), 0, st, n->p, n->g,
                     n->m, n->v, n->pb, NP_DEV, lr, (float)b1, (float)b2,
                     (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, (float)c1, (float)c2);
  return hipGetLastError();
}

extern "C" int mlp_adam_step(mlp_net* n, float lr, void* stream) {
  if (!n) return set_error(SBLM_ESTATE, "mlp_adam_step: null network");
  if (!(lr >= 0.0f)) return set_error(SBLM_EINVAL, "mlp_adam_step: lr must be >= 0");
  return check_hip(adam(n, lr, (hipStream_t)stream), "mlp_adam_step");
}

// The captured training step: batch gather, forward, likelihood, backward,
// Adam with the split-K and column sums, the loss and the step advance.
// Every pointer it holds belongs
// to the net (the caller's data is read through the gather node), so one
// graph serves every step of a call and later calls with the same shape.
static hipError_t capture_train(mlp_net* n, const uint16_t* x, const float* y, int64_t per,
                                int batch) {
  hipStream_t w = n->work;
  const int ks = ksplit_for(batch);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(w, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const int64_t nx = (int64_t)batch * NB / 8 + (int64_t)batch * DM;
  hipLaunchKernelGGL(batch_gather_kernel, dim3(grid_for(nx)), dim3(256), 0, w, x, y, per, batch,
                     n->dstep, n->xbuf, n->ybuf);
  e = hipGetLastError();
  float* loss_slot = n->cpart + (int64_t)CS_RC * COLS_ALL;
  if (e == hipSuccess) e = loss_grad(n, n->xbuf, n->ybuf, batch, loss_slot, w, true);
  if (e == hipSuccess) {
    const double b1 = 0.9, b2 = 0.999;
    KParts kp;
    kp.part[0] = n->kpart + KPART_W3;
    kp.part[1] = n->kpart + KPART_W2;
    kp.part[2] = n->kpart + KPART_W1;
    kp.off[0] = OFF_W3;
    kp.off[1] = OFF_W2;
    kp.off[2] = OFF_W1;
    kp.mn[0] = (int64_t)NH * NOP;
    kp.mn[1] = (int64_t)NH * NH;
    kp.mn[2] = (int64_t)NB * NH;
    kp.ks = ks;
    // the column sums' partials as loss_grad left them (b3, b2, b1, loss)
    CParts cp;
    cp.part = n->cpart;
    cp.ncol_all = COLS_ALL;
    cp.off[0] = OFF_B3;
    cp.off[1] = OFF_B2;
    cp.off[2] = OFF_B1;
    cp.ncol[0] = NOP;
    cp.ncol[1] = NH;
    cp.ncol[2] = NH;
    cp.col0[0] = 0;
    cp.col0[1] = NOP;
    cp.col0[2] = NOP + NH;
    cp.loss_col = NOP + 2 * NH;
    hipLaunchKernelGGL(adam_graph_kernel, dim3(grid_for(NP_DEV)), dim3(256), 0, w, n->p, n->g,
                       n->m, n->v, n->pb, NP_DEV, n->sched, n->dstep, kp, cp, (float)b1,
                       (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f);
    e = hipGetLastError();
    if (e == hipSuccess) {
      hipLaunchKernelGGL(step_advance_kernel, dim3(1), dim3(1), 0, w, n->dstep, cp, n->losses);
      e = hipGetLastError();
    }
  }
  const hipError_t e_end = hipStreamEndCapture(w, &graph);
  if (e == hipSuccess) e = e_end;
  if (e == hipSuccess) {
    if (n->train_exec) (void)hipGraphExecDestroy(n->train_exec);
    n->train_exec = nullptr;
    e = hipGraphInstantiate(&n->train_exec, graph, nullptr, nullptr, 0);
  }
  if (graph) (void)hipGraphDestroy(graph);
  return e;
}

extern "C" int mlp_train(mlp_net* n, const uint16_t* x, const float* y, int64_t rows,
                         int32_t batch, int32_t epochs, float lr0, float lr1,
                         float* loss, void* stream) {
  if (!n) return set_error(SBLM_ESTATE, "mlp_train: null network");
  if (!x || !y) return set_error(SBLM_EINVAL, "mlp_train: null x or y");
  if (batch < 64 || batch % 64 != 0 || batch > n->batch_max)
    return set_error(SBLM_EINVAL, "mlp_train: batch = %d must be a multiple of 64 in [64, %d]",
                     batch, n->batch_max);
  if (epochs < 0 || rows < batch)
    return set_error(SBLM_EINVAL, "mlp_train: epochs = %d, rows = %lld (< batch?)", epochs,
                     (long long)rows);
  if (!(lr0 >= 0.0f) || !(lr1 >= 0.0f))
    return set_error(SBLM_EINVAL, "mlp_train: learning rates must be >= 0");
  const int64_t per = rows / batch;
  const int64_t total = per * epochs;
  if (total > ((int64_t)1 << 31))
    return set_error(SBLM_ERANGE, "mlp_train: %lld steps beyond 2^31", (long long)total);
  if (total == 0) return SBLM_OK;
  hipStream_t st = (hipStream_t)stream;
  // the step schedule on the host, as mlp_adam_step computes it: cosine
  // learning rate, bias corrections of step t = (steps so far) + k + 1
  float* sched_h = (float*)malloc((size_t)total * 3 * sizeof(float));
  if (!sched_h) return set_error(SBLM_ENOMEM, "mlp_train: host allocation");
  const double b1 = 0.9, b2 = 0.999;
  for (int64_t k = 0; k < total; ++k) {
    const double fr = total > 1 ? (double)k / (double)(total - 1) : 0.0;
    const double t = (double)(n->step + k + 1);
    sched_h[3 * k] = (float)(lr1 + 0.5 * (lr0 - lr1) * (1.0 + cos(M_PI * fr)));
    sched_h[3 * k + 1] = (float)(1.0 / (1.0 - pow(b1, t)));
    sched_h[3 * k + 2] = (float)(1.0 / (1.0 - pow(b2, t)));
  }
  int rc = SBLM_OK;
  // the net's work stream follows the caller's
  rc = check_hip(hipEventRecord(n->ev_in, st), "mlp_train: event");
  if (!rc) rc = check_hip(hipStreamWaitEvent(n->work, n->ev_in, 0), "mlp_train: wait");
  if (!rc && total > n->sched_cap) {
    // larger step buffers: the graph holds the old ones, so it is captured again
    rc = check_hip(hipStreamSynchronize(n->work), "mlp_train: synchronise");
    if (!rc) {
      if (n->sched) (void)hipFree(n->sched);
      if (n->losses) (void)hipFree(n->losses);
      n->sched = nullptr;
      n->losses = nullptr;
      n->sched_cap = 0;
      if (hipMalloc(&n->sched, (size_t)total * 3 * sizeof(float)) != hipSuccess ||
          hipMalloc(&n->losses, (size_t)total * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        rc = set_error(SBLM_ENOMEM, "mlp_train: device allocation");
      } else {
        n->sched_cap = total;
      }
    }
  }
  if (!rc)
    rc = check_hip(hipMemcpy(n->sched, sched_h, (size_t)total * 3 * sizeof(float),
                             hipMemcpyHostToDevice),
                   "mlp_train: schedule");
  free(sched_h);
  const int64_t key[4] = {batch, (int64_t)(uintptr_t)x ^ ((int64_t)(uintptr_t)y << 1), per,
                          (int64_t)(uintptr_t)n->sched};
  if (!rc && (!n->train_exec || memcmp(key, n->train_key, sizeof(key)) != 0)) {
    rc = check_hip(capture_train(n, x, y, per, batch), "mlp_train: capture");
    if (!rc) memcpy(n->train_key, key, sizeof(key));
  }
  // the step counter restarts at 0 (outside the graph)
  if (!rc) rc = check_hip(hipMemsetAsync(n->dstep, 0, 8, n->work), "mlp_train: counter");
  for (int64_t k = 0; !rc && k < total; ++k)
    rc = check_hip(hipGraphLaunch(n->train_exec, n->work), "mlp_train: step");
  if (!rc && loss)
    rc = check_hip(hipMemcpyAsync(loss, n->losses, (size_t)total * sizeof(float),
                                  hipMemcpyDeviceToDevice, n->work),
                   "mlp_train: losses");
  if (!rc) n->step += total;
  if (!rc) rc = check_hip(hipEventRecord(n->ev_out, n->work), "mlp_train: event");
  if (!rc) rc = check_hip(hipStreamWaitEvent(st, n->ev_out, 0), "mlp_train: wait");
  return rc;
}

// ---------------------------------------------------------- resampling

extern "C" int sblm_resample(const sblm_lcs* lcs, float* xf, uint16_t* xb, void* stream) {
  if (!lcs || !lcs->off || !lcs->t || !lcs->y || !lcs->w)
    return set_error(SBLM_EINVAL, "sblm_resample: null lightcurve descriptor or array");
  if (lcs->n_lc < 1) return set_error(SBLM_EINVAL, "sblm_resample: n_lc < 1");
  if (lcs->n_lc > (1 << 24)) return set_error(SBLM_ERANGE, "sblm_resample: n_lc beyond 2^24");
  if (!xf && !xb) return set_error(SBLM_EINVAL, "sblm_resample: no output");
  hipLaunchKernelGGL(resample_kernel, dim3(lcs->n_lc), dim3(NB), 0, (hipStream_t)stream,
                     lcs->off, lcs->t, lcs->y, lcs->w, xf, xb);
  return check_hip(hipGetLastError(), "sblm_resample launch");
}

extern "C" int mlp_make_data(uint64_t seed, int64_t first, int64_t n, uint16_t* xb,
                             float* xf, float* y, void* stream) {
  if (n < 0 || first < 0) return set_error(SBLM_EINVAL, "mlp_make_data: negative range");
  if (n == 0) return SBLM_OK;
  if (!y || (!xb && !xf)) return set_error(SBLM_EINVAL, "mlp_make_data: null output");
  if (n > (1LL << 26)) return set_error(SBLM_ERANGE, "mlp_make_data: n beyond 2^26");
  hipStream_t st = (hipStream_t)stream;
  const int64_t chunk = std::min<int64_t>(n, 1 << 16);
  double *theta = nullptr, *aux = nullptr, *A = nullptr, *u = nullptr;
  bool ok = hipMalloc(&theta, (size_t)chunk * 6 * 8) == hipSuccess &&
            hipMalloc(&aux, (size_t)chunk * NAUX * 8) == hipSuccess &&
            hipMalloc(&A, (size_t)chunk * NB * 8) == hipSuccess &&
            hipMalloc(&u, NB * 8) == hipSuccess;
  int rc = SBLM_OK;
  if (!ok) {
    (void)hipGetLastError();
    rc = set_error(SBLM_ENOMEM, "mlp_make_data: device allocation");
  }
  if (rc == SBLM_OK) {
    hipLaunchKernelGGL(bin_centres_kernel, dim3(1), dim3(NB), 0, st, u);
    rc = check_hip(hipGetLastError(), "mlp_make_data: launch");
  }
  for (int64_t s0 = 0; rc == SBLM_OK && s0 < n; s0 += chunk) {
    const int nc = (int)std::min<int64_t>(chunk, n - s0);
    hipLaunchKernelGGL(data_draw_kernel, dim3((nc + 255) / 256), dim3(256), 0, st, seed,
                       first + s0, nc, theta, aux, y + s0 * DM);
    rc = check_hip(hipGetLastError(), "mlp_make_data: draw launch");
    if (rc == SBLM_OK) rc = sblm_magnify(theta, nc, u, NB, SBLM_FP64, A, nullptr, nullptr, st);
    if (rc == SBLM_OK) {
      hipLaunchKernelGGL(data_finish_kernel, dim3(nc), dim3(NB), 0, st, seed, first + s0,
                         aux, A, xf ? xf + s0 * NB : nullptr, xb ? xb + s0 * NB : nullptr);
      rc = check_hip(hipGetLastError(), "mlp_make_data: finish launch");
    }
  }
  // the temporaries are released once the queued work has used them
  if (hipStreamSynchronize(st) != hipSuccess && rc == SBLM_OK)
    rc = check_hip(hipGetLastError(), "mlp_make_data: synchronise");
  if (theta) (void)hipFree(theta);
  if (aux) (void)hipFree(aux);
  if (A) (void)hipFree(A);
  if (u) (void)hipFree(u);
  return rc;
}

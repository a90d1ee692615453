// sblm_internal.h -- declarations shared by the library's translation units
// (kernels and host entry points).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sblm.h"

namespace sblm {

// Thread-local last-error message; returns `code` for convenient chaining.
int set_error(int code, const char* fmt, ...);
int check_hip(hipError_t e, const char* what);

// Arguments of the batched fitness kernels (one wave per individual).
struct FitArgs {
  // population: theta[j * n_ind + i] decoded, or encoded P with lo/hi
  const double* theta;
  int64_t n_ind;
  int32_t encoded;
  double lo[SBLM_NPAR], span[SBLM_NPAR];
  // epochs: either shared (off == nullptr, n_t epochs of t) or CSR per
  // lightcurve (individual i uses lightcurve i / pop)
  const int64_t* off;
  int32_t pop;
  const double* t;
  const double* y;
  const double* w;
  int64_t n_t;
  // outputs
  double* A;        // [n_ind][n_t] (magnify)
  int8_t* n_img;    // nullable (magnify)
  double* chi2;     // [n_ind] (chi2)
  double* Fs;
  double* Fb;
  sblm_stats* stats;  // nullable
  // schedule
  const int32_t* order;  // nullable: item -> individual permutation
  double* root_cache;     // nullable, G >= 64 only: [n_ind][G][10] roots of
                          // each lane's first epoch, read as its start
                          // (when finite) and rewritten after the solve
  const int32_t* cold;    // nullable (with root_cache): individual i ignores
                          // the cache when cold[i / cold_per] != 0
  int64_t cold_per;
  int32_t lanes_per_ind;  // 64, 32, 16 or 8 (a power of two dividing 64), or
                          // 128 / 256: several waves per individual (one-shot
                          // lockstep, wpb a multiple of G/64)
  unsigned int* queue;    // nullable: persistent launch; one shared work
                          // counter, or with xcd_start one per XCD (8)
  const int64_t* xcd_start;  // nullable: [9] order positions; the items at
                             // [xcd_start[x], xcd_start[x+1]) belong to XCD x
                          // (must read 0 when the kernel starts)
  int32_t async;          // 1: lanes step through their epochs independently
  const int32_t* skip;    // nullable (CSR only): individual i is evaluated
  int32_t skip_per;       // as empty when skip[i / skip_per] != 0
};

// Launch the FP64 or mixed fitness kernel; chi2 = false writes A/n_img.
// Lanes per individual for a launch of n_ind individuals: the fewest of 8,
// 16, 32, 64 that give the launch 2^20 lanes of work (fewer lanes, longer
// chains of warm-started epochs per lane, fewer cold starts); a launch whose
// 64-lane groups would not fill one residency of the chip (2^17 lanes: 256
// compute units x 8 waves) takes the widest group, up to 256 lanes over
// several waves, that fits one.
inline int default_lanes(int64_t n_ind) {
  constexpr int64_t RESIDENT = 2048 * 64;
  if (n_ind * 64 <= RESIDENT) {
    int g = 64;
    while (g < 256 && n_ind * (2 * g) <= RESIDENT) g *= 2;
    return g;
  }
  for (int g = 8; g < 64; g *= 2)
    if (n_ind * g >= 8 * RESIDENT) return g;
  return 64;
}

hipError_t launch_fitness(const FitArgs& a, int mode, bool chi2,
                          hipStream_t stream, int waves_per_block);

// Batched downhill-simplex refinement (sblm_nm.hip): one simplex per
// lightcurve from x0 [6][n_lc] (encoded with lo/span); results as for
// nm_refine.  Allocates and frees its workspace; synchronises `st`.
// Iterated simplex (nm_iterated): `runs` random starts per slot and where
// the best per lightcurve goes.
struct NmIterated {
  uint64_t seed;
  int32_t runs;
  double* x;
  double* chi2;
  double* Fs;
  double* Fb;
  int64_t* n_iter;
};
// One simplex per (lightcurve, rep) from x0, or with `iter` the iterated
// form from drawn starts (x0 and the per-simplex outputs unused).
// `workspace` (nullable): a device block of nm_work_bytes(n_lc * reps) bytes
// that replaces the allocation of the simplices' state; with it the trial
// points take 64 lanes and no root cache, and nothing is allocated.
int nm_run(const sblm_lcs& lcs, int32_t reps, const double* lo, const double* span,
           const double* x0, const nm_config& cfg, double* x, double* chi2, double* Fs,
           double* Fb, int32_t* n_iter, sblm_stats* stats, hipStream_t st,
           const NmIterated* iter = nullptr, void* workspace = nullptr);
size_t nm_work_bytes(int64_t n_simplices);
int nm_check(const nm_config* cfg, const char* who);

}  // namespace sblm

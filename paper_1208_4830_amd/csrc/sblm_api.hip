// sblm_api.hip -- host entry points of the fitness part of the C ABI
// (sblm_magnify, sblm_chi2, sblm_last_error): argument checks, schedule
// choice and kernel launch.  The kernels are in sblm_fitness.hip.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sblm_internal.h"

namespace sblm {

static thread_local char g_err[512] = "";

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return SBLM_OK;
  return set_error(SBLM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Lanes per individual of the stateless calls: the rule of the EA states
// (default_lanes), so that sblm_chi2 of a population equals the state's own
// evaluation bit for bit.  Overridable with SBLM_LANES (8 ... 256) for tuning
// runs.
static int choose_group(int64_t n_ind) {
  const char* env = getenv("SBLM_LANES");
  if (env) {
    int g = atoi(env);
    if (g == 8 || g == 16 || g == 32 || g == 64 || g == 128 || g == 256) return g;
  }
  return default_lanes(n_ind);
}


// Epoch stepping of the stateless calls: lockstep unless SBLM_ASYNC=1 (the
// asynchronous form measured slower on the MI355X for 200-5000-epoch
// lightcurves: 6.8 vs 4.6 ms per batched evaluation).
static int async_stepping() {
  const char* env = getenv("SBLM_ASYNC");
  return (env && atoi(env) == 1) ? 1 : 0;
}

static int waves_per_block() {
  const char* env = getenv("SBLM_WAVES_PER_BLOCK");
  if (env) {
    int w = atoi(env);
    if (w == 1 || w == 2 || w == 4) return w;  // blocks of <= 256 threads
  }
  return 4;
}

// Waves per block for a group of g lanes (several waves per individual need
// whole individuals in a block).
static int block_waves(int g) { return g > 64 ? 4 : waves_per_block(); }

}  // namespace sblm

using namespace sblm;

extern "C" const char* sblm_last_error(void) { return g_err; }

extern "C" int sblm_magnify(const double* theta, int64_t n, const double* t,
                            int64_t n_t, int mode, double* A, int8_t* n_img,
                            sblm_stats* stats, void* stream) {
  if (mode != SBLM_FP64 && mode != SBLM_MIXED)
    return set_error(SBLM_EINVAL, "sblm_magnify: unknown mode %d", mode);
  if (n < 1) return set_error(SBLM_EINVAL, "sblm_magnify: n = %lld < 1", (long long)n);
  if (n_t < 0) return set_error(SBLM_EINVAL, "sblm_magnify: n_t < 0");
  if (n > (1LL << 26) || n_t > (1LL << 24))
    return set_error(SBLM_ERANGE, "sblm_magnify: n = %lld or n_t = %lld beyond limits",
                     (long long)n, (long long)n_t);
  if (n_t == 0) return SBLM_OK;
  if (!theta || !t || !A)
    return set_error(SBLM_EINVAL, "sblm_magnify: null theta, t or A");
  FitArgs a;
  memset(&a, 0, sizeof(a));
  a.theta = theta;
  a.n_ind = n;
  a.t = t;
  a.n_t = n_t;
  a.A = A;
  a.n_img = n_img;
  a.stats = stats;
  a.lanes_per_ind = choose_group(n);
  a.async = async_stepping() && a.lanes_per_ind <= 64;
  return check_hip(launch_fitness(a, mode, false, (hipStream_t)stream,
                                  block_waves(a.lanes_per_ind)),
                   "sblm_magnify launch");
}

extern "C" int sblm_chi2(const sblm_lcs* lcs, const double* theta, int32_t pop,
                         int mode, double* chi2, double* Fs, double* Fb,
                         sblm_stats* stats, void* stream) {
  if (mode != SBLM_FP64 && mode != SBLM_MIXED)
    return set_error(SBLM_EINVAL, "sblm_chi2: unknown mode %d", mode);
  if (!lcs || !lcs->off || !lcs->t || !lcs->y || !lcs->w)
    return set_error(SBLM_EINVAL, "sblm_chi2: null lightcurve descriptor or array");
  if (lcs->n_lc < 1 || pop < 1)
    return set_error(SBLM_EINVAL, "sblm_chi2: n_lc = %d, pop = %d", lcs->n_lc, pop);
  if (lcs->n_lc > (1 << 20) || pop > 65536 || (int64_t)lcs->n_lc * pop > (1LL << 31) - 1)
    return set_error(SBLM_ERANGE, "sblm_chi2: n_lc = %d, pop = %d beyond limits",
                     lcs->n_lc, pop);
  if (!theta || !chi2 || !Fs || !Fb)
    return set_error(SBLM_EINVAL, "sblm_chi2: null theta or output");
  FitArgs a;
  memset(&a, 0, sizeof(a));
  a.theta = theta;
  a.n_ind = (int64_t)lcs->n_lc * pop;
  a.off = lcs->off;
  a.pop = pop;
  a.t = lcs->t;
  a.y = lcs->y;
  a.w = lcs->w;
  a.chi2 = chi2;
  a.Fs = Fs;
  a.Fb = Fb;
  a.stats = stats;
  a.lanes_per_ind = choose_group(a.n_ind);
  a.async = async_stepping() && a.lanes_per_ind <= 64;
  return check_hip(launch_fitness(a, mode, true, (hipStream_t)stream,
                                  block_waves(a.lanes_per_ind)),
                   "sblm_chi2 launch");
}

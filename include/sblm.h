/*
 * sblm.h -- C ABI of libsblm: batched fitness evaluation and evolutionary
 * fitting of static binary-lens (SBLM) point-source microlensing lightcurves
 * on AMD Instinct MI355X (gfx950).
 *
 * The operations follow Rajpaul (2012), "Evolutionary algorithm-based
 * analysis of gravitational microlensing lightcurves":
 *   - forward model: source trajectory (Sec. 2.2, Eq. sourcePos and the
 *     dimensionless time tau), the binary lens equation (Eq. lensing), its
 *     fifth-order complex polynomial form (Eq. lensingPoly), rejection of the
 *     two spurious roots by substitution into the lens equation, and the
 *     magnification A = sum_i 1/|det J_i| (Sec. 2.2, per-image amplification);
 *   - fitness: chi^2 (Sec. 4.1) of the blended flux model F = Fs*A + Fb
 *     (Sec. 4.4, Eq. blend, with Fs and Fb obtained by linear least squares);
 *   - optimiser: the array-style evolutionary algorithm of Appendix A
 *     (initialisation A.1, encoding A.2, ranking A.3, tournament selection
 *     A.4, reproduction with elitism A.5, creep and jump mutation A.6,
 *     stagnation handling and restarts A.7).
 *
 * Conventions shared by every entry point
 *   - Parameter vector theta (decoded, physical), always stored as six
 *     contiguous planes (structure of arrays), plane j holding parameter j of
 *     every individual:
 *        j = 0  log10 q   mass ratio secondary/primary, q = 10^(log10 q)
 *        j = 1  d         lens separation (paper's a), primary-theta_E units
 *        j = 2  u0        impact parameter (paper's b) w.r.t. the primary
 *        j = 3  alpha     trajectory angle (paper's theta), radians
 *        j = 4  tE        Einstein crossing time, days
 *        j = 5  t0        time of closest approach to the primary (paper's
 *                         t_m), days
 *     Origin at the primary lens, secondary on the +x axis at z = d.
 *   - All array arguments are DEVICE pointers on the current HIP device
 *     unless stated otherwise; the caller owns them and keeps them alive
 *     until the work queued on `stream` has completed.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Every call only enqueues work and returns; results are valid once the
 *     stream has been synchronised.
 *   - Every call returns an sblm_status.  Argument errors are detected on the
 *     host before anything is launched; nothing aborts or throws across the
 *     ABI.  sblm_last_error() returns a thread-local message describing the
 *     last failure of the calling thread.
 *   - Numerical events (a degree drop of the lens polynomial, an iteration
 *     cap reached, a degenerate least-squares system, NaN fitness) are not
 *     errors; they are counted in the optional sblm_stats block.
 */
#ifndef SBLM_H
#define SBLM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SBLM_OK = 0,
  SBLM_EINVAL = -1,  /* bad argument (null pointer, size out of range)     */
  SBLM_EDEVICE = -2, /* a HIP runtime call or kernel launch failed          */
  SBLM_ENOMEM = -3,  /* device allocation failed (ea_create only)           */
  SBLM_ESTATE = -4,  /* state object invalid or snapshot does not match     */
  SBLM_ERANGE = -5   /* size beyond a documented limit                      */
} sblm_status;

typedef enum {
  SBLM_FP64 = 0,  /* root solve, polish, image test, det J and chi^2 in FP64 */
  SBLM_MIXED = 1  /* root iteration in FP32, then at most two FP64 Newton
                     steps per root (FP64 sweeps only where those do not
                     converge); image test, det J and chi^2 in FP64       */
} sblm_mode;

#define SBLM_NPAR 6

/* Device-side counters of numerical events, accumulated (not reset) by every
 * call that receives a non-NULL pointer.  64-bit device integers. */
typedef struct {
  unsigned long long n_solves;     /* polynomials solved                      */
  unsigned long long n_iter;       /* simultaneous-iteration sweeps, summed   */
  unsigned long long n_capped;     /* solves that reached the iteration cap,
                                      also after the cold retry (see
                                      n_unsettled)                          */
  unsigned long long n_fallback;   /* MIXED: solves whose FP32 roots were not
                                      polished to the FP64 tolerance by two
                                      Newton steps and went on to FP64
                                      simultaneous-iteration sweeps           */
  unsigned long long n_degree4;    /* leading coefficient negligible          */
  unsigned long long n_degenerate; /* chi^2 fits with a singular 2x2 system   */
  unsigned long long n_wave_iter;  /* sweeps the wavefront executed, summed
                                      over the solves of its lanes (lockstep
                                      cost; n_iter is the lanes' own need)    */
  unsigned long long n_iter_fp32;  /* MIXED: the FP32 part of n_iter          */
  unsigned long long n_polished;   /* images refined on the lens equation     */
  unsigned long long n_retried;    /* warm-started solves that failed and were
                                      solved again from the cold start        */
  unsigned long long n_unsettled;  /* capped solves whose roots were not finite
                                      or still moved by more than 1e-4
                                      relative in the last sweep: their
                                      magnification is NaN (n_img 0), and so
                                      is the chi^2 they enter (it ranks last);
                                      the other capped solves have stalled at
                                      the rounding level next to merging
                                      images (a fold or a cusp of the
                                      caustic), and their images are refined
                                      on the lens equation                    */
  unsigned long long n_newton;     /* MIXED: FP64 Newton polish passes over the
                                      five roots, summed                      */
} sblm_stats;

/* Ragged batch of lightcurves in CSR form.  Lightcurve k owns epochs
 * [off[k], off[k+1]) of t, y and w.  off is a DEVICE array of n_lc+1
 * non-decreasing int64 values with off[0] = 0; t in days, y the observed
 * flux, w = 1/sigma^2 the statistical weight (w >= 0). */
typedef struct {
  int32_t n_lc;
  const int64_t* off;
  const double* t;
  const double* y;
  const double* w;
} sblm_lcs;

/*
 * sblm_magnify -- magnification of every (individual, epoch) pair.
 * Defines: Sec. 2.2 (Eq. sourcePos, tau, Eq. lensing, Eq. lensingPoly, the
 * spurious-root elimination and the per-image amplification, with det J
 * = 1 - |1/conj(z)^2 + q/(d - conj(z))^2|^2).
 *   theta  [6][n]      decoded parameters (layout above)
 *   n      individuals, 1 <= n <= 2^26
 *   t      [n_t]       epochs (days), shared by all individuals
 *   n_t    epochs, 0 <= n_t <= 2^24 (n_t = 0 is a no-op)
 *   mode   SBLM_FP64 or SBLM_MIXED
 *   A      [n][n_t]    out: total magnification of the accepted images
 *   n_img  [n][n_t]    out (nullable): accepted image count, 3 or 5
 *   stats  (nullable)  device counters, see sblm_stats
 * Errors: SBLM_EINVAL for null theta/t/A with n_t > 0, n < 1 or a bad mode;
 * SBLM_ERANGE for sizes beyond the limits; SBLM_EDEVICE on launch failure.
 */
int sblm_magnify(const double* theta, int64_t n, const double* t, int64_t n_t,
                 int mode, double* A, int8_t* n_img, sblm_stats* stats,
                 void* stream);

/*
 * sblm_chi2 -- fitness of a population against a ragged batch.
 * Defines: Sec. 4.1 (chi^2 minimisation) with the blend model of Sec. 4.4
 * (Eq. blend) written in flux, F_k = Fs*A_k + Fb, Fs and Fb profiled by the
 * weighted linear least-squares solution for every individual:
 *     chi2 = min_{Fs,Fb} sum_k w_k (y_k - Fs*A_k - Fb)^2.
 * If the 2x2 normal matrix is singular to 1e-14 relative
 * (det <= 1e-14 * sum(wA^2) * sum(w)), the fit falls back to Fs = 0,
 * Fb = weighted mean of y.
 *   lcs    ragged lightcurves (device CSR, see sblm_lcs); 1 <= n_lc <= 2^20,
 *          every lightcurve at most 2^20 epochs
 *   theta  [6][n_lc*pop] decoded parameters; individual i is fitted to
 *          lightcurve i / pop
 *   pop    individuals per lightcurve, 1 <= pop <= 65536
 *   mode   SBLM_FP64 or SBLM_MIXED
 *   chi2, Fs, Fb  [n_lc*pop] out
 *   stats  (nullable)  device counters
 * An empty lightcurve gives chi2 = 0, Fs = 0, Fb = 0.
 * Errors: SBLM_EINVAL (null pointers, n_lc < 1, pop < 1, bad mode),
 * SBLM_ERANGE, SBLM_EDEVICE.
 */
int sblm_chi2(const sblm_lcs* lcs, const double* theta, int32_t pop, int mode,
              double* chi2, double* Fs, double* Fb, sblm_stats* stats,
              void* stream);

/* ---------------------------------------------------------------------- */
/* Evolutionary algorithm (Appendix A)                                     */
/* ---------------------------------------------------------------------- */

/* Random numbers.  Every random draw of the EA is one 64-bit word of the
 * Philox4x64-10 counter-based generator (Salmon, Moraes, Dror & Shaw 2011)
 * with key = (seed, lightcurve index) and counter = (generation, purpose,
 * row, j / 4), word j % 4.  Purposes: 1 initialisation (row = individual,
 * j = gene), 2 tournament (row = pairing, j = draw), 3 crossover mode and
 * weights (row = pairing, j = 0 mode, 1 + g weight of gene g), 4 creep
 * (row = offspring, j = 2g sign, 2g + 1 step), 5 jump (row = offspring,
 * j = 2g trigger, 2g + 1 new value).  A word x maps to the open unit
 * interval as ((x >> 12) + 0.5) * 2^-52 and to {0..n-1} as
 * ((x >> 32) * n) >> 32. */
#define EA_PURPOSE_INIT 1
#define EA_PURPOSE_TOURN 2
#define EA_PURPOSE_MODE 3
#define EA_PURPOSE_CREEP 4
#define EA_PURPOSE_JUMP 5
#define EA_PURPOSE_SEED 6 /* ea_seed: row = seeded row, j = draw (see there) */

typedef struct {
  int32_t pop;           /* N_pop, 2 <= pop <= 1024                        */
  int32_t n_tourn;       /* N_tourn; 0 selects ceil(pop / 25) (Sec. A.4)    */
  double p_mut0;         /* initial jump probability (Sec. A.6), e.g. 0.01 */
  double p_mut_min;      /* floor of the throttled probability             */
  double p_mut_max;      /* ceiling of the boosted probability             */
  double stag_frac;      /* relative improvement threshold (Sec. A.7), 0.01 */
  int32_t stag_window;   /* generations looked back (Sec. A.7), 10         */
  int32_t restart_after; /* consecutive stagnation flags before a restart  */
  double lo[SBLM_NPAR];  /* Omega_j = [lo_j, hi_j] (Sec. A.2)              */
  double hi[SBLM_NPAR];
  int32_t mode;          /* sblm_mode used by ea_fit's fitness evaluation  */
  /* Island form (Sec. 5.3): every lightcurve has n_islands populations of
   * pop rows that evolve independently and exchange their fittest rows.
   * Island i of lightcurve k is an Appendix-A EA of its own whose draws use
   * the lightcurve index k * n_islands + i (so n_islands = 1 is the plain
   * EA).  Migration, in ea_fit, before the generation step of generation g
   * (generations completed) when g > 0 and g % mig_every == 0: on a ring,
   * island i sends its n_migrants fittest rows (stable ascending chi^2, NaN
   * last) with their fitness to island (i + 1) % n_islands, where the r-th
   * fittest replaces the row of rank pop - 1 - r; all islands send from the
   * state before any receives.  The rows of lightcurve k are
   * [k * n_islands * pop, (k + 1) * n_islands * pop), island-major. */
  int32_t n_islands;     /* 1 <= n_islands <= 256                           */
  int32_t mig_every;     /* >= 0; 0 = never                                */
  int32_t n_migrants;    /* 0 <= n_migrants <= pop / 2; 0 = never           */
} ea_config;

/* Fills cfg with the defaults used by this library: pop 256, N_tourn =
 * ceil(pop/25), p_mut0 0.01, p_mut in [1e-4, 0.5], 1% over 10 generations,
 * restart after 10 consecutive flags, Omega = {log10 q in [-3,0], d in
 * [0.5,2], u0 in [0,0.5], alpha in [0,2pi], tE in [10,100], t0 in [-10,10]},
 * FP64 fitness, one island (no migration).  Host pointer. */
void ea_default_config(ea_config* cfg);

typedef struct ea_state ea_state; /* opaque */

/* Per-lightcurve summary, host-side copy (ea_summary).  With islands, every
 * field is that of the island holding the lightcurve's best chi^2 (the
 * lowest island index among equals). */
typedef struct {
  double best_chi2;      /* best chi^2 seen since ea_create (all restarts) */
  double best_Fs, best_Fb;
  double best_theta[SBLM_NPAR]; /* decoded parameters of that individual  */
  int64_t best_gen;      /* generation at which it was first seen         */
  double p_mut;          /* current jump probability                      */
  int32_t stag_count;    /* consecutive stagnation flags                  */
  int32_t n_restarts;
  int64_t gen;           /* generations completed                         */
  int64_t gen_restart;   /* first generation of the current sequence      */
} ea_lc_summary;

/*
 * ea_create -- allocate the device workspace of a fit of lcs->n_lc
 * independent lightcurves and initialise generation 0 (Sec. A.1: rows
 * i < pop/2 uniform, row i + pop/2 = 1 - row i, an odd last row uniform).
 *   cfg    host pointer, validated (pop range, lo < hi, 0 < p_mut, ...)
 *   lcs    host pointer to a descriptor of device CSR arrays; the arrays
 *          must stay alive and unchanged for the life of the state
 *   seed   64-bit seed (Philox key word 0)
 *   out    host pointer receiving the new state
 * With islands every island is initialised so, from its own draws.
 * n_lc * n_islands * pop <= 2^31 - 1.
 * The only entry point that allocates device memory.  Errors: SBLM_EINVAL,
 * SBLM_ERANGE, SBLM_ENOMEM, SBLM_EDEVICE.
 */
int ea_create(const ea_config* cfg, const sblm_lcs* lcs, uint64_t seed,
              ea_state** out);

/*
 * ea_generation -- one generation of Appendix A after the fitness of the
 * current population is known: rank (stable, NaN ranks last), update the
 * best-ever record, fill rows 1..pop-1 with offspring of tournament-selected
 * pairs (row 0 keeps the fittest individual), apply creep then jump mutation
 * to every offspring gene, then the stagnation test, the p_mut update and a
 * restart when the flags have repeated restart_after times.
 *   chi2, Fs, Fb  [n_lc*n_islands*pop] device, fitness of the current
 *          population in its current row order (as written by sblm_chi2 with
 *          n_islands*pop individuals per lightcurve, or by ea_evaluate)
 * Every island takes its own generation; no migration (see ea_migrate).
 * Errors: SBLM_EINVAL, SBLM_ESTATE, SBLM_EDEVICE.
 */
int ea_generation(ea_state* st, const double* chi2, const double* Fs,
                  const double* Fb, void* stream);

/* ea_evaluate -- decode the current population (Eq. EMMA-encoding) and
 * write its fitness into the state's own chi2/Fs/Fb buffers (the same
 * computation as sblm_chi2 in cfg->mode). */
int ea_evaluate(ea_state* st, sblm_stats* stats, void* stream);

/*
 * ea_fit -- run n_gen generations of the evolutionary loop of Appendix A
 * (evaluate the fitness of every individual, then rank, select, reproduce
 * and mutate, test for stagnation and restart, repeated generation after
 * generation), each = ea_evaluate + (when due, the migration of ea_config,
 * Sec. 5.3) + ea_generation on the state's own buffers, replayed from one
 * captured HIP graph.
 *   n_gen  >= 0; 0 only captures the graph (bound to `stats`) when it is
 *          not captured yet, so that a later timed call replays at once
 *   stats  nullable device pointer; accumulates the counters of every
 *          generation's fitness evaluation
 * Errors: SBLM_EINVAL, SBLM_ESTATE, SBLM_EDEVICE.
 */
int ea_fit(ea_state* st, int32_t n_gen, sblm_stats* stats, void* stream);

/*
 * ea_freeze -- stop or resume the EA of chosen lightcurves in a batch (for a
 * caller that has settled some fits and keeps evolving the rest; the paper's
 * loop of App. A runs per lightcurve, so the others are unaffected).
 *   mask  HOST int32[n_lc]: nonzero freezes lightcurve k, 0 lets it run
 *   n_lc  the mask's length, which must be the state's lightcurve count
 * A frozen lightcurve's population, records and generation counter stay as
 * they are: later generations skip its selection, offspring and migration,
 * and its fitness evaluations treat it as empty (its per-row chi2, Fs, Fb in
 * ea_buffers then read 0 until it runs again; ea_best and ea_records keep its
 * records).  Every other lightcurve evolves bit for bit as without the
 * freeze.  Copies the mask in order on `stream` and synchronises `stream`;
 * the mask is not part of ea_save's snapshot (ea_load leaves it as it is).
 * Errors: SBLM_ESTATE (null state), SBLM_EINVAL (null mask or another
 * length), SBLM_EDEVICE.
 */
int ea_freeze(ea_state* st, const int32_t* mask, int32_t n_lc, void* stream);

/*
 * ea_time_fitness -- instrumentation, not part of the method: with enable =
 * 1 every generation that ea_fit replays stamps the device's constant-rate
 * wall clock just before and just after its fitness kernel (two one-thread
 * kernels in the captured graph) and adds the interval to a sum in the
 * state; enable = 0 removes the stamps.  Either way the sum and the launch
 * count are cleared (in order on `stream`).  The interval includes the
 * dispatch gaps next to the kernel (microseconds against milliseconds).
 * ea_fitness_time -- the sum in milliseconds (host out *ms) and the number
 * of timed launches (host out *launches) since the last ea_time_fitness;
 * synchronises the state's work.  Errors: SBLM_EINVAL, SBLM_ESTATE,
 * SBLM_EDEVICE.
 */
int ea_time_fitness(ea_state* st, int32_t enable, void* stream);
int ea_fitness_time(ea_state* st, double* ms, int64_t* launches);

/*
 * ea_autotune -- choose the fitness schedule of this state by timing it on
 * the state's own population and lightcurves (coordinate descent over the
 * epoch stepping {asynchronous, lockstep}, waves per block {1, 2, 4} and a
 * persistent work-counter launch vs a one-shot grid; with 128 or 256 lanes
 * per individual only the waves per block that hold whole individuals, the
 * one-shot grid and lockstep stepping), starting from the current schedule
 * and moving only to a candidate more than 2% faster (so that repeated tuning
 * settles on the same choice despite timing jitter), then re-capture the
 * generation graph.  None of these knobs changes a result bit, so a tuned fit
 * is bit-identical to the untuned one.  The lanes per individual are not
 * tuned: each lane warm-starts the root solves along its own chunk of a
 * lightcurve's epochs, so their number decides where the chains of warm
 * starts begin (roots differ at the rounding level) and is part of the
 * fit's definition, set at ea_create (see ea_get_schedule).  `report`
 * (host, nullable) receives one line per candidate.  Synchronises `stream`.
 */
int ea_autotune(ea_state* st, char* report, size_t report_len, void* stream);

/*
 * ea_autotune_cached -- ea_autotune with a kept choice (App. A's fits are
 * run again and again on workloads of one shape).  `path` (host string)
 * names a text file of earlier choices, one line per device and workload:
 * a 64-bit key in hex (FNV-1a of the device's architecture and compute-unit
 * count and of the state's workload: precision form, population, islands,
 * lightcurve count, lanes per individual, and how many lightcurves have
 * floor(log2(L + 1)) = b for every b), then lanes, waves per block,
 * persistent, asynchronous, then the key's text.  A key found in the file
 * installs its schedule without timing (*tuned = 0, nullable); else the
 * state is tuned as by ea_autotune and a line appended (*tuned = 1).  A kept
 * schedule changes no result bit against the untuned one.  Lines that do
 * not parse are skipped.  Errors: those of ea_autotune and ea_set_schedule;
 * SBLM_ESTATE for a null state; SBLM_EINVAL for a null or empty path, a
 * file that cannot be appended, or an entry whose lanes differ from the
 * state's.  Calls that append to one file at once may interleave lines.
 */
int ea_autotune_cached(ea_state* st, const char* path, int32_t* tuned, char* report,
                       size_t report_len, void* stream);

/* Current schedule as int32[4] {lanes per individual, waves per block,
 * persistent, asynchronous stepping}; ea_set_schedule validates (lanes
 * 8/16/32/64, waves per block 1/2/4, persistent 0/1, asynchronous 0/1; or
 * lanes 128/256 with waves per block a multiple of lanes/64, one-shot,
 * lockstep; SBLM_EINVAL otherwise) and installs one (and re-captures the
 * graph).  Results depend on the lanes per individual only (see
 * ea_autotune).  ea_create starts from 4 waves per block, lockstep, the
 * persistent grid, and the fewest lanes in {8, 16, 32, 64} that give 2^20
 * lanes of work (n_ind x lanes >= 2^20, else 64); a state of at most 2048
 * individuals takes the widest lanes (up to 256, one-shot grid) with
 * n_ind x lanes <= 2^17, the lanes of one residency of the chip. */
int ea_get_schedule(ea_state* st, int32_t* sched);
int ea_set_schedule(ea_state* st, const int32_t* sched);

/*
 * ea_migrate -- one ring migration among the islands of every lightcurve
 * now, whatever the generation (the exchange that ea_fit makes when it is
 * due, Sec. 5.3 and ea_config): rows of the population and the matching
 * entries of chi2, Fs and Fb ([n_lc*n_islands*pop] device, modified in
 * place) are overwritten.  NULL fitness pointers select the state's own
 * buffers.  Errors: SBLM_ESTATE when the state has one island or no
 * migrants; SBLM_EINVAL when only some of the pointers are NULL.
 */
int ea_migrate(ea_state* st, double* chi2, double* Fs, double* Fb, void* stream);

/* Device pointers into the state (valid until ea_destroy):
 * P [6][n_lc*n_islands*pop] encoded population, chi2/Fs/Fb
 * [n_lc*n_islands*pop] the buffers ea_evaluate writes.  Any pointer argument
 * may be NULL. */
int ea_buffers(ea_state* st, double** P, double** chi2, double** Fs,
               double** Fb);

/* Copies the per-lightcurve summaries to host memory out[n_lc].
 * Synchronises `stream`. */
int ea_summary(ea_state* st, ea_lc_summary* out, void* stream);

/* ea_save -- snapshot of the whole state (config, seed, population and
 * per-lightcurve records: the best-ever solution that App. A.7 keeps across
 * restarts, p_mut, the stagnation counters and the history of best chi^2
 * the stagnation test reads) into host memory buf (caller-owned, *len
 * bytes).  With buf == NULL, *len receives the size; SBLM_EINVAL when *len
 * is too small.  Synchronises `stream`.
 * ea_load -- restore such a snapshot (host buf of len bytes) into a state
 * created with the same config, lightcurve count and seed (SBLM_ESTATE
 * otherwise, or for a short snapshot); the continued run is bit-identical
 * to an uninterrupted one, since every random draw is keyed by (seed,
 * lightcurve, generation) and not by the history of calls (App. A.7 resumes
 * from the saved record). */
int ea_save(ea_state* st, void* buf, size_t* len, void* stream);
int ea_load(ea_state* st, const void* buf, size_t len, void* stream);

void ea_destroy(ea_state* st);

/* ---------------------------------------------------------------------- */
/* Simplex fine-tuning ("EA with amoeba", Sec. 4.1, Tables 2-3)            */
/* ---------------------------------------------------------------------- */
/*
 * The downhill simplex of Nelder & Mead (1965) in the form of Lagarias,
 * Reeds, Wright & Wright (1998), which the paper applies to the fittest
 * solution of the EA.  One simplex per lightcurve, in the EA's encoded domain
 * [0, 1]^6 (Eq. EMMA-encoding), chi^2 as in sblm_chi2:
 *   - coefficients: reflection 1, expansion 2, contraction 1/2, shrink 1/2;
 *   - initial simplex: x0 (clipped) and, for k = 0..5, x0 with coordinate k
 *     multiplied by 1.05 (set to 0.00025 where it is 0), a value above 1
 *     reflected to 2 - value, then clipped to [0, 1];
 *   - every trial point (reflection, expansion, contractions, shrunk
 *     vertices) is clipped to [0, 1];
 *   - vertices are kept in ascending chi^2, equal values in their previous
 *     order (a new vertex after older equal ones); NaN counts as +inf;
 *   - before each step the run stops if every vertex lies within tol_x of
 *     the best in every coordinate and within tol_f of its chi^2, or after
 *     max_iter steps (a shrink counts as one step).
 */
typedef struct {
  double tol_x;     /* encoded units, default 1e-4                        */
  double tol_f;     /* chi^2 units, default 1e-4                          */
  int32_t max_iter; /* simplex steps, default 200 x 6 = 1200; <= 10^6     */
  int32_t mode;     /* sblm_mode of the fitness evaluations, default FP64 */
} nm_config;

void nm_default_config(nm_config* cfg);

/*
 * nm_refine -- refine one start point per lightcurve.
 *   lcs     ragged lightcurves (device CSR), 1 <= n_lc <= 2^24
 *   lo, hi  HOST double[6], the domain of the encoding (lo < hi)
 *   x0      [6][n_lc] device, encoded start points
 *   x       [6][n_lc] device out, best vertex (may alias x0)
 *   chi2, Fs, Fb  [n_lc] device out (nullable), its chi^2 and fluxes
 *   n_iter  [n_lc] device int32 out (nullable), simplex steps taken
 *   stats   (nullable) fitness counters
 * A round evaluates, per running simplex, its step's reflection (then, in
 * the next round, the one other point the step needs) while more than 256
 * simplices run, else all four points of a step at once; either way the
 * simplices are those of the sequential method.
 * Allocates and frees a workspace of ~1 KB per simplex, a work order of
 * 32 B per simplex, and saved roots of 80 B per lane: the trial points of a
 * round are spread over 64, 128 or 256 lanes each, the fewest that give
 * 2^19 lanes for the round's trial points (read every 16 rounds), each
 * width with its own saved roots (140 KB per simplex for the three; where
 * they would pass 1 GiB, one width: 256 lanes, else 128, else 64 without
 * saved roots).  The widths and the form of a round change results at the
 * rounding level only, and are a function of the simplices, so calls are
 * repeatable.  Synchronises `stream`.
 * Errors: SBLM_EINVAL, SBLM_ERANGE, SBLM_ENOMEM, SBLM_EDEVICE.
 */
int nm_refine(const sblm_lcs* lcs, const double* lo, const double* hi,
              const double* x0, const nm_config* cfg, double* x, double* chi2,
              double* Fs, double* Fb, int32_t* n_iter, sblm_stats* stats,
              void* stream);

/*
 * nm_refine_noalloc -- nm_refine for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same simplices, arguments, outputs and errors as
 * nm_refine, with no hipMalloc, hipFree or other allocation.  The
 * simplices' state (~0.8 KB per lightcurve) lives in a static device array
 * of 8 MiB that every GPU the library runs on holds until the process ends,
 * so 1 <= n_lc <= 9936 (SBLM_ERANGE beyond, with the limit in the message).
 * Trial points are spread over 64 lanes without saved roots: the results are
 * those of nm_refine run with 64 lanes per trial point (bit for bit), and
 * they do not depend on what an earlier call left in the array (every
 * simplex's state is initialised by the call).  All calls on one GPU share
 * its array: calls that overlap on one GPU (other streams, other threads)
 * race and must not be made.  Synchronises `stream`.
 */
int nm_refine_noalloc(const sblm_lcs* lcs, const double* lo, const double* hi,
                      const double* x0, const nm_config* cfg, double* x, double* chi2,
                      double* Fs, double* Fb, int32_t* n_iter, sblm_stats* stats,
                      void* stream);

/*
 * nm_refine_multi -- as nm_refine with `reps` independent simplices per
 * lightcurve (several start points: the fittest solution of every island,
 * or the random starts of an iterated simplex).  Simplex j = k * reps + i
 * works on lightcurve k; x0, x [6][n_lc * reps], chi2, Fs, Fb, n_iter
 * [n_lc * reps].  1 <= reps, n_lc * reps <= 2^24.  nm_refine is reps = 1.
 */
int nm_refine_multi(const sblm_lcs* lcs, int32_t reps, const double* lo,
                    const double* hi, const double* x0, const nm_config* cfg,
                    double* x, double* chi2, double* Fs, double* Fb,
                    int32_t* n_iter, sblm_stats* stats, void* stream);

/*
 * nm_iterated -- the iterated simplex (the comparison algorithm of Sec. 4.1):
 * simplices deployed at random start points, each run ended by convergence
 * or max_iter steps, the best of all runs kept.  Every lightcurve has
 * reps * runs starts and reps slots: slot i begins with start i, and a slot
 * whose run ends takes the lightcurve's next unstarted start in the same
 * round (slots ending together in slot order), so long runs do not hold up
 * the starts behind them; the result does not depend on which slot ran a
 * start (the first round of every run starts its root solves cold, never
 * from roots that another run left in the slot).  Start s of lightcurve
 * k, coordinate g: ((w >> 12) + 0.5) * 2^-52 for the Philox4x64-10 word
 * w = word g % 4 of key (seed, k), counter (0, NM_PURPOSE_START, s, g / 4):
 * uniform over the encoded domain (the prior box).  Each run is the simplex
 * of nm_refine (settings above, cfg->max_iter per run).
 *   reps, runs  >= 1; reps <= 1024; n_lc * reps <= 2^24; reps * runs < 2^31;
 *                runs * (max_iter + 1) < 2^31
 *   x       [6][n_lc] device out, encoded best point over the reps * runs
 *           starts (lowest chi^2; the lowest start index among equals)
 *   chi2, Fs, Fb  [n_lc] device out (nullable)
 *   n_iter  [n_lc] device int64 out (nullable), steps of all runs
 * Allocates and frees ~1.2 KB per slot, plus saved roots as nm_refine;
 * synchronises `stream`.  Errors: SBLM_EINVAL, SBLM_ERANGE, SBLM_ENOMEM,
 * SBLM_EDEVICE.
 */
#define NM_PURPOSE_START 7
int nm_iterated(const sblm_lcs* lcs, int32_t reps, int32_t runs, uint64_t seed,
                const double* lo, const double* hi, const nm_config* cfg, double* x,
                double* chi2, double* Fs, double* Fb, int64_t* n_iter,
                sblm_stats* stats, void* stream);

/* ea_best -- the fittest solution seen so far by every lightcurve's EA:
 * x [6][n_lc] device (encoded), chi2 [n_lc] device (nullable).  With
 * islands: the best island record (the lowest island index among equals). */
int ea_best(ea_state* st, double* x, double* chi2, void* stream);

/* ea_records -- the record of every island: x [6][n_lc * n_islands] device
 * (encoded), chi2 [n_lc * n_islands] device (nullable), island-major within
 * each lightcurve.  Without islands the same as ea_best. */
int ea_records(ea_state* st, double* x, double* chi2, void* stream);

/*
 * ea_refine -- a simplex (as nm_refine) from every record (ea_records: one
 * per lightcurve, or one per island), in the state's domain; where the
 * simplex finds a lower chi^2 that record (best chi^2, parameters, fluxes,
 * generation) is replaced.  The population is not touched.  n_iter
 * [n_lc * n_islands] device (nullable), the steps of each simplex.
 * Synchronises `stream`.
 */
int ea_refine(ea_state* st, const nm_config* cfg, int32_t* n_iter, sblm_stats* stats,
              void* stream);

/* ---------------------------------------------------------------------- */
/* Learned proposal network                                                */
/* ---------------------------------------------------------------------- */
/*
 * Not part of the paper's method: its neural-network approach (Sec. 4.1) is a
 * competing fitter, whereas this network only proposes starting points for
 * part of the initial population; the EA's chi^2 (Sec. 4.1, 4.4) ranks them
 * like any other individual and the uniform rows (Sec. A.1) remain.
 *
 * Input: a lightcurve resampled to MLP_NBINS normalised bins (sblm_resample),
 * stored as BF16 (uint16 bit patterns, row-major [rows][256]).
 * Network: 256 -> 512 (ReLU) -> 512 (ReLU) -> 120, BF16 weights and
 * activations with FP32 accumulation on the matrix cores, FP32 master
 * weights.  Output row (FP32, padded to MLP_NOUT_PAD = 128 columns):
 *   [0, 8)     mixture logits of the K = 8 components,
 *   [8, 64)    means, component k, target d at 8 + 7k + d,
 *   [64, 120)  log standard deviations at 64 + 7k + d,
 *   [120, 128) zero.
 * Targets (the "target map", float [rows][7]):
 *   0 (log10 q + 3)/3, 1 (d - 0.5)/1.5, 2 u0/0.5, 3 alpha/(2 pi) (periodic
 *   on [0, 1)), 4 (t0 - t_first)/span, 5 tE/span, 6 Fs/(Fs + Fb),
 * with t_first and span the first epoch and the time covered by the
 * lightcurve.  Loss: the negative log-likelihood of the targets under the
 * mixture averaged over the rows, the residual of target 3 wrapped into
 * [-1/2, 1/2).
 * Canonical parameter order (host arrays of MLP_NPARAMS floats): W1
 * [256][512] (input-major), b1 [512], W2 [512][512], b2 [512], W3 [512][120],
 * b3 [120].
 */
#define MLP_NBINS 256
#define MLP_HIDDEN 512
#define MLP_K 8
#define MLP_D 7
#define MLP_PERIODIC 3
#define MLP_NOUT 120
#define MLP_NOUT_PAD 128
#define MLP_NPARAMS 455800

typedef struct mlp_net mlp_net; /* opaque */

/*
 * sblm_resample -- every lightcurve of a ragged batch to 256 normalised
 * bins over its observed span (epochs ascending within each lightcurve):
 * epoch e of a lightcurve with first/last epochs t_a, t_b falls in bin
 * min(floor((t_e - t_a)/(t_b - t_a) * 256), 255) (bin 0 if t_b = t_a); a bin
 * holds the w-weighted mean flux of its epochs; bins without weight take the
 * linear interpolation of the nearest filled bins (the nearest filled value
 * beyond the first/last); then v -> (v - median)/max(max - median, 1e-12),
 * the median being the mean of the 128th and 129th smallest values.  A
 * lightcurve without weight gives zeros.
 *   lcs   ragged lightcurves (device CSR), 1 <= n_lc <= 2^24
 *   xf    [n_lc][256] FP32 out (nullable)
 *   xb    [n_lc][256] BF16 out, round-to-nearest-even (nullable; not both)
 */
int sblm_resample(const sblm_lcs* lcs, float* xf, uint16_t* xb, void* stream);

/*
 * mlp_make_data -- training samples first .. first+n-1 of the stream keyed
 * by `seed`: parameters uniform over the default EA domain, Fs = 1,
 * Fb ~ U[0, 0.5], observed through nightly windows over t0 +- 2 tE with a
 * Poisson epoch count per bin and Gaussian flux noise, magnified by the
 * forward model of Sec. 2.2 (FP64) at the bin centres, then binned and
 * normalised as by sblm_resample.  Sample s depends only on (seed, s).
 *   xb [n][256] BF16 and/or xf [n][256] FP32 (one may be NULL), y [n][7]
 *   targets (the target map above).  Device pointers.
 * Allocates and frees temporary device memory; synchronises `stream`.
 * Errors: SBLM_EINVAL, SBLM_ERANGE (n > 2^26), SBLM_ENOMEM, SBLM_EDEVICE.
 */
int mlp_make_data(uint64_t seed, int64_t first, int64_t n, uint16_t* xb,
                  float* xf, float* y, void* stream);

/*
 * mlp_create -- a network with He-normal hidden weights (std sqrt(2/fan_in)),
 * output weights of std 0.01 and zero biases (Philox, key (seed, 0)), Adam
 * moments zero, and activation buffers for batch_max rows.
 *   batch_max  positive multiple of 64, at most 2^20
 * Allocates device memory on the current device.  Errors: SBLM_EINVAL,
 * SBLM_ERANGE, SBLM_ENOMEM, SBLM_EDEVICE.
 */
int mlp_create(int32_t batch_max, uint64_t seed, mlp_net** out);
void mlp_destroy(mlp_net* net);

/* Host copies of the FP32 master parameters (canonical order above).
 * mlp_set_params also refreshes the BF16 shadow and zeroes the Adam moments
 * and step count.  Both synchronise the device. */
int mlp_set_params(mlp_net* net, const float* params);
int mlp_get_params(mlp_net* net, float* params);

/*
 * mlp_forward -- network output for `rows` inputs.
 *   x    [rows][256] BF16, device;   out  [rows][128] FP32, device
 * Any rows >= 0; processed in chunks of batch_max through the network's own
 * buffers (so calls on one network must not overlap).
 */
int mlp_forward(mlp_net* net, const uint16_t* x, int64_t rows, float* out,
                void* stream);

/*
 * mlp_loss_grad -- forward pass, loss and gradient of the loss with respect
 * to every parameter (kept in the network; mlp_get_grad copies it out).
 *   x [rows][256] BF16, y [rows][7] FP32 targets, device;
 *   rows a multiple of 64 in [64, batch_max];
 *   loss (nullable) device float receiving the mean loss.
 * The backward GEMMs take BF16 copies of the output gradient and of the
 * hidden-layer gradients; bias gradients are FP32 column sums.
 */
int mlp_loss_grad(mlp_net* net, const uint16_t* x, const float* y, int32_t rows,
                  float* loss, void* stream);
int mlp_get_grad(mlp_net* net, float* grad);

/* One Adam step (Kingma & Ba 2015: beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected as p -= lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps)) with
 * the last gradient; t counts the steps since creation or mlp_set_params. */
int mlp_adam_step(mlp_net* net, float lr, void* stream);

/*
 * mlp_train -- epochs x floor(rows/batch) steps of mlp_loss_grad + Adam
 * over consecutive batches of (x, y), the learning rate following a cosine
 * from lr0 (first step) to lr1 (last step).  loss (nullable, device float
 * [epochs*floor(rows/batch)]) receives the loss of every step.  The steps
 * are the ones that mlp_loss_grad and mlp_adam_step would take one call at
 * a time, bit for bit; here one step is captured as a HIP graph (batch
 * gather, forward, likelihood, backward, Adam, all reading the step index
 * from device memory) and replayed on the net's own stream, which follows
 * `stream` and which `stream` then waits for.  The graph is kept with the
 * net for later calls of the same shape and data; step buffers of 16 B per
 * step grow as needed (with a synchronisation of the net's stream).
 * Errors: SBLM_EINVAL, SBLM_ERANGE (more than 2^31 steps), SBLM_ENOMEM,
 * SBLM_EDEVICE.
 */
int mlp_train(mlp_net* net, const uint16_t* x, const float* y, int64_t rows,
              int32_t batch, int32_t epochs, float lr0, float lr1, float* loss,
              void* stream);

/*
 * ea_seed -- overwrite rows 0 .. n_seed-1 of every lightcurve's current
 * population (of every island) with draws from the network's proposal
 * mixture; island i of lightcurve k draws with lightcurve index
 * k * n_islands + i and the network output and epochs of lightcurve k.
 *   out     [n_lc][ld_out] FP32 device, network output for each lightcurve
 *           (mlp_forward of its sblm_resample bins), ld_out >= 120
 *   n_seed  0 <= n_seed <= pop
 *   flags   0, or EA_SEED_AT_RESTARTS: keep `out` attached so that every
 *           later restart (Sec. A.7; the fresh population of Sec. A.1) also
 *           re-draws rows 0 .. n_seed-1 from the mixture.  The caller keeps
 *           `out` alive and unchanged while it is attached; a call with
 *           flags 0 or n_seed 0 detaches it.  Attaching or detaching
 *           re-captures the generation graph (synchronises the state).
 * Row r of lightcurve l at generation g (the lightcurve's current generation
 * here, the first generation of the new sequence at a restart) draws key
 * (seed, l), counter (g, EA_PURPOSE_SEED, r, j/4): word 0 -> u, component =
 * the first k with u * sum(e) < e_0 + ... + e_k, e_k = exp(logit_k - max
 * logit); words 1..8 -> four Box-Muller pairs (sqrt(-2 ln u1) cos(2 pi u2),
 * sqrt(-2 ln u1) sin(2 pi u2)) giving z_0..z_6; x_d = mean_kd + exp(logstd_kd)
 * z_d, x_3 reduced mod 1; decoded through the target map with t_first/span
 * of lightcurve l; re-encoded into the state's domain (Eq. EMMA-encoding) and
 * clamped to [0, 1].  Lightcurves without epochs are left alone.  Seeding
 * before ea_fit takes effect at once (ea_fit evaluates first).
 * With flags | EA_SEED_WINDOW_ONLY (`out` and ld_out unused, may be NULL /
 * 0) the rows come from the observation window alone -- the ablation that
 * separates what the network learns from what the window gives: x_0..x_3 =
 * u(word 1..4) (uniform over the ranges of log10 q, d, u0, alpha), x_4 =
 * 0.5 (t0 at the middle of the observed span), x_5 = 0.25 (tE a quarter of
 * it), through the same target map and encoding.
 */
#define EA_SEED_AT_RESTARTS 1
#define EA_SEED_WINDOW_ONLY 2
int ea_seed(ea_state* st, const float* out, int32_t ld_out, int32_t n_seed,
            int32_t flags, void* stream);

/* ---------------------------------------------------------------------- */
/* Diagnostics (used by the parity tests)                                  */
/* ---------------------------------------------------------------------- */

/* ea_draws -- the raw 64-bit Philox4x64-10 words the EA uses: out[k] =
 * word (j0 + k) % 4 of the block at key (seed, lc), counter (gen, purpose,
 * row, (j0 + k) / 4), for k < n.  out: DEVICE uint64 [n], 0 <= n <= 2^24. */
int ea_draws(uint64_t seed, uint64_t lc, uint64_t gen, uint64_t purpose,
             uint64_t row, uint64_t j0, int64_t n, uint64_t* out,
             void* stream);

/* ea_generation_traced -- ea_generation that also writes the parent ranks
 * chosen by every tournament: parents DEVICE int32
 * [n_lc][2*floor(pop/2)], pairing k of lightcurve l at
 * parents[l*2*floor(pop/2) + 2k] (first parent) and [... + 2k + 1]. */
int ea_generation_traced(ea_state* st, const double* chi2, const double* Fs,
                         const double* Fb, int32_t* parents, void* stream);

/* mlp_set_grad -- replace the network's gradient buffer with host values
 * (canonical order, MLP_NPARAMS floats), so that mlp_adam_step can be
 * checked on a given gradient.  Synchronises the device. */
int mlp_set_grad(mlp_net* net, const float* grad);

/* Thread-local description of the last error of this thread. */
const char* sblm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SBLM_H */

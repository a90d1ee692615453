"""Benchmark of the batched binary-lens fitness + EA generation on one MI355X.

Headline workload (the batched FP64 fitting configuration): 256 synthetic
lightcurves of 1000 uniform epochs over t0 +- 2 tE (sigma = 1% of the flux),
population 256 per lightcurve.  A step is one generation of the whole hot
path for the whole batch: decode, magnification of all 256 x 256 x 1000
(individual, epoch) pairs, least-squares fluxes and chi^2, then the EA
generation, replayed from one HIP graph.  The default run times a full fit
(500 generations) in the plain FP64 form and in the mixed-precision form,
with the fitness kernel's duration stamped on the device inside every
replayed generation (the roofline), the success rate (best chi^2 <= chi^2 of
the true parameters + 10) and fits/hour.

Chosen form (the batching workload): 4096 lightcurves of 200-5000 irregular
epochs, population 128, autotuned schedule, a full 500-generation fit timed
the same way.  On the same lightcurves the time to 90% success is measured
for the plain EA and for the EA seeded by the proposal network (the learned
form), each with the paper's simplex fine-tuning of the fittest solution at
every checkpoint, and for the learned form that then spends more effort on
the lightcurves whose fit is still poor by its own reduced chi^2, freezing
each in the batch once its fit is good (options:
the EA seeded by the window alone, the ablation; the learned form on
islands); fits/hour at >= 90% success follows.  The CPU oracle is timed on a
bounded sample of the headline workload.

Prints ONE JSON line (a summary line goes to stderr just before it).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FLOPs per call of the fitness arithmetic, as counted by the
# counting build of the kernel's own code (paper_1208_4830_amd/csrc/
# flop_count.cpp over csrc/sblm_math.h; tests/test_flop_count.py checks that
# these are its output): source position + polynomial, warm start, one
# simultaneous-iteration sweep (FP64, FP32), image test + det J + sum over
# three images, one more accepted image, an image refined on the lens
# equation (one or two Newton steps), one residual evaluation, one
# least-squares row.  fma = 2, reciprocal estimate = 1.
FLOP_COUNTS = {"coef": 151, "warm": 72, "sweep64": 696, "sweep32": 691, "images": 380,
               "image_extra": 10, "refine1": 145, "refine": 227, "eval": 50, "lsq": 48,
               "newton": 490, "nearest": 70}


def flop_per_magnification(sweeps64, sweeps32, refined, newton=0.0, polishes=0.0):
    """Algorithmic FLOPs of one magnification + fit update at the lanes' own
    mean counts per solve: FP64 and FP32 sweeps, refined images, FP64 Newton
    polish passes and polishes (each judged on two sets of nearest-root
    distances).  Iterations a wavefront runs past a lane's convergence are
    not credited; three accepted images are counted (a fifth-image epoch
    costs 2 x image_extra more)."""
    c = FLOP_COUNTS
    return (c["coef"] + c["warm"] + sweeps64 * c["sweep64"] + sweeps32 * c["sweep32"]
            + c["images"] + c["lsq"] + refined * c["refine"] + newton * c["newton"]
            + polishes * 2 * c["nearest"])


# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (fma) x 2.4 GHz, the same
# for FP64 and for unpacked FP32 (packed FP32 is not used)
PEAK_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
N_GEN_FIT = 500
# HBM traffic of one launch of the FP64 chi^2 fitness kernel on the default
# workload and schedule, from rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by a
# copy kernel of known size (profiles/fitness_kernel_fp64_256lc_1000ep_pop256_
# traffic.md).  Valid only for the kernel sources it was taken on (the kernel
# file and the arithmetic it shares).
FITNESS_TRAFFIC = dict(source_sha256_16="3eb16ce76bfdd35b", bytes_per_launch=13.75e6,
                       algorithmic_bytes_per_launch=10.86e6)
FITNESS_SOURCES = ("sblm_fitness.hip", "sblm_math.h", "sblm_internal.h")


def fitness_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in FITNESS_SOURCES:
        with open(os.path.join(ROOT, "paper_1208_4830_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def fitness_traffic():
    return FITNESS_TRAFFIC["bytes_per_launch"] \
        if fitness_sources_sha() == FITNESS_TRAFFIC["source_sha256_16"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=N_GEN_FIT)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-lc", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=1000)
    ap.add_argument("--pop", type=int, default=256)
    ap.add_argument("--forms", default="fp64,mixed")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target wall time of the CPU-oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--ragged-lc", type=int, default=4096,
                    help="lightcurves of the chosen-form (ragged) workload (0 = skip it)")
    ap.add_argument("--ragged-steps", type=int, default=N_GEN_FIT,
                    help="generations of the chosen form's timed fit")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tune-after", type=int, default=30,
                    help="generations the scratch state evolves before the autotuner")
    ap.add_argument("--success-max-gen", type=int, default=1600,
                    help="generation cap of the time-to-90%% success runs on the chosen-form "
                         "lightcurves (0 = skip them)")
    ap.add_argument("--success-every", type=int, default=200)
    ap.add_argument("--success-forms", default="plain,learned,learned_adaptive",
                    help="forms of the success study: plain EA (plain), window-only seeding "
                         "(window), network seeding (learned), network seeding on islands "
                         "(learned_islands), network seeding with effort where the fit is "
                         "poor (learned_adaptive)")
    ap.add_argument("--iterated", default="",
                    help="iterated-simplex comparison on the headline lightcurves: slots per "
                         "lightcurve,runs per slot,max steps per run (e.g. 16,4,10000)")
    ap.add_argument("--paper-lc", type=int, default=0,
                    help="lightcurves per paper-shaped experiment (Tables 2-3); 0 skips")
    ap.add_argument("--paper-checkpoints", default="500,1000,3000")
    ap.add_argument("--islands", default="",
                    help="island form in the success study: islands,migrate every,migrants "
                         "(e.g. 8,50,2); also the islands of the learned_islands form "
                         "(default 4,50,2)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device 4 times (a kernel of "
                         "known traffic that scales the profiler's byte counters)")
    ap.add_argument("--train-network", action="store_true",
                    help="train the proposal network even when no success run uses it")
    ap.add_argument("--precision-pairs", type=int, default=8_000_000,
                    help="single-epoch pairs of the precision-form comparison (0 skips it)")
    ap.add_argument("--mlp-samples", type=int, default=1 << 20)
    ap.add_argument("--mlp-epochs", type=int, default=32)
    ap.add_argument("--mlp-batch", type=int, default=1024)
    ap.add_argument("--mlp-lr", type=float, default=2e-3, help="initial learning rate (cosine "
                    "schedule to 1e-5)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_batch(sblm, torch, wl):
    """Device lightcurves; observations from the library's own forward model."""
    dev = "cuda"
    t = torch.as_tensor(wl.t, device=dev)
    A = torch.empty(wl.t.size, dtype=torch.float64, device=dev)
    for k in range(wl.n_lc):  # each lightcurve has its own epochs
        a, b = int(wl.off[k]), int(wl.off[k + 1])
        A[a:b] = sblm.sblm_magnify(torch.as_tensor(wl.theta[:, k:k + 1].copy(), device=dev),
                                   t[a:b].contiguous())[0]
    A = A.cpu().numpy()
    L = np.diff(wl.off)
    F = np.repeat(wl.Fs, L) * A + np.repeat(wl.Fb, L)
    sig = wl.sfrac * F
    y = F + sig * wl.noise
    w = 1.0 / sig ** 2
    lcs = sblm.Lightcurves(torch.as_tensor(wl.off, device=dev), t,
                           torch.as_tensor(y, device=dev), torch.as_tensor(w, device=dev))
    return y, w, lcs


def run_form(sblm, torch, lcs, wl, chi2_true, pop, steps, args, mode, tune=True):
    """A fit of `args.warmup` untimed generations, then `steps` timed ones:
    wall time of the replayed graphs, and the fitness kernel's own duration
    in every one of them (device clock stamped by graph nodes just before
    and after it)."""
    n_lc = wl.n_lc
    mags_per_gen = pop * int(wl.off[-1])
    cfg = sblm.ea_default_config()
    cfg.pop = pop
    cfg.mode = mode
    # warm-up and schedule choice on a scratch state (same shapes), tuned
    # after some generations: the initial uniform population solves very
    # differently from the evolved ones the fit spends its time on
    scratch = sblm.EAState(cfg, lcs, 999)
    scratch.fit(max(args.warmup, args.tune_after))
    torch.cuda.synchronize()
    report = ""
    if tune and not args.no_autotune:
        report = scratch.autotune()
        log("bench: autotune\n" + report.strip())
    sched = scratch.schedule()
    scratch.close()

    # the timed fit: fresh state with the chosen schedule, fitness counters
    # and kernel stamps on; its first `warmup` generations untimed (the
    # stamps' sums and the counters cleared after them), then `steps` timed
    state = sblm.EAState(cfg, lcs, 1)
    state.set_schedule(*sched)
    state.time_fitness(True)
    st = sblm.new_stats()
    state.fit(0, stats=st)  # capture the graph with the counters bound
    if args.warmup > 0:
        state.fit(args.warmup, stats=st)
        state.time_fitness(True)
        st.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    state.fit(steps, stats=st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k_ms_sum, launches = state.fitness_time()
    k_ms = k_ms_sum / max(launches, 1)
    summ = state.summary()
    best = np.array([summ[k].best_chi2 for k in range(n_lc)])
    success = float(np.mean(best <= chi2_true + 10.0))
    # cross-check: the same kernel on the final population, HIP events on
    # the stream it runs on (the state's work stream is joined to it)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    state.evaluate(stream=stream)
    e0.record(stream)
    for _ in range(args.kernel_reps):
        state.evaluate(stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    k_ms_final = e0.elapsed_time(e1) / args.kernel_reps
    state.close()

    s = sblm.stats_dict(st)
    n = max(s["n_solves"], 1)
    sweeps = s["n_iter"] / n
    n32 = s["n_iter_fp32"] / n
    refined = s["n_polished"] / n
    newton = s["n_newton"] / n
    # MIXED: every solve with an FP32 phase is polished (all but degree-4
    # polynomials and far roots, a few in 10^6)
    polishes = (1.0 - s["n_degree4"] / n) if mode == sblm.MIXED else 0.0
    flop = flop_per_magnification(sweeps - n32, n32, refined, newton, polishes)
    # what the wavefronts executed: lockstep sweeps (n_wave_iter) instead of
    # the lanes' own need
    wave = s["n_wave_iter"] / n
    flop_exec = flop + (wave - sweeps) * FLOP_COUNTS["sweep64"]
    ms_step = dt * 1e3 / steps
    return dict(
        mags_per_s=mags_per_gen * steps / dt,
        ms_per_step=ms_step,
        fits_per_hour=n_lc * 3600.0 / (steps * ms_step / 1e3),
        success=success, generations=steps, warmup_generations=args.warmup,
        kernel_ms=k_ms, kernel_launches=launches, kernel_ms_final_population=k_ms_final,
        kernel_mags_per_s=mags_per_gen / (k_ms / 1e3),
        sweeps_per_solve=sweeps, fp32_sweeps_per_solve=n32, flop_per_mag=flop,
        newton_passes_per_solve=newton,
        kernel_tflops=flop * mags_per_gen / (k_ms / 1e3) / 1e12,
        kernel_tflops_executed=flop_exec * mags_per_gen / (k_ms / 1e3) / 1e12,
        capped=s["n_capped"], unsettled=s["n_unsettled"], fallback=s["n_fallback"],
        wave_sweeps_per_solve=wave, polished_per_solve=refined,
        schedule=dict(zip(("lanes", "waves_per_block", "persistent", "asynchronous"), sched)))


def success_run(sblm, torch, lcs, chi2_true, pop, mode, sched, lo, hi, proposals=None,
                max_gen=1600, every=100, target=0.9, seed=7, passes=3, islands=None,
                window=False):
    """EA with optional proposal seeding; at every checkpoint the fittest
    solution of each lightcurve is fine-tuned by `passes` simplex passes, each
    restarted from the last (on a copy: the EA continues untouched), as the
    paper's "EA with amoeba".  `sched` is the chosen form's tuned schedule:
    the knobs the tuner turns change no result bit, so these runs are
    reproducible whatever it chose.
    Success = chi^2 <= chi^2 of the true parameters + 10.  GPU time of a
    checkpoint = EA time so far + that checkpoint's simplex time.
    islands = (n_islands, migrate every, migrants): the island form with the
    same total population (pop // n_islands rows per island); its simplex
    passes start from every island's record (the best island record for
    the EA alone)."""
    cfg = sblm.ea_default_config()
    cfg.pop = pop
    cfg.mode = mode
    if islands:
        cfg.n_islands, cfg.mig_every, cfg.n_migrants = islands
        cfg.pop = pop // cfg.n_islands
    state = sblm.EAState(cfg, lcs, seed)
    state.set_schedule(*sched)
    n_lc = len(chi2_true)
    sync = torch.cuda.synchronize
    ea_s = 0.0
    if proposals is not None:  # resampling + inference done by the caller
        sync()
        t0 = time.perf_counter()
        state.seed(proposals, cfg.pop // 2, at_restarts=True)
        sync()
        ea_s += time.perf_counter() - t0
    elif window:  # the ablation: seeds from the observation window alone
        sync()
        t0 = time.perf_counter()
        state.seed_window(cfg.pop // 2, at_restarts=True)
        sync()
        ea_s += time.perf_counter() - t0
    nm_cfg = sblm.nm_default_config()
    nm_cfg.mode = mode
    gens, curve, hit_ea, hit_nm = 0, [], None, None
    while gens < max_gen:
        sync()
        t0 = time.perf_counter()
        state.fit(every)
        sync()
        ea_s += time.perf_counter() - t0
        gens += every
        reps = cfg.n_islands
        x, c0 = state.records() if reps > 1 else state.best()
        sync()
        t0 = time.perf_counter()
        c2 = c0.clone()
        for _ in range(passes):
            x, c, _, _, _ = sblm.nm_refine(lcs, lo, hi, x, nm_cfg, reps=reps)
            c2 = torch.minimum(c2, c)
        c0 = c0.view(n_lc, reps).min(dim=1).values
        c2 = c2.view(n_lc, reps).min(dim=1).values
        sync()
        nm_s = time.perf_counter() - t0
        c0 = c0.cpu().numpy()
        c2 = c2.cpu().numpy()
        s_ea = float(np.mean(c0 <= chi2_true + 10.0))
        s_nm = float(np.mean(c2 <= chi2_true + 10.0))
        curve.append(dict(gen=gens, ea=round(s_ea, 4), ea_amoeba=round(s_nm, 4),
                          ea_seconds=round(ea_s, 3), amoeba_seconds=round(nm_s, 3)))
        log(f"bench:   checkpoint {json.dumps(curve[-1])}")
        if hit_ea is None and s_ea >= target:
            hit_ea = (gens, ea_s)
        if hit_nm is None and s_nm >= target:
            hit_nm = (gens, ea_s + nm_s)
        if hit_nm is not None:
            break
    state.close()
    per_hour = lambda h: n_lc * 3600.0 / h[1] if h else f"not reached by generation {gens}"
    return dict(target=target, curve=curve,
                ea_amoeba=dict(reached=hit_nm is not None,
                               generations=hit_nm[0] if hit_nm else None,
                               gpu_seconds=hit_nm[1] if hit_nm else None,
                               fits_per_hour=per_hour(hit_nm)),
                ea_alone=dict(reached=hit_ea is not None,
                              generations=hit_ea[0] if hit_ea else None,
                              gpu_seconds=hit_ea[1] if hit_ea else None,
                              fits_per_hour=per_hour(hit_ea)))


def simplex_passes(sblm, torch, lcs, lo, hi, x, c, passes, nm_cfg):
    """`passes` simplex passes, each restarted from the last result; the
    best point and chi^2 seen (the start's included)."""
    xb, cb = x.clone(), c.clone()
    for _ in range(passes):
        x, cp, _, _, _ = sblm.nm_refine(lcs, lo, hi, x, nm_cfg)
        better = cp < cb
        xb = torch.where(better, x, xb)
        cb = torch.minimum(cb, cp)
    return xb, cb


def subset_batch(sblm, torch, lcs, idx):
    """The lightcurves idx of a device batch as a batch of their own."""
    off = lcs.off.cpu().numpy()
    L = np.diff(off)[idx]
    sub_off = np.concatenate([[0], np.cumsum(L)]).astype(np.int64)
    sel = np.concatenate([np.arange(off[k], off[k + 1]) for k in idx]) if len(idx) else \
        np.zeros(0, np.int64)
    sel = torch.as_tensor(sel, device=lcs.t.device)
    return sblm.Lightcurves(torch.as_tensor(sub_off, device=lcs.t.device), lcs.t[sel].contiguous(),
                            lcs.y[sel].contiguous(), lcs.w[sel].contiguous())


def adaptive_run(sblm, torch, lcs, chi2_true, pop, sched, lo, hi, proposals, stage1_gen=400,
                 pop2=1024, every=100, max_gen2=1000, red_thr=1.05, target=0.9, seed=7,
                 passes=3, freeze=True, stage1_every=None, freeze_thr=None):
    """The learned form with effort where the fit asks for it.  Stage 1: the
    learned form on every lightcurve for `stage1_gen` generations, then twice
    `passes` simplex passes from each fittest solution.  Lightcurves whose
    fit is still poor by its own measure (reduced chi^2 = chi^2 / (L - 6)
    above `red_thr`; the data's errors are known, so a good fit sits near 1)
    get stage 2: a fresh network-seeded EA of population `pop2` on those
    lightcurves alone, with `passes` simplex passes from its fittest
    solutions every `every` generations; a lightcurve keeps the best of its
    fits.  With `freeze`, a lightcurve whose best fit has come down to the
    threshold is frozen (ea_freeze): its EA stops and later passes skip it,
    so the remaining effort goes to the fits still poor; with `stage1_every`
    stage 1 also takes `passes` passes every so many generations and freezes
    the same way (off by default: the threshold is loose enough that stage-1
    fits frozen there would still have improved).  GPU time: the EA
    time so far, stage 1's passes included, plus the stage-2 passes (all
    checkpoints' with `freeze`, since frozen fits come from earlier
    checkpoints; else that checkpoint's, as in success_run)."""
    sync = torch.cuda.synchronize
    n_lc = len(chi2_true)
    fthr = red_thr if freeze_thr is None else freeze_thr  # reduced chi^2 that freezes
    nm_cfg = sblm.nm_default_config()
    cfg = sblm.ea_default_config()
    cfg.pop = pop
    sync()
    t0 = time.perf_counter()
    st = sblm.EAState(cfg, lcs, seed)
    st.set_schedule(*sched)
    st.seed(proposals, pop // 2, at_restarts=True)
    L = np.diff(lcs.off.cpu().numpy())
    dof = np.maximum(L - 6, 1)
    c1 = np.full(n_lc, np.inf)
    frozen1 = np.zeros(n_lc, np.int32)
    curve = []
    g1 = 0
    while g1 < stage1_gen:
        step = min(stage1_every, stage1_gen - g1) if (freeze and stage1_every) else stage1_gen
        st.fit(step)
        g1 += step
        x, c = st.best()
        run = np.nonzero(frozen1 == 0)[0]
        npass = 2 * passes if g1 >= stage1_gen else passes
        if len(run) < n_lc:
            sel = torch.as_tensor(run, device=x.device)
            _, cr = simplex_passes(sblm, torch, subset_batch(sblm, torch, lcs, run), lo, hi,
                                   x[:, sel].contiguous(), c[sel].contiguous(), npass, nm_cfg)
        else:
            _, cr = simplex_passes(sblm, torch, lcs, lo, hi, x, c, npass, nm_cfg)
        c1[run] = np.minimum(c1[run], cr.cpu().numpy())
        if g1 < stage1_gen:
            frozen1 = (c1 / dof <= fthr).astype(np.int32)
            st.freeze(frozen1)
            sync()
            curve.append(dict(gen=g1, stage=1, success=round(float(np.mean(c1 <= chi2_true + 10.0)),
                                                             4),
                              gpu_seconds=round(time.perf_counter() - t0, 3),
                              running=int(len(run))))
            log(f"bench:   checkpoint {json.dumps(curve[-1])}")
    sync()
    base_s = time.perf_counter() - t0
    st.close()
    idx = np.nonzero(c1 / dof > red_thr)[0]
    s1 = float(np.mean(c1 <= chi2_true + 10.0))
    curve.append(dict(gen=stage1_gen, stage=1, success=round(s1, 4), gpu_seconds=round(base_s, 3),
                      running=int(len(run)), flagged=int(len(idx))))
    log(f"bench:   stage 1 {json.dumps(curve[-1])}")
    hit = (stage1_gen, base_s) if s1 >= target else None
    if hit is None and len(idx):
        sync()
        t0 = time.perf_counter()
        lcs2 = subset_batch(sblm, torch, lcs, idx)
        props2 = proposals[torch.as_tensor(idx, device=proposals.device)].contiguous()
        cfg2 = sblm.ea_default_config()
        cfg2.pop = pop2
        st2 = sblm.EAState(cfg2, lcs2, seed + 4)
        st2.seed(props2, pop2 // 2, at_restarts=True)
        sync()
        ea_s = base_s + time.perf_counter() - t0
        nm_all = 0.0
        best = c1.copy()
        frozen = np.zeros(len(idx), np.int32)
        gens = 0
        while gens < max_gen2:
            sync()
            t0 = time.perf_counter()
            st2.fit(every)
            sync()
            ea_s += time.perf_counter() - t0
            gens += every
            x2, c2 = st2.best()
            run = np.nonzero(frozen == 0)[0]
            sync()
            t0 = time.perf_counter()
            if freeze and len(run) < len(idx):
                sel = torch.as_tensor(run, device=x2.device)
                _, c2r = simplex_passes(sblm, torch, subset_batch(sblm, torch, lcs2, run), lo, hi,
                                        x2[:, sel].contiguous(), c2[sel].contiguous(), passes,
                                        nm_cfg)
            else:
                _, c2r = simplex_passes(sblm, torch, lcs2, lo, hi, x2, c2, passes, nm_cfg)
            sync()
            nm_s = time.perf_counter() - t0
            nm_all += nm_s
            c2r = c2r.cpu().numpy()
            if freeze:
                best[idx[run]] = np.minimum(best[idx[run]], c2r)
            else:
                best[idx] = np.minimum(c1[idx], c2r)
            succ = float(np.mean(best <= chi2_true + 10.0))
            spent = ea_s + (nm_all if freeze else nm_s)
            curve.append(dict(gen=stage1_gen + gens, stage=2, success=round(succ, 4),
                              gpu_seconds=round(spent, 3), running=int(len(run))))
            log(f"bench:   checkpoint {json.dumps(curve[-1])}")
            if succ >= target:
                hit = (stage1_gen + gens, spent)
                break
            if freeze:
                frozen = (best[idx] / dof[idx] <= fthr).astype(np.int32)
                if frozen.all():
                    break
                st2.freeze(frozen)
        st2.close()
    last = curve[-1]["gen"]
    return dict(target=target, curve=curve,
                config=dict(stage1_generations=stage1_gen, stage1_passes=2 * passes,
                            reduced_chi2_above=red_thr, pop_stage2=pop2, every=every,
                            stage2_max_generations=max_gen2, freeze=freeze,
                            stage1_every=stage1_every if freeze else None),
                ea_amoeba=dict(reached=hit is not None,
                               generations=hit[0] if hit else None,
                               gpu_seconds=hit[1] if hit else None,
                               fits_per_hour=(n_lc * 3600.0 / hit[1] if hit else
                                              f"not reached by generation {last}")))


def iterated_run(sblm, torch, lcs, chi2_true, lo, hi, reps, runs, max_iter, seed=7):
    """The paper's iterated simplex (Sec. 4.1) on the GPU fitness: reps * runs
    random starts per lightcurve, each run to convergence or max_iter steps,
    the best kept; success and GPU time of the whole call."""
    cfg = sblm.nm_default_config()
    cfg.max_iter = max_iter
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, c, _, _, it = sblm.nm_iterated(lcs, lo, hi, reps, runs, seed, cfg)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dict(starts_per_lightcurve=reps * runs, slots=reps, runs_per_slot=runs,
                max_steps_per_run=max_iter,
                success=round(float(np.mean(c.cpu().numpy() <= chi2_true + 10.0)), 4),
                gpu_seconds=round(dt, 3),
                mean_steps_per_run=round(it.double().mean().item() / (reps * runs), 1))


def train_proposals(sblm, torch, args):
    """Proposal network trained on generated lightcurves (timed)."""
    sync = torch.cuda.synchronize
    sync()
    t0 = time.perf_counter()
    xb, _, yt = sblm.mlp_make_data(11, 0, args.mlp_samples)
    sync()
    t_data = time.perf_counter() - t0
    batch = args.mlp_batch
    net = sblm.MLP(batch_max=batch, seed=2)
    steps = args.mlp_epochs * (args.mlp_samples // batch)
    t0 = time.perf_counter()
    loss = net.train(xb, yt, batch=batch, epochs=args.mlp_epochs, lr0=args.mlp_lr,
                     lr1=1e-5)
    sync()
    t_train = time.perf_counter() - t0
    lc = loss.cpu().numpy()
    # held-out loss: fresh samples of the same generator, no update
    xh, _, yh = sblm.mlp_make_data(12, 0, 4 * batch)
    held = float(np.mean([net.loss_grad(xh[i * batch:(i + 1) * batch],
                                        yh[i * batch:(i + 1) * batch]).item()
                          for i in range(4)]))
    step_s = t_train / max(steps, 1)
    mfma_tflops = 6.0 * batch * MLP_GEMM_WEIGHTS / step_s / 1e12
    info = dict(samples=args.mlp_samples, epochs=args.mlp_epochs, batch=batch, steps=steps,
                data_seconds=t_data, train_seconds=t_train, us_per_step=step_s * 1e6,
                loss_first=float(lc[:16].mean()), loss_last=float(lc[-16:].mean()),
                loss_held_out=held,
                mfma_tflops=mfma_tflops, mfma_frac=mfma_tflops / PEAK_BF16_TFLOPS)
    return net, info


def propose(sblm, torch, net, lcs):
    """Resampling + network forward pass for every lightcurve (timed)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xr, _ = sblm.sblm_resample(lcs)
    out = net.forward(xr)
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


# Matrix-core FLOPs of one training step per sample: forward 2 P, backward
# 4 P (data and weight gradients), P = 256*512 + 512*512 + 512*128 weights
# as the kernels multiply them (output layer padded to 128 columns)
MLP_GEMM_WEIGHTS = 256 * 512 + 512 * 512 + 512 * 128
PEAK_BF16_TFLOPS = 2500.0


def success_study(sblm, torch, lcs, chi2_true, pop, sched, lo, hi, net, train_info, args):
    """Time to 90% success on the chosen-form lightcurves for the forms in
    --success-forms: the plain EA, the EA half seeded (at the start and at
    every restart) from the observation window alone, the EA half seeded by
    the proposal network (the learned form; also on islands), each with the
    simplex fine-tuning of the fittest solution at every checkpoint and
    stopped once 90% of the lightcurves succeed; and the learned form with
    a second stage on the lightcurves whose fit is poor (adaptive_run)."""
    forms = [f for f in args.success_forms.split(",") if f]
    out = dict(workload=f"{len(chi2_true)} lightcurves, pop {pop}, {pop // 2} rows seeded at "
                        f"the start and at every restart; EA + three simplex passes from the "
                        f"fittest solution every {args.success_every} generations",
               training=train_info)
    t_inf = 0.0
    props = None
    isl = tuple(int(v) for v in (args.islands or "4,50,2").split(","))
    for f in forms:
        log(f"bench: success study, form {f}")
        kw = {}
        if f in ("learned", "learned_islands", "learned_adaptive"):
            if props is None:
                props, t_inf = propose(sblm, torch, net, lcs)
                out["inference_seconds"] = t_inf
            kw["proposals"] = props
        elif f == "window":
            kw["window"] = True
        if f == "learned_islands":
            # the learned form on islands: half of every island's rows seeded,
            # a simplex from every island's record at each checkpoint
            kw["islands"] = isl
        if f == "learned_adaptive":
            r = adaptive_run(sblm, torch, lcs, chi2_true, pop, sched, lo, hi, kw["proposals"])
        else:
            r = success_run(sblm, torch, lcs, chi2_true, pop, sblm.FP64, sched, lo, hi,
                            max_gen=args.success_max_gen, every=args.success_every, **kw)
        if f == "learned_islands":
            r["config"] = dict(islands=isl[0], pop_per_island=pop // isl[0],
                               migrate_every=isl[1], migrants=isl[2])
        if f.startswith("learned") and r["ea_amoeba"]["reached"]:  # inference is its time too
            r["ea_amoeba"]["gpu_seconds"] += t_inf
            r["ea_amoeba"]["fits_per_hour"] = len(chi2_true) * 3600.0 / \
                r["ea_amoeba"]["gpu_seconds"]
        out[f] = r
        log(f"bench: success {f}: {json.dumps(r)}")
    if args.islands:
        out["islands"] = success_run(sblm, torch, lcs, chi2_true, pop, sblm.FP64, sched, lo, hi,
                                     max_gen=args.success_max_gen, every=args.success_every,
                                     islands=isl)
        out["islands"]["config"] = dict(islands=isl[0], pop_per_island=pop // isl[0],
                                        migrate_every=isl[1], migrants=isl[2])
    return out


def cpu_baseline(wl, y, w, pop, target_s):
    """The CPU oracle's chi^2 on a sample of the same workload."""
    import oracle as O
    # the host share of one GPU is 16 cores
    nthreads = min(16, len(os.sched_getaffinity(0)))
    rng = np.random.default_rng(5)
    from paper_1208_4830_amd import inputs

    def run(n_ind_per_lc, n_lcs):
        off = wl.off[:n_lcs + 1]
        sl = slice(0, int(off[-1]))
        th = inputs.draw_theta(rng, n_lcs * n_ind_per_lc)
        t0 = time.perf_counter()
        O.chi2(off, wl.t[sl], y[sl], w[sl], th, n_ind_per_lc, nthreads=nthreads)
        return time.perf_counter() - t0, n_lcs * n_ind_per_lc * int(off[1] - off[0])

    dt, mags = run(nthreads, 1)  # calibration
    rate = mags / dt
    n_ind = max(nthreads, int(target_s * rate / 1000))
    n_lcs = min(wl.n_lc, max(1, n_ind // pop))
    per = max(1, n_ind // n_lcs)
    dt, mags = run(per, n_lcs)
    # one core on a smaller sample (about a fifth of the wall time)
    n1 = max(1, int(0.2 * target_s * rate / nthreads / 1000))
    t0 = time.perf_counter()
    off1 = wl.off[:2]
    th1 = inputs.draw_theta(rng, n1)
    O.chi2(off1, wl.t[:int(off1[1])], y[:int(off1[1])], w[:int(off1[1])], th1, n1, nthreads=1)
    dt1 = time.perf_counter() - t0
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=mags / dt, unit="magnifications/s", cores=nthreads, kind="oracle",
                sample=f"{n_lcs} lightcurves x {per} individuals x {int(wl.off[1])} epochs "
                       f"({mags} magnifications + chi^2, {dt:.1f} s)",
                one_core_value=n1 * int(off1[1]) / dt1,
                one_core_sample=f"1 lightcurve x {n1} individuals x {int(off1[1])} epochs "
                                f"({dt1:.1f} s)",
                host_cpus=os.cpu_count(), cpu_model=cpu_model)


def single_fit(sblm, torch, nthreads):
    """The single-lightcurve configuration in full (400 uniform epochs over
    t0 +- 2 tE, sigma = 1% of the flux, population 48, 100 generations): on
    the GPU (one graph per generation) and with the CPU oracle (its chi^2 on
    `nthreads` threads and its EA generation), same seeds."""
    import oracle as O
    from paper_1208_4830_amd import inputs
    wl = inputs.uniform_workload(1, 1, 400)
    A, _ = O.magnify(wl.theta, wl.t)  # observations from the oracle's forward model
    F = wl.Fs[0] * A[0] + wl.Fb[0]
    sig = wl.sfrac * F
    y, w = F + sig * wl.noise, 1.0 / sig ** 2
    pop, gens, seed = 48, 100, 3
    lo, hi = inputs.PRIOR_LO, inputs.PRIOR_HI
    c_true = O.chi2(wl.off, wl.t, y, w, wl.theta, 1, nthreads=1)[0][0]
    cu = lambda a, dt=torch.float64: torch.as_tensor(a, dtype=dt, device="cuda")
    lcs = sblm.Lightcurves(cu(wl.off, torch.int64), cu(wl.t), cu(y), cu(w))
    cfg = sblm.ea_default_config()
    cfg.pop = pop
    st = sblm.EAState(cfg, lcs, seed)
    st.fit(2)  # warm-up (graph, code objects)
    st.close()
    st = sblm.EAState(cfg, lcs, seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.fit(gens)
    torch.cuda.synchronize()
    gpu_s = time.perf_counter() - t0
    gpu_best = st.summary()[0].best_chi2
    st.close()
    ea = O.EA(pop, seed, 0)
    t0 = time.perf_counter()
    for _ in range(gens):
        th = O.decode(ea.P.T.copy(), lo, hi)
        c, fs, fb = O.chi2(wl.off, wl.t, y, w, th, pop, nthreads=nthreads)
        ea.generation(c, fs, fb)
    cpu_s = time.perf_counter() - t0
    return dict(workload="1 lightcurve x 400 uniform epochs, pop 48, 100 generations",
                gpu_seconds=gpu_s, cpu_seconds=cpu_s, cpu_threads=nthreads,
                gpu_best_chi2=gpu_best, cpu_best_chi2=ea.summary()["best_chi2"],
                chi2_true=c_true)


def precision_forms(sblm, torch, lcs, n_lc, args):
    """FP64 against the precision form (FP32 iteration + FP64 Newton polish)
    where cold starts dominate: single-epoch magnifications (every solve
    cold) and the simplex passes (each lane's first epoch of a round starts
    from the last round's roots, the rest warm)."""
    from paper_1208_4830_amd import inputs
    rng = np.random.default_rng(31)
    n = args.precision_pairs
    th = inputs.draw_theta(rng, n)
    th[5] = -rng.uniform(-2.0, 2.0, n) * th[4]  # the epoch t = 0 at tau ~ U[-2, 2]
    theta = torch.as_tensor(th, device="cuda")
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    A = torch.empty((n, 1), dtype=torch.float64, device="cuda")
    out = {"single_epoch_magnify": {}, "simplex_pass": {}}
    for name, mode in (("fp64", sblm.FP64), ("mixed", sblm.MIXED)):
        st = sblm.new_stats()
        sblm.sblm_magnify(theta, t, mode=mode, A=A, stats=st)  # warm-up, counters
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        stream = torch.cuda.current_stream()
        e0.record(stream)
        for _ in range(3):
            sblm.sblm_magnify(theta, t, mode=mode, A=A, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        s = sblm.stats_dict(st)
        out["single_epoch_magnify"][name] = dict(
            pairs=n, ms=ms, mags_per_s=n / (ms / 1e3),
            sweeps_per_solve=s["n_iter"] / n, fp32_sweeps_per_solve=s["n_iter_fp32"] / n,
            newton_passes_per_solve=s["n_newton"] / n, fallback_per_solve=s["n_fallback"] / n)
    lo, hi = inputs.PRIOR_LO, inputs.PRIOR_HI
    x0 = torch.as_tensor(np.clip(rng.random((6, n_lc)), 0, 1), device="cuda")
    for name, mode in (("fp64", sblm.FP64), ("mixed", sblm.MIXED)):
        cfg = sblm.nm_default_config()
        cfg.mode = mode
        cfg.max_iter = 300
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, c, _, _, it = sblm.nm_refine(lcs, lo, hi, x0, cfg)
        torch.cuda.synchronize()
        out["simplex_pass"][name] = dict(seconds=time.perf_counter() - t0,
                                         steps=int(it.sum().item()),
                                         workload=f"{n_lc} simplices from random starts, "
                                                  f"<= {cfg.max_iter} steps")
    for k in out:
        f64, mx = out[k]["fp64"], out[k]["mixed"]
        out[k]["mixed_over_fp64_time"] = (mx["ms"] / f64["ms"] if "ms" in mx
                                          else mx["seconds"] / f64["seconds"])
    return out


def roofline_of(form, kernel):
    return {"bound": "alu", "achieved": form["kernel_tflops"], "peak": PEAK_VALU_TFLOPS,
            "unit": "TFLOP/s", "frac": form["kernel_tflops"] / PEAK_VALU_TFLOPS,
            "kernel": kernel, "kernel_ms": form["kernel_ms"],
            "kernel_launches": form["kernel_launches"],
            "flop_per_magnification": form["flop_per_mag"],
            "executed_tflops": form["kernel_tflops_executed"],
            "executed_frac": form["kernel_tflops_executed"] / PEAK_VALU_TFLOPS}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the fit shards by "
                          "lightcurve, and no multi-GPU path is implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_1208_4830_amd import sblm
    sblm.load()
    assert torch.cuda.is_available()
    from paper_1208_4830_amd import inputs
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib << 18  # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copied {args.copy_calibration_mib} MiB x 4 (counter calibration)")
        del src, dst
    log(f"bench: {args.n_lc} lightcurves x {args.epochs} epochs, pop {args.pop}, "
        f"{args.steps} generations")
    wl = inputs.uniform_workload(2, args.n_lc, args.epochs)
    y, w, lcs = make_batch(sblm, torch, wl)
    th_true = torch.as_tensor(wl.theta.copy(), device="cuda")
    c_true, _, _ = sblm.sblm_chi2(lcs, th_true, 1)
    chi2_true = c_true.cpu().numpy()

    forms = {}
    for name in args.forms.split(","):
        mode = sblm.FP64 if name == "fp64" else sblm.MIXED
        log(f"bench: form {name}")
        forms[name] = run_form(sblm, torch, lcs, wl, chi2_true, args.pop, args.steps, args, mode)
        log(f"bench: {name}: {json.dumps(forms[name])}")
    main_form = forms.get("fp64") or next(iter(forms.values()))
    lo, hi = inputs.PRIOR_LO, inputs.PRIOR_HI  # the default EA domain
    if args.precision_pairs > 0:
        log("bench: precision forms where cold starts dominate")
        forms["cold_dominated"] = precision_forms(sblm, torch, lcs, args.n_lc, args)
        log(f"bench: cold-dominated: {json.dumps(forms['cold_dominated'])}")

    iterated = None
    if args.iterated:
        iterated = iterated_run(sblm, torch, lcs, chi2_true, lo, hi,
                                *(int(v) for v in args.iterated.split(",")))
        log(f"bench: iterated simplex: {json.dumps(iterated)}")

    paper = None
    if args.paper_lc > 0:
        from paper_1208_4830_amd import experiments
        cps = tuple(int(v) for v in args.paper_checkpoints.split(","))
        paper = {}
        for exp in (1, 2):
            log(f"bench: paper experiment {exp} (Table {exp + 1} shape), {args.paper_lc} "
                f"lightcurves of 100 points, pop 1000")
            paper[f"experiment_{exp}"] = experiments.run_experiment(
                sblm, torch, exp, n_lc=args.paper_lc, pop=1000, checkpoints=cps)
            log(f"bench: paper {exp}: {json.dumps(paper[f'experiment_{exp}'])}")

    chosen = None
    study = None
    if args.ragged_lc > 0:
        log(f"bench: chosen form, {args.ragged_lc} lightcurves of 200-5000 epochs, pop 128, "
            f"{args.ragged_steps} generations")
        wr = inputs.ragged_workload(4, args.ragged_lc)
        yr, wr_w, lcs_r = make_batch(sblm, torch, wr)
        c_true_r, _, _ = sblm.sblm_chi2(lcs_r, torch.as_tensor(wr.theta.copy(), device="cuda"), 1)
        c_true_r = c_true_r.cpu().numpy()
        chosen = run_form(sblm, torch, lcs_r, wr, c_true_r, 128, args.ragged_steps, args,
                          sblm.FP64)
        chosen["workload"] = (f"{args.ragged_lc} lightcurves, L ~ U{{200..5000}} "
                              f"(total {int(wr.off[-1])} epochs), nightly cadence, pop 128, "
                              f"FP64, autotuned schedule, {args.ragged_steps} generations")
        chosen["roofline"] = roofline_of(chosen, "fitness_kernel (FP64, chosen schedule)")
        log(f"bench: chosen: {json.dumps(chosen)}")
        if args.success_max_gen > 0:
            net = train_info = None
            if any(f.startswith("learned") for f in args.success_forms.split(",")):
                log("bench: training the proposal network on generated lightcurves")
                net, train_info = train_proposals(sblm, torch, args)
                log(f"bench: training: {json.dumps(train_info)}")
            sched_r = tuple(chosen["schedule"][k] for k in
                            ("lanes", "waves_per_block", "persistent", "asynchronous"))
            study = success_study(sblm, torch, lcs_r, c_true_r, 128, sched_r, lo, hi,
                                  net, train_info, args)
            if net is not None:
                net.close()
        del lcs_r
    elif args.train_network:
        net, train_info = train_proposals(sblm, torch, args)
        log(f"bench: training: {json.dumps(train_info)}")
        net.close()

    cpu = None
    if not args.no_cpu:
        log("bench: CPU oracle sample")
        cpu = cpu_baseline(wl, y, w, args.pop, args.cpu_seconds)
        cpu["single_fit"] = single_fit(sblm, torch, cpu["cores"])
        log(f"bench: cpu {json.dumps(cpu)}")

    at90 = None
    if study:
        forms_done = [f for f in ("plain", "window", "learned", "learned_islands",
                                  "learned_adaptive", "islands") if f in study]
        at90 = {f: study[f]["ea_amoeba"]["fits_per_hour"] for f in forms_done}
        at90["gpu_seconds"] = {f: study[f]["ea_amoeba"]["gpu_seconds"] for f in forms_done}
        at90["workload"] = "the chosen-form lightcurves (EA + simplex fine-tuning, FP64)"
    roof = roofline_of(main_form, "fitness_kernel (FP64)")
    roof["traffic"] = fitness_traffic()
    roof["traffic_unit"] = "B/launch"
    roof["algorithmic_bytes"] = FITNESS_TRAFFIC["algorithmic_bytes_per_launch"]
    out = {
        "metric": "binary-lens magnifications/s; fits/hour at >=90% success, plain vs chosen "
                  "form",
        "value": main_form["mags_per_s"],
        "unit": "magnifications/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main_form["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.n_lc} lightcurves x {args.epochs} uniform epochs, "
                               f"population {args.pop}, FP64 chi^2 with profiled Fs, Fb, "
                               f"{args.steps}-generation fit",
                   "n_lc": args.n_lc, "epochs": args.epochs, "pop": args.pop,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fits_per_hour": main_form["fits_per_hour"],
        "success_rate": main_form["success"],
        "chosen_form": chosen,
        "fits_per_hour_at_90pct": at90,
        "success_study": study,
        "forms": forms,
        "iterated_simplex": iterated,
        "paper_tables": paper,
    }
    summary = dict(
        plain_mags_per_s=main_form["mags_per_s"], plain_ms_per_step=main_form["ms_per_step"],
        plain_roofline_frac=roof["frac"],
        mixed_mags_per_s=forms.get("mixed", {}).get("mags_per_s"),
        chosen_mags_per_s=chosen["mags_per_s"] if chosen else None,
        chosen_ms_per_step=chosen["ms_per_step"] if chosen else None,
        chosen_roofline_frac=chosen["roofline"]["frac"] if chosen else None,
        chosen_fits_per_hour=chosen["fits_per_hour"] if chosen else None,
        fits_per_hour_at_90pct={k: v for k, v in (at90 or {}).items()
                                if k not in ("gpu_seconds", "workload")})
    log("bench: summary " + json.dumps(summary))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

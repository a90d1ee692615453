"""Benchmark of the batched binary-lens fitness + EA generation on one MI355X.

Workload (the batched FP64 fitting configuration): 256 synthetic lightcurves
of 1000 uniform epochs over t0 +- 2 tE (sigma = 1% of the flux), population
256 per lightcurve.  A step is one generation of the whole hot path for the
whole batch: decode, magnification of all 256 x 256 x 1000 (individual,
epoch) pairs, least-squares fluxes and chi^2, then the EA generation, replayed
from one HIP graph.  The default run times a full fit (500 generations) in
the plain FP64 form and in the mixed-precision form, reports the success rate
(best chi^2 <= chi^2 of the true parameters + 10) and fits/hour, the fitness
kernel's roofline fraction, and the CPU oracle timed on a bounded sample.
Time to 90% success is measured for the plain EA and for the learned form
(proposal seeding), each with the paper's simplex fine-tuning of the
fittest solution at every checkpoint.  Then the ragged batching workload (4096 lightcurves of 200-5000 irregular
epochs, population 128) is timed per generation, and on the same lightcurves
the plain EA is compared with the learned form: a proposal network trained
on generated lightcurves seeds half of every population (at the start and at
each restart) and the EA's chi^2 decides.

Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FLOPs of one magnification + fit update as the fitness kernel
# computes it (counted from its source; fma = 2, reciprocal = 1 plus its
# Newton refinement steps): source position and polynomial coefficients,
# per sweep of the simultaneous root iteration over the five roots, image
# test + det J + magnification, and the weighted least-squares row update.
FLOP_COEF = 106
FLOP_SWEEP64 = 760
FLOP_SWEEP32 = 680
FLOP_IMAGES = 345
FLOP_LSQ = 50
# per image refined on the lens equation: one residual/g evaluation at the
# root, one Newton step, one evaluation at the new point
FLOP_POLISH = 150
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (fma) x 2.4 GHz, the same
# for FP64 and for unpacked FP32 (packed FP32 is not used)
PEAK_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
N_GEN_FIT = 500
# HBM traffic of one launch of the FP64 chi^2 fitness kernel on the default
# workload and schedule, from rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by a
# copy kernel of known size (profiles/fitness_kernel_fp64_256lc_1000ep_pop256_
# traffic.md).  Valid only for the kernel source it was taken on.
FITNESS_TRAFFIC = dict(source_sha256_16="9f43dbfc9d015751", bytes_per_launch=15.35e6,
                       algorithmic_bytes_per_launch=10.86e6)


def fitness_traffic():
    import hashlib
    src = os.path.join(ROOT, "paper_1208_4830_amd", "csrc", "sblm_fitness.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return FITNESS_TRAFFIC["bytes_per_launch"] if sha == FITNESS_TRAFFIC["source_sha256_16"] \
        else None


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
                    help="lightcurves of the ragged workload (0 = skip it)")
    ap.add_argument("--ragged-steps", type=int, default=30)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tune-after", type=int, default=30,
                    help="generations the scratch state evolves before the autotuner")
    ap.add_argument("--success-max-gen", type=int, default=1600,
                    help="generation cap of the time-to-90%%-success runs (0 = skip them)")
    ap.add_argument("--success-every", type=int, default=100)
    ap.add_argument("--learned-gens", type=int, default=300,
                    help="generations of the plain-vs-learned comparison on the ragged "
                         "workload (0 = skip it)")
    ap.add_argument("--learned-every", type=int, default=100)
    ap.add_argument("--iterated", default="16,4,10000",
                    help="iterated-simplex comparison: slots per lightcurve,runs per slot,"
                         "max steps per run (empty: skip)")
    ap.add_argument("--paper-lc", type=int, default=256,
                    help="lightcurves per paper-shaped experiment (Tables 2-3); 0 skips")
    ap.add_argument("--paper-checkpoints", default="500,1000,3000")
    ap.add_argument("--islands", default="8,50,2",
                    help="island form for the success comparison: islands,migrate every,"
                         "migrants (empty: skip)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device 4 times (a kernel of "
                         "known traffic that scales the profiler's byte counters)")
    ap.add_argument("--train-network", action="store_true",
                    help="train the proposal network even when no success run uses it")
    ap.add_argument("--mlp-samples", type=int, default=1 << 20)
    ap.add_argument("--mlp-epochs", type=int, default=32)
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
    # sweeps per solve (lane level) for the algorithmic FLOP count
    st = sblm.new_stats()
    scratch.evaluate(stats=st)
    torch.cuda.synchronize()
    s = sblm.stats_dict(st)
    sweeps = s["n_iter"] / max(s["n_solves"], 1)
    # dominant kernel: fitness evaluation, timed with events on the stream
    # it is launched on (the current stream)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.kernel_reps):
        scratch.evaluate(stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    k_ms = e0.elapsed_time(e1) / args.kernel_reps
    scratch.close()

    # the timed fit: fresh state with the chosen schedule, `steps` generations
    state = sblm.EAState(cfg, lcs, 1)
    state.set_schedule(*sched)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    state.fit(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    summ = state.summary()
    best = np.array([summ[k].best_chi2 for k in range(n_lc)])
    success = float(np.mean(best <= chi2_true + 10.0))
    state.close()

    polished = s["n_polished"] / max(s["n_solves"], 1)
    if mode == sblm.FP64:
        flop = FLOP_COEF + sweeps * FLOP_SWEEP64 + FLOP_IMAGES + FLOP_LSQ
    else:  # FP32 sweeps, then FP64 sweeps
        n32 = s["n_iter_fp32"] / max(s["n_solves"], 1)
        flop = FLOP_COEF + n32 * FLOP_SWEEP32 + (sweeps - n32) * FLOP_SWEEP64 \
            + FLOP_IMAGES + FLOP_LSQ
    flop += polished * FLOP_POLISH
    # what the wavefronts executed: lockstep sweeps (n_wave_iter) instead of
    # the lanes' own need
    wave = s["n_wave_iter"] / max(s["n_solves"], 1)
    flop_exec = flop + (wave - sweeps) * FLOP_SWEEP64
    ms_step = dt * 1e3 / steps
    return dict(
        mags_per_s=mags_per_gen * steps / dt,
        ms_per_step=ms_step,
        fits_per_hour=n_lc * 3600.0 / (N_GEN_FIT * ms_step / 1e3),
        success=success, generations=steps,
        kernel_ms=k_ms, kernel_mags_per_s=mags_per_gen / (k_ms / 1e3),
        sweeps_per_solve=sweeps, flop_per_mag=flop,
        kernel_tflops=flop * mags_per_gen / (k_ms / 1e3) / 1e12,
        kernel_tflops_executed=flop_exec * mags_per_gen / (k_ms / 1e3) / 1e12,
        capped=s["n_capped"], fallback=s["n_fallback"],
        wave_sweeps_per_solve=s["n_wave_iter"] / max(s["n_solves"], 1),
        polished_per_solve=s["n_polished"] / max(s["n_solves"], 1),
        schedule=dict(zip(("lanes", "waves_per_block", "persistent", "asynchronous"), sched)))


def success_run(sblm, torch, lcs, chi2_true, pop, mode, sched, lo, hi, proposals=None,
                max_gen=1600, every=100, target=0.9, seed=7, passes=3, islands=None):
    """EA with optional proposal seeding; at every checkpoint the fittest
    solution of each lightcurve is fine-tuned by `passes` simplex passes, each
    restarted from the last (on a copy: the EA continues untouched), as the
    paper's "EA with amoeba".  `sched` is fixed, not autotuned: lanes per
    individual and the epoch stepping change the roots at the rounding level
    and with them the EA's path, so a fixed schedule makes these runs
    reproducible on any device.
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
        if hit_ea is None and s_ea >= target:
            hit_ea = (gens, ea_s)
        if hit_nm is None and s_nm >= target:
            hit_nm = (gens, ea_s + nm_s)
        if hit_nm is not None:
            break
    state.close()
    per_hour = lambda h: n_lc * 3600.0 / h[1] if h else None
    return dict(target=target, curve=curve,
                ea_amoeba=dict(reached=hit_nm is not None,
                               generations=hit_nm[0] if hit_nm else None,
                               gpu_seconds=hit_nm[1] if hit_nm else None,
                               fits_per_hour=per_hour(hit_nm)),
                ea_alone=dict(reached=hit_ea is not None,
                              generations=hit_ea[0] if hit_ea else None,
                              gpu_seconds=hit_ea[1] if hit_ea else None,
                              fits_per_hour=per_hour(hit_ea)))


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
    net = sblm.MLP(batch_max=1024, seed=2)
    batch = 1024
    steps = args.mlp_epochs * (args.mlp_samples // batch)
    t0 = time.perf_counter()
    loss = net.train(xb, yt, batch=batch, epochs=args.mlp_epochs, lr0=2e-3, lr1=1e-5)
    sync()
    t_train = time.perf_counter() - t0
    lc = loss.cpu().numpy()
    step_s = t_train / max(steps, 1)
    mfma_tflops = 6.0 * batch * MLP_GEMM_WEIGHTS / step_s / 1e12
    info = dict(samples=args.mlp_samples, epochs=args.mlp_epochs, batch=batch, steps=steps,
                data_seconds=t_data, train_seconds=t_train, us_per_step=step_s * 1e6,
                loss_first=float(lc[:16].mean()), loss_last=float(lc[-16:].mean()),
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


def learned_form(sblm, torch, lcs, chi2_true, pop, sched, lo, hi, net, train_info, args):
    """Plain EA vs the EA whose population is half seeded (and re-seeded at
    every restart) by the proposal network, both with the simplex
    fine-tuning at every checkpoint."""
    out, t_inf = propose(sblm, torch, net, lcs)
    plain = success_run(sblm, torch, lcs, chi2_true, pop, sblm.FP64, sched, lo, hi,
                        max_gen=args.learned_gens, every=args.learned_every)
    learned = success_run(sblm, torch, lcs, chi2_true, pop, sblm.FP64, sched, lo, hi,
                          proposals=out, max_gen=args.learned_gens, every=args.learned_every)
    n_lc = len(chi2_true)
    last_p, last_l = plain["curve"][-1], learned["curve"][-1]
    # GPU time for the learned form to match the plain form's last success
    hit = next((c for c in learned["curve"] if c["ea_amoeba"] >= last_p["ea_amoeba"]), None)
    return dict(
        workload=f"{n_lc} lightcurves, pop {pop}, {pop // 2} rows seeded at the start and at "
                 f"every restart; EA + three simplex passes from the fittest solution",
        training=train_info, inference_seconds=t_inf, plain=plain, learned=learned,
        learned_matches_plain_last=dict(
            plain_success=last_p["ea_amoeba"],
            plain_gpu_seconds=last_p["ea_seconds"] + last_p["amoeba_seconds"],
            learned_generations=hit["gen"] if hit else None,
            learned_gpu_seconds=(hit["ea_seconds"] + hit["amoeba_seconds"] + t_inf)
            if hit else None),
        gpu_seconds_per_fit_last=dict(
            plain=(last_p["ea_seconds"] + last_p["amoeba_seconds"]) / n_lc,
            learned=(last_l["ea_seconds"] + last_l["amoeba_seconds"] + t_inf) / n_lc,
            learned_with_training=(last_l["ea_seconds"] + last_l["amoeba_seconds"] + t_inf
                                   + train_info["data_seconds"] + train_info["train_seconds"])
            / n_lc))


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
    # success runs: a fixed schedule (see success_run)
    sched = (16, 4, 1, 0)
    net = train_info = None
    if args.success_max_gen > 0 or args.learned_gens > 0 or args.train_network:
        log("bench: training the proposal network on generated lightcurves")
        net, train_info = train_proposals(sblm, torch, args)
        log(f"bench: training: {json.dumps(train_info)}")
    success = None
    if args.success_max_gen > 0:
        log("bench: time to 90% success, plain and learned, EA + simplex fine-tuning")
        out_p, t_inf = propose(sblm, torch, net, lcs)
        success = dict(
            plain=success_run(sblm, torch, lcs, chi2_true, args.pop, sblm.FP64, sched, lo, hi,
                              max_gen=args.success_max_gen, every=args.success_every),
            learned=success_run(sblm, torch, lcs, chi2_true, args.pop, sblm.FP64, sched, lo,
                                hi, proposals=out_p, max_gen=args.success_max_gen,
                                every=args.success_every),
            inference_seconds=t_inf)
        if args.islands:
            isl = tuple(int(v) for v in args.islands.split(","))
            success["islands"] = success_run(sblm, torch, lcs, chi2_true, args.pop, sblm.FP64,
                                             sched, lo, hi, max_gen=args.success_max_gen,
                                             every=args.success_every, islands=isl)
            success["islands"]["config"] = dict(islands=isl[0], pop_per_island=args.pop // isl[0],
                                                migrate_every=isl[1], migrants=isl[2])
        if args.iterated:
            success["iterated_simplex"] = iterated_run(sblm, torch, lcs, chi2_true, lo, hi,
                                                       *(int(v) for v in
                                                         args.iterated.split(",")))
        lrn = success["learned"]["ea_amoeba"]
        if lrn["gpu_seconds"] is not None:  # proposals are part of the learned fit's GPU time
            lrn["gpu_seconds"] += t_inf
            lrn["fits_per_hour"] = args.n_lc * 3600.0 / lrn["gpu_seconds"]
        log(f"bench: success: {json.dumps(success)}")

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

    ragged = None
    learned = None
    if args.ragged_lc > 0:
        log(f"bench: ragged workload, {args.ragged_lc} lightcurves of 200-5000 epochs, pop 128")
        wr = inputs.ragged_workload(4, args.ragged_lc)
        yr, wr_w, lcs_r = make_batch(sblm, torch, wr)
        c_true_r, _, _ = sblm.sblm_chi2(lcs_r, torch.as_tensor(wr.theta.copy(), device="cuda"), 1)
        ragged = run_form(sblm, torch, lcs_r, wr, c_true_r.cpu().numpy(), 128,
                          args.ragged_steps, args, sblm.FP64)
        ragged["workload"] = (f"{args.ragged_lc} lightcurves, L ~ U{{200..5000}} "
                              f"(total {int(wr.off[-1])} epochs), nightly cadence, pop 128")
        log(f"bench: ragged: {json.dumps(ragged)}")
        if args.learned_gens > 0:
            log("bench: learned form (proposal network) vs plain EA on the ragged workload")
            learned = learned_form(sblm, torch, lcs_r, c_true_r.cpu().numpy(), 128,
                                   (8, 4, 1, 0), lo, hi, net, train_info, args)
            log(f"bench: learned: {json.dumps(learned)}")
        del lcs_r
    if net is not None:
        net.close()

    cpu = None
    if not args.no_cpu:
        log("bench: CPU oracle sample")
        cpu = cpu_baseline(wl, y, w, args.pop, args.cpu_seconds)
        cpu["single_fit"] = single_fit(sblm, torch, cpu["cores"])
        log(f"bench: cpu {json.dumps(cpu)}")

    out = {
        "metric": "binary-lens magnifications/s (batched fitness + EA generation)",
        "value": main_form["mags_per_s"],
        "unit": "magnifications/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main_form["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.n_lc} lightcurves x {args.epochs} uniform epochs, "
                               f"population {args.pop}, FP64 chi^2 with profiled Fs, Fb",
                   "n_lc": args.n_lc, "epochs": args.epochs, "pop": args.pop,
                   "parallelism": "single GPU"},
        "fits_per_hour": main_form["fits_per_hour"],
        "fits_per_hour_at_90pct": ({f: success[f]["ea_amoeba"]["fits_per_hour"]
                                    for f in ("plain", "learned", "islands") if f in success}
                                   if success else None),
        "time_to_90pct_success": success,
        "success_rate": main_form["success"],
        "forms": forms,
        "ragged": ragged,
        "learned": learned,
        "paper_tables": paper,
        "roofline": {"bound": "alu", "achieved": main_form["kernel_tflops"],
                     "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": main_form["kernel_tflops"] / PEAK_VALU_TFLOPS,
                     "traffic": fitness_traffic(), "traffic_unit": "B/launch",
                     "algorithmic_bytes": FITNESS_TRAFFIC["algorithmic_bytes_per_launch"],
                     "executed_tflops": main_form["kernel_tflops_executed"],
                     "executed_frac": main_form["kernel_tflops_executed"] / PEAK_VALU_TFLOPS,
                     "kernel": "fitness_kernel (FP64)",
                     "flop_per_magnification": main_form["flop_per_mag"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

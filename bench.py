"""Benchmark: full population-annealing runs of the 2D Ising model on one GPU.

Workload (the paper's sample-program defaults): L = 64, R = 20000, theta = 100,
beta 0 -> 1 in 200 fixed steps of 0.005, random initial spins.  One benchmark
"step" is one complete PA run: initial state, then 200 x (resample, theta
sweeps, measurement), through the C ABI's pa_anneal (the schedule in one call,
one host round trip per temperature step).  The metric is attempted spin flips
per ns over the whole run, L^2 theta sum_i R_i / t_run (the inverse of the
paper's time per spin flip).  The same runs driven one call at a time from
Python are reported beside it.

Prints one JSON line.  The dominant kernel (the sweep) is timed by the library
with HIP events on the run's stream, inside the timed runs; its roofline is the
VALU issue rate (the sweep is bound by integer ALU work for the random numbers,
not by HBM).  The CPU oracle is timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

L, R, THETA, DBETA, NSTEPS = 64, 20000, 100, 0.005, 200

# ALU roofline of the sweep:
#   peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 VALU lane-slots/s
#   (one full-rate 32-bit VALU operation on one lane = one slot; the
#   32x32->64 multiply runs at full rate on gfx950).
#   work per attempted flip: the minimal evaluation of the chain's random
#   numbers for a 32-site word is the first 2 Philox4x32-10 blocks (8 bit planes
#   decide a site except with probability 2^-8), 10 rounds x (2 multiplies +
#   2 three-input xors) = 40 slots each, plus about 32 slots of bit-sliced
#   neighbour, class and comparison logic: (2*40 + 32) / 32 = 3.5 slots.
VALU_PEAK_SLOTS = 256 * 4 * 16 * 2.4e9
HBM_PEAK = 8.0e12  # bytes/s
SLOTS_PER_FLIP = 3.5
PROFILE = os.path.join(ROOT, "profiles", "sweep_kernel_L64_R20000_theta100.md")
KERNEL_SRCS = [os.path.join(ROOT, "paper_1703_03676_amd", "csrc", f)
               for f in ("pa_internal.h", "pa_device.h", "pa_sweep.hip")]


def kernel_source_hash():
    """First 16 hex digits of the sha256 of the sweep kernel's sources."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_counters():
    """From the committed counter profile of the sweep: HBM bytes per launch
    and VALU instructions per 32-site word and half sweep, or (None, None)
    when the kernel source has changed since the counters were taken."""
    import re
    try:
        txt = open(PROFILE).read()
        want = re.search(r"sha256\[:16\] = ([0-9a-f]{16})", txt).group(1)
        val = float(re.search(r"traffic_bytes_per_launch = ([0-9.e+]+)", txt).group(1))
        valu = float(re.search(r"VALU instructions per 32-site word and half sweep: [^=]*= ([0-9.]+)", txt).group(1))
    except (OSError, AttributeError, ValueError):
        return None, None
    return (val, valu) if kernel_source_hash() == want else (None, None)


def measured_traffic():
    """HBM bytes per sweep launch from the committed counter profile (None if stale)."""
    return measured_counters()[0]


def one_run(pa, torch, seed, layout, sweep_events=None):
    """One full run through the single-step calls (pa_resample, pa_sweep,
    pa_observables per temperature step, from Python)."""
    run = pa.Run(L, R, seed=seed, layout=layout)
    stream = torch.cuda.current_stream()
    run.observables()
    flips = 0
    for i in range(1, NSTEPS + 1):
        run.resample(i * DBETA)
        n = run.state()["R"]
        if sweep_events is not None:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run.sweep(THETA)
            e1.record(stream)
            sweep_events.append((e0, e1, n))
        else:
            run.sweep(THETA)
        flips += L * L * THETA * n
        run.observables()
    last = run.observables()
    run.close()
    return flips, last


def anneal_run(pa, seed, layout, sweeps=None, heatbath=False, lcg=False):
    """One full run through pa_anneal (the whole schedule in one call, one
    host round trip per temperature step).  The library times every sweep
    launch with HIP events on the run's stream; (ms, flips) pairs are appended
    to `sweeps`."""
    run = pa.Run(L, R, seed=seed, layout=layout, heatbath=heatbath, lcg=lcg)
    run.observables()
    obs, ms = run.anneal(beta_f=1.0, dbeta=DBETA, theta=THETA, mode="fixed", sweep_times=True)
    run.close()
    assert len(obs) == NSTEPS
    flips = [L * L * THETA * o["R"] for o in obs]
    if sweeps is not None:
        sweeps.extend(zip(ms, flips))
    return sum(flips), obs[-1]


UPDATES = {"metropolis": {}, "heatbath": {"heatbath": True}, "lcg": {"lcg": True}}


def time_layout(pa, torch, layout, steps, warmup, update="metropolis"):
    """Timed full runs through pa_anneal (the headline: Metropolis)."""
    kw = UPDATES[update]
    for w in range(warmup):
        anneal_run(pa, 1 + w % 3, layout, **kw)
    torch.cuda.synchronize()
    sweeps = []
    total_flips = 0
    t0 = time.perf_counter()
    for k in range(steps):
        f, last = anneal_run(pa, 1 + k % 3, layout, sweeps, **kw)
        total_flips += f
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    sweep_ms = [m for m, _ in sweeps]
    sweep_flips = [f for _, f in sweeps]
    return {
        "flips": total_flips,
        "seconds": t,
        "flips_per_ns": total_flips / (t * 1e9),
        "ms_per_run": 1e3 * t / steps,
        "sweep_ms_avg": sum(sweep_ms) / len(sweep_ms),
        "sweep_flips_avg": sum(sweep_flips) / len(sweep_flips),
        "sweep_share": sum(sweep_ms) / (1e3 * t),
        "e_final": last["e"],
        "betaF_per_N_final": last["betaF_per_N"],
    }


def time_step_calls(pa, torch, layout, steps):
    """The same runs driven one C-ABI call at a time from Python, for
    comparison with pa_anneal (not the headline)."""
    one_run(pa, torch, 1, layout)
    torch.cuda.synchronize()
    events = []
    total_flips = 0
    t0 = time.perf_counter()
    for k in range(steps):
        f, _ = one_run(pa, torch, 1 + k % 3, layout, events)
        total_flips += f
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    sweep_ms = [a.elapsed_time(b) for a, b, _ in events]
    return {"flips_per_ns": total_flips / (t * 1e9), "ms_per_run": 1e3 * t / steps,
            "sweep_ms_avg": sum(sweep_ms) / len(sweep_ms)}


def host_cores():
    """Cores this process may run on, at most 16 (the host CPU share of one
    GPU on the measurement machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _oracle_leg(Rs, threads, seconds_target):
    """The oracle on L = 64, theta = 100, fixed dbeta = 0.005 with Rs
    replicas, for the first temperature steps until about seconds_target."""
    import oracle

    o = oracle.Run(L, Rs, seed=1)
    o.set_threads(threads)
    o.init()
    o.measure()
    flips = 0
    t0 = time.perf_counter()
    i = 0
    while time.perf_counter() - t0 < seconds_target and i < NSTEPS:
        i += 1
        o.resample(i * DBETA)
        n = o.population
        o.sweep(THETA)
        o.measure()
        flips += L * L * THETA * n
    t = time.perf_counter() - t0
    return {
        "value": flips / (t * 1e9),
        "unit": "attempted spin flips/ns",
        "cores": threads,
        "kind": "oracle",
        "sample": "L=64, theta=100, dbeta=0.005, R=%d replicas, first %d temperature steps (%.2e flips, %.1f s), "
                  "%d thread(s) over replicas; host CPU: %s"
                  % (Rs, i, flips, t, threads, platform.processor() or platform.machine()),
    }


def cpu_baseline(seconds_target=10.0):
    """The oracle on the host's cores (OpenMP over replicas, at most 16
    threads), and on one core beside it, each on a bounded sample of the
    same workload."""
    n = host_cores()
    out = _oracle_leg(400 * n, n, seconds_target) if n > 1 else _oracle_leg(400, 1, seconds_target)
    out["single_core"] = _oracle_leg(400, 1, seconds_target) if n > 1 else dict(out)
    return out


def _exact_betaF(L, beta):
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import exact  # exact finite-torus solution, used only to report accuracy
    return exact.torus_exact(L, beta)["betaF_per_N"]


def run_plain_adaptive(pa, L, R_, theta, alpha, beta_f, seed, mhr=False):
    """One run through the single-run C ABI with host bisection each step."""
    run = pa.Run(L, R_, seed=seed, layout="bits", mhr=mhr)
    run.observables()
    flips = 0
    nsteps = 0
    while run.state()["beta"] < beta_f:
        b = run.adapt_beta(alpha, beta_f)
        run.resample(b)
        flips += L * L * theta * run.state()["R"]
        run.sweep(theta)
        run.observables()
        nsteps += 1
    return run, flips, nsteps


def anneal_adaptive(pa, torch, L, R_, theta, alpha, seed, mhr=False):
    """The same adaptive run through pa_anneal (one host round trip per step,
    the resampling copy fused into the sweep's load, the statistics taken in
    the sweep's epilogue).  Returns the run, the wall time and the step
    observables."""
    run = pa.Run(L, R_, seed=seed, layout="bits", mhr=mhr)
    run.observables()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    obs = run.anneal(beta_f=1.0, alpha_star=alpha, theta=theta, mode="adaptive")
    torch.cuda.synchronize()
    return run, time.perf_counter() - t0, obs


def _anneal_line(L, theta, t, obs, plain_last):
    """Summary of a pa_anneal run, with whether it ended in the plain run's state."""
    flips = sum(L * L * theta * o["R"] for o in obs)
    return {"run_wall_time_s": t, "flips_per_ns": flips / (t * 1e9), "temperature_steps": len(obs),
            "same_final_observables_as_plain": all(obs[-1][k] == plain_last[k]
                                                   for k in ("beta", "R", "sumE", "sumE2", "sumM4"))}


def workload_l128_adaptive(pa, torch):
    """L=128, R=50000, theta=50, adaptive dbeta (alpha*=0.85), multi-histogram
    reweighting on a 1000-point beta grid; plain single-run form, then the
    same run through pa_anneal."""
    import numpy as np
    L, R_, theta = 128, 50000, 50
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run, flips, nsteps = run_plain_adaptive(pa, L, R_, theta, 0.85, 1.0, seed=1, mhr=True)
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    t1 = time.perf_counter()
    rw = run.reweight(np.linspace(0.0, 1.0, 1000))
    t_rw = time.perf_counter() - t1
    last = run.observables()
    run.close()
    arun, t_a, obs = anneal_adaptive(pa, torch, L, R_, theta, 0.85, seed=1, mhr=True)
    arun.close()
    return {
        "workload": "L=128, R=50000, theta=50, adaptive alpha*=0.85, beta 0->1, MHR on 1000 betas",
        "flips_per_ns": flips / (t_run * 1e9), "run_wall_time_s": t_run, "temperature_steps": nsteps,
        "reweight_s": t_rw, "betaF_per_N_final": last["betaF_per_N"],
        "betaF_per_N_exact": _exact_betaF(L, 1.0),
        "mhr_C_peak_beta": float(np.linspace(0.0, 1.0, 1000)[int(np.argmax([o["C"] for o in rw]))]),
        "pa_anneal": _anneal_line(L, theta, t_a, obs, last),
    }


BATCH64_LR = [(L, R_) for L in (16, 32, 64, 128) for R_ in (5000, 20000)]


def _batch64_runs(seed0):
    return [dict(L=L, R=R_, seed=seed0 + 8 * k + s, layout="bits")
            for k, (L, R_) in enumerate(BATCH64_LR) for s in range(8)]


def _batch_errors(b, runs):
    return [abs(b.history(r)[-1]["betaF_per_N"] - _exact_betaF(sp["L"], 1.0)) for r, sp in enumerate(runs)]


def workload_batch64(pa, torch, sequential=True):
    """64 runs, (L, R) in {16,32,64,128} x {5000,20000}, theta=20, adaptive
    alpha*=0.85, beta 0->1: plain adaptive one run at a time, batched
    adaptive (one graph replay per step for all runs) and batched learned."""
    import numpy as np
    theta, alpha = 20, 0.85
    out = {"workload": "64 runs, (L,R) in {16,32,64,128}x{5000,20000}, 8 seeds each, theta=20, "
                       "adaptive alpha*=0.85, beta 0->1"}
    runs = _batch64_runs(1)
    if sequential:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        errs, flips, steps = [], 0, 0
        for sp in runs:
            run, f, n = run_plain_adaptive(pa, sp["L"], sp["R"], theta, alpha, 1.0, sp["seed"])
            errs.append(abs(run.observables()["betaF_per_N"] - _exact_betaF(sp["L"], 1.0)))
            flips += f
            steps += n
            run.close()
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out["plain_adaptive"] = {"s_per_run": t / len(runs), "total_s": t, "flips_per_ns": flips / (t * 1e9),
                                 "steps": steps, "mean_abs_dbetaF_per_N": float(np.mean(errs))}
    sched = dict(beta_f=1.0, alpha_star=alpha, alpha_tol=0.01, theta=theta, mode="adaptive")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = pa.Batch(runs, sched)
    b.run()
    t = time.perf_counter() - t0
    steps = sum(len(b.history(r)) - 1 for r in range(len(runs)))
    flips = sum(sp["L"] ** 2 * theta * o["R"] for r, sp in enumerate(runs) for o in b.history(r)[1:])
    ev_a = sum(b.choice_stats(r)[0] for r in range(len(runs)))
    host_a = sum(b.choice_stats(r)[1] for r in range(len(runs)))
    out["batched_adaptive"] = {"s_per_run": t / len(runs), "total_s": t, "flips_per_ns": flips / (t * 1e9),
                               "steps": steps, "mean_abs_dbetaF_per_N": float(np.mean(_batch_errors(b, runs))),
                               "overlap_evals_per_step": ev_a / steps, "host_us_choosing_per_step": 1e6 * host_a / steps}
    # learned: train on the bisection pairs of the adaptive batch, then new seeds
    x, tt = b.training_pairs()
    b.close()
    m = pa.Mlp(max_batch=512, seed=0)
    xc, tc = torch.from_numpy(x).cuda(), torch.from_numpy(tt).cuda()
    t0 = time.perf_counter()
    m.fit_norm(xc, tc)
    losses = m.train(xc, tc, batch=256, epochs=200, lr=3e-3, momentum=0.9, seed=1)
    t_train = time.perf_counter() - t0
    params, norm = m.params()
    runs2 = _batch64_runs(1001)
    sched2 = dict(sched, mode="learned")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bl = pa.Batch(runs2, sched2)
    bl.set_model(params, norm)
    bl.run()
    t = time.perf_counter() - t0
    props = sum(bl.learned_stats(r)[0] for r in range(len(runs2)))
    acc = sum(bl.learned_stats(r)[1] for r in range(len(runs2)))
    steps = sum(len(bl.history(r)) - 1 for r in range(len(runs2)))
    flips = sum(sp["L"] ** 2 * theta * o["R"] for r, sp in enumerate(runs2) for o in bl.history(r)[1:])
    ev_l = sum(bl.choice_stats(r)[0] for r in range(len(runs2)))
    host_l = sum(bl.choice_stats(r)[1] for r in range(len(runs2)))
    out["batched_learned"] = {"s_per_run": t / len(runs2), "total_s": t, "flips_per_ns": flips / (t * 1e9),
                              "steps": steps, "proposals": props, "accepted": acc,
                              "overlap_evals_per_step": ev_l / steps, "host_us_choosing_per_step": 1e6 * host_l / steps,
                              "mean_abs_dbetaF_per_N": float(np.mean(_batch_errors(bl, runs2))),
                              "training_pairs": int(len(tt)), "train_s": t_train,
                              "train_loss_first_last": [float(losses[0]), float(losses[-1])]}
    # shared schedule (Sec. 2.3, several runs): per (L, R) the first seed adapts,
    # the other seven follow it, and the eight runs are combined by the
    # free-energy-weighted average of Sec. 2.2
    runs3 = _batch64_runs(2001)
    sched3 = []
    for k in range(len(BATCH64_LR)):
        sched3.append(dict(sched, mode="adaptive"))
        sched3.extend(dict(beta_f=1.0, theta=theta, mode="follow", leader=8 * k) for _ in range(7))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bs = pa.Batch(runs3, sched3)
    bs.run()
    t = time.perf_counter() - t0
    steps = sum(len(bs.history(r)) - 1 for r in range(len(runs3)))
    flips = sum(sp["L"] ** 2 * theta * o["R"] for r, sp in enumerate(runs3) for o in bs.history(r)[1:])
    single, combined = [], []
    for k, (L_, _) in enumerate(BATCH64_LR):
        hs = [bs.history(8 * k + s) for s in range(8)]
        ex = _exact_betaF(L_, 1.0)
        single.extend(abs(h[-1]["betaF_per_N"] - ex) for h in hs)
        combined.append(abs(pa.weighted_average(hs, L_ * L_)[-1]["betaF_per_N"] - ex))
    out["batched_shared_schedule"] = {"s_per_run": t / len(runs3), "total_s": t, "flips_per_ns": flips / (t * 1e9),
                                      "steps": steps, "mean_abs_dbetaF_per_N_single": float(np.mean(single)),
                                      "mean_abs_dbetaF_per_N_weighted_8": float(np.mean(combined))}
    bs.close()
    out["_model"] = (params, norm)
    return out


def workload_l256_learned(pa, torch):
    """L=256, R=100000, theta=20, beta 0->1: plain adaptive single run, then a
    batched learned run with a proposer trained on the adaptive pairs of the 64-run batch."""
    c4 = workload_batch64(pa, torch, sequential=False)
    params, norm = c4.pop("_model")
    L, R_, theta = 256, 100000, 20
    out = {"workload": "L=256, R=100000, theta=20, beta 0->1, adaptive vs learned (alpha*=0.85)"}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run, flips, nsteps = run_plain_adaptive(pa, L, R_, theta, 0.85, 1.0, seed=5)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    last = run.observables()
    out["plain_adaptive"] = {"run_wall_time_s": t, "flips_per_ns": flips / (t * 1e9), "steps": nsteps,
                             "betaF_per_N_error": abs(last["betaF_per_N"] - _exact_betaF(L, 1.0))}
    run.close()
    arun, t_a, obs = anneal_adaptive(pa, torch, L, R_, theta, 0.85, seed=5)
    arun.close()
    out["pa_anneal_adaptive"] = _anneal_line(L, theta, t_a, obs, last)
    b = pa.Batch([dict(L=L, R=R_, seed=6, layout="bits")],
                 dict(beta_f=1.0, alpha_star=0.85, alpha_tol=0.01, theta=theta, mode="learned"))
    b.set_model(params, norm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run()
    t = time.perf_counter() - t0
    h = b.history(0)
    flips = sum(L * L * theta * o["R"] for o in h[1:])
    p, a = b.learned_stats(0)
    out["batched_learned"] = {"run_wall_time_s": t, "flips_per_ns": flips / (t * 1e9), "steps": len(h) - 1,
                              "proposals": p, "accepted": a,
                              "betaF_per_N_error": abs(h[-1]["betaF_per_N"] - _exact_betaF(L, 1.0))}
    return out


def workload_l64_heatbath(pa, torch):
    """The headline workload (L=64, R=20000, theta=100, 200 fixed steps of
    dbeta = 0.005, bit store, through pa_anneal) with each update rule in the
    same process: Metropolis with the bit-sliced Philox uniforms, heat-bath,
    and Metropolis with the in-line LCG uniforms of the paper's multi-spin
    variant.  Run time, sweep kernel time and the free-energy error at
    beta = 1 against the exact finite-torus value, over three seeds each."""
    exact_bf = _exact_betaF(L, 1.0)
    out = {"workload": "L=64, R=20000, theta=100, beta 0->1 in 200 steps of 0.005, bit store, pa_anneal: "
                       "Metropolis vs heat-bath vs LCG-variant sweeps"}
    for name, hb, lcg in (("metropolis", False, False), ("heatbath", True, False), ("lcg", False, True)):
        anneal_run(pa, 9, "bits", heatbath=hb, lcg=lcg)  # warm-up
        torch.cuda.synchronize()
        sweeps, errs, flips = [], [], 0
        t0 = time.perf_counter()
        for seed in (1, 2, 3):
            f, last = anneal_run(pa, seed, "bits", sweeps, heatbath=hb, lcg=lcg)
            flips += f
            errs.append(abs(last["betaF_per_N"] - exact_bf))
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out[name] = {"ms_per_run": 1e3 * t / 3, "flips_per_ns": flips / (t * 1e9),
                     "sweep_ms_avg": sum(m for m, _ in sweeps) / len(sweeps),
                     "betaF_per_N_abs_error": errs}
    return out


def _paper_run(pa, torch, L_, R_, theta, layout):
    """One full run beta 0 -> 1 in 200 fixed steps of 0.005 through pa_anneal;
    returns (t_SF in ns, share of the run spent in sweep launches)."""
    run = pa.Run(L_, R_, seed=1, layout=layout)
    run.observables()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    obs, ms = run.anneal(beta_f=1.0, dbeta=0.005, theta=theta, mode="fixed", cap=256, sweep_times=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    run.close()
    flips = sum(L_ * L_ * theta * o["R"] for o in obs)
    return 1e9 * t / flips, 1e-3 * sum(ms) / t


def workload_paper_tables(pa, torch):
    """The paper's own timing tables re-run on one MI355X: t_SF = run time /
    attempted flips for full runs beta 0 -> 1 (200 steps of dbeta = 0.005; the
    paper does not state its dbeta), Table 2 (theta = 500, R = 50000,
    L = 16 ... 256, both stores) and Table 3 (L = 128, R in {2k, 10k, 50k,
    100k}, theta in {1, 5, 10, 50, 100, 200, 500}, bit store), with the share
    of each run spent in sweep launches (the quantity of Table 4)."""
    out = {"workload": "paper Tables 2-4 shapes: full runs beta 0->1, 200 steps of dbeta=0.005, pa_anneal",
           "table2": {}, "table3": {}}
    _paper_run(pa, torch, 64, 2000, 10, "bits")  # warm-up
    for L_ in (16, 32, 64, 128, 256):
        for layout in ("int8", "bits"):
            tsf, share = _paper_run(pa, torch, L_, 50000, 500, layout)
            out["table2"]["L=%d %s" % (L_, layout)] = {"t_SF_ns": tsf, "flips_per_ns": 1.0 / tsf,
                                                       "sweep_share": share}
            print("table2 L=%d %s t_SF %.5f ns" % (L_, layout, tsf), file=sys.stderr, flush=True)
    for R_ in (2000, 10000, 50000, 100000):
        for theta in (1, 5, 10, 50, 100, 200, 500):
            tsf, share = _paper_run(pa, torch, 128, R_, theta, "bits")
            out["table3"]["R=%d theta=%d" % (R_, theta)] = {"t_SF_ns": tsf, "flips_per_ns": 1.0 / tsf,
                                                           "sweep_share": share}
            print("table3 R=%d theta=%d t_SF %.5f ns" % (R_, theta, tsf), file=sys.stderr, flush=True)
    return out


def workload_resample_l256(pa, torch):
    """Resampling alone at L=256, R=100000 (both stores): 20 steps of dbeta =
    0.0005 from the initial population, no sweeps.  The replica copy moves
    2 x R x (N/8 or N) bytes per step and is the HBM-bound kernel of the path;
    the time per pa_resample call (counts, scan, scatter, copy, one host
    round trip) is reported with the bytes the copy moves."""
    L_, R_ = 256, 100000
    out = {"workload": "resampling only, L=256, R=100000, 20 steps of dbeta=0.0005, no sweeps"}
    for layout in ("bits", "int8"):
        run = pa.Run(L_, R_, seed=3, layout=layout)
        run.resample(0.0005)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        copied = 0
        for k in range(2, 22):
            info = run.resample(0.0005 * k)
            copied += info["R_new"]
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        rep = L_ * L_ // 8 if layout == "bits" else L_ * L_
        moved = 2 * copied * rep
        out[layout] = {"ms_per_resample": 1e3 * t / 20, "copy_bytes_per_step": moved / 20,
                       "GB_per_s_whole_call": moved / t / 1e9}
        run.close()
    return out


def workload_sweeps(pa, torch):
    """pa_sweep alone at each lattice size, bit store, beta = 0.44 (near the
    critical point), after one resampling from the initial population: three
    timed launches per shape (HIP events on the run's stream), the shortest
    reported.  Shapes: L=16 R=100000, L=32 R=50000, L=64 R=20000 (theta=100;
    register path) and L=128 R=50000 (theta=20), L=256 R=20000 (theta=5) (LDS
    path)."""
    out = {"workload": "pa_sweep alone, bit store, beta=0.44, one launch of theta sweeps per shape"}
    s = torch.cuda.current_stream()
    for L_, R_, theta in ((16, 100000, 100), (32, 50000, 100), (64, 20000, 100), (128, 50000, 20),
                          (256, 20000, 5)):
        run = pa.Run(L_, R_, seed=7, layout="bits")
        run.resample(0.44)
        run.sweep(theta)
        ev = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            run.sweep(theta)
            e1.record(s)
            ev.append((e0, e1))
        torch.cuda.synchronize()
        ms = min(a.elapsed_time(b) for a, b in ev)
        n = run.state()["R"]
        out["L=%d" % L_] = {"R": n, "theta": theta, "ms_per_launch": ms,
                            "flips_per_ns": L_ * L_ * theta * n / (ms * 1e6)}
        print("sweeps L=%d R=%d %.3f ms" % (L_, n, ms), file=sys.stderr, flush=True)
        run.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--layouts", default="bits,int8")
    ap.add_argument("--no-step-calls", action="store_true",
                    help="skip the comparison runs driven one C-ABI call at a time")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="end with one pa_resample of a fresh L=64, R=20000 population, whose replica copy "
                         "(known bytes) calibrates the HBM counters of a profiling run")
    ap.add_argument("--update", default="metropolis", choices=sorted(UPDATES),
                    help="update rule of the l64 workload's sweeps (the headline is metropolis)")
    ap.add_argument("--workload", default="l64",
                    choices=["l64", "l128_adaptive", "batch64", "l256_learned", "resample_l256", "l64_heatbath",
                             "l64_update_rules",
                             "paper_tables", "sweeps"],
                    help="l64 (default) is the headline workload; the others print their own JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(population annealing would shard by replica, one population share per GPU)", file=sys.stderr)
        return 2

    import torch
    import paper_1703_03676_amd as pa

    if not os.path.exists(pa.LIB_PATH):
        from paper_1703_03676_amd import build as hip_build
        hip_build.build()
    torch.cuda.set_device(0)
    if args.workload != "l64":
        fn = {"l128_adaptive": workload_l128_adaptive, "batch64": workload_batch64,
              "l256_learned": workload_l256_learned, "resample_l256": workload_resample_l256,
              "l64_heatbath": workload_l64_heatbath, "l64_update_rules": workload_l64_heatbath,
              "paper_tables": workload_paper_tables,
              "sweeps": workload_sweeps}[args.workload]
        res = fn(pa, torch)
        res.pop("_model", None)
        print(json.dumps(res), flush=True)
        return 0
    layouts = args.layouts.split(",")
    res = {lay: time_layout(pa, torch, lay, args.steps, args.warmup, args.update) for lay in layouts}
    steps_cmp = None if args.no_step_calls else time_step_calls(pa, torch, layouts[0], 2)
    if args.calibration_copy:
        cal = pa.Run(L, R, seed=9, layout=layouts[0])
        cal.observables()
        cal.resample(DBETA)
        torch.cuda.synchronize()
        cal.close()
    head = res[layouts[0]]
    achieved = head["sweep_flips_avg"] * SLOTS_PER_FLIP / (head["sweep_ms_avg"] * 1e-3)
    # the committed counter profile is of the Metropolis sweep on the bit store
    profiled = args.update == "metropolis" and layouts[0] == "bits"
    traffic, valu_per_word = measured_counters() if profiled else (None, None)
    # algorithmic HBM bytes of one sweep launch: every replica's spins read and
    # written once for all theta sweeps (N/8 or N bytes each way) plus E and M
    rep_bytes = L * L // 8 if layouts[0] == "bits" else L * L
    n_rep = head["sweep_flips_avg"] / (L * L * THETA)
    alg_bytes = 2 * n_rep * rep_bytes + 8 * n_rep
    out = {
        "metric": "attempted spin flips/ns + PA run wall-time (L=64,R=20000) on 1 MI355X vs HBM roofline",
        "value": round(head["flips_per_ns"], 3),
        "unit": "attempted spin flips/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_run"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "population annealing, 2D Ising L=64 periodic, R=20000, theta=100, "
                        "beta 0->1 fixed dbeta=0.005 (200 steps), random initial spins, "
                        "spin store: %s; one step = one full PA run (pa_anneal)" % layouts[0],
            "L": L, "R": R, "theta": THETA, "dbeta": DBETA, "temperature_steps": NSTEPS,
            "layout": layouts[0],
            "update": args.update,
        },
        "run_wall_time_s": round(head["ms_per_run"] / 1e3, 4),
        "roofline": {
            "bound": "alu",
            "kernel": ("rp_sweep_kernel<64>" if layouts[0] == "interleaved"
                       else "sweep_kernel<64,%s>" % layouts[0]),
            "achieved": round(achieved / 1e12, 3),
            "peak": round(VALU_PEAK_SLOTS / 1e12, 2),
            "unit": "Tops/s (VALU lane-slots, %.1f per attempted flip)" % SLOTS_PER_FLIP,
            "frac": round(achieved / VALU_PEAK_SLOTS, 4),
            "traffic": traffic,
            # counters of the same kernel (committed profile): VALU instructions per
            # 32-site word and half sweep, and what they make of the issue peak at
            # the measured launch time (4 cycles per wave64 instruction)
            "valu_instr_per_word": valu_per_word,
            "valu_issue_frac": (round(valu_per_word * head["sweep_flips_avg"] / 32 / 64 * 4
                                      / (head["sweep_ms_avg"] * 1e-3 * 2.4e9 * 1024), 4)
                                if valu_per_word else None),
            "hbm_frac": (round(traffic / (head["sweep_ms_avg"] * 1e-3) / HBM_PEAK, 5) if traffic else None),
            "hbm_bytes_algorithmic": round(alg_bytes),
            "hbm_frac_algorithmic": round(alg_bytes / (head["sweep_ms_avg"] * 1e-3) / HBM_PEAK, 5),
            "kernel_ms_avg": round(head["sweep_ms_avg"], 4),
            "flips_per_launch": head["sweep_flips_avg"],
            "kernel_share_of_run": round(head["sweep_share"], 4),
        },
        "layouts": {lay: {k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}
                    for lay, r in res.items()},
    }
    if steps_cmp:
        out["step_calls_%s" % layouts[0]] = {k: round(v, 4) for k, v in steps_cmp.items()}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Benchmark: full population-annealing runs of the 2D Ising model on one GPU.

Workload (the paper's sample-program defaults): L = 64, R = 20000, theta = 100,
beta 0 -> 1 in 200 fixed steps of 0.005, random initial spins.  One benchmark
"step" is one complete PA run: initial state, then 200 x (resample, theta
sweeps, measurement), all through the C ABI.  The metric is attempted spin
flips per ns over the whole run, L^2 theta sum_i R_i / t_run (the inverse of
the paper's time per spin flip).

Prints one JSON line.  The dominant kernel (the sweep) is timed with HIP events
on the run's stream; its roofline is the VALU issue rate (the sweep is bound by
integer ALU work for the random numbers, not by HBM).  The CPU oracle is timed
on a bounded sample of the same workload.
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
SLOTS_PER_FLIP = 3.5
PROFILE = os.path.join(ROOT, "profiles", "sweep_kernel_L64_R20000_theta100.md")
KERNEL_SRC = os.path.join(ROOT, "paper_1703_03676_amd", "csrc", "pa_kernels.hip")


def measured_traffic():
    """HBM bytes per sweep launch from the committed counter profile, or None
    when the kernel source has changed since the counters were taken."""
    import hashlib
    import re
    try:
        txt = open(PROFILE).read()
        want = re.search(r"sha256\[:16\] = ([0-9a-f]{16})", txt).group(1)
        val = float(re.search(r"traffic_bytes_per_launch = ([0-9.e+]+)", txt).group(1))
    except (OSError, AttributeError, ValueError):
        return None
    have = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]
    return val if have == want else None


def one_run(pa, torch, seed, layout, sweep_events=None):
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


def time_layout(pa, torch, layout, steps, warmup):
    for w in range(warmup):
        one_run(pa, torch, 1 + w % 3, layout)
    torch.cuda.synchronize()
    events = []
    total_flips = 0
    t0 = time.perf_counter()
    for k in range(steps):
        f, last = one_run(pa, torch, 1 + k % 3, layout, events)
        total_flips += f
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    sweep_ms = [a.elapsed_time(b) for a, b, _ in events]
    sweep_flips = [L * L * THETA * n for _, _, n in events]
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


def cpu_baseline(seconds_target=15.0):
    """The oracle, single-threaded, on a bounded sample of the same workload:
    L = 64, theta = 100, fixed dbeta = 0.005, with R = 400 replicas for the
    first temperature steps until about seconds_target of CPU time."""
    import oracle

    Rs = 400
    o = oracle.Run(L, Rs, seed=1)
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
        "cores": 1,
        "kind": "oracle",
        "sample": "L=64, theta=100, dbeta=0.005, R=%d replicas, first %d temperature steps (%.2e flips, %.1f s); "
                  "host CPU: %s" % (Rs, i, flips, t, platform.processor() or platform.machine()),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--layouts", default="bits,int8")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(population annealing shards by replica; see DESIGN.md)", file=sys.stderr)
        return 2

    import torch
    import paper_1703_03676_amd as pa

    if not os.path.exists(pa.LIB_PATH):
        from paper_1703_03676_amd import build as hip_build
        hip_build.build()
    torch.cuda.set_device(0)
    layouts = args.layouts.split(",")
    res = {lay: time_layout(pa, torch, lay, args.steps, args.warmup) for lay in layouts}
    head = res[layouts[0]]
    achieved = head["sweep_flips_avg"] * SLOTS_PER_FLIP / (head["sweep_ms_avg"] * 1e-3)
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
                        "spin store: %s; one step = one full PA run" % layouts[0],
            "L": L, "R": R, "theta": THETA, "dbeta": DBETA, "temperature_steps": NSTEPS,
            "layout": layouts[0],
        },
        "run_wall_time_s": round(head["ms_per_run"] / 1e3, 4),
        "roofline": {
            "bound": "alu",
            "kernel": "sweep_kernel<64,bits>",
            "achieved": round(achieved / 1e12, 3),
            "peak": round(VALU_PEAK_SLOTS / 1e12, 2),
            "unit": "Tops/s (VALU lane-slots, %.1f per attempted flip)" % SLOTS_PER_FLIP,
            "frac": round(achieved / VALU_PEAK_SLOTS, 4),
            "traffic": measured_traffic(),
            "kernel_ms_avg": round(head["sweep_ms_avg"], 4),
            "flips_per_launch": head["sweep_flips_avg"],
            "kernel_share_of_run": round(head["sweep_share"], 4),
        },
        "layouts": {lay: {k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}
                    for lay, r in res.items()},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

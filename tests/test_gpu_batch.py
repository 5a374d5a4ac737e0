"""Batched runs through the C ABI: every run of a mixed batch (lattice sizes,
stores, fixed and adaptive schedules, multi-histogram) is bit-identical to an
independent oracle run with the same seed and schedule; a run that fails stops
alone with its state at the last good step."""
import numpy as np
import pytest

import oracle

import paper_1703_03676_amd as pa  # noqa: E402  (a broken package fails, never skips)
import torch  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _close(a, b, rel=1e-12):
    return a == b or abs(a - b) <= rel * max(abs(a), abs(b))


def _same_obs(go, oo):
    for k in ("sumE", "sumE2", "sumAbsM", "sumM2", "sumM4", "R"):
        assert go[k] == oo[k], k
    for k in ("beta", "e", "C", "abs_m", "m2", "m4", "betaF_per_N", "S_per_N", "lnQ"):
        assert _close(go[k], oo[k]), (k, go[k], oo[k])


RUNS = [
    dict(L=16, R=300, seed=11, layout="bits"),
    dict(L=32, R=200, seed=12, run_id=5, layout="int8"),
    dict(L=64, R=40, seed=13, layout="bits", mhr=True),
    dict(L=16, R=500, seed=14, layout="int8", mhr=True),
    dict(L=128, R=6, seed=15, layout="bits"),
    dict(L=256, R=3, seed=16, layout="int8"),
    dict(L=32, R=150, seed=17, layout="bits"),
    dict(L=128, R=5, seed=18, layout="int8", heatbath=True),
]
SCHED = [
    dict(beta_f=1.0, dbeta=0.05, theta=5, mode="fixed"),
    dict(beta_f=1.0, alpha_star=0.85, theta=3, mode="adaptive"),
    dict(beta_f=0.8, dbeta=0.1, theta=2, mode="fixed"),
    dict(beta_f=1.2, alpha_star=0.8, theta=4, mode="adaptive"),
    dict(beta_f=0.6, dbeta=0.2, theta=1, mode="fixed"),
    dict(beta_f=0.5, dbeta=0.25, theta=1, mode="fixed"),
    dict(beta_f=0.9, alpha_star=0.9, theta=2, mode="adaptive"),
    dict(beta_f=0.6, dbeta=0.15, theta=3, mode="fixed"),
]


_TRACES = {}


def _oracle_trace(spec, sched):
    key = (tuple(sorted(spec.items())), tuple(sorted(sched.items())))
    if key not in _TRACES:
        _TRACES[key] = _make_oracle_trace(spec, sched)
    return _TRACES[key]


def _make_oracle_trace(spec, sched):
    o = oracle.Run(spec["L"], spec["R"], seed=spec["seed"], run_id=spec.get("run_id", 0),
                   heatbath=spec.get("heatbath", False))
    o.init()
    trace = [o.measure()]
    i = 0
    while o.beta < sched["beta_f"]:
        i += 1
        if sched["mode"] == "fixed":
            nb = max(1, int(round(sched["beta_f"] / sched["dbeta"])))
            b = sched["beta_f"] if i >= nb else i * sched["dbeta"]
            b = min(b, sched["beta_f"])
        else:
            b = o.adapt_beta(sched["alpha_star"], sched["beta_f"])
        o.resample(b)
        o.sweep(sched["theta"])
        trace.append(o.measure())
    return o, trace


@pytest.mark.parametrize("wpb,qcap", [(0, None), (1, None), (2, None), (4, None), (8, None), (2, 0), (4, 8)])
def test_mixed_batch_matches_independent_oracle_runs(wpb, qcap):
    # every sweep shape (waves per block; L = 256 takes at most 4, the largest
    # that fits its LDS) and, with qcap, the overflow route of the LDS path's
    # tie queue
    print("case mixed batch wpb=%d qcap=%s" % (wpb, qcap), flush=True)
    b = pa.Batch(RUNS, SCHED, waves_per_block=wpb)
    if wpb:
        for r, spec in enumerate(RUNS):
            assert b.waves_per_block(r) == (min(wpb, 4) if spec["L"] == 256 else wpb)
    if qcap is not None:
        b.set_tie_queue_cap(qcap)
    b.run()
    for r, (spec, sc) in enumerate(zip(RUNS, SCHED)):
        print("  run %d L=%d" % (r, spec["L"]), flush=True)
        assert b.status(r) == pa.PA_OK
        o, trace = _oracle_trace(spec, sc)
        hist = b.history(r)
        assert len(hist) == len(trace)
        for go, oo in zip(hist, trace):
            _same_obs(go, oo)
        gs, gE, gM = b.download_population(r)
        os_, oE, oM = o.get_population()
        assert np.array_equal(gE, oE) and np.array_equal(gM, oM) and np.array_equal(gs, os_)
        st = b.state(r)
        assert st["beta"] == sc["beta_f"] and st["lnZ"] == o.lnZ and st["sweeps"] == o.sweeps
        if spec.get("mhr"):
            betas = np.linspace(0.0, sc["beta_f"], 17)
            for go, oo in zip(b.reweight(r, betas), o.reweight(betas)):
                for k in ("e", "C", "abs_m", "m2", "m4", "betaF_per_N", "S_per_N"):
                    assert _close(go[k], oo[k]), (k, go[k], oo[k])


def test_batch_with_resampling_only_runs():
    """Runs with theta = 0 resample without sweeping, so they need the separate
    replica copy, whose step graph the batch replays only in steps where such
    a run resamples; here mixed with sweeping runs in the same steps (and the
    sweeping runs go on alone after the others have finished)."""
    print("case batch with theta = 0 runs", flush=True)
    runs = [dict(L=16, R=300, seed=31, layout="bits"), dict(L=64, R=40, seed=32, layout="int8"),
            dict(L=128, R=6, seed=33, layout="bits"), dict(L=32, R=150, seed=34, layout="int8"),
            dict(L=256, R=3, seed=35, layout="bits")]
    scheds = [dict(beta_f=0.6, dbeta=0.1, theta=0, mode="fixed"),
              dict(beta_f=0.6, dbeta=0.1, theta=2, mode="fixed"),
              dict(beta_f=0.4, dbeta=0.1, theta=0, mode="fixed"),
              dict(beta_f=0.9, alpha_star=0.85, theta=0, mode="adaptive"),
              dict(beta_f=0.8, dbeta=0.1, theta=1, mode="fixed")]
    b = pa.Batch(runs, scheds)
    b.run()
    for r, (spec, sc) in enumerate(zip(runs, scheds)):
        print("  run %d L=%d theta=%d" % (r, spec["L"], sc["theta"]), flush=True)
        assert b.status(r) == pa.PA_OK
        o, trace = _oracle_trace(spec, sc)
        hist = b.history(r)
        assert len(hist) == len(trace)
        for go, oo in zip(hist, trace):
            _same_obs(go, oo)
        gs, gE, gM = b.download_population(r)
        os_, oE, oM = o.get_population()
        assert np.array_equal(gE, oE) and np.array_equal(gM, oM) and np.array_equal(gs, os_)


def test_batch_equals_single_runs():
    # the same run alone through the single-run API
    print("case batch vs single", flush=True)
    spec, sc = RUNS[0], SCHED[0]
    b = pa.Batch([spec], [sc])
    b.run()
    g = pa.Run(spec["L"], spec["R"], seed=spec["seed"], layout=spec["layout"])
    trace = [g.observables()]
    for i in range(1, 21):
        g.resample(min(i * sc["dbeta"], 1.0) if i < 20 else 1.0)
        g.sweep(sc["theta"])
        trace.append(g.observables())
    for go, bo in zip(trace, b.history(0)):
        _same_obs(go, bo)


def test_failed_run_stops_alone():
    print("case failing run", flush=True)
    # capacity == R: the first upward fluctuation of R_i stops the run
    runs = [dict(L=16, R=64, seed=s, capacity=64, layout="bits") for s in range(1, 9)]
    runs.append(dict(L=16, R=300, seed=99, layout="bits"))
    sched = dict(beta_f=1.0, dbeta=0.05, theta=2, mode="fixed")
    b = pa.Batch(runs, sched)
    b.run()
    statuses = [b.status(r) for r in range(len(runs))]
    assert pa.PA_ECAPACITY in statuses[:-1]
    assert statuses[-1] == pa.PA_OK and b.state(len(runs) - 1)["beta"] == 1.0
    for r, spec in enumerate(runs[:-1]):
        o = oracle.Run(16, 64, seed=spec["seed"], capacity=64)
        o.init()
        o.measure()
        i = 0
        failed = False
        while o.beta < 1.0:
            i += 1
            try:
                o.resample(min(i * 0.05, 1.0) if i < 20 else 1.0)
            except OverflowError:
                failed = True
                break
            o.sweep(2)
            o.measure()
        assert failed == (statuses[r] == pa.PA_ECAPACITY)
        st = b.state(r)
        assert st["step"] == o.step and st["beta"] == o.beta and st["lnZ"] == o.lnZ
        gs, gE, gM = b.download_population(r)
        os_, oE, oM = o.get_population()
        assert np.array_equal(gs, os_) and np.array_equal(gE, oE)


def test_batch_argument_errors():
    with pytest.raises(pa.PaError):
        pa.Batch([dict(L=17, R=10, seed=1)], dict(beta_f=1.0, dbeta=0.1, theta=1))
    with pytest.raises(pa.PaError):
        pa.Batch([dict(L=16, R=10, seed=1)], dict(beta_f=1.0, dbeta=0.0, theta=1, mode="fixed"))
    with pytest.raises(pa.PaError):
        pa.Batch([dict(L=16, R=10, seed=1)], dict(beta_f=1.0, alpha_star=1.5, theta=1, mode="adaptive"))


def test_shared_schedule_and_weighted_average():
    """Run 0 adapts its temperatures; runs 1-4 (other seeds, both stores) follow
    it step for step.  Every follower equals an oracle run replaying the
    leader's temperatures, and the library's weighted average of the five runs
    equals the oracle's (Sec. 2.2)."""
    print("case shared schedule", flush=True)
    L, R, theta = 16, 400, 3
    runs = [dict(L=L, R=R, seed=100 + k, layout=("bits", "int8")[k % 2]) for k in range(5)]
    scheds = [dict(beta_f=1.0, alpha_star=0.85, theta=theta, mode="adaptive")] + \
        [dict(beta_f=5.0, theta=theta, mode="follow", leader=0) for _ in range(4)]
    b = pa.Batch(runs, scheds)
    b.run()
    hists = [b.history(r) for r in range(5)]
    betas = [o["beta"] for o in hists[0]]
    assert betas[-1] == 1.0 and len(betas) > 5
    for r in range(5):
        assert b.status(r) == pa.PA_OK
        assert [o["beta"] for o in hists[r]] == betas
    for r in range(1, 5):
        o = oracle.Run(L, R, seed=100 + r)
        o.init()
        trace = [o.measure()]
        for beta in betas[1:]:
            o.resample(beta)
            o.sweep(theta)
            trace.append(o.measure())
        for go, oo in zip(hists[r], trace):
            _same_obs(go, oo)
    from oracle import weighted
    got = pa.weighted_average(hists, L * L)
    want = weighted.weighted_average(hists, L * L)
    for g, w in zip(got, want):
        for k in ("e", "C", "abs_m", "m2", "m4", "betaF_per_N", "S_per_N"):
            assert _close(g[k], w[k]), k


def test_follow_schedule_validation():
    runs = [dict(L=16, R=50, seed=1), dict(L=16, R=50, seed=2)]
    with pytest.raises(pa.PaError):
        pa.Batch(runs, [dict(beta_f=1.0, dbeta=0.1, mode="fixed"), dict(mode="follow", leader=1)])
    with pytest.raises(pa.PaError):
        pa.Batch(runs, [dict(mode="follow", leader=1), dict(mode="follow", leader=0)])
    with pytest.raises(pa.PaError):
        pa.Batch(runs, [dict(beta_f=1.0, dbeta=0.1, mode="fixed"), dict(mode="follow", leader=7)])

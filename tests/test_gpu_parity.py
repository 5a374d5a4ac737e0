"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Spins, energies, magnetisations, copy counts, population sizes and the
adaptive inverse temperatures must be bit-identical; FP64 quantities derived
from them (free energy, entropy, observables, reweighting) agree to 1e-12
relative.  Inputs are seeded: the method's own initial state, or synthetic
populations from tests/inputs.py.
"""
import numpy as np
import pytest

import inputs
import oracle

import paper_1703_03676_amd as pa  # noqa: E402  (a broken package fails, never skips)
import torch  # noqa: E402

pytestmark = pytest.mark.gpu

LAYOUTS = ["int8", "bits"]
# population sizes spanning several blocks with a ragged last one
R_OF_L = {16: 300, 32: 70, 64: 9, 128: 5, 256: 3}
FP_REL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _same_population(g, o):
    gs, gE, gM = g.download_population()
    os_, oE, oM = o.get_population()
    assert gs.shape == os_.shape
    assert np.array_equal(gE, oE)
    assert np.array_equal(gM, oM)
    assert np.array_equal(gs, os_)


def _close(a, b, rel=FP_REL):
    return a == b or abs(a - b) <= rel * max(abs(a), abs(b))


def _same_obs(go, oo):
    for k in ("sumE", "sumE2", "sumAbsM", "sumM2", "sumM4", "R"):
        assert go[k] == oo[k], k
    for k in ("beta", "e", "C", "abs_m", "m2", "m4", "betaF_per_N", "S_per_N", "lnQ"):
        assert _close(go[k], oo[k]), (k, go[k], oo[k])


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("L", [16, 32, 64, 128, 256])
def test_init_matches_oracle(L, layout):
    R = R_OF_L[L]
    print("case init L=%d layout=%s R=%d" % (L, layout, R), flush=True)
    g = pa.Run(L, R, seed=7, run_id=3, layout=layout)
    o = oracle.Run(L, R, seed=7, run_id=3)
    o.init()
    _same_population(g, o)
    _same_obs(g.observables(), o.measure())


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("L", [16, 32, 64, 128, 256])
@pytest.mark.parametrize("beta", [0.0, 1e-12, 0.2, 0.4406868, 0.9, 3.0])
def test_sweep_matches_oracle(L, layout, beta):
    R = R_OF_L[L]
    nsw = 4 if L <= 64 else 2
    print("case sweep L=%d layout=%s beta=%g" % (L, layout, beta), flush=True)
    spins = inputs.mixed_spins(R, L, seed=L + 1)
    g = pa.Run(L, R, seed=11, layout=layout)
    g.upload_population(spins, step=3, sweeps=17, beta=beta)
    o = oracle.Run(L, R, seed=11)
    o.set_population(spins, step=3, sweeps=17, beta=beta)
    _same_population(g, o)
    g.sweep(nsw)
    o.sweep(nsw)
    _same_population(g, o)
    assert g.state()["sweeps"] == o.sweeps == 17 + nsw


@pytest.mark.parametrize("layout", LAYOUTS)
def test_many_sweeps_exercise_ties(layout):
    # ~5e5 random decisions: about eight reach the low 16 bits (ties)
    L, R = 64, 9
    print("case ties layout=%s" % layout, flush=True)
    spins = inputs.random_spins(R, L, seed=5)
    g = pa.Run(L, R, seed=3, layout=layout)
    g.upload_population(spins, beta=0.6)
    o = oracle.Run(L, R, seed=3)
    o.set_population(spins, beta=0.6)
    g.sweep(25)
    o.sweep(25)
    _same_population(g, o)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("L", [16, 32, 64, 128, 256])
def test_resample_matches_oracle(L, layout):
    # replica sizes from 32 B to 64 KiB: every team width of the copy kernel
    # (16, 64 and 256 threads per child; 64 at L = 32 int8 and L = 128 bits)
    R = {16: 1500, 32: 900, 64: 700, 128: 120, 256: 40}[L]
    print("case resample L=%d layout=%s" % (L, layout), flush=True)
    spins = inputs.mixed_spins(R, L, seed=3)
    g = pa.Run(L, R, seed=5, layout=layout)
    o = oracle.Run(L, R, seed=5)
    g.upload_population(spins, step=4, sweeps=9, beta=0.3, lnZ=10.5)
    o.set_population(spins, step=4, sweeps=9, beta=0.3, lnZ=10.5)
    for beta in (0.3, 0.31, 0.45, 0.9):
        gi = g.resample(beta)
        oi = o.resample(beta)
        assert gi["R_new"] == oi["R_new"]
        assert gi["E_min"] == oi["E_min"]
        assert gi["lnQ"] == oi["lnQ"]  # same FP64 operations in the same order
        assert np.array_equal(g.download_counts(g.capacity), o.get_counts())
        _same_population(g, o)
        st = g.state()
        assert st["lnZ"] == o.lnZ and st["step"] == o.step and st["beta"] == o.beta


@pytest.mark.parametrize("heatbath", [False, True])
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("L,R,nsw", [(128, 6, 6), (256, 3, 3)])
@pytest.mark.parametrize("cap", [0, 8])
def test_tie_queue_overflow_route(cap, L, R, nsw, layout, heatbath):
    # a wave's tie queue limited to `cap` entries: the chunks with more tied
    # sites than that (every chunk with a tie at cap 0) are decided lane by
    # lane instead of through the queue; the chain is the same
    print("case tie queue cap=%d L=%d layout=%s hb=%d" % (cap, L, layout, heatbath), flush=True)
    spins = inputs.mixed_spins(R, L, seed=L + 7)
    g = pa.Run(L, R, seed=19, layout=layout, heatbath=heatbath)
    g.set_tie_queue_cap(cap)
    g.upload_population(spins, step=2, sweeps=5, beta=0.55)
    o = oracle.Run(L, R, seed=19, heatbath=heatbath)
    o.set_population(spins, step=2, sweeps=5, beta=0.55)
    g.sweep(nsw)
    o.sweep(nsw)
    _same_population(g, o)
    g.set_tie_queue_cap(256)
    g.sweep(1)
    o.sweep(1)
    _same_population(g, o)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("L,R", [(32, 700), (128, 60)])
def test_anneal_without_sweeps(L, R, layout):
    # theta = 0: pa_anneal resamples with the separate copy kernel (no sweep
    # to fuse it into) and measures; compared with the oracle step by step
    print("case anneal theta=0 L=%d layout=%s" % (L, layout), flush=True)
    spins = inputs.mixed_spins(R, L, seed=4)
    g = pa.Run(L, R, seed=8, layout=layout)
    g.upload_population(spins, step=0, sweeps=0, beta=0.0, lnZ=float(L * L) * np.log(2.0))
    o = oracle.Run(L, R, seed=8)
    o.set_population(spins, step=0, sweeps=0, beta=0.0, lnZ=float(L * L) * np.log(2.0))
    res = g.anneal(beta_f=0.3, dbeta=0.05, theta=0)
    assert len(res) == 6
    for i, go in enumerate(res, start=1):
        o.resample(min(i * 0.05, 0.3) if i < 6 else 0.3)
        _same_obs(go, o.measure())
    _same_population(g, o)


def test_resample_many_blocks_uses_the_block_scan():
    """More than 1024 blocks of 256 parents: the scatter takes the block totals
    from a single-block scan instead of summing them itself; counts, R_i,
    parents (through the copied population) and the statistics that follow
    match the oracle."""
    L, R = 16, 300000
    print("case resample many blocks L=%d R=%d" % (L, R), flush=True)
    g = pa.Run(L, R, seed=5, layout="bits")
    o = oracle.Run(L, R, seed=5)
    o.init()
    gi, oi = g.resample(0.35), o.resample(0.35)
    assert gi == oi
    assert np.array_equal(g.download_counts(g.capacity), o.get_counts())
    _same_population(g, o)
    _same_obs(g.observables(), o.measure())


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("L,R,kind", [(64, 600, "ordered"), (64, 600, "mixed"), (128, 300, "mixed")])
def test_statistics_windows_and_multi_histogram(L, R, kind, layout):
    """Population statistics and the multi-histogram accumulators for narrow
    per-block energy windows (ordered) and for windows wider than the
    kernels' LDS tables (mixed: ordered and random replicas in one block),
    over several blocks with a ragged last one."""
    print("case stats L=%d R=%d %s layout=%s" % (L, R, kind, layout), flush=True)
    if kind == "ordered":
        spins = inputs.ordered_spins(R, L, seed=21, n_flipped_max=40)
    else:
        spins = inputs.mixed_spins(R, L, seed=22)
    g = pa.Run(L, R, seed=13, layout=layout, mhr=True)
    o = oracle.Run(L, R, seed=13)
    g.upload_population(spins, step=2, sweeps=5, beta=0.35, lnZ=3.0)
    o.set_population(spins, step=2, sweeps=5, beta=0.35, lnZ=3.0)
    _same_obs(g.observables(), o.measure())
    for beta in (0.36, 0.4):
        assert g.resample(beta) == o.resample(beta)
        g.sweep(1)
        o.sweep(1)
        _same_obs(g.observables(), o.measure())
    betas = np.linspace(0.3, 0.5, 11)
    for go, oo in zip(g.reweight(betas), o.reweight(betas)):
        for k in ("e", "C", "abs_m", "m2", "m4", "betaF_per_N", "S_per_N"):
            assert _close(go[k], oo[k], 1e-12), (k, go["beta"], go[k], oo[k])


@pytest.mark.parametrize("path", ["epilogue", "auto"])
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("L,R,kind", [(16, 3000, "mixed"), (64, 700, "ordered"), (64, 700, "mixed"),
                                      (128, 130, "mixed"), (256, 20, "mixed")])
def test_statistics_from_the_sweep_epilogue_single_calls(L, R, kind, layout, path):
    """Without the multi-histogram record, the statistics of a population made
    by a sweep (or by the recount after an upload) come from the sweep's
    epilogue and its gather; after a resampling with no sweep, from the
    statistics kernel.  Ordered and mixed populations give narrow and very
    wide energy windows; every measurement matches the oracle."""
    print("case epilogue stats single calls L=%d R=%d %s layout=%s path=%s" % (L, R, kind, layout, path),
          flush=True)
    if kind == "ordered":
        spins = inputs.ordered_spins(R, L, seed=41, n_flipped_max=40)
    else:
        spins = inputs.mixed_spins(R, L, seed=42)
    g = pa.Run(L, R, seed=23, layout=layout)
    g.set_stats_path(path)
    o = oracle.Run(L, R, seed=23)
    g.upload_population(spins, step=1, sweeps=3, beta=0.3, lnZ=2.0)
    o.set_population(spins, step=1, sweeps=3, beta=0.3, lnZ=2.0)
    _same_obs(g.observables(), o.measure())       # recount's epilogue
    for beta in (0.32, 0.5):
        assert g.resample(beta) == o.resample(beta)
        _same_obs(g.observables(), o.measure())   # statistics kernel
        g.sweep(2)
        o.sweep(2)
        g.sweep(1)                                # two sweeps in a row: only the last one's count
        o.sweep(1)
        _same_obs(g.observables(), o.measure())   # the last sweep's epilogue
    _same_population(g, o)


@pytest.mark.parametrize("kind", ["ordered", "mixed"])
def test_statistics_more_chunks_than_workgroups(kind):
    """The statistics kernel runs a bounded number of workgroups that take
    256-replica chunks in turn: R = 40000 gives 157 chunks, more than the
    workgroups, with a ragged last chunk.  Statistics, the multi-histogram
    accumulators and the reweighted observables match the oracle."""
    L, R = 16, 40000
    print("case stats chunks L=%d R=%d %s" % (L, R, kind), flush=True)
    if kind == "ordered":
        spins = inputs.ordered_spins(R, L, seed=31, n_flipped_max=30)
    else:
        spins = inputs.mixed_spins(R, L, seed=32)
    g = pa.Run(L, R, seed=17, layout="bits", mhr=True)
    o = oracle.Run(L, R, seed=17)
    g.upload_population(spins, step=2, sweeps=5, beta=0.35, lnZ=3.0)
    o.set_population(spins, step=2, sweeps=5, beta=0.35, lnZ=3.0)
    _same_obs(g.observables(), o.measure())
    for beta in (0.36, 0.4):
        assert g.resample(beta) == o.resample(beta)
        g.sweep(1)
        o.sweep(1)
        _same_obs(g.observables(), o.measure())
    _same_population(g, o)
    betas = np.linspace(0.3, 0.5, 11)
    for go, oo in zip(g.reweight(betas), o.reweight(betas)):
        for k in ("e", "C", "abs_m", "m2", "m4", "betaF_per_N", "S_per_N"):
            assert _close(go[k], oo[k], 1e-12), (k, go["beta"], go[k], oo[k])


def _l16_trace(run, nsteps, theta, dbeta, measure):
    trace = [measure()]
    for i in range(1, nsteps + 1):
        run.resample(i * dbeta)
        run.sweep(theta)
        trace.append(measure())
    return trace


@pytest.fixture(scope="module")
def oracle_l16_run():
    """L=16, R=1000, theta=10, dbeta=0.01, beta 0 -> 1 (100 steps), seed 1."""
    o = oracle.Run(16, 1000, seed=1)
    o.init()
    trace = _l16_trace(o, 100, 10, 0.01, o.measure)
    return o, trace


@pytest.mark.parametrize("layout", LAYOUTS)
def test_full_run_l16_r1000(layout, oracle_l16_run):
    print("case l16 run layout=%s" % layout, flush=True)
    o, otrace = oracle_l16_run
    g = pa.Run(16, 1000, seed=1, layout=layout)
    gtrace = _l16_trace(g, 100, 10, 0.01, g.observables)
    for go, oo in zip(gtrace, otrace):
        _same_obs(go, oo)
    _same_population(g, o)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_anneal_l16_run(layout, oracle_l16_run):
    """pa_anneal (one host round trip per step) against the oracle's step-by-
    step L=16, R=1000 run: every step's observables and the final population."""
    print("case anneal l16 run layout=%s" % layout, flush=True)
    o, trace = oracle_l16_run
    g = pa.Run(16, 1000, seed=1, layout=layout)
    _same_obs(g.observables(), trace[0])
    obs = g.anneal(beta_f=1.0, dbeta=0.01, theta=10, mode="fixed")
    assert len(obs) == 100
    for go, oo in zip(obs, trace[1:]):
        _same_obs(go, oo)
    _same_population(g, o)
    st = g.state()
    assert st["step"] == 100 and st["sweeps"] == 1000 and st["beta"] == 1.0 and st["lnZ"] == o.lnZ
    assert g.anneal(beta_f=1.0, dbeta=0.01, theta=10) == []  # already at beta_f


@pytest.mark.parametrize("layout", LAYOUTS)
def test_anneal_adaptive_with_reweighting(layout):
    """Adaptive pa_anneal with the multi-histogram record against the oracle
    stepped by hand, then interrupted and resumed (max_steps)."""
    print("case anneal adaptive layout=%s" % layout, flush=True)
    L, R, theta = 16, 2000, 5
    g = pa.Run(L, R, seed=9, layout=layout, mhr=True)
    o = oracle.Run(L, R, seed=9)
    o.init()
    _same_obs(g.observables(), o.measure())
    trace = []
    while o.beta < 1.0:
        b = o.adapt_beta(0.85, 1.0)
        o.resample(b)
        o.sweep(theta)
        trace.append(o.measure())
    first = g.anneal(beta_f=1.0, alpha_star=0.85, theta=theta, mode="adaptive", max_steps=3)
    rest = g.anneal(beta_f=1.0, alpha_star=0.85, theta=theta, mode="adaptive")
    assert len(first) == 3 and len(first) + len(rest) == len(trace)
    for go, oo in zip(first + rest, trace):
        _same_obs(go, oo)
    _same_population(g, o)
    betas = np.linspace(0.0, 1.2, 31)
    for go, oo in zip(g.reweight(betas), o.reweight(betas)):
        for k in ("e", "C", "abs_m", "m2", "m4", "betaF_per_N", "S_per_N"):
            assert _close(go[k], oo[k], 1e-12), (k, go["beta"], go[k], oo[k])


def _fixed_betas(step0, beta0, beta_f, dbeta):
    """Inverse temperatures of a fixed schedule after step step0 (the host's
    rule: i * dbeta, beta_f from step round(beta_f / dbeta) on)."""
    nb = max(1, round(beta_f / dbeta))
    out, i, b = [], step0, beta0
    while b < beta_f:
        i += 1
        b = max(beta_f if i >= nb else min(i * dbeta, beta_f), b)
        out.append(b)
    return out


@pytest.mark.parametrize("path", ["epilogue", "pass"])
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("L,R", [(16, 900), (32, 333), (64, 130), (128, 21), (256, 5)])
def test_anneal_statistics_from_the_sweep_epilogue(L, R, layout, path):
    """pa_anneal takes each step's statistics in the sweep's epilogue (per-wave
    atomics into accumulator slots and histogram copies, summed by a gather
    pass that clears them again) or in a separate pass, each forced here at
    every lattice size: every step's sums against the oracle, with partial last
    waves at L = 16 and 32, over two calls on one run, so leftovers of a step
    or of a call would show."""
    print("case anneal statistics L=%d R=%d layout=%s path=%s" % (L, R, layout, path), flush=True)
    theta = 2
    g = pa.Run(L, R, seed=13, layout=layout)
    g.set_stats_path(path)
    o = oracle.Run(L, R, seed=13)
    o.init()
    _same_obs(g.observables(), o.measure())
    got = g.anneal(beta_f=0.3, dbeta=0.1, theta=theta, mode="fixed")
    got += g.anneal(beta_f=0.6, dbeta=0.1, theta=theta, mode="fixed")
    want = _fixed_betas(0, 0.0, 0.3, 0.1) + _fixed_betas(3, 0.3, 0.6, 0.1)
    assert [go["beta"] for go in got] == want
    for go in got:
        o.resample(go["beta"])
        o.sweep(theta)
        _same_obs(go, o.measure())
    _same_population(g, o)


@pytest.mark.parametrize("path", ["epilogue", "pass"])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_anneal_refusal_in_the_middle_of_a_run(layout, path):
    """A step refused for capacity after other steps of the same pa_anneal
    call leaves the run at the last completed step, equal to the oracle's;
    runs that are not refused match the oracle at every step.  With the
    statistics in the sweep's epilogue, the refused step has published the
    refused population's statistics, which the run must not take for those
    of its current one."""
    print("case anneal refusal mid-run layout=%s path=%s" % (layout, path), flush=True)
    refused_late = 0
    for seed in range(1, 31):
        g = pa.Run(16, 100, seed=seed, capacity=100, layout=layout)
        g.set_stats_path(path)
        o = oracle.Run(16, 100, seed=seed, capacity=100)
        s = np.ones((3, 16, 16), np.int8)
        g.upload_population(s, step=1, beta=0.1)
        o.set_population(s, step=1, beta=0.1)
        trace, refused_at = [], None
        for k, b in enumerate(_fixed_betas(1, 0.1, 0.6, 0.1)):
            try:
                o.resample(b)
            except OverflowError:
                refused_at = k
                break
            o.sweep(2)
            trace.append(o.measure())
        if refused_at is None:
            obs = g.anneal(beta_f=0.6, dbeta=0.1, theta=2)
            assert len(obs) == len(trace)
            for go, oo in zip(obs, trace):
                _same_obs(go, oo)
        else:
            refused_late += refused_at > 0
            with pytest.raises(pa.CapacityError):
                g.anneal(beta_f=0.6, dbeta=0.1, theta=2)
            st = g.state()
            assert st["step"] == 1 + refused_at and st["sweeps"] == 2 * refused_at
            _same_obs(g.observables(), o.measure())
        _same_population(g, o)
        g.sweep(1)
        o.sweep(1)
        _same_population(g, o)
    assert refused_late > 0


@pytest.mark.parametrize("layout", LAYOUTS)
def test_anneal_from_an_ordered_population(layout):
    """pa_anneal from an ordered population (one energy bin) at high
    temperature, where the energy window widens by two orders of magnitude
    within the first steps.  Every step matches the oracle."""
    print("case anneal wide window layout=%s" % layout, flush=True)
    L, R, theta = 64, 400, 5
    g = pa.Run(L, R, seed=3, layout=layout)
    o = oracle.Run(L, R, seed=3)
    s = np.ones((R, L, L), np.int8)
    g.upload_population(s, step=1, beta=0.05)
    o.set_population(s, step=1, beta=0.05)
    trace = []
    for b in _fixed_betas(1, 0.05, 0.3, 0.05):
        o.resample(b)
        o.sweep(theta)
        trace.append(o.measure())
    obs = g.anneal(beta_f=0.3, dbeta=0.05, theta=theta)
    assert len(obs) == len(trace) == 5
    for go, oo in zip(obs, trace):
        _same_obs(go, oo)
    _same_population(g, o)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_anneal_capacity_refusal_keeps_state(layout):
    """A step refused for capacity inside pa_anneal leaves the run at the last
    completed step, usable, and equal to the oracle's."""
    print("case anneal capacity layout=%s" % layout, flush=True)
    refused = 0
    for seed in range(1, 25):
        g = pa.Run(16, 100, seed=seed, capacity=100, layout=layout)
        o = oracle.Run(16, 100, seed=seed, capacity=100)
        s = np.ones((3, 16, 16), np.int8)
        # step 1 at beta 0.1: the fixed schedule's next step is beta_2 = 0.2
        g.upload_population(s, step=1, beta=0.1)
        o.set_population(s, step=1, beta=0.1)
        try:
            o.resample(0.2)
            o.sweep(2)
            ok = True
        except OverflowError:
            ok = False
        if ok:
            obs = g.anneal(beta_f=0.2, dbeta=0.1, theta=2)
            assert len(obs) == 1
            _same_obs(obs[0], o.measure())
        else:
            refused += 1
            with pytest.raises(pa.CapacityError):
                g.anneal(beta_f=0.2, dbeta=0.1, theta=2)
            st = g.state()
            assert st["step"] == 1 and st["R"] == 3 and st["sweeps"] == 0 and st["beta"] == 0.1
            _same_obs(g.observables(), o.measure())
            g.sweep(1)
            o.sweep(1)
        _same_population(g, o)
    assert 0 < refused < 24


@pytest.mark.parametrize("layout", LAYOUTS)
def test_l64_r20000_full_size_sampled(layout):
    """L=64, R=20000, theta=100: full-size init and resampling compared
    element by element; the 100 sweeps compared on sampled replicas swept by
    the oracle alone at their slots; invariants checked on every replica."""
    L, R, theta = 64, 20000, 100
    print("case l64 r20000 layout=%s" % layout, flush=True)
    g = pa.Run(L, R, seed=1, layout=layout)
    o = oracle.Run(L, R, seed=1)
    o.init()
    _same_population(g, o)
    _same_obs(g.observables(), o.measure())
    gi, oi = g.resample(0.005), o.resample(0.005)
    assert gi == oi
    assert np.array_equal(g.download_counts(g.capacity), o.get_counts())
    _same_population(g, o)
    pre, _, _ = o.get_population()
    n = o.population
    g.sweep(theta)
    gs, gE, gM = g.download_population()
    rng = np.random.default_rng(0)
    slots = np.unique(np.concatenate([[0, 1, 63, 64, n - 1], rng.integers(0, n, 4)]))
    so = oracle.Run(L, R, seed=1)
    so.set_population(pre[slots], step=1, sweeps=0, beta=0.005)
    so.set_slots(slots)
    so.sweep(theta)
    ss, sE, sM = so.get_population()
    assert np.array_equal(ss, gs[slots]) and np.array_equal(sE, gE[slots]) and np.array_equal(sM, gM[slots])
    # every replica: E and M are those of its spins
    s = gs.astype(np.int32)
    assert np.array_equal(-(s * (np.roll(s, -1, 2) + np.roll(s, -1, 1))).sum(axis=(1, 2)), gE)
    assert np.array_equal(s.sum(axis=(1, 2)), gM)
    obs = g.observables()
    assert obs["sumE"] == int(gE.astype(np.int64).sum()) and obs["R"] == n


def _energy_of(spins):
    s = spins.astype(np.int32)
    return -(s * (np.roll(s, -1, 2) + np.roll(s, -1, 1))).sum(axis=(1, 2)), s.sum(axis=(1, 2))


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("L,R,theta,beta", [(128, 50000, 2, 0.44), (256, 100000, 1, 0.44)])
def test_full_size_lds_path_sampled(L, R, theta, beta, layout):
    """The LDS-path sweep at the full L=128 (R=50000) and L=256 (R=100000)
    workload sizes, in the benchmark's launch configuration: sampled replicas
    are swept again by the oracle alone at their slots; every replica's E and
    M sum to the population statistics."""
    print("case full-size L=%d R=%d layout=%s" % (L, R, layout), flush=True)
    g = pa.Run(L, R, seed=2, layout=layout)
    g.resample(beta)
    st = g.state()
    n = st["R"]
    rng = np.random.default_rng(1)
    slots = np.unique(np.concatenate([[0, 1, 63, 64, n - 1], rng.integers(0, n, 4)])).astype(np.int32)
    pre, pE, pM = g.download_replicas(slots)
    assert np.array_equal(_energy_of(pre)[0], pE) and np.array_equal(_energy_of(pre)[1], pM)
    g.sweep(theta)
    gs, gE, gM = g.download_replicas(slots)
    so = oracle.Run(L, len(slots), seed=2)
    so.set_population(pre, step=st["step"], sweeps=st["sweeps"], beta=st["beta"])
    so.set_slots(slots)
    so.sweep(theta)
    ss, sE, sM = so.get_population()
    assert np.array_equal(ss, gs) and np.array_equal(sE, gE) and np.array_equal(sM, gM)
    E, M = g.download_energies()
    obs = g.observables()
    assert obs["R"] == n == len(E)
    assert obs["sumE"] == int(E.astype(np.int64).sum())
    assert obs["sumAbsM"] == int(np.abs(M.astype(np.int64)).sum())


@pytest.mark.parametrize("layout", LAYOUTS)
def test_capacity_overflow_and_extinction(layout):
    print("case capacity layout=%s" % layout, flush=True)
    outcomes = []
    for seed in range(1, 25):
        # R = 100 from 3 equal replicas: R_new in 99..102, capacity 100
        g = pa.Run(4 * 4, 100, seed=seed, capacity=100, layout=layout)
        o = oracle.Run(16, 100, seed=seed, capacity=100)
        s = np.ones((3, 16, 16), np.int8)
        g.upload_population(s, beta=0.1)
        o.set_population(s, beta=0.1)
        try:
            o.resample(0.2)
            ok = True
        except OverflowError:
            ok = False
        if ok:
            g.resample(0.2)
        else:
            with pytest.raises(pa.CapacityError):
                g.resample(0.2)
            assert g.state()["step"] == 0 and g.state()["R"] == 3
            # the run stays usable after the refusal
            g.sweep(1)
            o.sweep(1)
        _same_population(g, o)
        outcomes.append(ok)
    assert not all(outcomes) and any(outcomes)
    # extinction: R = 1 from two equal replicas survives with probability 3/4
    ext = []
    for seed in range(1, 25):
        g = pa.Run(16, 1, seed=seed, capacity=8, layout=layout)
        o = oracle.Run(16, 1, seed=seed, capacity=8)
        s = np.ones((2, 16, 16), np.int8)
        g.upload_population(s, beta=0.1)
        o.set_population(s, beta=0.1)
        try:
            o.resample(0.2)
            dead = False
        except ArithmeticError:
            dead = True
        if dead:
            with pytest.raises(pa.ExtinctError):
                g.resample(0.2)
            assert g.state()["R"] == 2
        else:
            g.resample(0.2)
        _same_population(g, o)
        ext.append(dead)
    assert any(ext) and not all(ext)


def test_stats_path_hook_rejects_unknown_modes():
    g = pa.Run(16, 10, seed=1)
    for bad in (-1, 3):
        with pytest.raises(pa.PaError):
            g.set_stats_path(bad)
    for mode in ("auto", "epilogue", "pass"):
        g.set_stats_path(mode)


@pytest.mark.parametrize("path", ["epilogue", "pass"])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_anneal_extinction_keeps_state(layout, path):
    """A pa_anneal step that would leave no replica (R = 1 from two equal
    replicas dies with probability 1/4) sweeps an empty population, whose
    statistics are empty: the call raises, the run stays at its last step
    with the oracle's population and statistics, and carries on."""
    print("case anneal extinction layout=%s path=%s" % (layout, path), flush=True)
    ext = []
    for seed in range(1, 25):
        g = pa.Run(16, 1, seed=seed, capacity=8, layout=layout)
        g.set_stats_path(path)
        o = oracle.Run(16, 1, seed=seed, capacity=8)
        s = np.ones((2, 16, 16), np.int8)
        g.upload_population(s, step=1, beta=0.1)
        o.set_population(s, step=1, beta=0.1)
        try:
            o.resample(0.2)
            dead = False
        except ArithmeticError:
            dead = True
        if dead:
            with pytest.raises(pa.ExtinctError):
                g.anneal(beta_f=0.2, dbeta=0.1, theta=3)
            st = g.state()
            assert st["R"] == 2 and st["step"] == 1 and st["beta"] == 0.1
            _same_obs(g.observables(), o.measure())
            g.sweep(2)
            o.sweep(2)
            _same_obs(g.observables(), o.measure())
        else:
            o.sweep(3)
            got = g.anneal(beta_f=0.2, dbeta=0.1, theta=3)
            assert len(got) == 1
            _same_obs(got[0], o.measure())
        _same_population(g, o)
        ext.append(dead)
    assert any(ext) and not all(ext)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_adaptive_run_and_reweighting(layout):
    """Adaptive steps (alpha* = 0.85) with multi-histogram reweighting."""
    print("case adaptive layout=%s" % layout, flush=True)
    L, R, theta = 16, 2000, 5
    g = pa.Run(L, R, seed=9, layout=layout, mhr=True)
    o = oracle.Run(L, R, seed=9)
    o.init()
    _same_obs(g.observables(), o.measure())
    steps = 0
    while o.beta < 1.0:
        bo = o.adapt_beta(0.85, 1.0)
        bg = g.adapt_beta(0.85, 1.0)
        assert bg == bo
        assert g.alpha(bo) == o.alpha(bo)
        assert g.resample(bg) == o.resample(bo)
        g.sweep(theta)
        o.sweep(theta)
        _same_obs(g.observables(), o.measure())
        steps += 1
    assert steps > 5
    _same_population(g, o)
    betas = np.linspace(0.0, 1.2, 61)
    for go, oo in zip(g.reweight(betas), o.reweight(betas)):
        for k in ("e", "C", "abs_m", "m2", "m4", "betaF_per_N", "S_per_N"):
            assert _close(go[k], oo[k], 1e-12), (k, go["beta"], go[k], oo[k])


def test_runs_are_deterministic_and_keyed():
    print("case determinism", flush=True)
    a = pa.Run(32, 100, seed=4)
    b = pa.Run(32, 100, seed=4)
    c = pa.Run(32, 100, seed=4, run_id=1)
    for r in (a, b, c):
        r.resample(0.3)
        r.sweep(3)
    sa, sb, sc = (r.download_population()[0] for r in (a, b, c))
    assert np.array_equal(sa, sb)
    assert not np.array_equal(sa, sc)


def test_argument_errors_on_device_runs():
    g = pa.Run(16, 10, seed=1)
    with pytest.raises(pa.PaError):
        g.sweep(-1)
    with pytest.raises(pa.PaError):
        g.resample(-0.1)  # below the current beta
    with pytest.raises(pa.PaError):
        g.adapt_beta(1.5, 1.0)
    with pytest.raises(pa.PaError):
        g.reweight([0.1])  # run without the multi-histogram flag
    with pytest.raises(pa.PaError):
        g.upload_population(np.zeros((2, 16, 16), np.int8))  # spins must be +-1
    g.sweep(0)
    assert g.state()["sweeps"] == 0

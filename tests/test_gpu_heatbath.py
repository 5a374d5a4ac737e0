"""GPU parity of the heat-bath update (PA_FLAG_HEATBATH) against the oracle's
heat-bath mode: spins, E and M bit-identical after sweeps for every lattice
size, both stores and inverse temperatures from 0 to 3 (register and LDS
paths, tie resolution), a full pa_anneal run, sampled replicas at the full
L = 64 and L = 128 workload sizes, and heat-bath runs inside a batch next to
Metropolis runs."""
import numpy as np
import pytest

import inputs
import oracle

import paper_1703_03676_amd as pa  # noqa: E402  (a broken package fails, never skips)
import torch  # noqa: E402

pytestmark = pytest.mark.gpu

LAYOUTS = ["int8", "bits"]
R_OF_L = {16: 300, 32: 70, 64: 9, 128: 5, 256: 3}


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


def _same_population(g, o):
    gs, gE, gM = g.download_population()
    os_, oE, oM = o.get_population()
    assert np.array_equal(gE, oE)
    assert np.array_equal(gM, oM)
    assert np.array_equal(gs, os_)


def _energy_of(spins):
    s = spins.astype(np.int32)
    return -(s * (np.roll(s, -1, 2) + np.roll(s, -1, 1))).sum(axis=(1, 2)), s.sum(axis=(1, 2))


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("L", [16, 32, 64, 128, 256])
@pytest.mark.parametrize("beta", [0.0, 0.2, 0.4406868, 0.9, 3.0])
def test_heatbath_sweep_matches_oracle(L, layout, beta):
    R = R_OF_L[L]
    nsw = 4 if L <= 64 else 2
    print("case hb sweep L=%d layout=%s beta=%g" % (L, layout, beta), flush=True)
    spins = inputs.mixed_spins(R, L, seed=L + 3)
    g = pa.Run(L, R, seed=11, layout=layout, heatbath=True)
    g.upload_population(spins, step=2, sweeps=9, beta=beta)
    o = oracle.Run(L, R, seed=11, heatbath=True)
    o.set_population(spins, step=2, sweeps=9, beta=beta)
    g.sweep(nsw)
    o.sweep(nsw)
    _same_population(g, o)
    assert g.state()["sweeps"] == o.sweeps == 9 + nsw


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("L,R,nsw", [(64, 9, 25), (128, 5, 12), (256, 3, 4)])
def test_heatbath_many_sweeps_exercise_ties(L, R, nsw, layout):
    # every site draws a uniform, so ties past the high 16 bits occur about
    # once per 65536 decisions: these cases make several hundred thousand
    print("case hb ties L=%d layout=%s" % (L, layout), flush=True)
    spins = inputs.random_spins(R, L, seed=5)
    g = pa.Run(L, R, seed=3, layout=layout, heatbath=True)
    g.upload_population(spins, beta=0.6)
    o = oracle.Run(L, R, seed=3, heatbath=True)
    o.set_population(spins, beta=0.6)
    g.sweep(nsw)
    o.sweep(nsw)
    _same_population(g, o)


@pytest.mark.parametrize("heatbath", [True, False])
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("L", [16, 32, 64, 128, 256])
@pytest.mark.parametrize("kind", ["cols", "rows", "checker", "up"])
def test_structured_populations_match_oracle(kind, L, layout, heatbath):
    # regular patterns put every site of a replica in one class: stripes
    # have k = 0 everywhere (heat-bath decides them by the top bit of the
    # uniform, Metropolis flips them without one), the checkerboard k = -4,
    # all-up k = 4; on the LDS path one wave holds one replica, so no site of
    # the wave needs the later planes
    R = 4 if L >= 128 else 40
    print("case structured %s L=%d layout=%s hb=%d" % (kind, L, layout, heatbath), flush=True)
    spins = inputs.structured_spins(R, L, kind)
    for nsw in (1, 2):
        g = pa.Run(L, R, seed=21, layout=layout, heatbath=heatbath)
        g.upload_population(spins, step=1, sweeps=4, beta=0.3)
        o = oracle.Run(L, R, seed=21, heatbath=heatbath)
        o.set_population(spins, step=1, sweeps=4, beta=0.3)
        g.sweep(nsw)
        o.sweep(nsw)
        _same_population(g, o)
        g.close()


def test_metropolis_and_heatbath_runs_differ_on_the_gpu():
    spins = inputs.random_spins(9, 64, seed=2)
    runs = []
    for hb in (False, True):
        g = pa.Run(64, 9, seed=5, heatbath=hb)
        g.upload_population(spins, beta=0.4)
        g.sweep(3)
        runs.append(g.download_population()[0])
    assert not np.array_equal(runs[0], runs[1])


@pytest.fixture(scope="module")
def oracle_hb_l16_run():
    """Heat-bath L=16, R=1000, theta=10, dbeta=0.01, beta 0 -> 1, seed 4."""
    o = oracle.Run(16, 1000, seed=4, heatbath=True)
    o.init()
    trace = [o.measure()]
    for i in range(1, 101):
        o.resample(i * 0.01)
        o.sweep(10)
        trace.append(o.measure())
    return o, trace


@pytest.mark.parametrize("layout", LAYOUTS)
def test_heatbath_anneal_l16_run(layout, oracle_hb_l16_run):
    print("case hb anneal l16 layout=%s" % layout, flush=True)
    o, trace = oracle_hb_l16_run
    g = pa.Run(16, 1000, seed=4, layout=layout, heatbath=True)
    _same_obs(g.observables(), trace[0])
    obs = g.anneal(beta_f=1.0, dbeta=0.01, theta=10, mode="fixed")
    assert len(obs) == 100
    for go, oo in zip(obs, trace[1:]):
        _same_obs(go, oo)
    _same_population(g, o)
    assert g.state()["lnZ"] == o.lnZ


@pytest.mark.parametrize("layout", LAYOUTS)
def test_heatbath_l64_r20000_anneal_sampled(layout):
    """The benchmark's configuration with heat-bath sweeps: one pa_anneal step
    at L=64, R=20000, theta=100 (resampling copy fused into the sweep, grid
    sized by the capacity).  The oracle resamples the whole population; sampled
    replicas are then swept by the oracle alone at their slots.  E and M of
    every replica match its spins."""
    L, R, theta = 64, 20000, 100
    print("case hb l64 r20000 anneal layout=%s" % layout, flush=True)
    g = pa.Run(L, R, seed=6, layout=layout, heatbath=True)
    o = oracle.Run(L, R, seed=6, heatbath=True)
    o.init()
    obs = g.anneal(beta_f=0.005, dbeta=0.005, theta=theta, mode="fixed")
    o.resample(0.005)
    pre, _, _ = o.get_population()
    n = o.population
    assert obs[0]["R"] == n
    rng = np.random.default_rng(2)
    slots = np.unique(np.concatenate([[0, 1, 63, 64, n - 1], rng.integers(0, n, 4)])).astype(np.int32)
    gs, gE, gM = g.download_replicas(slots)
    so = oracle.Run(L, len(slots), seed=6, heatbath=True)
    so.set_population(pre[slots], step=1, sweeps=0, beta=0.005)
    so.set_slots(slots)
    so.sweep(theta)
    ss, sE, sM = so.get_population()
    assert np.array_equal(ss, gs) and np.array_equal(sE, gE) and np.array_equal(sM, gM)
    s_all, E_all, M_all = g.download_population()
    E2, M2 = _energy_of(s_all)
    assert np.array_equal(E2, E_all) and np.array_equal(M2, M_all)
    assert obs[0]["sumE"] == int(E_all.astype(np.int64).sum())


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("L,R,theta", [(128, 50000, 2), (256, 100000, 1)])
def test_heatbath_lds_path_full_size_sampled(L, R, theta, layout):
    """LDS-path heat-bath sweeps at the full L=128 and L=256 workload sizes:
    sampled replicas are swept again by the oracle alone at their slots."""
    print("case hb full-size L=%d R=%d layout=%s" % (L, R, layout), flush=True)
    g = pa.Run(L, R, seed=6, layout=layout, heatbath=True)
    g.resample(0.44)
    st = g.state()
    n = st["R"]
    rng = np.random.default_rng(2)
    slots = np.unique(np.concatenate([[0, 1, 63, 64, n - 1], rng.integers(0, n, 4)])).astype(np.int32)
    pre, _, _ = g.download_replicas(slots)
    g.sweep(theta)
    gs, gE, gM = g.download_replicas(slots)
    so = oracle.Run(L, len(slots), seed=6, heatbath=True)
    so.set_population(pre, step=st["step"], sweeps=st["sweeps"], beta=st["beta"])
    so.set_slots(slots)
    so.sweep(theta)
    ss, sE, sM = so.get_population()
    assert np.array_equal(ss, gs) and np.array_equal(sE, gE) and np.array_equal(sM, gM)
    E, M = g.download_energies()
    obs = g.observables()
    assert obs["R"] == n == len(E) and obs["sumE"] == int(E.astype(np.int64).sum())


def test_heatbath_runs_in_a_batch():
    """Heat-bath and Metropolis runs of the same lattice size and store in one
    batch: separate sweep groups, each run bit-identical to its oracle run."""
    print("case hb batch", flush=True)
    runs = [dict(L=32, R=200, seed=21, layout="bits", heatbath=True),
            dict(L=32, R=200, seed=22, layout="bits"),
            dict(L=128, R=20, seed=23, layout="int8", heatbath=True, mhr=True),
            dict(L=16, R=300, seed=24, layout="int8", heatbath=True)]
    scheds = [dict(beta_f=1.0, dbeta=0.05, theta=4, mode="fixed"),
              dict(beta_f=1.0, dbeta=0.05, theta=4, mode="fixed"),
              dict(beta_f=0.8, dbeta=0.1, theta=2, mode="fixed"),
              dict(beta_f=1.0, alpha_star=0.9, theta=3, mode="adaptive")]
    b = pa.Batch(runs, scheds)
    b.run()
    for r, (spec, sc) in enumerate(zip(runs, scheds)):
        print("  run %d L=%d hb=%s" % (r, spec["L"], spec.get("heatbath", False)), flush=True)
        assert b.status(r) == pa.PA_OK
        o = oracle.Run(spec["L"], spec["R"], seed=spec["seed"], heatbath=spec.get("heatbath", False))
        o.init()
        trace = [o.measure()]
        i = 0
        while o.beta < sc["beta_f"]:
            i += 1
            if sc["mode"] == "fixed":
                nb = int(round(sc["beta_f"] / sc["dbeta"]))
                bn = sc["beta_f"] if i >= nb else i * sc["dbeta"]
            else:
                bn = o.adapt_beta(sc["alpha_star"], sc["beta_f"])
            o.resample(bn)
            o.sweep(sc["theta"])
            trace.append(o.measure())
        hist = b.history(r)
        assert len(hist) == len(trace)
        for go, oo in zip(hist, trace):
            _same_obs(go, oo)
        gs, gE, gM = b.download_population(r)
        os_, oE, oM = o.get_population()
        assert np.array_equal(gE, oE) and np.array_equal(gM, oM) and np.array_equal(gs, os_)

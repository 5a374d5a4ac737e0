"""GPU parity of the in-line LCG variant of the sweep (PA_FLAG_LCG; Sec. 4,
one base-generator draw per word and update seeds an LCG that supplies the
word's uniforms) against the oracle's LCG mode: spins, E and M bit-identical
after sweeps for every lattice size, both stores and inverse temperatures
from 0 to 3, regular patterns, a full pa_anneal run, the full L = 64,
R = 20000 workload on sampled replicas, and LCG runs inside a batch."""
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


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("L", [16, 32, 64, 128, 256])
@pytest.mark.parametrize("beta", [0.0, 1e-12, 0.2, 0.4406868, 0.9, 3.0])
def test_lcg_sweep_matches_oracle(L, layout, beta):
    R = R_OF_L[L]
    nsw = 4 if L <= 64 else 2
    print("case lcg sweep L=%d layout=%s beta=%g" % (L, layout, beta), flush=True)
    spins = inputs.mixed_spins(R, L, seed=L + 5)
    g = pa.Run(L, R, seed=13, run_id=2, layout=layout, lcg=True)
    g.upload_population(spins, step=3, sweeps=11, beta=beta)
    o = oracle.Run(L, R, seed=13, run_id=2, lcg=True)
    o.set_population(spins, step=3, sweeps=11, beta=beta)
    g.sweep(nsw)
    o.sweep(nsw)
    _same_population(g, o)
    g.close()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("L", [16, 64, 128, 256])
@pytest.mark.parametrize("kind", ["cols", "checker", "up"])
def test_lcg_structured_populations(kind, L, layout):
    R = 4 if L >= 128 else 40
    print("case lcg structured %s L=%d layout=%s" % (kind, L, layout), flush=True)
    spins = inputs.structured_spins(R, L, kind)
    g = pa.Run(L, R, seed=22, layout=layout, lcg=True)
    g.upload_population(spins, step=1, sweeps=4, beta=0.3)
    o = oracle.Run(L, R, seed=22, lcg=True)
    o.set_population(spins, step=1, sweeps=4, beta=0.3)
    g.sweep(2)
    o.sweep(2)
    _same_population(g, o)
    g.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_lcg_anneal_l16_run(layout):
    # L=16, R=1000, theta=10, dbeta=0.01, beta 0 -> 1 (100 steps) through
    # pa_anneal, every step's observables against the oracle
    print("case lcg anneal L=16 layout=%s" % layout, flush=True)
    g = pa.Run(16, 1000, seed=1, layout=layout, lcg=True)
    o = oracle.Run(16, 1000, seed=1, lcg=True)
    o.init()
    g.observables()
    o.measure()
    res = g.anneal(beta_f=1.0, dbeta=0.01, theta=10)
    assert len(res) == 100
    for i, go in enumerate(res, start=1):
        o.resample(1.0 if i == 100 else i * 0.01)
        o.sweep(10)
        _same_obs(go, o.measure())
    _same_population(g, o)
    g.close()


def test_lcg_and_philox_runs_differ_and_agree_statistically():
    spins = inputs.random_spins(9, 64, seed=2)
    runs = []
    for lcg in (False, True):
        g = pa.Run(64, 9, seed=5, lcg=lcg)
        g.upload_population(spins, beta=0.4)
        g.sweep(3)
        runs.append(g.download_population()[0])
        g.close()
    assert not np.array_equal(runs[0], runs[1])


@pytest.mark.parametrize("layout", LAYOUTS)
def test_lcg_l64_r20000_anneal_full_size(layout):
    # the headline workload's shape (L = 64, R = 20000, theta = 100, dbeta =
    # 0.005), its first two temperature steps through pa_anneal, every
    # replica compared with the oracle (OpenMP over replicas)
    L, R, theta = 64, 20000, 100
    print("case lcg L=64 R=20000 layout=%s" % layout, flush=True)
    g = pa.Run(L, R, seed=2, layout=layout, lcg=True)
    o = oracle.Run(L, R, seed=2, lcg=True)
    o.set_threads(16)
    o.init()
    g.observables()
    res = g.anneal(beta_f=1.0, dbeta=0.005, theta=theta, max_steps=2)
    assert len(res) == 2
    for i, go in enumerate(res, start=1):
        o.resample(i * 0.005)
        o.sweep(theta)
        _same_obs(go, o.measure())
    _same_population(g, o)
    g.close()


def test_lcg_runs_in_a_batch():
    runs = [dict(L=32, R=200, seed=31, layout="bits", lcg=True),
            dict(L=128, R=6, seed=32, layout="int8", lcg=True),
            dict(L=32, R=200, seed=31, layout="bits")]
    sched = dict(beta_f=0.6, dbeta=0.1, theta=3, mode="fixed")
    print("case lcg batch", flush=True)
    b = pa.Batch(runs, sched)
    b.run()
    for r, spec in enumerate(runs):
        o = oracle.Run(spec["L"], spec["R"], seed=spec["seed"], lcg=spec.get("lcg", False))
        o.init()
        for i in range(1, 7):
            o.resample(0.6 if i == 6 else i * 0.1)
            o.sweep(3)
        gs, gE, gM = b.download_population(r)
        os_, oE, oM = o.get_population()
        assert np.array_equal(gE, oE) and np.array_equal(gM, oM) and np.array_equal(gs, os_)
    b.close()


def test_lcg_with_heatbath_is_refused():
    with pytest.raises(pa.PaError):
        pa.Run(16, 10, seed=1, heatbath=True, lcg=True)

"""Full-size parity over whole populations and several temperature steps.

* L = 64, R = 20000, theta = 100, fixed dbeta = 0.005 (the headline workload),
  through pa_anneal, the benchmark's launch configuration: the first two
  temperature steps, every replica and every observable.
* L = 128, R = 50000, theta = 50, adaptive steps to alpha* = 0.85 with the
  multi-histogram record (the L = 128 workload): the first three steps, the
  adaptive inverse temperatures bit-equal, every replica, and the reweighted
  observables.
* L = 128, R = 50000 and L = 256, R = 100000: the initial state and the first
  resampling of the whole population, element by element.

The oracle shares its replicas out among the host's cores (at most 16
threads) so that these sizes finish in minutes; its results do not depend on
the thread count.
"""
import os

import numpy as np
import pytest

import oracle

import paper_1703_03676_amd as pa  # noqa: E402  (a broken package fails, never skips)
import torch  # noqa: E402

pytestmark = pytest.mark.gpu

FP_REL = 1e-12
INT_KEYS = ("sumE", "sumE2", "sumAbsM", "sumM2", "sumM4", "R")
FP_KEYS = ("beta", "e", "C", "abs_m", "m2", "m4", "betaF_per_N", "S_per_N", "lnQ")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _close(a, b, rel=FP_REL):
    return a == b or abs(a - b) <= rel * max(abs(a), abs(b))


def _same_obs(go, oo, where):
    for k in INT_KEYS:
        assert go[k] == oo[k], (where, k, go[k], oo[k])
    for k in FP_KEYS:
        assert _close(go[k], oo[k]), (where, k, go[k], oo[k])


def _same_population(g, o, where):
    gs, gE, gM = g.download_population()
    os_, oE, oM = o.get_population()
    assert gs.shape == os_.shape, where
    assert np.array_equal(gE, oE), where
    assert np.array_equal(gM, oM), where
    assert np.array_equal(gs, os_), where


@pytest.fixture(scope="module")
def oracle_l64_two_steps():
    """Oracle run at L = 64, R = 20000: observables at beta_0 and after each of
    the first two fixed steps, and the population after each step."""
    L, R, theta, dbeta = 64, 20000, 100, 0.005
    print("case oracle L=64 R=20000, two steps, %d threads" % _threads(), flush=True)
    o = oracle.Run(L, R, seed=1)
    o.set_threads(_threads())
    o.init()
    obs = [o.measure()]
    pops = []
    for i in (1, 2):
        o.resample(i * dbeta)
        o.sweep(theta)
        obs.append(o.measure())
        pops.append(o.get_population())
        print("  oracle step %d done" % i, flush=True)
    return obs, pops


@pytest.mark.parametrize("layout", ["bits", "int8"])
def test_l64_r20000_first_two_steps_every_replica(layout, oracle_l64_two_steps):
    obs, pops = oracle_l64_two_steps
    print("case l64 r20000 two anneal steps layout=%s" % layout, flush=True)
    g = pa.Run(64, 20000, seed=1, layout=layout)
    _same_obs(g.observables(), obs[0], "beta0")
    for i in (1, 2):
        got = g.anneal(beta_f=1.0, dbeta=0.005, theta=100, max_steps=1)
        assert len(got) == 1
        _same_obs(got[0], obs[i], "step %d" % i)
        gs, gE, gM = g.download_population()
        os_, oE, oM = pops[i - 1]
        assert np.array_equal(gE, oE) and np.array_equal(gM, oM) and np.array_equal(gs, os_), i
    g.close()


def test_l128_r50000_adaptive_first_three_steps():
    L, R, theta, alpha = 128, 50000, 50, 0.85
    print("case l128 r50000 adaptive three steps, %d oracle threads" % _threads(), flush=True)
    g = pa.Run(L, R, seed=3, layout="bits", mhr=True)
    o = oracle.Run(L, R, seed=3)
    o.set_threads(_threads())
    o.init()
    _same_obs(g.observables(), o.measure(), "beta0")
    got = g.anneal(beta_f=1.0, alpha_star=alpha, theta=theta, mode="adaptive", max_steps=3)
    assert len(got) == 3
    for i in range(3):
        b = o.adapt_beta(alpha, 1.0)
        assert got[i]["beta"] == b, (i, got[i]["beta"], b)
        o.resample(b)
        o.sweep(theta)
        _same_obs(got[i], o.measure(), "step %d" % (i + 1))
        print("  step %d beta %.6f equal" % (i + 1, b), flush=True)
    _same_population(g, o, "after three steps")
    betas = np.linspace(0.0, got[-1]["beta"] * 1.5, 9)
    for go, oo in zip(g.reweight(betas), o.reweight(betas)):
        for k in ("e", "C", "abs_m", "m2", "m4", "betaF_per_N", "S_per_N"):
            assert _close(go[k], oo[k]), (k, go[k], oo[k])
    g.close()


@pytest.mark.parametrize("L,R", [(128, 50000), (256, 100000)])
def test_full_size_init_and_resample_every_replica(L, R):
    print("case full-size init + resample L=%d R=%d, %d oracle threads" % (L, R, _threads()), flush=True)
    o = oracle.Run(L, R, seed=4, run_id=2)
    o.set_threads(_threads())
    o.init()
    oo0 = o.measure()
    os0, oE0, oM0 = o.get_population()
    # a typical adaptive step at L = 128; at L = 256 a large one, where a few
    # low-energy parents take almost all of the population
    beta = 0.002 if L == 128 else 0.2
    oi = o.resample(beta)
    ocounts = o.get_counts()
    oo1 = o.measure()
    os1, oE1, oM1 = o.get_population()
    del o
    for layout in ("bits", "int8"):
        print("  layout %s" % layout, flush=True)
        g = pa.Run(L, R, seed=4, run_id=2, layout=layout)
        _same_obs(g.observables(), oo0, "init")
        gs, gE, gM = g.download_population()
        assert np.array_equal(gE, oE0) and np.array_equal(gM, oM0)
        assert np.array_equal(gs, os0)
        del gs
        gi = g.resample(beta)
        assert gi == oi, (gi, oi)
        assert np.array_equal(g.download_counts(g.capacity), ocounts)
        _same_obs(g.observables(), oo1, "resample")
        gs, gE, gM = g.download_population()
        assert np.array_equal(gE, oE1) and np.array_equal(gM, oM1)
        assert np.array_equal(gs, os1)
        del gs
        g.close()

"""Pins of the oracle's full PA runs against exact results: brute-force
enumeration at L = 4 and the exact finite-torus solution at L = 8 (free energy,
energy, specific heat, magnetisation moments), multi-histogram reweighting, and
the adaptive-step postconditions (Sec. 2.1-2.4)."""
import numpy as np
import pytest

import exact
import oracle


@pytest.fixture(scope="module")
def run_L4():
    r = oracle.Run(4, 20000, seed=1)
    r.init()
    obs = [r.measure()]
    for i in range(1, 21):
        r.resample(0.05 * i)
        r.sweep(5)
        obs.append(r.measure())
    return r, obs


@pytest.fixture(scope="module")
def run_L8():
    r = oracle.Run(8, 4000, seed=1)
    r.init()
    obs = [r.measure()]
    for i in range(1, 41):
        r.resample(0.025 * i)
        r.sweep(10)
        obs.append(r.measure())
    return r, obs


def test_beta0_measurement(run_L4):
    _, obs = run_L4
    o = obs[0]
    assert o["beta"] == 0.0 and o["R"] == 20000
    assert o["betaF_per_N"] == pytest.approx(-np.log(2.0), rel=1e-15)
    assert o["S_per_N"] == pytest.approx(np.log(2.0), rel=1e-15)
    assert o["C"] == 0.0


def test_population_estimates_L4(run_L4):
    _, obs = run_L4
    for o in obs[1:]:
        ex = exact.brute_observables(4, o["beta"])
        lnZ = -o["betaF_per_N"] * 16
        assert abs(lnZ - ex["lnZ"]) < 0.03
        assert abs(o["e"] - ex["e"]) < 0.03
        assert abs(o["abs_m"] - ex["abs_m"]) < 0.03
        assert abs(o["m2"] - ex["m2"]) < 0.03
        assert abs(o["m4"] - ex["m4"]) < 0.03
        assert abs(o["S_per_N"] - ex["S_per_N"]) < 0.01
        assert o["C"] == pytest.approx(ex["C"], rel=0.4)
        assert abs(o["R"] - 20000) < 5 * np.sqrt(20000 / 4)


def test_population_estimates_L8(run_L8):
    _, obs = run_L8
    Cs = []
    for o in obs[1:]:
        ex = exact.torus_exact(8, o["beta"])
        assert abs(o["betaF_per_N"] - ex["betaF_per_N"]) < 0.004
        assert abs(o["e"] - ex["e"]) < 0.03
        Cs.append((o["C"], ex["C"]))
    Cs = np.array(Cs)
    assert np.abs(Cs[:, 0] / Cs[:, 1] - 1).mean() < 0.1


def test_measurement_sums_are_the_population_sums(run_L4):
    r, obs = run_L4
    _, E, M = r.get_population()
    o = obs[-1]
    E = E.astype(object)
    M = M.astype(object)
    assert o["sumE"] == sum(E) and o["sumE2"] == sum(e * e for e in E)
    assert o["sumAbsM"] == sum(abs(m) for m in M) and o["sumM2"] == sum(m * m for m in M)
    assert o["sumM4"] == sum(m ** 4 for m in M)


def test_multi_histogram_L4(run_L4):
    r, _ = run_L4
    betas = np.linspace(0.0, 1.0, 21)
    for o, b in zip(r.reweight(betas), betas):
        ex = exact.brute_observables(4, b)
        assert abs(o["betaF_per_N"] - ex["betaF_per_N"]) < 2e-3
        assert abs(o["e"] - ex["e"]) < 0.01
        assert abs(o["m2"] - ex["m2"]) < 0.01
        assert abs(o["abs_m"] - ex["abs_m"]) < 0.01
        if b > 0:
            assert o["C"] == pytest.approx(ex["C"], rel=0.05)


def test_multi_histogram_L8(run_L8):
    r, obs = run_L8
    betas = np.linspace(0.05, 1.0, 20)
    for o, b in zip(r.reweight(betas), betas):
        ex = exact.torus_exact(8, b)
        assert abs(o["betaF_per_N"] - ex["betaF_per_N"]) < 2e-3
        assert abs(o["e"] - ex["e"]) < 0.01
        assert o["C"] == pytest.approx(ex["C"], rel=0.05)
    # self-consistency: ln Z from the histograms at beta_i equals the PA estimate
    bi = np.array([o["beta"] for o in obs[1:]])
    for o, p in zip(r.reweight(bi), obs[1:]):
        assert o["betaF_per_N"] == pytest.approx(p["betaF_per_N"], abs=2e-3)


def test_adaptive_step_postconditions():
    alpha_star = 0.85
    r = oracle.Run(8, 2000, seed=4)
    r.init()
    betas = [0.0]
    while r.beta < 1.0:
        b = r.adapt_beta(alpha_star, 1.0)
        assert b > r.beta
        a = r.alpha(b)
        if b < 1.0:
            assert a >= alpha_star
            # a slightly larger step falls below the target
            assert r.alpha(b + 1e-9) < alpha_star
        else:
            assert a >= alpha_star
        # a fine scan finds no larger beta below the crossing
        if b < 1.0:
            grid = np.linspace(r.beta, 1.0, 400)
            ok = [g for g in grid if r.alpha(g) >= alpha_star]
            assert max(ok) <= b + (grid[1] - grid[0])
        r.resample(b)
        r.sweep(5)
        betas.append(b)
    assert betas[-1] == 1.0
    assert len(betas) > 10


def test_overlap_limits():
    r = oracle.Run(8, 1000, seed=4)
    r.init()
    assert r.alpha(0.0) == pytest.approx(1.0)
    assert 0.0 < r.alpha(5.0) < r.alpha(0.5) < r.alpha(0.1) <= 1.0

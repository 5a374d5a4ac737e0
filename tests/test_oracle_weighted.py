"""Pins of the oracle's weighted averaging of independent runs (Sec. 2.2,
Eq. (weighted-average)): closed forms, invariances, and, at L = 4, the
enumerated partition function."""
import numpy as np
import pytest

import exact
import oracle
from oracle import weighted


def _obs(beta, lnZ, N, e=-1.0, R=100, **kw):
    d = {"beta": beta, "R": R, "e": e, "C": 0.5, "abs_m": 0.25, "m2": 0.125, "m4": 0.0625,
         "betaF_per_N": -lnZ / N}
    d.update(kw)
    return d


def test_single_run_is_unchanged():
    N = 16
    run = [_obs(0.1 * i, 10.0 + i, N, e=-0.1 * i) for i in range(5)]
    out = weighted.weighted_average([run], N)
    for o, r in zip(out, run):
        for k in ("e", "C", "abs_m", "m2", "m4", "betaF_per_N"):
            assert o[k] == pytest.approx(r[k], rel=1e-15, abs=1e-15)
        assert o["S_per_N"] == pytest.approx(o["beta"] * o["e"] - o["betaF_per_N"], rel=1e-14)


def test_equal_free_energies_give_the_plain_mean():
    N = 64
    runs = [[_obs(0.5, 40.0, N, e=e, abs_m=a)] for e, a in ((-1.0, 0.1), (-1.2, 0.3), (-0.8, 0.8))]
    o = weighted.weighted_average(runs, N)[0]
    assert o["e"] == pytest.approx(-1.0, rel=1e-15)
    assert o["abs_m"] == pytest.approx(0.4, rel=1e-15)
    assert o["betaF_per_N"] == pytest.approx(-40.0 / N, rel=1e-15)
    assert o["R"] == 300


def test_two_runs_closed_form():
    # Z_2 = 3 Z_1: weights 1/4 and 3/4; pooled Z = 2 Z_1
    N, a = 32, 55.0
    runs = [[_obs(0.3, a, N, e=-1.0)], [_obs(0.3, a + np.log(3.0), N, e=-2.0)]]
    o = weighted.weighted_average(runs, N)[0]
    assert o["e"] == pytest.approx(0.25 * -1.0 + 0.75 * -2.0, rel=1e-14)
    assert -N * o["betaF_per_N"] == pytest.approx(a + np.log(2.0), rel=1e-14)
    assert o["S_per_N"] == pytest.approx(0.3 * o["e"] + (a + np.log(2.0)) / N, rel=1e-14)


def test_weights_follow_the_partition_function_and_ignore_a_common_shift():
    lnZ = np.array([[1.0, 5.0], [3.0, -60.0], [2.0, 5.0]])
    w = weighted.weights(lnZ)
    assert np.allclose(w.sum(axis=0), 1.0, rtol=0, atol=1e-15)
    assert w[1, 0] > w[2, 0] > w[0, 0]  # the larger Z weighs more
    assert w[1, 1] < 1e-25 and w[0, 1] == pytest.approx(0.5, rel=1e-14)
    assert np.allclose(weighted.weights(lnZ + 700.0), w, rtol=1e-14, atol=0)
    direct = np.exp(lnZ[:, 0]) / np.exp(lnZ[:, 0]).sum()
    assert np.allclose(w[:, 0], direct, rtol=1e-14, atol=0)


def test_runs_must_share_the_temperatures():
    N = 16
    with pytest.raises(ValueError):
        weighted.weighted_average([[_obs(0.1, 1.0, N)], [_obs(0.2, 1.0, N)]], N)
    with pytest.raises(ValueError):
        weighted.weighted_average([[_obs(0.1, 1.0, N)], [_obs(0.1, 1.0, N), _obs(0.2, 1.0, N)]], N)


@pytest.fixture(scope="module")
def l4_runs():
    """400 independent oracle runs at L = 4, R = 12, theta = 1, beta 0 -> 1 in
    20 steps: small populations, so single-run estimates are visibly biased."""
    runs = []
    for seed in range(1, 401):
        o = oracle.Run(4, 12, seed=seed)
        o.init()
        trace = [o.measure()]
        for i in range(1, 21):
            o.resample(i / 20)
            o.sweep(1)
            trace.append(o.measure())
        runs.append(trace)
    return runs


def test_pooled_partition_function_is_unbiased_at_l4(l4_runs):
    """The PA estimate of Z (not of ln Z) is unbiased, so the pooled free
    energy approaches the enumerated one while the mean of ln Z_m stays low."""
    N = 16
    ex = exact.brute_observables(4, 1.0)
    lnZ = weighted.log_z(l4_runs, N)[:, -1]
    ratio = np.exp(lnZ - ex["lnZ"])
    assert abs(ratio.mean() - 1.0) < 3 * ratio.std() / np.sqrt(len(ratio))
    se = lnZ.std() / np.sqrt(len(lnZ))
    assert ex["lnZ"] - lnZ.mean() > 3 * se  # Jensen: E[ln Z_m] < ln Z
    pooled = -N * weighted.weighted_average(l4_runs, N)[-1]["betaF_per_N"]
    assert abs(pooled - ex["lnZ"]) < 0.5 * (ex["lnZ"] - lnZ.mean())


def test_weighted_energy_at_l4(l4_runs):
    N = 16
    out = weighted.weighted_average(l4_runs, N)
    for i in (5, 10, 20):
        ex = exact.brute_observables(4, i / 20)
        e = np.array([r[i]["e"] for r in l4_runs])
        assert abs(out[i]["e"] - ex["e"]) < 4 * e.std() / np.sqrt(len(e))

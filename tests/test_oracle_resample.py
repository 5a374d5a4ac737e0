"""Pins of the oracle's resampling (Sec. 2.1, Eqs. (Q) and (resampling
factors)): special cases with closed forms, normalisation, expected copy
counts, compaction order, population fluctuations and capacity."""
import numpy as np
import pytest

import inputs
import oracle


def _run_with(spins, beta=0.0, R=None, capacity=0, seed=1):
    n, L, _ = spins.shape
    r = oracle.Run(L, R or n, seed=seed, capacity=capacity)
    r.set_population(spins, beta=beta)
    return r


def test_zero_step_keeps_population():
    # dbeta = 0 and R_{i-1} = R: tau_hat = 1 exactly, thr = 0, so every replica
    # keeps exactly one copy unless its uniform is 0 (probability 2^-32).
    s = inputs.mixed_spins(300, 8, 2)
    r = _run_with(s, beta=0.3)
    info = r.resample(0.3)
    assert info["R_new"] == 300
    assert np.all(r.get_counts() == 1)
    assert np.array_equal(r.get_population()[0], s)
    assert info["lnQ"] == pytest.approx(0.0, abs=1e-15)


def test_single_energy_population():
    # All replicas at one energy E: Q = exp(-dbeta E) exactly, tau_hat = R/R_{i-1}.
    L = 8
    s = np.ones((500, L, L), np.int8)
    r = _run_with(s, R=400)
    info = r.resample(0.2)
    E = -2 * L * L
    assert info["lnQ"] == pytest.approx(-0.2 * E, rel=1e-15)
    counts = r.get_counts()
    assert set(np.unique(counts)) <= {0, 1}
    # tau_hat = 0.8: expected survivors 400, binomial sd sqrt(500*0.8*0.2)
    assert abs(info["R_new"] - 400) < 5 * np.sqrt(500 * 0.16)


def test_tables_normalisation():
    rng = np.random.default_rng(4)
    N = 256
    for trial in range(20):
        hist = np.zeros(N + 1, np.int64)
        lo = rng.integers(0, N - 40)
        hist[lo: lo + 40] = rng.integers(0, 60, 40)
        hist[lo] = max(hist[lo], 1)
        R = int(rng.integers(100, 5000))
        Rprev = int(hist.sum())
        dbeta = float(rng.uniform(0.0, 0.3))
        base, thr, lnQ = oracle.tables(N, R, Rprev, hist, dbeta)
        occ = hist > 0
        tau = base[occ] + thr[occ] / 2.0 ** 32
        # sum_b n(b) tau_hat(b) = R (normalisation of Eq. (resampling factors))
        assert (hist[occ] * tau).sum() == pytest.approx(R, rel=1e-9)
        # Q from the definition, computed with a different formula
        E = 4 * np.arange(N + 1) - 2 * N
        Q = (hist[occ] * np.exp(-dbeta * E[occ].astype(np.float64))).sum() / Rprev
        assert lnQ == pytest.approx(np.log(Q), rel=1e-12, abs=1e-12)


def test_expected_copy_counts_by_energy():
    # E[count | b] = base + (thr + 1) / 2^32, i.e. tau_hat(b) to 2^-32.
    L = 6
    s = inputs.ordered_spins(40000, L, 5, 3)
    r = _run_with(s, capacity=80000)
    _, E0, _ = r.get_population()
    info = r.resample(0.35)
    counts = r.get_counts().astype(np.float64)
    Ev = np.unique(E0)
    hist = np.zeros(L * L + 1, np.int64)
    for e in Ev:
        hist[(e + 2 * L * L) // 4] = (E0 == e).sum()
    base, thr, _ = oracle.tables(L * L, 40000, 40000, hist, 0.35)
    for e in Ev:
        sel = E0 == e
        b = (e + 2 * L * L) // 4
        tau = base[b] + thr[b] / 2.0 ** 32
        mean = counts[sel].mean()
        assert set(np.unique(counts[sel])) <= {base[b], base[b] + 1}
        sd = np.sqrt(max((tau - np.floor(tau)) * (1 - (tau - np.floor(tau))), 1e-12) / sel.sum())
        assert abs(mean - tau) < 5 * sd + 1e-12
    # lower energies are favoured when cooling
    order = np.argsort(Ev)
    means = [counts[E0 == Ev[k]].mean() for k in order]
    assert all(a >= b for a, b in zip(means, means[1:]))


def test_compaction_order():
    s = inputs.mixed_spins(200, 8, 3)
    r = _run_with(s)
    r.resample(0.5)
    counts = r.get_counts()
    new, E, M = r.get_population()
    assert np.array_equal(new, np.repeat(s, counts, axis=0))
    assert len(new) == counts.sum()


def test_population_fluctuations_small():
    # nearest-integer resampling: Var(R_i) <= sum_j frac(1-frac) <= R/4
    R = 5000
    r = oracle.Run(8, R, seed=13)
    r.init()
    for i in range(1, 11):
        info = r.resample(0.05 * i)
        assert abs(info["R_new"] - R) < 5 * np.sqrt(R / 4.0)
        r.sweep(2)


def test_capacity_overflow_leaves_state():
    # Three equal-energy replicas with target R = 100: tau_hat = 100/3, so
    # R_new is 99..102 and exceeds a capacity of 100 with probability 7/27.
    s = np.ones((3, 4, 4), np.int8)
    overflowed = 0
    for seed in range(1, 41):
        r = oracle.Run(4, 100, seed=seed, capacity=100)
        r.set_population(s, beta=0.1)
        before = r.get_population()
        try:
            info = r.resample(0.2)
            assert 99 <= info["R_new"] <= 100
        except OverflowError:
            overflowed += 1
            after = r.get_population()
            assert r.step == 0 and r.beta == 0.1 and r.population == 3
            for a, b in zip(before, after):
                assert np.array_equal(a, b)
    assert overflowed > 0

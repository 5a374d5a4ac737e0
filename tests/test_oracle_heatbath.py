"""Pins of the oracle's heat-bath sweep (reading of Sec. 2.1, which names
heat-bath dynamics as an alternative update): the law P(flip | k) =
1 / (1 + e^{2 beta k}) in its detailed-balance form, the per-class flip
frequencies of one colour, beta = 0, the exact Boltzmann distribution at
L = 4, bookkeeping, and a full PA run at L = 4 against enumeration."""
import numpy as np
import pytest

import exact
import inputs
import oracle

TWO32 = 2 ** 32


def _chi2(counts, probs):
    n = counts.sum()
    m = probs * n
    keep = m > 5
    chi2 = ((counts[keep] - m[keep]) ** 2 / m[keep]).sum()
    return chi2, keep.sum() - 1


def test_thresholds_detailed_balance():
    """Heat-bath flips obey P(flip | k) / P(flip | -k) = e^{-2 beta k}; with
    integer thresholds rounded up the ratio is exact to 4 * 2^-32."""
    assert oracle.hb_thresholds(0.0) == (TWO32 // 2, TWO32 // 2)
    prev = (TWO32 // 2, TWO32 // 2)
    for beta in np.linspace(0.01, 2.0, 30):
        U2, U4 = oracle.hb_thresholds(beta)
        assert 1 <= U4 <= U2 <= TWO32 // 2
        assert U2 <= prev[0] and U4 <= prev[1]
        for k, U in ((2, U2), (4, U4)):
            ratio = U / (TWO32 - U)
            assert abs(ratio - np.exp(-2.0 * beta * k)) <= 4.0 * 2.0 ** -32
        prev = (U2, U4)


def _colour0_k(s):
    """k = s h of every colour-0 site of each replica, and the site mask."""
    h = np.roll(s, 1, 1) + np.roll(s, -1, 1) + np.roll(s, 1, 2) + np.roll(s, -1, 2)
    L = s.shape[1]
    y, x = np.mgrid[0:L, 0:L]
    c0 = ((x + y) & 1) == 0
    return (s.astype(int) * h)[:, c0], c0


@pytest.mark.parametrize("beta", [0.3, 0.8])
def test_flip_frequency_of_each_class(beta):
    """Colour 0 is updated first, against the initial neighbours, so its sites
    flip with probability 1 / (1 + e^{2 beta k}) for the k of the initial
    configuration; every class k in {-4, -2, 0, 2, 4} is checked."""
    L, R = 8, 4000
    s0 = inputs.random_spins(R, L, 31)
    r = oracle.Run(L, R, seed=17, heatbath=True)
    r.set_population(s0, beta=beta)
    r.sweep(1)
    s1, _, _ = r.get_population()
    k, c0 = _colour0_k(s0)
    # colour-1 updates never touch colour-0 sites, so a colour-0 change is a flip
    flipped = (s1 != s0)[:, c0]
    for kk in (-4, -2, 0, 2, 4):
        sel = k == kk
        n = sel.sum()
        assert n > 1000
        p = 1.0 / (1.0 + np.exp(2.0 * beta * kk))
        f = flipped[sel].mean()
        assert abs(f - p) < 5 * np.sqrt(p * (1 - p) / n), (kk, f, p)


def test_beta_zero_flips_half_the_spins():
    """At beta = 0 every site takes a fresh uniform spin (Metropolis, by
    contrast, negates the configuration)."""
    L, R = 8, 2000
    s0 = inputs.random_spins(R, L, 4)
    r = oracle.Run(L, R, seed=9, heatbath=True)
    r.set_population(s0, beta=0.0)
    r.sweep(1)
    s1, _, _ = r.get_population()
    changed = (s1 != s0).mean()
    assert abs(changed - 0.5) < 5 * 0.5 / np.sqrt(s0.size)


def test_bookkeeping_matches_recount():
    L, R = 8, 40
    r = oracle.Run(L, R, seed=2, heatbath=True)
    r.set_population(inputs.mixed_spins(R, L, 1), beta=0.37)
    r.sweep(7)
    s, E, M = r.get_population()
    Es = -(s.astype(int) * (np.roll(s, -1, 2) + np.roll(s, -1, 1))).sum(axis=(1, 2))
    assert np.array_equal(Es, E)
    assert np.array_equal(s.astype(int).sum(axis=(1, 2)), M)


def test_metropolis_and_heatbath_chains_differ():
    L, R = 8, 20
    a = oracle.Run(L, R, seed=5)
    b = oracle.Run(L, R, seed=5, heatbath=True)
    s0 = inputs.random_spins(R, L, 2)
    for r in (a, b):
        r.set_population(s0, beta=0.4)
        r.sweep(3)
    assert not np.array_equal(a.get_population()[0], b.get_population()[0])


@pytest.mark.parametrize("beta", [0.25, float(exact.BETA_C), 0.7])
def test_heatbath_samples_boltzmann_L4(beta):
    L, R = 4, 6000
    r = oracle.Run(L, R, seed=23, heatbath=True)
    r.set_population(inputs.random_spins(R, L, 8), beta=beta)
    r.sweep(60)
    _, E, M = r.get_population()
    ex = exact.brute_observables(4, beta)
    cE = np.array([(E == e).sum() for e in ex["Ev"]])
    chi2, dof = _chi2(cE, ex["pE"])
    assert chi2 < dof + 6 * np.sqrt(2 * dof), (chi2, dof)
    absv = np.unique(np.abs(ex["Mv"]))
    pabs = np.array([ex["pM"][np.abs(ex["Mv"]) == a].sum() for a in absv])
    cM = np.array([(np.abs(M) == a).sum() for a in absv])
    chi2, dof = _chi2(cM, pabs)
    assert chi2 < dof + 6 * np.sqrt(2 * dof), (chi2, dof)


def test_heatbath_pa_run_L4_against_enumeration():
    r = oracle.Run(4, 6000, seed=3, heatbath=True)
    r.init()
    for i in range(1, 11):
        r.resample(0.1 * i)
        r.sweep(5)
        o = r.measure()
        ex = exact.brute_observables(4, o["beta"])
        assert abs(o["betaF_per_N"] - ex["betaF_per_N"]) < 4e-3
        assert abs(o["e"] - ex["e"]) < 0.04

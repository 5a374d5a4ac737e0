"""Pins of the oracle's in-line LCG variant of the sweep (Sec. 4: one draw
of the base generator per word and update seeds a linear congruential
generator that supplies the word's uniforms; reading R11 in the oracle).

The variant is a different Markov chain from the Philox sweep but must
sample the same distribution: the exact Boltzmann distribution at L = 4
(enumeration), the exact finite-torus free energy and energy at L = 8 from a
PA run, independent decisions for the sites of one word, and numbers of its
own for every update.  Initial state and resampling are unchanged."""
import numpy as np
import pytest

import exact
import inputs
import oracle
import stream_pins


def _chi2(counts, probs):
    m = probs * counts.sum()
    keep = m > 5
    return ((counts[keep] - m[keep]) ** 2 / m[keep]).sum(), keep.sum() - 1


@pytest.mark.parametrize("beta", [0.2, 0.4406868, 0.8])
def test_lcg_chains_reach_the_boltzmann_distribution_L4(beta):
    R = 6000
    r = oracle.Run(4, R, seed=13, lcg=True)
    r.set_population(inputs.random_spins(R, 4, 2), beta=beta)
    r.sweep(60)
    _, E, M = r.get_population()
    ex = exact.brute_observables(4, beta)
    chi2, dof = _chi2(np.array([(E == e).sum() for e in ex["Ev"]]), ex["pE"])
    assert chi2 < dof + 6 * np.sqrt(2 * dof)
    assert abs((M.astype(float) ** 2).mean() / 256 - ex["m2"]) < 0.03


def test_lcg_population_annealing_matches_exact_torus_L8():
    L, R = 8, 4000
    r = oracle.Run(L, R, seed=3, lcg=True)
    r.init()
    out = []
    for i in range(1, 21):
        r.resample(0.05 * i)
        r.sweep(10)
        out.append(r.measure())
    for o in out[4::5]:
        ex = exact.torus_exact(L, o["beta"])
        assert abs(o["betaF_per_N"] - ex["betaF_per_N"]) < 2e-3
        assert abs(o["e"] - ex["e"]) < 0.03


def test_lcg_site_decisions_and_numbers_are_independent():
    lib = oracle.lib()
    assert stream_pins.site_pairs_independent(lib, lcg=True)
    assert stream_pins.site_uniforms_independent(lib, lcg=True)
    assert stream_pins.uniforms_distinct_across_updates(lib, lcg=True)


def test_lcg_is_its_own_chain_with_the_same_start_and_resampling():
    spins = inputs.mixed_spins(50, 16, 4)
    pops = []
    for lcg in (False, True):
        r = oracle.Run(16, 50, seed=6, lcg=lcg)
        r.init()
        init = r.get_population()[0]
        r.set_population(spins, beta=0.5)
        r.sweep(2)
        pops.append((init, r.get_population()[0]))
        r.set_population(spins, beta=0.5)
        counts = (r.resample(0.7), r.get_counts())
        pops[-1] += (counts[0]["R_new"], counts[1])
    (ia, pa_, ra, ca), (ib, pb, rb, cb) = pops
    assert np.array_equal(ia, ib)          # INIT stream shared
    assert not np.array_equal(pa_, pb)     # a different sweep chain
    assert ra == rb and np.array_equal(ca, cb)  # RESAMPLE stream shared

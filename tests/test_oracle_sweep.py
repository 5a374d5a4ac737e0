"""Pins of the oracle's initial state and Metropolis sweep (Sec. 2.1 steps 1
and 3; Sec. 3): closed forms at beta = 0, the exact Boltzmann distribution at
L = 4, and bookkeeping invariants."""
import numpy as np
import pytest

import exact
import inputs
import oracle
import stream_pins


def _chi2(counts, probs):
    n = counts.sum()
    m = probs * n
    keep = m > 5
    chi2 = ((counts[keep] - m[keep]) ** 2 / m[keep]).sum()
    dof = keep.sum() - 1
    return chi2, dof


def test_init_closed_forms_beta0():
    L, R = 8, 20000
    N = L * L
    r = oracle.Run(L, R, seed=11)
    r.init()
    s, E, M = r.get_population()
    E = E.astype(np.float64)
    M = M.astype(np.float64)
    # independent +-1 spins: <E> = 0, <E^2> = 2N, <M^2> = N, <M^4> = 3N^2 - 2N
    for val, target in ((E, 0.0), (E ** 2, 2.0 * N), (M ** 2, float(N)), (M ** 4, 3.0 * N * N - 2.0 * N)):
        se = val.std() / np.sqrt(R)
        assert abs(val.mean() - target) < 5 * se
    assert abs((s == -1).mean() - 0.5) < 5 * 0.5 / np.sqrt(s.size)


def test_init_energy_distribution_L4():
    L, R = 4, 60000
    r = oracle.Run(L, R, seed=3)
    r.init()
    _, E, _ = r.get_population()
    Ev, _, g = exact.brute_force(4)
    p = g.sum(axis=1) / 2.0 ** 16
    counts = np.array([(E == e).sum() for e in Ev])
    assert counts.sum() == R
    chi2, dof = _chi2(counts, p)
    assert chi2 < dof + 6 * np.sqrt(2 * dof)


def test_init_reproducible_and_keyed():
    a = oracle.Run(8, 50, seed=5)
    a.init()
    b = oracle.Run(8, 50, seed=5)
    b.init()
    c = oracle.Run(8, 50, seed=5, run_id=1)
    c.init()
    assert np.array_equal(a.get_population()[0], b.get_population()[0])
    assert not np.array_equal(a.get_population()[0], c.get_population()[0])


def test_sites_of_one_word_decide_independently():
    # one uniform per spin update (Sec. 3): the colour-0 word of an all-up
    # 8 x 8 lattice (k = 4 at every site) flips each site with T_4 / 2^32,
    # and the pairs (q, q + 16) and (q, q ^ 1) flip independently
    f, p = stream_pins.colour0_word_flips(oracle.lib())
    assert abs(f.mean() - p) < 5 * np.sqrt(p * (1 - p) / f.size)
    assert stream_pins.chi2_independent(f[:, :16].ravel(), f[:, 16:].ravel()) < 25.0
    assert stream_pins.chi2_independent(f[:, 0::2].ravel(), f[:, 1::2].ravel()) < 25.0
    assert stream_pins.site_pairs_independent(oracle.lib())


def test_site_uniforms_share_no_halves():
    assert stream_pins.site_uniforms_independent(oracle.lib())


def test_runs_have_streams_of_their_own():
    # (seed_hi = 1, run 0) and (seed_hi = 0, run 1) are different runs
    assert stream_pins.runs_have_own_streams(oracle.lib())
    with pytest.raises(ValueError):
        oracle.Run(8, 10, seed=1, run_id=1 << 28)


def test_incremental_bookkeeping_matches_recount():
    L, R = 8, 40
    r = oracle.Run(L, R, seed=2)
    r.set_population(inputs.mixed_spins(R, L, 1), beta=0.37)
    r.sweep(7)
    s, E, M = r.get_population()
    for j in range(R):
        assert (E[j], M[j]) == r.recount(j)
    # and straight from the Hamiltonian
    Es = -(s.astype(int) * (np.roll(s, -1, 2) + np.roll(s, -1, 1))).sum(axis=(1, 2))
    assert np.array_equal(Es, E)
    assert np.array_equal(s.astype(int).sum(axis=(1, 2)), M)
    assert r.sweeps == 7


def test_beta_zero_sweep_flips_every_spin():
    # At beta = 0 the thresholds are 2^32: every proposed flip is accepted, so a
    # sweep negates the configuration (colour 0, then colour 1).
    assert oracle.thresholds(0.0) == (2 ** 32, 2 ** 32)
    L, R = 6, 5
    r = oracle.Run(L, R, seed=9)
    s0 = inputs.random_spins(R, L, 4)
    r.set_population(s0, beta=0.0)
    r.sweep(1)
    s1, E1, M1 = r.get_population()
    assert np.array_equal(s1, -s0)


def test_thresholds_monotone_and_bounded():
    prev = (2 ** 32, 2 ** 32)
    for beta in np.linspace(0.01, 3.0, 40):
        t2, t4 = oracle.thresholds(beta)
        assert 1 <= t4 <= t2 <= 2 ** 32
        assert t2 < prev[0] or t2 == prev[0]
        # acceptance probability T/2^32 is the Metropolis factor rounded up
        assert abs(t2 / 2 ** 32 - np.exp(-4 * beta)) <= 2.0 ** -32
        assert abs(t4 / 2 ** 32 - np.exp(-8 * beta)) <= 2.0 ** -32
        prev = (t2, t4)


@pytest.mark.parametrize("beta", [0.25, float(exact.BETA_C), 0.7])
def test_metropolis_samples_boltzmann_L4(beta):
    """Independent chains (no resampling) started from random states and swept
    long enough at fixed beta sample the exact Boltzmann distribution."""
    L, R = 4, 6000
    r = oracle.Run(L, R, seed=21)
    r.set_population(inputs.random_spins(R, L, 8), beta=beta)
    r.sweep(60)
    _, E, M = r.get_population()
    ex = exact.brute_observables(4, beta)
    cE = np.array([(E == e).sum() for e in ex["Ev"]])
    chi2, dof = _chi2(cE, ex["pE"])
    assert chi2 < dof + 6 * np.sqrt(2 * dof), (chi2, dof)
    aM = np.abs(M)
    absv = np.unique(np.abs(ex["Mv"]))
    pabs = np.array([ex["pM"][np.abs(ex["Mv"]) == a].sum() for a in absv])
    cM = np.array([(aM == a).sum() for a in absv])
    chi2, dof = _chi2(cM, pabs)
    assert chi2 < dof + 6 * np.sqrt(2 * dof), (chi2, dof)


@pytest.mark.parametrize("heatbath", [False, True])
def test_threads_over_replicas_give_the_same_run(heatbath):
    # the OpenMP loop over replicas (timing only) changes nothing
    pops = []
    for threads in (1, 4):
        r = oracle.Run(16, 301, seed=9, heatbath=heatbath)
        r.set_threads(threads)
        r.init()
        r.resample(0.2)
        r.sweep(3)
        r.resample(0.45)
        r.sweep(2)
        pops.append((r.get_population(), r.measure()))
    (a, oa), (b, ob) = pops
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert oa == ob

"""Pins on the oracle's random streams (reading R3), for the oracle tests and
the mutant battery.  Each takes a loaded oracle library and returns True when
the property holds.

The paper uses one uniform random number per spin update (Sec. 3, spin
updates); the sites of one 32-site word must therefore decide independently,
and every run must have streams of its own.  These checks look at what the
streams produce (flip statistics, the site uniforms), not at how they are
computed.
"""
import numpy as np

import oracle


def colour0_word_flips(lib, R=3000, seed=29, lcg=False):
    """Colour-0 flips of R all-up 8 x 8 replicas after one sweep at a beta
    where T_4 / 2^32 is about 1/2: colour 0 is one word (q = 0..31), every
    site has k = 4 and is updated against the initial neighbours, so each
    flips with probability T_4 / 2^32 independently.  Returns ([R, 32] flips
    in q order, p)."""
    beta = np.log(2.0) / 8.0
    r = oracle.Run(8, R, seed=seed, lib_=lib, lcg=lcg)
    s0 = np.ones((R, 8, 8), np.int8)
    r.set_population(s0, beta=beta)
    r.sweep(1)
    s1, _, _ = r.get_population()
    q = np.arange(32)
    y = q // 4
    x = 2 * (q % 4) + (y & 1)
    flips = (s1 != s0).reshape(R, 64)[:, y * 8 + x]
    p = oracle.thresholds(beta, lib)[1] / 2.0 ** 32
    return flips, p


def chi2_independent(a, b):
    """Pearson chi-square (1 dof) of the 2 x 2 table of paired booleans."""
    n = a.size
    t = np.array([[np.sum(a & b), np.sum(a & ~b)], [np.sum(~a & b), np.sum(~a & ~b)]], float)
    e = np.outer(t.sum(1), t.sum(0)) / n
    return float(((t - e) ** 2 / e).sum())


def site_pairs_independent(lib, limit=25.0, lcg=False):
    """Joint flips of sites (q, q + 16) and (q, q ^ 1) of one word follow the
    product of their marginals (chi-square below `limit`, p ~ 6e-7), and each
    site flips at rate p."""
    f, p = colour0_word_flips(lib, lcg=lcg)
    if abs(f.mean() - p) > 5 * np.sqrt(p * (1 - p) / f.size):
        return False
    pairs = ((f[:, :16], f[:, 16:]), (f[:, 0::2], f[:, 1::2]))
    return all(chi2_independent(a.ravel(), b.ravel()) < limit for a, b in pairs)


def site_uniforms_independent(lib, words=2000, lcg=False):
    """The 32 site uniforms of a word: no two sites share their high or
    their low 16 bits more often than chance (expected about 15 equal halves
    of each kind over 2000 words x 496 pairs; a shared half would add 16 per
    word), and the top and bottom bytes are uniform (chi-square, 255 dof)."""
    r = oracle.Run(8, 10, seed=31, lib_=lib, lcg=lcg)
    keys = [(g, c, j) for g in range(100) for c in (0, 1) for j in range(10)][:words]
    us = [r.word_uniforms(g, c, j, 0).astype(np.int64) for g, c, j in keys]
    equal = {"hi": 0, "lo": 0}
    for u in us:
        for name, half in (("hi", u >> 16), ("lo", u & 0xFFFF)):
            _, cnt = np.unique(half, return_counts=True)
            equal[name] += int((cnt * (cnt - 1) // 2).sum())
    if equal["hi"] > 60 or equal["lo"] > 60:
        return False
    u = np.concatenate(us)
    for byte in (u >> 24, u & 0xFF):
        cnt = np.bincount(byte, minlength=256)
        e = u.size / 256.0
        if ((cnt - e) ** 2 / e).sum() > 255 + 6 * np.sqrt(2 * 255):
            return False
    return True


def runs_have_own_streams(lib):
    """Distinct (seed, run_id) pairs give distinct initial populations, also
    for pairs that trade the run number against the seed's high word."""
    pops = []
    for seed, run in ((5, 0), (5, 1), (5 + (1 << 32), 0), (5 + (1 << 32), 1)):
        r = oracle.Run(8, 40, seed=seed, run_id=run, lib_=lib)
        r.init()
        pops.append(r.get_population()[0])
    return all(not np.array_equal(pops[a], pops[b]) for a in range(4) for b in range(a + 1, 4))


def uniforms_distinct_across_updates(lib, lcg=False):
    """Every update of a word (sweep g, colour c) gets numbers of its own:
    among the 3200 site uniforms of one word over 50 sweeps and both
    colours, equal values are as rare as chance makes them (about 0.001
    expected; at most 2 allowed)."""
    r = oracle.Run(8, 4, seed=37, lib_=lib, lcg=lcg)
    u = np.concatenate([r.word_uniforms(g, c, 1, 0) for g in range(50) for c in (0, 1)])
    _, cnt = np.unique(u, return_counts=True)
    return int((cnt * (cnt - 1) // 2).sum()) <= 2

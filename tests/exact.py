"""Exact reference results for the 2D Ising model on an L x L torus.

Independent of the oracle and of the GPU path; used to pin both.

* ``brute_force(L)`` enumerates all 2^(L*L) states (L <= 4) and returns the
  exact density of states g(E, M).
* ``torus_lnZ(L, beta)`` is the exact finite-torus partition function of
  Kaufman (1949) in the form of Ferdinand and Fisher (1969), evaluated with
  mpmath at 40 significant digits; energy and specific heat follow from its
  derivatives in beta.
"""
import functools

import mpmath
import numpy as np


@functools.lru_cache(maxsize=None)
def brute_force(L):
    """Density of states of the L x L periodic Ising model (J = 1, h = 0).

    Returns (E_values, M_values, g) with g[a, b] the number of states with
    energy E_values[a] and magnetisation M_values[b].  The energy counts each
    of the 2N bonds (right and down neighbour of each site) once.
    """
    N = L * L
    assert N <= 16, "brute force is for L <= 4"
    states = np.arange(2 ** N, dtype=np.int64)
    bits = (states[:, None] >> np.arange(N)) & 1
    s = (1 - 2 * bits).reshape(-1, L, L).astype(np.int64)
    E = -(s * (np.roll(s, -1, axis=2) + np.roll(s, -1, axis=1))).sum(axis=(1, 2))
    M = s.sum(axis=(1, 2))
    Ev = np.unique(E)
    Mv = np.unique(M)
    g = np.zeros((len(Ev), len(Mv)), np.int64)
    np.add.at(g, (np.searchsorted(Ev, E), np.searchsorted(Mv, M)), 1)
    return Ev, Mv, g


def brute_observables(L, beta):
    """Exact canonical averages from the enumerated density of states."""
    Ev, Mv, g = brute_force(L)
    N = L * L
    Ev_f = Ev.astype(np.float64)
    shift = -beta * Ev_f.min()
    wE = np.exp(-beta * Ev_f - shift)  # relative Boltzmann factor per energy
    w = g * wE[:, None]
    Z = w.sum()
    lnZ = np.log(Z) + shift
    pE = w.sum(axis=1) / Z
    pM = w.sum(axis=0) / Z
    mE = (pE * Ev_f).sum()
    varE = (pE * (Ev_f - mE) ** 2).sum()
    Mf = Mv.astype(np.float64)
    return {
        "lnZ": lnZ,
        "e": mE / N,
        "C": beta * beta * varE / N,
        "abs_m": (pM * np.abs(Mf)).sum() / N,
        "m2": (pM * Mf ** 2).sum() / N ** 2,
        "m4": (pM * Mf ** 4).sum() / N ** 4,
        "betaF_per_N": -lnZ / N,
        "S_per_N": beta * mE / N + lnZ / N,
        "pE": pE,
        "Ev": Ev,
        "pM": pM,
        "Mv": Mv,
    }


def _torus_Z_mp(n, m, K):
    """Exact partition function of the n x m periodic Ising model at coupling K."""
    two = mpmath.mpf(2)
    c2k = mpmath.cosh(2 * K)
    coth2k = mpmath.coth(2 * K)

    def gamma(l):
        if l == 0:
            return 2 * K + mpmath.log(mpmath.tanh(K))  # sign kept
        return mpmath.acosh(c2k * coth2k - mpmath.cos(mpmath.pi * l / n))

    z1 = z2 = z3 = z4 = mpmath.mpf(1)
    for r in range(n):
        go = gamma(2 * r + 1)
        ge = gamma(2 * r)
        z1 *= two * mpmath.cosh(m * go / 2)
        z2 *= two * mpmath.sinh(m * go / 2)
        z3 *= two * mpmath.cosh(m * ge / 2)
        z4 *= two * mpmath.sinh(m * ge / 2)
    return (two * mpmath.sinh(2 * K)) ** (n * m / two) / 2 * (z1 + z2 + z3 + z4)


def torus_lnZ_mp(L, beta):
    with mpmath.workdps(40):
        return mpmath.log(_torus_Z_mp(L, L, mpmath.mpf(beta)))


@functools.lru_cache(maxsize=None)
def torus_exact(L, beta):
    """ln Z, e, C, beta F / N and S / N of the L x L torus at inverse temperature beta."""
    N = L * L
    with mpmath.workdps(40):
        b = mpmath.mpf(beta)
        f = lambda x: mpmath.log(_torus_Z_mp(L, L, x))
        lnZ = f(b)
        d1 = mpmath.diff(f, b, 1)
        d2 = mpmath.diff(f, b, 2)
        e = -d1 / N
        C = b * b * d2 / N
        return {
            "lnZ": float(lnZ),
            "e": float(e),
            "C": float(C),
            "betaF_per_N": float(-lnZ / N),
            "S_per_N": float(b * e + lnZ / N),
        }


BETA_C = 0.5 * np.log(1.0 + np.sqrt(2.0))

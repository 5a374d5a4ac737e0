"""Seeded synthetic inputs shared by the oracle and GPU tests.

Holds none of the method's arithmetic: only numpy-seeded random spin
configurations and structured populations.
"""
import numpy as np


def random_spins(R, L, seed, p_down=0.5):
    """R independent L x L configurations of int8 +-1 spins (row-major)."""
    rng = np.random.default_rng(seed)
    down = rng.random((R, L, L)) < p_down
    return np.where(down, -1, 1).astype(np.int8)


def ordered_spins(R, L, seed, n_flipped_max):
    """Mostly-up configurations with a random number (<= n_flipped_max) of
    down spins at random sites: a population spread over a few low energies."""
    rng = np.random.default_rng(seed)
    s = np.ones((R, L * L), np.int8)
    for j in range(R):
        k = rng.integers(0, n_flipped_max + 1)
        s[j, rng.choice(L * L, size=k, replace=False)] = -1
    return s.reshape(R, L, L)


def mixed_spins(R, L, seed):
    """Population mixing ordered and random replicas (wide energy spread)."""
    rng = np.random.default_rng(seed)
    p = rng.random(R)[:, None, None] * 0.5
    return np.where(rng.random((R, L, L)) < p, -1, 1).astype(np.int8)


def structured_spins(R, L, kind):
    """R copies of one regular pattern: 'cols' s(x, y) = (-1)^x, 'rows'
    s(x, y) = (-1)^y, 'checker' s(x, y) = (-1)^(x + y), 'up' all +1."""
    y, x = np.mgrid[0:L, 0:L]
    pattern = {"cols": x % 2, "rows": y % 2, "checker": (x + y) % 2, "up": np.zeros((L, L), int)}[kind]
    one = np.where(pattern == 1, -1, 1).astype(np.int8)
    return np.broadcast_to(one, (R, L, L)).copy()

"""Pins of the exact references themselves: the finite-torus partition
function (Kaufman; Ferdinand-Fisher form) must equal brute-force enumeration."""
import numpy as np
import pytest

import exact


@pytest.mark.parametrize("L", [2, 4])
@pytest.mark.parametrize("beta", [0.05, 0.2, 0.35, float(exact.BETA_C), 0.55, 0.8, 1.3])
def test_torus_formula_equals_enumeration(L, beta):
    b = exact.brute_observables(L, beta)
    t = exact.torus_exact(L, beta)
    for key in ("lnZ", "e", "C", "betaF_per_N", "S_per_N"):
        assert t[key] == pytest.approx(b[key], rel=1e-12, abs=1e-14), key


def test_enumeration_closed_forms():
    # 2^N states; E and M symmetric; ground states E = -2N (all up / all down).
    for L in (2, 4):
        Ev, Mv, g = exact.brute_force(L)
        N = L * L
        assert g.sum() == 2 ** N
        assert Ev.min() == -2 * N and g[0].sum() == 2
        # infinite temperature: <E> = 0, <E^2> = 2N (independent bonds, L >= 3)
        pE = g.sum(axis=1) / 2 ** N
        assert (pE * Ev).sum() == pytest.approx(0.0, abs=1e-12)
        if L >= 3:
            assert (pE * Ev ** 2).sum() == pytest.approx(2 * N)
        pM = g.sum(axis=0) / 2 ** N
        assert (pM * Mv ** 2).sum() == pytest.approx(N)
        assert (pM * Mv ** 4).sum() == pytest.approx(3 * N * N - 2 * N)


def test_torus_known_limits():
    # beta -> 0: ln Z -> N ln 2; the critical point is where C peaks (L = 32)
    assert exact.torus_exact(8, 1e-9)["lnZ"] == pytest.approx(64 * np.log(2.0), rel=1e-8)
    betas = np.linspace(0.38, 0.5, 13)
    C = [exact.torus_exact(32, float(b))["C"] for b in betas]
    assert 0.40 < betas[int(np.argmax(C))] < exact.BETA_C + 0.01

"""Statistical physics of the GPU runs against the exact finite-torus solution
(Kaufman; Ferdinand and Fisher; tests/exact.py, itself pinned to brute force)
at L = 16, 64 and 128, the lattice sizes of the small, headline and adaptive
configurations.

For each case several independent seeds run on the GPU; the mean of the
population-annealing estimates of the free energy, the energy per site and the
specific heat must lie within K standard errors of the exact value, plus a
small floor for the method's own O(1/R) bias (the paper states no tolerance;
the floors are a few times the run-to-run spread measured at these sizes).
"""
import numpy as np
import pytest

import exact

import paper_1703_03676_amd as pa  # noqa: E402  (a broken package fails, never skips)
import torch  # noqa: E402

pytestmark = pytest.mark.gpu

K = 5.0
# absolute floors: beta F / N, e (per site), and C relative
FLOOR_F, FLOOR_E, FLOOR_C_REL = 3e-5, 3e-4, 0.05


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _check(name, values, exact_value, floor):
    v = np.asarray(values, dtype=np.float64)
    m = float(v.mean())
    se = float(v.std(ddof=1) / np.sqrt(len(v))) if len(v) > 1 else 0.0
    print("  %-10s mean %.8g  exact %.8g  diff %.2e  se %.2e" % (name, m, exact_value, m - exact_value, se),
          flush=True)
    assert abs(m - exact_value) <= K * se + floor, (name, m, exact_value, se)


@pytest.mark.parametrize("L,R,theta,dbeta,seeds", [(16, 2000, 10, 0.01, 8), (64, 20000, 100, 0.005, 4)])
def test_fixed_schedule_matches_exact_torus(L, R, theta, dbeta, seeds):
    print("case physics L=%d R=%d theta=%d, %d seeds" % (L, R, theta, seeds), flush=True)
    targets = (0.44, 1.0)
    idx = {b: int(round(b / dbeta)) - 1 for b in targets}  # observables after step i are at beta = (i+1) dbeta
    got = {b: {"F": [], "e": [], "C": []} for b in targets}
    for s in range(1, seeds + 1):
        g = pa.Run(L, R, seed=100 + s, layout="bits")
        g.observables()
        obs = g.anneal(beta_f=1.0, dbeta=dbeta, theta=theta, mode="fixed")
        g.close()
        for b in targets:
            o = obs[idx[b]]
            assert abs(o["beta"] - b) < 1e-12
            got[b]["F"].append(o["betaF_per_N"])
            got[b]["e"].append(o["e"])
            got[b]["C"].append(o["C"])
    for b in targets:
        ex = exact.torus_exact(L, b)
        print(" beta %.2f" % b, flush=True)
        _check("betaF/N", got[b]["F"], ex["betaF_per_N"], FLOOR_F)
        _check("e", got[b]["e"], ex["e"], FLOOR_E)
        _check("C", got[b]["C"], ex["C"], FLOOR_C_REL * ex["C"])


def test_adaptive_l128_with_reweighting_matches_exact_torus():
    """L = 128, R = 50000, theta = 50, adaptive steps to alpha* = 0.85 with the
    multi-histogram record: the estimates at beta = 1, and the reweighted ones
    at beta = 0.44 (near the critical point) and 0.6."""
    L, R, theta, seeds = 128, 50000, 50, 3
    print("case physics L=128 adaptive, %d seeds" % seeds, flush=True)
    betas = np.array([0.44, 0.6])
    fin = {"F": [], "e": [], "C": []}
    rw = {b: {"F": [], "e": [], "C": []} for b in betas}
    for s in range(1, seeds + 1):
        g = pa.Run(L, R, seed=200 + s, layout="bits", mhr=True)
        g.observables()
        obs = g.anneal(beta_f=1.0, alpha_star=0.85, theta=theta, mode="adaptive")
        assert obs[-1]["beta"] == 1.0
        fin["F"].append(obs[-1]["betaF_per_N"])
        fin["e"].append(obs[-1]["e"])
        fin["C"].append(obs[-1]["C"])
        for b, o in zip(betas, g.reweight(betas)):
            rw[b]["F"].append(o["betaF_per_N"])
            rw[b]["e"].append(o["e"])
            rw[b]["C"].append(o["C"])
        g.close()
    ex = exact.torus_exact(L, 1.0)
    print(" beta 1.00", flush=True)
    _check("betaF/N", fin["F"], ex["betaF_per_N"], FLOOR_F)
    _check("e", fin["e"], ex["e"], FLOOR_E)
    _check("C", fin["C"], ex["C"], FLOOR_C_REL * ex["C"])
    for b in betas:
        ex = exact.torus_exact(L, float(b))
        print(" beta %.2f (reweighted)" % b, flush=True)
        _check("betaF/N", rw[b]["F"], ex["betaF_per_N"], FLOOR_F)
        _check("e", rw[b]["e"], ex["e"], FLOOR_E)
        _check("C", rw[b]["C"], ex["C"], FLOOR_C_REL * ex["C"])

"""Weighted averages of independent PA runs (Sec. 2.2, Eq. (weighted-average)).

TEST INFRASTRUCTURE ONLY (the library's pa_weighted_average is checked
against it).

M independent runs of the same system and target population size, measured
at the same inverse temperatures beta_i.  Run m's free-energy estimator
(Eq. (free energy)) gives ln Z_m(beta_i) = -beta_i F_m(beta_i) = -N (beta F/N)_m.
An observable is combined as

    A~(beta_i) = sum_m w_m(beta_i) A_m(beta_i),
    w_m(beta_i) = exp(-beta_i F_m(beta_i)) / sum_m' exp(-beta_i F_m'(beta_i)).

Readings where the paper is silent:
  * the combined free energy is that of the pooled estimate of Z, the mean of
    the M estimates:  -beta F~ = ln((1/M) sum_m Z_m);
  * the entropy of the combination follows Eq. (entropy) from the combined
    energy and free energy:  S~/N = beta e~ - beta F~/N;
  * the combined population size is the sum of the runs' sizes.
Exponentials are taken relative to the largest ln Z_m at each beta (the same
quotient, without overflow).
"""
import numpy as np

OBSERVABLES = ("e", "C", "abs_m", "m2", "m4")


def log_z(obs_runs, N):
    """ln Z_m(beta_i) = -N (beta F/N)_m, as an [M, nb] array."""
    return np.array([[-N * o["betaF_per_N"] for o in run] for run in obs_runs], dtype=np.float64)


def weights(lnZ):
    """w_m(beta_i) for lnZ [M, nb]: exp(ln Z_m) / sum_m' exp(ln Z_m')."""
    lnZ = np.asarray(lnZ, dtype=np.float64)
    top = lnZ.max(axis=0)
    z = np.exp(lnZ - top)
    return z / z.sum(axis=0)


def weighted_average(obs_runs, N):
    """Combine M runs (lists of per-beta observable dicts with keys beta, R, e,
    C, abs_m, m2, m4, betaF_per_N) measured at the same betas; returns one
    dict per beta."""
    M = len(obs_runs)
    nb = len(obs_runs[0])
    for run in obs_runs:
        if len(run) != nb:
            raise ValueError("runs measured at different numbers of temperatures")
        for o, o0 in zip(run, obs_runs[0]):
            if o["beta"] != o0["beta"]:
                raise ValueError("runs measured at different temperatures")
    lnZ = log_z(obs_runs, N)
    w = weights(lnZ)
    top = lnZ.max(axis=0)
    lnZ_comb = top + np.log(np.exp(lnZ - top).sum(axis=0)) - np.log(M)
    out = []
    for i in range(nb):
        beta = obs_runs[0][i]["beta"]
        d = {"beta": beta, "R": sum(run[i]["R"] for run in obs_runs)}
        for k in OBSERVABLES:
            d[k] = float(sum(w[m, i] * obs_runs[m][i][k] for m in range(M)))
        d["betaF_per_N"] = float(-lnZ_comb[i] / N)
        d["S_per_N"] = float(beta * d["e"] + lnZ_comb[i] / N)
        out.append(d)
    return out

"""Learned temperature steps: pairs logged by the bisection of adaptive runs
train the proposer on the GPU; learned runs then mostly skip the bisection
(the exact overlap test accepts the proposal), which saves overlap
evaluations, and reach the same free-energy accuracy against the exact
finite-torus result as plain adaptive runs.  Every learned run is also
replayed on the oracle with its own temperature schedule and must match it
bit for bit at every step."""
import os
import time

import numpy as np
import pytest

import exact
import oracle

import paper_1703_03676_amd as pa  # noqa: E402  (a broken package fails, never skips)
import torch  # noqa: E402

pytestmark = pytest.mark.gpu

ALPHA, THETA, BF = 0.85, 5, 1.0


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _runs(seeds):
    return [dict(L=16 if s % 2 else 32, R=1000, seed=int(s), layout="bits") for s in seeds]


@pytest.fixture(scope="module")
def trained():
    print("case learned: collect and train", flush=True)
    b = pa.Batch(_runs(range(1, 25)), dict(beta_f=BF, alpha_star=ALPHA, theta=THETA, mode="adaptive"))
    b.run()
    x, t = b.training_pairs()
    assert len(t) > 500 and np.all(np.isfinite(x)) and np.all(np.isfinite(t))
    m = pa.Mlp(max_batch=256, seed=0)
    xc, tc = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    m.fit_norm(xc, tc)
    losses = m.train(xc, tc, batch=64, epochs=300, lr=3e-3, momentum=0.9, seed=1)
    params, norm = m.params()
    # the target ln(dbeta sigma_E) varies little; what is left of its spread is
    # largely the bisection's own noise from finite populations, so the check
    # is on the residual in natural units: ln-step error below 0.1
    rms = float(np.sqrt(losses[-1])) * float(norm[17])
    print("learned: target spread %.3f, residual %.3f" % (float(norm[17]), rms), flush=True)
    assert losses[-1] < 0.8 * losses[0] and rms < 0.1
    return params, norm, float(losses[-1])


def _run_batch(seeds, mode, model=None):
    b = pa.Batch(_runs(seeds), dict(beta_f=BF, alpha_star=ALPHA, alpha_tol=0.01, theta=THETA, mode=mode))
    if model is not None:
        b.set_model(*model)
    t0 = time.perf_counter()
    b.run()
    return b, time.perf_counter() - t0


def _close(a, b, rel=1e-12):
    return a == b or abs(a - b) <= rel * max(abs(a), abs(b))


def _replay_on_oracle(b, r, spec, theta):
    """The run's temperature schedule from its history, replayed by the oracle
    (resample to each beta_i, theta sweeps, measure): every step's integer
    sums and population size, and the final population, must be equal."""
    hist = b.history(r)
    o = oracle.Run(spec["L"], spec["R"], seed=spec["seed"], run_id=spec.get("run_id", 0))
    o.set_threads(min(8, os.cpu_count() or 1))
    o.init()
    first = o.measure()
    for k in ("sumE", "sumE2", "sumAbsM", "sumM2", "sumM4", "R"):
        assert hist[0][k] == first[k], k
    for i, go in enumerate(hist[1:], start=1):
        o.resample(go["beta"])
        o.sweep(theta)
        oo = o.measure()
        for k in ("sumE", "sumE2", "sumAbsM", "sumM2", "sumM4", "R"):
            assert go[k] == oo[k], (i, k)
        for k in ("beta", "e", "C", "abs_m", "m2", "m4", "betaF_per_N", "S_per_N", "lnQ"):
            assert _close(go[k], oo[k]), (i, k, go[k], oo[k])
    gs, gE, gM = b.download_population(r)
    os_, oE, oM = o.get_population()
    assert np.array_equal(gE, oE) and np.array_equal(gM, oM) and np.array_equal(gs, os_)
    return len(hist) - 1


def test_learned_runs_accept_proposals_and_match_accuracy(trained):
    params, norm, loss = trained
    seeds = range(101, 117)
    ba, ta = _run_batch(seeds, "adaptive")
    bl, tl = _run_batch(seeds, "learned", (params, norm))
    props = acc = 0
    evals_a = evals_l = 0
    host_a = host_l = 0.0
    steps_a = steps_l = 0
    err_a, err_l = [], []
    for r, spec in enumerate(_runs(seeds)):
        assert ba.status(r) == pa.PA_OK and bl.status(r) == pa.PA_OK
        assert bl.state(r)["beta"] == BF
        p, a = bl.learned_stats(r)
        props += p
        acc += a
        na, sa = ba.choice_stats(r)
        nl, sl = bl.choice_stats(r)
        evals_a, evals_l, host_a, host_l = evals_a + na, evals_l + nl, host_a + sa, host_l + sl
        steps_a += len(ba.history(r)) - 1
        steps_l += len(bl.history(r)) - 1
        # overlap evaluations: 1 per proposal, 51 per bisection that does not
        # reach beta_f at once (1 for alpha(beta_f) and 50 halvings)
        assert nl <= p + 51 * (len(bl.history(r)) - 1 - a)
        assert na >= 51 * (len(ba.history(r)) - 2) + 1
        ex = exact.torus_exact(spec["L"], BF)["betaF_per_N"]
        err_a.append(ba.history(r)[-1]["betaF_per_N"] - ex)
        err_l.append(bl.history(r)[-1]["betaF_per_N"] - ex)
        # every step of the learned schedule keeps enough overlap: R_i stays near R
        for o in bl.history(r)[1:]:
            assert abs(o["R"] - spec["R"]) < 5 * np.sqrt(spec["R"])
    rate = acc / max(props, 1)
    print("learned: %d proposals, %d accepted (%.2f); adaptive %.3f s, learned %.3f s; "
          "|dF| adaptive %.2e learned %.2e; final training loss %.3f"
          % (props, acc, rate, ta, tl, np.mean(np.abs(err_a)), np.mean(np.abs(err_l)), loss), flush=True)
    print("learned: overlap evaluations per step %.1f (adaptive) vs %.1f (learned); host time choosing "
          "%.1f us vs %.1f us per step"
          % (evals_a / steps_a, evals_l / steps_l, 1e6 * host_a / steps_a, 1e6 * host_l / steps_l), flush=True)
    assert props > 0 and rate > 0.5
    # the deterministic saving: accepted proposals replace bisections
    assert evals_l / steps_l < 0.5 * evals_a / steps_a
    # the learned schedules themselves are reproduced by the oracle
    for r, spec in enumerate(_runs(seeds)[:6]):
        print("  replay learned run %d L=%d" % (r, spec["L"]), flush=True)
        _replay_on_oracle(bl, r, spec, THETA)
    # equal free-energy accuracy within the statistical spread of the runs
    sd = np.std(err_a) / np.sqrt(len(err_a)) + np.std(err_l) / np.sqrt(len(err_l))
    assert abs(np.mean(err_l)) < abs(np.mean(err_a)) + 4 * sd + 1e-4


def test_features_are_the_population_moments(trained):
    params, norm, _ = trained
    b = pa.Batch(_runs([7]), dict(beta_f=0.4, alpha_star=ALPHA, alpha_tol=0.01, theta=THETA, mode="learned"))
    b.set_model(params, norm)
    for _ in range(3):
        b.step()
    x, valid, prop = b.features(0)
    _, E, _ = b.download_population(0)
    st = b.state(0)
    hist = b.history(0)
    E = E.astype(np.float64)
    mu, sd = E.mean(), E.std()
    assert valid
    assert x[0] == pytest.approx(mu / 256, rel=1e-6)
    assert x[1] == pytest.approx(np.log(sd), rel=1e-6)
    assert x[2] == pytest.approx(((E - mu) ** 3).mean() / sd ** 3, rel=1e-4, abs=1e-5)
    assert x[3] == pytest.approx(((E - mu) ** 4).mean() / sd ** 4 - 3, rel=1e-4, abs=1e-5)
    assert x[4] == pytest.approx(st["beta"], rel=1e-7)
    assert x[5] == pytest.approx(np.log(16.0)) and x[6] == pytest.approx(np.log(1000.0))
    assert x[7] == pytest.approx(np.log(hist[-1]["beta"] - hist[-2]["beta"]), rel=1e-6)
    assert np.isfinite(prop)


def test_learned_run_at_l256_replays_on_the_oracle(trained):
    """A learned run at the lattice size of the L = 256 workload (population
    and temperature range reduced so the oracle replays it in seconds): the
    proposer was trained on L <= 32 only; its accepted steps and the fallback
    bisections make one schedule, which the oracle reproduces exactly."""
    params, norm, _ = trained
    # R as in training: ln R is constant there, so the network has no scale
    # for other R and its proposals for them are refused as non-finite
    spec = dict(L=256, R=1000, seed=5, layout="bits")
    print("case learned L=256 replay", flush=True)
    b = pa.Batch([spec], dict(beta_f=0.06, alpha_star=ALPHA, alpha_tol=0.01, theta=2, mode="learned"))
    b.set_model(params, norm)
    b.run()
    assert b.status(0) == pa.PA_OK and b.state(0)["beta"] == 0.06
    p, a = b.learned_stats(0)
    n = _replay_on_oracle(b, 0, spec, 2)
    print("learned L=256: %d steps, %d proposals, %d accepted" % (n, p, a), flush=True)
    assert p > 0 and n > 5

"""Planted mistakes in the oracle must fail its pins.

Each case copies the oracle's C source, plants one plausible mistake (a wrong
constant, sign, index, operand or comparison), builds it on the CPU and runs a
fast battery of the same pins the oracle tests use: published Philox vectors,
independence of the sites of one word and of runs in the random streams,
the exact Boltzmann distribution and exact free energy at L = 4, closed forms at
beta = 0, the heat-bath flip law per class, resampling normalisation and order, multi-histogram reweighting and
the adaptive-step postcondition.  The unmodified source must pass the battery
and every mutant must fail it.
"""
import os
import subprocess

import numpy as np
import pytest

import exact
import inputs
import oracle
import stream_pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "pa_oracle.c")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")

MUTANTS = {
    "philox_multiplier": ("0xD2511F53u", "0xD2511F55u"),
    "philox_key_schedule": ("k1 += PHILOX_W1;", "k1 += 0;"),
    "philox_lo_hi": ("uint32_t n1 = lo1;", "uint32_t n1 = hi1;"),
    "init_bias": ("((w >> (p & 31)) & 1) ? -1 : 1", "((w >> (p & 31)) & 3) ? -1 : 1"),
    "bond_index": ("int down = s[((y + 1) % L) * L + x];", "int down = s[((y + 1) % L) * L + (x + 1) % L];"),
    "zero_move_draws": ("if (k <= 0) {", "if (k < 0) {"),
    "thresholds_swapped": ("uint64_t T = (k == 2) ? T2 : T4;", "uint64_t T = (k == 2) ? T4 : T2;"),
    "threshold_exponent": ("exp(-4.0 * beta)", "exp(-2.0 * beta)"),
    "neighbour_index": ("s[y * L + (x + L - 1) % L]", "s[y * L + (x + 1) % L]"),
    "energy_bookkeeping": ("r->E[j] += 2 * k;", "r->E[j] += k;"),
    "magnetisation_bookkeeping": ("r->M[j] -= 2 * si;", "r->M[j] += 2 * si;"),
    "acceptance_direction": ("flip = ((uint64_t)x < T);", "flip = ((uint64_t)x >= T);"),
    "weight_sign": ("w[b] = exp(-(dbeta * d));", "w[b] = exp(dbeta * d);"),
    "tau_normalisation": ("double tau = ((double)r->R * w[b]) / W;", "double tau = ((double)r->Rcur * w[b]) / W;"),
    "count_comparison": ("(x <= thr[b] ? 1u : 0u)", "(x > thr[b] ? 1u : 0u)"),
    "lnQ_shift_sign": ("- dbeta * (double)Emin;", "+ dbeta * (double)Emin;"),
    "lnZ_accumulation": ("r->lnZ += lnQ;", "r->lnZ -= lnQ;"),
    "copy_parent_index": ("spin_at(r, r->spin, j), (size_t)r->N);", "spin_at(r, r->spin, (int)(off % r->Rcur)), (size_t)r->N);"),
    "specific_heat_beta": ("o->C = (beta * beta * (double)D)", "o->C = (beta * (double)D)"),
    "m4_normalisation": ("(R * N * N * N * N)", "(R * N * N * N)"),
    "entropy_sign": ("o->S_per_N = beta * o->e + r->lnZ / N;", "o->S_per_N = beta * o->e - r->lnZ / N;"),
    "mhr_beta_sign": ("- r->m_beta[i] * E;", "+ r->m_beta[i] * E;"),
    "mhr_moment_index": ("mM2 += p * ((double)r->SM2[b] / h);", "mM2 += p * ((double)r->SA[b] / h);"),
    "bisection_side": ("if (orc_alpha(r, mid) >= alpha_star)", "if (orc_alpha(r, mid) < alpha_star)"),
    "hb_negative_k": ("if (k == -2) return two32 - U2;", "if (k == -2) return U2;"),
    "hb_zero_k": ("if (k == 0) return two32 / 2;", "if (k == 0) return two32;"),
    "hb_exponent_sign": ("1.0 / (1.0 + exp(4.0 * beta))", "1.0 / (1.0 + exp(-4.0 * beta))"),
    "hb_exponent_scale": ("1.0 / (1.0 + exp(8.0 * beta))", "1.0 / (1.0 + exp(4.0 * beta))"),
    "hb_direction": ("flip = ((uint64_t)x < U);", "flip = ((uint64_t)x > U);"),
    # stream mapping: sites q and q + 16 share their high 16 bits
    "plane_alias": ("int bit = q & 31;", "int bit = q & 15;"),
    # stream mapping: sites q and q ^ 1 share one half of a SWEEP-LOW word
    "low_half_shared": ("uint32_t lo = (q & 1) ? (low_word & 0xFFFFu) : (low_word >> 16);",
                        "uint32_t lo = low_word >> 16;"),
    # stream mapping: the run number left out of the counters
    "run_tag_dropped": ("r->tag = run_id << 4;", "r->tag = 0;"),
    # in-line LCG variant (Sec. 4): multiplier, state update, seed counters
    "lcg_multiplier": ("#define LCG_A 1664525u", "#define LCG_A 1u"),
    "lcg_state_frozen": ("        x = lcg_next(x);\n        out[b] = x;", "        out[b] = lcg_next(x);"),
    "lcg_seed_colour": ("r->tag | 4, c);", "r->tag | 4, 0);"),
    "lcg_seed_sweep": ("(uint32_t)v, (uint32_t)g, (uint32_t)j, r->tag | 4", "(uint32_t)v, 0u, (uint32_t)j, r->tag | 4"),
    # the run number xored into the key (seed_hi = 1, run 0 == seed_hi = 0, run 1)
    "run_in_key": ("r->key1 = (uint32_t)(seed >> 32);\n    r->tag = run_id << 4;",
                   "r->key1 = (uint32_t)(seed >> 32) ^ run_id;\n    r->tag = 0;"),
}


def _check(cond, name, failures):
    if not cond:
        failures.append(name)
        raise StopIteration


def battery(lib, full=False):
    """Run the pins against the library; return the names of failed pins."""
    failures = []
    try:
        for line in open(GOLDEN):
            if line.strip() and not line.startswith("#"):
                v = [int(x, 16) for x in line.split()]
                _check(oracle.philox(v[0:4], v[4:6], lib) == v[6:10], "philox_kat", failures)

        # random streams: independent sites within a word, runs keyed apart
        _check(stream_pins.site_pairs_independent(lib), "site_pairs_independent", failures)
        _check(stream_pins.site_uniforms_independent(lib), "site_uniforms_independent", failures)
        _check(stream_pins.runs_have_own_streams(lib), "runs_have_own_streams", failures)
        _check(stream_pins.uniforms_distinct_across_updates(lib), "distinct_updates", failures)
        _check(stream_pins.site_pairs_independent(lib, lcg=True), "lcg_site_pairs_independent", failures)
        _check(stream_pins.uniforms_distinct_across_updates(lib, lcg=True), "lcg_distinct_updates", failures)

        # beta = 0 closed forms (independent spins)
        r = oracle.Run(8, 4000, seed=11, lib_=lib)
        r.init()
        s, E, M = r.get_population()
        Ef, Mf = E.astype(float), M.astype(float)
        for val, target in ((Ef, 0.0), (Ef ** 2, 128.0), (Mf ** 2, 64.0)):
            _check(abs(val.mean() - target) < 5 * val.std() / np.sqrt(4000), "beta0_moments", failures)
        Es = -(s.astype(int) * (np.roll(s, -1, 2) + np.roll(s, -1, 1))).sum(axis=(1, 2))
        _check(np.array_equal(Es, E), "init_energy", failures)

        # bookkeeping after sweeps
        r = oracle.Run(6, 30, seed=2, lib_=lib)
        r.set_population(inputs.mixed_spins(30, 6, 1), beta=0.4)
        r.sweep(5)
        s, E, M = r.get_population()
        Es = -(s.astype(int) * (np.roll(s, -1, 2) + np.roll(s, -1, 1))).sum(axis=(1, 2))
        _check(np.array_equal(Es, E) and np.array_equal(s.astype(int).sum(axis=(1, 2)), M), "bookkeeping", failures)

        # exact Boltzmann distribution at L = 4
        for beta in (0.3, 0.6):
            r = oracle.Run(4, 4000, seed=21, lib_=lib)
            r.set_population(inputs.random_spins(4000, 4, 8), beta=beta)
            r.sweep(40)
            _, E, _ = r.get_population()
            ex = exact.brute_observables(4, beta)
            cnt = np.array([(E == e).sum() for e in ex["Ev"]])
            m = ex["pE"] * cnt.sum()
            keep = m > 5
            chi2 = ((cnt[keep] - m[keep]) ** 2 / m[keep]).sum()
            dof = keep.sum() - 1
            _check(chi2 < dof + 6 * np.sqrt(2 * dof), "boltzmann_L4", failures)

        # the in-line LCG variant reaches the same distribution at L = 4
        r = oracle.Run(4, 4000, seed=25, lib_=lib, lcg=True)
        r.set_population(inputs.random_spins(4000, 4, 9), beta=0.44)
        r.sweep(40)
        _, E, _ = r.get_population()
        ex = exact.brute_observables(4, 0.44)
        cnt = np.array([(E == e).sum() for e in ex["Ev"]])
        m = ex["pE"] * cnt.sum()
        keep = m > 5
        chi2 = ((cnt[keep] - m[keep]) ** 2 / m[keep]).sum()
        dof = keep.sum() - 1
        _check(chi2 < dof + 6 * np.sqrt(2 * dof), "lcg_boltzmann_L4", failures)

        # heat-bath: flip frequency of each class k of colour 0 (updated first,
        # against the initial neighbours) and the Boltzmann distribution at L = 4
        s0 = inputs.random_spins(1500, 8, 31)
        r = oracle.Run(8, 1500, seed=17, lib_=lib, heatbath=True)
        r.set_population(s0, beta=0.3)
        r.sweep(1)
        s1, _, _ = r.get_population()
        h = np.roll(s0, 1, 1) + np.roll(s0, -1, 1) + np.roll(s0, 1, 2) + np.roll(s0, -1, 2)
        yy, xx = np.mgrid[0:8, 0:8]
        c0 = ((xx + yy) & 1) == 0
        k = (s0.astype(int) * h)[:, c0]
        flipped = (s1 != s0)[:, c0]
        for kk in (-4, -2, 0, 2, 4):
            p = 1.0 / (1.0 + np.exp(0.6 * kk))
            sel = k == kk
            _check(abs(flipped[sel].mean() - p) < 5 * np.sqrt(p * (1 - p) / sel.sum()), "hb_class_rates", failures)
        r = oracle.Run(4, 4000, seed=23, lib_=lib, heatbath=True)
        r.set_population(inputs.random_spins(4000, 4, 8), beta=0.5)
        r.sweep(40)
        _, E, _ = r.get_population()
        ex = exact.brute_observables(4, 0.5)
        cnt = np.array([(E == e).sum() for e in ex["Ev"]])
        m = ex["pE"] * cnt.sum()
        keep = m > 5
        chi2 = ((cnt[keep] - m[keep]) ** 2 / m[keep]).sum()
        dof = keep.sum() - 1
        _check(chi2 < dof + 6 * np.sqrt(2 * dof), "hb_boltzmann_L4", failures)

        # resampling: zero step, order, normalisation, lnQ
        s0 = inputs.mixed_spins(200, 6, 3)
        r = oracle.Run(6, 200, seed=1, lib_=lib)
        r.set_population(s0, beta=0.2)
        info = r.resample(0.2)
        _check(info["R_new"] == 200 and abs(info["lnQ"]) < 1e-14, "zero_step", failures)
        r.resample(0.6)
        counts = r.get_counts()
        new, E, M = r.get_population()
        _check(np.array_equal(new, np.repeat(s0, counts, axis=0)), "compaction_order", failures)
        Es = -(new.astype(int) * (np.roll(new, -1, 2) + np.roll(new, -1, 1))).sum(axis=(1, 2))
        _check(np.array_equal(Es, E), "copy_keeps_energy", failures)
        _check(abs(r.population - 200) < 5 * np.sqrt(50), "population_size", failures)
        # population pulled back to the target size R from R_{i-1} = 150
        r = oracle.Run(4, 100, seed=1, capacity=400, lib_=lib)
        r.set_population(np.ones((150, 4, 4), np.int8), beta=0.1)
        _check(abs(r.resample(0.3)["R_new"] - 100) <= 25, "target_population", failures)
        hist = np.zeros(37, np.int64)
        hist[3:9] = [5, 0, 7, 30, 2, 9]
        base, thr, lnQ = oracle.tables(36, 300, 53, hist, 0.17, lib)
        occ = hist > 0
        _check(abs((hist[occ] * (base[occ] + thr[occ] / 2.0 ** 32)).sum() / 300 - 1) < 1e-9, "tables_norm", failures)
        Ev = 4 * np.arange(37) - 72
        _check(abs(lnQ - np.log((hist * np.exp(-0.17 * Ev)).sum() / 53)) < 1e-12, "lnQ_closed_form", failures)

        # a full PA run at L = 4 against enumeration, plus multi-histogram
        r = oracle.Run(4, 6000, seed=1, lib_=lib)
        r.init()
        obs = [r.measure()]
        for i in range(1, 11):
            r.resample(0.1 * i)
            r.sweep(5)
            obs.append(r.measure())
        for o in obs[1:]:
            ex = exact.brute_observables(4, o["beta"])
            _check(abs(o["betaF_per_N"] - ex["betaF_per_N"]) < 4e-3, "pa_free_energy", failures)
            _check(abs(o["e"] - ex["e"]) < 0.04, "pa_energy", failures)
            _check(abs(o["S_per_N"] - ex["S_per_N"]) < 0.02, "pa_entropy", failures)
            _check(abs(o["m2"] - ex["m2"]) < 0.04 and abs(o["m4"] - ex["m4"]) < 0.04, "pa_magnetisation", failures)
        Cr = np.array([o["C"] / exact.brute_observables(4, o["beta"])["C"] for o in obs[1:]])
        _check(abs(Cr.mean() - 1) < 0.15, "pa_specific_heat", failures)
        for o in r.reweight(np.array([0.2, 0.45, 0.8])):
            ex = exact.brute_observables(4, o["beta"])
            _check(abs(o["betaF_per_N"] - ex["betaF_per_N"]) < 3e-3 and abs(o["e"] - ex["e"]) < 0.02, "mhr", failures)
            _check(abs(o["m2"] - ex["m2"]) < 0.02 and abs(o["C"] / ex["C"] - 1) < 0.1, "mhr_moments", failures)

        # adaptive step postcondition
        r = oracle.Run(6, 1500, seed=4, lib_=lib)
        r.init()
        b = r.adapt_beta(0.85, 1.0)
        _check(r.alpha(b) >= 0.85 and (b == 1.0 or r.alpha(b + 1e-9) < 0.85), "adaptive_step", failures)
    except StopIteration:
        pass
    except (OverflowError, ValueError) as exc:  # run aborted by the mutant
        failures.append("aborted:" + type(exc).__name__)
    return failures


def _build(tmp_path, name, source):
    c = tmp_path / (name + ".c")
    c.write_text(source)
    so = tmp_path / ("lib" + name + ".so")
    subprocess.check_call(["gcc", *oracle.CFLAGS, str(c), "-o", str(so), "-lm"])
    return oracle.load(str(so))


def test_unmodified_oracle_passes_battery(tmp_path):
    lib = _build(tmp_path, "control", open(SRC).read())
    assert battery(lib) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert old in src, "mutation site missing: " + old
    lib = _build(tmp_path, name, src.replace(old, new, 1))
    assert battery(lib) != [], "planted mistake %s passed every pin" % name

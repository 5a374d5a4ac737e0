// Host FP64 arithmetic of the method, shared by the single-run C ABI
// (pa_api.hip) and the batched driver (pa_batch.hip).  Everything here works
// on energy bins (E_b = 4 b - 2N) and a few scalars; nothing is per replica.
//
// Values that decide integers (thresholds, copy-count tables, the bisection)
// use a fixed operation order over ascending bins and are compiled without
// contraction, so they are reproducible bit for bit.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "pa.h"
#include "pa_internal.h"

namespace pa {
namespace host {

// Occupied window [bmin, bmax] of an energy histogram n[0..N].
struct Hist {
    const uint32_t* n;
    int bmin, bmax, N;
    int32_t energy(int b) const { return 4 * b - 2 * N; }
};

inline Hist hist_window(const uint32_t* n, const DevStats& s, int N)
{
    return Hist{n, (s.emin + 2 * N) / 4, (s.emax + 2 * N) / 4, N};
}

// Metropolis thresholds ceil(2^32 exp(-2 beta k)), k = 2, 4 (Sec. 3 table of
// Metropolis factors), split into a high part compared plane by plane and the
// low 16 bits.
inline void thresholds(double beta, uint32_t* t2h, uint32_t* t2l, uint32_t* t4h, uint32_t* t4l)
{
    const uint64_t t2 = (uint64_t)std::ceil(std::ldexp(std::exp(-4.0 * beta), 32));
    const uint64_t t4 = (uint64_t)std::ceil(std::ldexp(std::exp(-8.0 * beta), 32));
    *t2h = (uint32_t)(t2 >> 16);
    *t2l = (uint32_t)(t2 & 0xFFFFu);
    *t4h = (uint32_t)(t4 >> 16);
    *t4l = (uint32_t)(t4 & 0xFFFFu);
}

// Heat-bath thresholds U_k = ceil(2^32 / (1 + exp(2 beta k))), k = 2, 4: a site
// with k = s h flips with probability 1 / (1 + e^{2 beta k}) (heat-bath update,
// the alternative to Metropolis named in Sec. 2.1); U_0 = 2^31 and
// U_{-k} = 2^32 - U_k are applied in the kernel.  Same split as thresholds().
inline void hb_thresholds(double beta, uint32_t* u2h, uint32_t* u2l, uint32_t* u4h, uint32_t* u4l)
{
    const uint64_t u2 = (uint64_t)std::ceil(std::ldexp(1.0 / (1.0 + std::exp(4.0 * beta)), 32));
    const uint64_t u4 = (uint64_t)std::ceil(std::ldexp(1.0 / (1.0 + std::exp(8.0 * beta)), 32));
    *u2h = (uint32_t)(u2 >> 16);
    *u2l = (uint32_t)(u2 & 0xFFFFu);
    *u4h = (uint32_t)(u4 >> 16);
    *u4l = (uint32_t)(u4 & 0xFFFFu);
}

// The thresholds of a run's update rule at beta.
inline void sweep_thresholds(bool heatbath, double beta, uint32_t* t2h, uint32_t* t2l, uint32_t* t4h, uint32_t* t4l)
{
    if (heatbath)
        hb_thresholds(beta, t2h, t2l, t4h, t4l);
    else
        thresholds(beta, t2h, t2l, t4h, t4l);
}

// Weights exp(-dbeta d) for d = 4 k, k = 0, 1, ...: exactly the expression
// weight_sum evaluates for a bin 4 k above E_min (energies are multiples of 4),
// so a table filled ahead of time, while the GPU sweeps, gives identical
// values.
struct WeightTable {
    double dbeta = -1.0;
    std::vector<double> w;
    void fill(double db, size_t n)
    {
        dbeta = db;
        w.resize(n);
        for (size_t k = 0; k < n; ++k) w[k] = std::exp(-(db * (double)(int32_t)(4 * k)));
    }
    bool covers(double db, int nwin) const { return db == dbeta && (size_t)nwin <= w.size(); }
};

// W = sum over occupied bins (ascending) of n(b) w(b), w(b) = exp(-dbeta (E_b - E_min)):
// the normalisation of Eq. (Q) shifted by E_min.  With a table that covers the
// window (same dbeta), its values are used instead of evaluating exp again.
inline double weight_sum(const Hist& h, double dbeta, double* w, const WeightTable* pre = nullptr)
{
    const int32_t Emin = h.energy(h.bmin);
    const double* tw = (pre && pre->covers(dbeta, h.bmax - h.bmin + 1)) ? pre->w.data() : nullptr;
    double W = 0.0;
    for (int b = h.bmin; b <= h.bmax; ++b) {
        const uint32_t n = h.n[b];
        if (n == 0) continue;
        const double d = (double)(h.energy(b) - Emin);
        const double wb = tw ? tw[b - h.bmin] : std::exp(-(dbeta * d));
        if (w) w[b - h.bmin] = wb;
        W += (double)n * wb;
    }
    return W;
}

// Copy-count tables of Eq. (resampling factors): for every bin, base =
// floor(tau_hat) and thr = floor(2^32 frac(tau_hat)), tau_hat = R w / W.
// tab holds 2 entries per bin of the window; returns ln Q of Eq. (Q).
inline double resample_tables(const Hist& h, int64_t R, int64_t Rprev, double dbeta, uint32_t* tab,
                              std::vector<double>& w, const WeightTable* pre = nullptr)
{
    w.assign((size_t)(h.bmax - h.bmin + 1), 0.0);
    const double W = weight_sum(h, dbeta, w.data(), pre);
    for (int b = h.bmin; b <= h.bmax; ++b) {
        uint32_t base = 0, thr = 0;
        if (h.n[b] != 0) {
            const double tau = ((double)R * w[b - h.bmin]) / W;
            const double fl = std::floor(tau);
            base = (uint32_t)fl;
            thr = (uint32_t)std::floor(std::ldexp(tau - fl, 32));
        }
        tab[2 * (b - h.bmin)] = base;
        tab[2 * (b - h.bmin) + 1] = thr;
    }
    return std::log(W) - std::log((double)Rprev) - dbeta * (double)h.energy(h.bmin);
}

// Histogram overlap alpha(beta_i, beta_i + dbeta) of Sec. 2.3 over bins:
// (1/R_{i-1}) sum_b n(b) min(1, tau_hat(b)).
inline double overlap(const Hist& h, int64_t R, int64_t Rprev, double dbeta, std::vector<double>& w)
{
    w.assign((size_t)(h.bmax - h.bmin + 1), 0.0);
    const double W = weight_sum(h, dbeta, w.data());
    double acc = 0.0;
    for (int b = h.bmin; b <= h.bmax; ++b) {
        const uint32_t n = h.n[b];
        if (n == 0) continue;
        const double tau = ((double)R * w[b - h.bmin]) / W;
        acc += (double)n * (tau < 1.0 ? tau : 1.0);
    }
    return acc / (double)Rprev;
}

// Adaptive step (Sec. 2.3): beta_f if alpha(beta_f) >= alpha_star, else the low
// end of 50 bisection halvings of [beta, beta_f] that keep alpha >= alpha_star.
// Returns false if no step above beta reaches the target.  `evals` (may be
// null) is increased by the number of overlap evaluations made.
inline bool adapt_beta(const Hist& h, int64_t R, int64_t Rprev, double beta, double beta_f, double alpha_star,
                       double* beta_next, double* alpha_next, std::vector<double>& w, int64_t* evals = nullptr)
{
    int64_t n_eval = 1;
    const double a_f = overlap(h, R, Rprev, beta_f - beta, w);
    if (a_f >= alpha_star) {
        if (evals) *evals += n_eval;
        *beta_next = beta_f;
        if (alpha_next) *alpha_next = a_f;
        return true;
    }
    double lo = beta, hi = beta_f;
    for (int it = 0; it < 50; ++it) {
        const double mid = lo + 0.5 * (hi - lo);
        ++n_eval;
        if (overlap(h, R, Rprev, mid - beta, w) >= alpha_star)
            lo = mid;
        else
            hi = mid;
    }
    if (evals) *evals += n_eval + (lo != beta && alpha_next ? 1 : 0);
    if (lo == beta) return false;
    *beta_next = lo;
    if (alpha_next) *alpha_next = overlap(h, R, Rprev, lo - beta, w);
    return true;
}

inline double u128_to_double(uint64_t lo, uint64_t hi)
{
    const unsigned __int128 v = ((unsigned __int128)hi << 64) | lo;
    return (double)v;
}

// Population averages of Eq. (observables) from the exact integer sums, the
// free energy of Eq. (free energy) and the entropy of Eq. (entropy).
inline void observables(const DevStats& s, int64_t R_cur, int N_, double beta, double lnZ, double lnQ, pa_obs* o)
{
    const int64_t sE = (int64_t)s.sumE, sE2 = (int64_t)s.sumE2;
    const double N = (double)N_, R = (double)R_cur;
    const __int128 D = (__int128)R_cur * (__int128)sE2 - (__int128)sE * (__int128)sE;
    o->beta = beta;
    o->e = (double)sE / (R * N);
    o->C = (beta * beta * (double)D) / (N * R * R);
    o->abs_m = (double)(int64_t)s.sumAbsM / (R * N);
    o->m2 = (double)(int64_t)s.sumM2 / (R * N * N);
    o->m4 = u128_to_double(s.sumM4_lo, s.sumM4_hi) / (R * N * N * N * N);
    o->betaF_per_N = -lnZ / N;
    o->S_per_N = beta * o->e + lnZ / N;
    o->lnQ = lnQ;
    o->R = R_cur;
    o->sumE = sE;
    o->sumE2 = sE2;
    o->sumAbsM = (int64_t)s.sumAbsM;
    o->sumM2 = (int64_t)s.sumM2;
    o->sumM4_lo = s.sumM4_lo;
    o->sumM4_hi = s.sumM4_hi;
}

// Multi-histogram reweighting (Sec. 2.4, Eq. (MHR)) from the per-energy
// accumulators H, sum|M|, sum M^2 (u64) and sum M^4 (u128 pairs) and the
// measurement history (beta_i, R_i, ln Z_i).  Writes nb observables.
inline void reweight(int N_, const uint64_t* H, const uint64_t* SA, const uint64_t* SM2, const uint64_t* SM4,
                     const std::vector<double>& m_beta, const std::vector<double>& m_lnZ,
                     const std::vector<int64_t>& m_R, const double* betas, int32_t nb, pa_obs* out)
{
    const size_t nbins = (size_t)N_ + 1;
    const double N = (double)N_;
    const size_t nm = m_beta.size();
    auto energy = [&](size_t b) { return (double)(4 * (int64_t)b - 2 * (int64_t)N_); };
    // ln Omega(E) = ln H(E) - ln sum_i R_i exp(-ln Z_i - beta_i E)
    std::vector<double> lnOmega(nbins, 0.0), lw(nbins, 0.0), terms(nm);
    for (size_t b = 0; b < nbins; ++b) {
        if (H[b] == 0) continue;
        const double E = energy(b);
        double mx = -INFINITY;
        for (size_t i = 0; i < nm; ++i) {
            terms[i] = std::log((double)m_R[i]) - m_lnZ[i] - m_beta[i] * E;
            if (terms[i] > mx) mx = terms[i];
        }
        double s = 0.0;
        for (size_t i = 0; i < nm; ++i) s += std::exp(terms[i] - mx);
        lnOmega[b] = std::log((double)H[b]) - (mx + std::log(s));
    }
    for (int32_t k = 0; k < nb; ++k) {
        const double beta = betas[k];
        double mx = -INFINITY;
        for (size_t b = 0; b < nbins; ++b) {
            if (H[b] == 0) continue;
            lw[b] = lnOmega[b] - beta * energy(b);
            if (lw[b] > mx) mx = lw[b];
        }
        double s = 0.0;
        for (size_t b = 0; b < nbins; ++b)
            if (H[b] != 0) s += std::exp(lw[b] - mx);
        const double lnZ = mx + std::log(s);
        double mE = 0.0, mA = 0.0, mM2 = 0.0, mM4 = 0.0;
        for (size_t b = 0; b < nbins; ++b) {
            if (H[b] == 0) continue;
            const double p = std::exp(lw[b] - lnZ);
            const double h = (double)H[b];
            mE += p * energy(b);
            mA += p * ((double)SA[b] / h);
            mM2 += p * ((double)SM2[b] / h);
            mM4 += p * (u128_to_double(SM4[2 * b], SM4[2 * b + 1]) / h);
        }
        double var = 0.0;
        for (size_t b = 0; b < nbins; ++b) {
            if (H[b] == 0) continue;
            const double p = std::exp(lw[b] - lnZ);
            const double d = energy(b) - mE;
            var += p * d * d;
        }
        pa_obs* o = &out[k];
        std::memset(o, 0, sizeof(*o));
        o->beta = beta;
        o->e = mE / N;
        o->C = beta * beta * var / N;
        o->abs_m = mA / N;
        o->m2 = mM2 / (N * N);
        o->m4 = mM4 / (N * N * N * N);
        o->betaF_per_N = -lnZ / N;
        o->S_per_N = beta * o->e + lnZ / N;
    }
}

// Weighted average of nruns runs measured at the same nb temperatures (Sec.
// 2.2, Eq. (weighted-average)); obs[m * nb + i].  Weights w_m =
// exp(ln Z_m) / sum exp(ln Z_m') with ln Z_m = -N (beta F/N)_m, taken relative
// to the largest ln Z_m; the combined free energy is that of the pooled
// estimate ln((1/M) sum_m Z_m).  Sums run over m in ascending order.  Returns
// false if the runs' temperatures differ.
inline bool weighted_average(int N_, int nruns, int nb, const pa_obs* obs, pa_obs* out)
{
    const double N = (double)N_;
    std::vector<double> lnZ((size_t)nruns), z((size_t)nruns);
    for (int i = 0; i < nb; ++i) {
        const double beta = obs[i].beta;
        double top = -INFINITY;
        for (int m = 0; m < nruns; ++m) {
            const pa_obs& o = obs[(size_t)m * nb + i];
            if (o.beta != beta) return false;
            lnZ[(size_t)m] = -N * o.betaF_per_N;
            if (lnZ[(size_t)m] > top) top = lnZ[(size_t)m];
        }
        double S = 0.0;
        for (int m = 0; m < nruns; ++m) {
            z[(size_t)m] = std::exp(lnZ[(size_t)m] - top);
            S += z[(size_t)m];
        }
        pa_obs r;
        std::memset(&r, 0, sizeof(r));
        r.beta = beta;
        for (int m = 0; m < nruns; ++m) {
            const pa_obs& o = obs[(size_t)m * nb + i];
            const double w = z[(size_t)m] / S;
            r.e += w * o.e;
            r.C += w * o.C;
            r.abs_m += w * o.abs_m;
            r.m2 += w * o.m2;
            r.m4 += w * o.m4;
            r.R += o.R;
        }
        const double lnZc = top + std::log(S) - std::log((double)nruns);
        r.betaF_per_N = -lnZc / N;
        r.S_per_N = beta * r.e + lnZc / N;
        out[i] = r;
    }
    return true;
}

// Bit store (colour 0 words then colour 1 words; bit q & 31 of word q >> 5 is
// within-colour site q = (y L + x) >> 1; set = spin -1) <-> int8 row-major.
inline void bits_to_int8(const uint32_t* words, int L, size_t n, int8_t* spins)
{
    const int N = L * L, half = N / 2, hw = L / 2, wpc = half / 32;
    for (size_t j = 0; j < n; ++j) {
        const uint32_t* wj = words + j * (size_t)(N / 32);
        int8_t* sj = spins + j * (size_t)N;
        for (int c = 0; c < 2; ++c)
            for (int q = 0; q < half; ++q) {
                const int y = q / hw, x = 2 * (q % hw) + ((y + c) & 1);
                sj[y * L + x] = ((wj[c * wpc + (q >> 5)] >> (q & 31)) & 1u) ? -1 : 1;
            }
    }
}

// Site rows of the interleaved store ([site][replica], n replicas per row as
// copied out of the store) <-> int8 row-major replicas ([replica][site]).
inline void interleaved_to_int8(const int8_t* rows, size_t N, size_t n, int8_t* spins)
{
    for (size_t s = 0; s < N; ++s)
        for (size_t j = 0; j < n; ++j) spins[j * N + s] = rows[s * n + j];
}

inline void int8_to_interleaved(const int8_t* spins, size_t N, size_t n, int8_t* rows)
{
    for (size_t s = 0; s < N; ++s)
        for (size_t j = 0; j < n; ++j) rows[s * n + j] = spins[j * N + s];
}

inline void int8_to_bits(const int8_t* spins, int L, size_t n, uint32_t* words)
{
    const int N = L * L, half = N / 2, hw = L / 2, wpc = half / 32;
    std::memset(words, 0, n * (size_t)(N / 8));
    for (size_t j = 0; j < n; ++j) {
        uint32_t* wj = words + j * (size_t)(N / 32);
        const int8_t* sj = spins + j * (size_t)N;
        for (int c = 0; c < 2; ++c)
            for (int q = 0; q < half; ++q) {
                const int y = q / hw, x = 2 * (q % hw) + ((y + c) & 1);
                if (sj[y * L + x] < 0) wj[c * wpc + (q >> 5)] |= 1u << (q & 31);
            }
    }
}

}  // namespace host
}  // namespace pa

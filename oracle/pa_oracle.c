/*
 * pa_oracle.c -- plain, serial CPU oracle for population annealing (PA) of the
 * 2D ferromagnetic Ising model.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this code.  The GPU product path never
 * calls it and shares no code with it.
 *
 * The oracle follows the paper (Barash, Weigel, Borovsky, Janke, Shchur,
 * "GPU accelerated population annealing algorithm", arXiv:1703.03676) step by
 * step, with every choice the paper leaves open fixed as stated below.  It is
 * written for clarity: int8 row-major spins, one site at a time, FP64 with no
 * contraction (build with -ffp-contract=off).  Only for timing, orc_init and
 * orc_sweep may share the replicas out among threads (OpenMP); replicas are
 * independent there, so results do not depend on it.
 *
 *   Sec. 2.1, enumerated algorithm ........ orc_init / orc_resample / orc_sweep
 *   Sec. 2.1, Eq. (Q) ...................... resample: Q_i via the energy histogram
 *   Sec. 2.1, Eq. (resampling factors) ..... resample: integer copy counts
 *   Sec. 2.1, Eq. (observables) ............ orc_measure
 *   Sec. 2.1, Eqs. (free energy), (entropy)  orc_measure
 *   Sec. 2.3, overlap alpha + bisection .... orc_alpha / orc_adapt_beta
 *   Sec. 2.4, Eq. (multi-histogram) ........ orc_reweight
 *   Sec. 3, Hamiltonian; checkerboard ...... site_energy / orc_sweep
 *   Sec. 3, Philox4x32-10 (Salmon et al.) .. philox4x32_10
 *
 * Readings of points the paper leaves open (each is also a documented design
 * reading of the project):
 *   R1  Colour of site (x,y) is (x+y)&1; colour 0 is updated first; one sweep is
 *       colour 0 then colour 1.  Within a colour the order is irrelevant because
 *       same-colour sites do not interact.
 *   R2  Within-colour index q = (y*L + x) >> 1 (a bijection onto [0, N/2)).
 *   R3  Random-number streams, all Philox4x32-10 with key (seed_lo, seed_hi).
 *       Counter word 3 carries the stream tag in its low 4 bits and the run
 *       number above them, t(s) = 16 run + s (run < 2^28), so that every
 *       (seed, run, stream) triple has streams of its own:
 *         SWEEP-HIGH  counter (4v+k, 2g+c, j, t(0)), k=0..3, output w -> plane 4k+w
 *                     (v = q>>5 is the 32-site word of the site, g the run's
 *                     global sweep number, j the replica slot).  The high 16 bits
 *                     of the site's uniform are bit (q&31) of planes 0..15,
 *                     plane 0 most significant.
 *         SWEEP-LOW   counter (q>>3, 2g+c, j, t(3)), output (q>>1)&3, upper half
 *                     for even q, lower half for odd q: the low 16 bits.
 *         RESAMPLE    counter (j>>2, i, 0, t(1)), output j&3 (i = temperature step).
 *         INIT        counter (p>>7, 0, j, t(2)), output (p>>5)&3, bit p&31, with
 *                     p = c*N/2 + q; a set bit means spin -1.
 *   R4  Metropolis: with k = s * (sum of the 4 neighbours), the energy change of a
 *       flip is 2k; k <= 0 always flips; k in {2,4} flips iff the site's 32-bit
 *       uniform x satisfies x < T_k = ceil(2^32 exp(-2 beta k)), i.e. u < p for
 *       u = x 2^-32.
 *   R5  Resampling tie r == frac gives floor+1 (literal reading); with
 *       thr = floor(2^32 frac) this is "count = floor(tau) + (x <= thr)".
 *   R6  Weights are shifted by the smallest energy E_min so exp never overflows;
 *       Q_i is recovered exactly: ln Q = ln W - ln R_{i-1} - dbeta E_min.
 *   R7  All FP64 sums run over energy bins in ascending order.
 *   R8  Adaptive step: if alpha(beta_f) >= alpha*, take beta_f; otherwise 50
 *       bisection halvings of [beta_{i-1}, beta_f], keeping the side with
 *       alpha >= alpha*; the result is the low end.
 *   R9  Multi-histogram reweighting uses every measurement taken (one per call
 *       of orc_measure), including the one at beta_0 = 0.
 *   R10 Heat-bath update (Sec. 2.1 names it as an alternative to Metropolis and
 *       gives no details): the site takes spin +1 with probability
 *       e^{beta h} / (e^{beta h} + e^{-beta h}), so with k = s h it flips with
 *       probability 1 / (1 + e^{2 beta k}).  It flips iff its 32-bit uniform x
 *       (the same streams as R3) satisfies x < U_k, with
 *       U_k = ceil(2^32 / (1 + e^{2 beta k})) for k = 2, 4, U_0 = 2^31 and
 *       U_{-k} = 2^32 - U_k, so that P(flip | k) + P(flip | -k) = 1 exactly.
 *   R11 In-line LCG variant of the multi-spin-coded sweep (Sec. 4: one draw of
 *       the base generator seeds, per word of spins and per update of it, a
 *       linear congruential generator r' = A r + C mod 2^32 with A = 1664525,
 *       C = 1013904223, which supplies the word's uniforms).  A word here is
 *       the 32 same-colour sites q = 32v .. 32v+31 of one replica; its seed
 *       for the update of colour c in sweep g is output c of Philox block
 *       (v, g, j, t(4)) (stream LCG-SEED); site q = 32v + b takes the
 *       (b+1)-th LCG output after the seed as its 32-bit uniform x, and
 *       flips as in R4.  Every site consumes its output whether or not it
 *       needs it, so positions are fixed.  Initial state and resampling keep
 *       the Philox streams of R3, as the paper's variant does.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random numbers:
 * as easy as 1, 2, 3").  A 4-word counter is mixed by ten rounds; each round
 * multiplies words 0 and 2 by fixed odd constants, takes the 64-bit products
 * apart and xors the high halves with the other two words and the round key.
 * The 2-word key is advanced by the Weyl constants between rounds.           */
/* ------------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint32_t philox_word(uint32_t key0, uint32_t key1, uint32_t a, uint32_t b,
                            uint32_t c, uint32_t d, int word)
{
    uint32_t ctr[4] = {a, b, c, d}, key[2] = {key0, key1}, out[4];
    philox4x32_10(ctr, key, out);
    return out[word];
}

/* ------------------------------------------------------------------------- */
/* Run state                                                                  */
/* ------------------------------------------------------------------------- */
typedef struct {
    double beta, e, C, abs_m, m2, m4, betaF_per_N, S_per_N, lnQ;
    int64_t R;
    int64_t sumE, sumE2, sumAbsM, sumM2;
    uint64_t sumM4_lo, sumM4_hi;
} orc_obs;

typedef struct {
    int L, N, R, capacity;
    uint32_t key0, key1;
    uint32_t tag;       /* 16 * run number: counter word 3 without the stream number */
    int Rcur;           /* R_i: current population size */
    int step;           /* i: number of resampling steps done */
    uint64_t sweeps;    /* g: number of sweeps done in this run */
    double beta;        /* beta_i */
    double lnZ;         /* ln Z(beta_i) estimate, Eq. (free energy) */
    double lnQ_last;
    int8_t *spin;       /* capacity x N, replica-major, row-major inside */
    int32_t *E, *M;
    int8_t *spin2;      /* resampling target */
    int32_t *E2, *M2;
    uint32_t *counts;   /* copy counts of the last resampling (per parent) */
    int counts_n;
    int32_t *slot;      /* optional: random-stream slot of each replica in a sweep
                           (NULL: replica j uses slot j); for sampled checks */
    int heatbath;       /* 0: Metropolis sweeps (R4); 1: heat-bath sweeps (R10) */
    int threads;        /* threads over replicas in orc_init / orc_sweep (1: serial) */
    int lcg;            /* 1: site uniforms from the in-line LCG of R11 (Metropolis only) */
    /* multi-histogram accumulators, one bin per energy level */
    int64_t *H, *SA, *SM2;
    unsigned __int128 *SM4;
    int nmeas, meas_cap;
    double *m_beta, *m_lnZ;
    int64_t *m_R;
} orc_run;

static int bin_of(const orc_run *r, int32_t E) { return (E + 2 * r->N) / 4; }
static int32_t energy_of_bin(const orc_run *r, int b) { return 4 * b - 2 * r->N; }

static int8_t *spin_at(orc_run *r, int8_t *base, int j) { return base + (size_t)j * r->N; }

/* Energy and magnetisation straight from the Hamiltonian (Sec. 3):
 * E = -sum over the 2N bonds (right and down neighbour of every site). */
static void count_EM(const orc_run *r, const int8_t *s, int32_t *E, int32_t *M)
{
    int L = r->L;
    int32_t e = 0, m = 0;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            int si = s[y * L + x];
            int right = s[y * L + (x + 1) % L];
            int down = s[((y + 1) % L) * L + x];
            e -= si * (right + down);
            m += si;
        }
    *E = e;
    *M = m;
}

orc_run *orc_new(int L, int R, int capacity, uint64_t seed, uint32_t run_id)
{
    if (L < 2 || (L & 1) || R < 1 || capacity < R || run_id >= (1u << 28)) return NULL;
    orc_run *r = (orc_run *)calloc(1, sizeof(orc_run));
    r->L = L;
    r->N = L * L;
    r->R = R;
    r->capacity = capacity;
    r->key0 = (uint32_t)seed;
    r->key1 = (uint32_t)(seed >> 32);
    r->tag = run_id << 4;
    r->threads = 1;
    size_t ns = (size_t)capacity * r->N;
    r->spin = (int8_t *)calloc(ns, 1);
    r->spin2 = (int8_t *)calloc(ns, 1);
    r->E = (int32_t *)calloc(capacity, 4);
    r->M = (int32_t *)calloc(capacity, 4);
    r->E2 = (int32_t *)calloc(capacity, 4);
    r->M2 = (int32_t *)calloc(capacity, 4);
    r->counts = (uint32_t *)calloc(capacity, 4);
    int nb = r->N + 1;
    r->H = (int64_t *)calloc(nb, 8);
    r->SA = (int64_t *)calloc(nb, 8);
    r->SM2 = (int64_t *)calloc(nb, 8);
    r->SM4 = (unsigned __int128 *)calloc(nb, sizeof(unsigned __int128));
    r->meas_cap = 64;
    r->m_beta = (double *)calloc(r->meas_cap, 8);
    r->m_lnZ = (double *)calloc(r->meas_cap, 8);
    r->m_R = (int64_t *)calloc(r->meas_cap, 8);
    return r;
}

void orc_free(orc_run *r)
{
    if (!r) return;
    free(r->spin); free(r->spin2); free(r->E); free(r->M); free(r->E2); free(r->M2);
    free(r->counts); free(r->H); free(r->SA); free(r->SM2); free(r->SM4);
    free(r->m_beta); free(r->m_lnZ); free(r->m_R); free(r->slot);
    free(r);
}

/* Step 1 of the algorithm at beta_0 = 0: simple sampling of independent
 * uniform spins; Z_{beta_0} = 2^N (Sec. 2.1).  Stream INIT, reading R3. */
void orc_init(orc_run *r)
{
    int L = r->L, N = r->N, half = N / 2;
#pragma omp parallel for schedule(static) num_threads(r->threads) if (r->threads > 1)
    for (int j = 0; j < r->R; ++j) {
        int8_t *s = spin_at(r, r->spin, j);
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                int c = (x + y) & 1;
                int q = (y * L + x) >> 1;
                uint32_t p = (uint32_t)(c * half + q);
                uint32_t w = philox_word(r->key0, r->key1, p >> 7, 0, (uint32_t)j, r->tag | 2, (int)((p >> 5) & 3));
                s[y * L + x] = ((w >> (p & 31)) & 1) ? -1 : 1;
            }
        count_EM(r, s, &r->E[j], &r->M[j]);
    }
    r->Rcur = r->R;
    r->step = 0;
    r->sweeps = 0;
    r->beta = 0.0;
    r->lnZ = (double)N * log(2.0);
    r->lnQ_last = 0.0;
    r->counts_n = 0;
}

/* Integer Metropolis thresholds T_k = ceil(2^32 exp(-2 beta k)), k = 2, 4
 * (the paper's table of exp(-beta dE), Sec. 3, with dE = 2k). */
void orc_thresholds(double beta, uint64_t *T2, uint64_t *T4)
{
    *T2 = (uint64_t)ceil(ldexp(exp(-4.0 * beta), 32));
    *T4 = (uint64_t)ceil(ldexp(exp(-8.0 * beta), 32));
}

/* Integer heat-bath thresholds of reading R10 for k = 2, 4:
 * U_k = ceil(2^32 / (1 + exp(2 beta k))); U_0 = 2^31 and U_{-k} = 2^32 - U_k
 * follow from them. */
void orc_hb_thresholds(double beta, uint64_t *U2, uint64_t *U4)
{
    *U2 = (uint64_t)ceil(ldexp(1.0 / (1.0 + exp(4.0 * beta)), 32));
    *U4 = (uint64_t)ceil(ldexp(1.0 / (1.0 + exp(8.0 * beta)), 32));
}

/* Threads over replicas in orc_init and orc_sweep (for timing only: the
 * replicas of a half sweep are independent, so the result does not depend on
 * it).  n < 1 means 1. */
void orc_set_threads(orc_run *r, int n) { r->threads = n < 1 ? 1 : n; }

/* Site uniforms of orc_sweep: 0 the Philox streams of R3, 1 the in-line LCG
 * of R11 (for either update rule). */
void orc_set_lcg(orc_run *r, int on) { r->lcg = on ? 1 : 0; }

/* The LCG of R11: one step r -> A r + C mod 2^32. */
#define LCG_A 1664525u
#define LCG_C 1013904223u
static uint32_t lcg_next(uint32_t x) { return LCG_A * x + LCG_C; }

/* R11: the 32 uniforms of word v (colour c, replica slot j, sweep g): the
 * word's seed from stream LCG-SEED, then one LCG output per site in bit
 * order. */
static void lcg_uniforms(const orc_run *r, uint64_t g, int c, int j, int v, uint32_t out[32])
{
    uint32_t x = philox_word(r->key0, r->key1, (uint32_t)v, (uint32_t)g, (uint32_t)j, r->tag | 4, c);
    for (int b = 0; b < 32; ++b) {
        x = lcg_next(x);
        out[b] = x;
    }
}

/* Select the update of orc_sweep: 0 Metropolis (R4), 1 heat-bath (R10). */
void orc_set_heatbath(orc_run *r, int on) { r->heatbath = on ? 1 : 0; }

/* Heat-bath threshold of a site with k = s h (reading R10). */
static uint64_t hb_threshold(int k, uint64_t U2, uint64_t U4)
{
    const uint64_t two32 = (uint64_t)1 << 32;
    if (k == 0) return two32 / 2;
    if (k == 2) return U2;
    if (k == 4) return U4;
    if (k == -2) return two32 - U2;
    return two32 - U4;
}

/* The sixteen SWEEP-HIGH planes of the 32-site word v (colour c, replica slot
 * j, sweep g): four Philox blocks, outputs in order, plane 0 first. */
static void sweep_planes(const orc_run *r, uint64_t g, int c, int j, uint32_t v, uint32_t planes[16])
{
    uint32_t ctr1 = (uint32_t)(2 * g + (uint64_t)c);
    for (uint32_t k = 0; k < 4; ++k) {
        uint32_t ctr[4] = {4 * v + k, ctr1, (uint32_t)j, r->tag | 0}, key[2] = {r->key0, r->key1}, out[4];
        philox4x32_10(ctr, key, out);
        for (int w = 0; w < 4; ++w) planes[4 * k + w] = out[w];
    }
}

/* The 32-bit uniform that decides a flip of site q: its high 16 bits are bit
 * (q & 31) of planes 0..15 (plane 0 most significant), its low 16 bits come
 * from the SWEEP-LOW stream (reading R3). */
static uint32_t site_uniform(const orc_run *r, uint64_t g, int c, int j, int q, const uint32_t planes[16])
{
    int bit = q & 31;
    uint32_t hi = 0;
    for (int p = 0; p < 16; ++p) hi = (hi << 1) | ((planes[p] >> bit) & 1u);
    uint32_t ctr1 = (uint32_t)(2 * g + (uint64_t)c);
    uint32_t low_word = philox_word(r->key0, r->key1, (uint32_t)q >> 3, ctr1, (uint32_t)j, r->tag | 3, (q >> 1) & 3);
    uint32_t lo = (q & 1) ? (low_word & 0xFFFFu) : (low_word >> 16);
    return (hi << 16) | lo;
}

/* Step 3 of the algorithm: theta rounds of checkerboard Metropolis updates at
 * the current beta (Sec. 2.1; checkerboard decomposition of Sec. 3), or of
 * heat-bath updates (reading R10) when selected.  Sites of one colour are
 * visited word by word in within-colour index order. */
void orc_sweep(orc_run *r, int nsweeps)
{
    int L = r->L, half = r->N / 2, hw = L / 2;
    uint64_t T2, T4, U2, U4;
    orc_thresholds(r->beta, &T2, &T4);
    orc_hb_thresholds(r->beta, &U2, &U4);
    for (int t = 0; t < nsweeps; ++t) {
        uint64_t g = r->sweeps;
        for (int c = 0; c < 2; ++c) {
            /* replicas are independent within a half sweep: with threads set,
             * they are shared out among them; the result is the same */
#pragma omp parallel for schedule(dynamic, 16) num_threads(r->threads) if (r->threads > 1)
            for (int j = 0; j < r->Rcur; ++j) {
                int8_t *s = spin_at(r, r->spin, j);
                int slot = r->slot ? r->slot[j] : j;
                for (int v = 0; 32 * v < half; ++v) {
                    uint32_t planes[16], lcg_u[32];
                    if (r->lcg) {
                        lcg_uniforms(r, g, c, slot, v, lcg_u);
                    } else {
                        sweep_planes(r, g, c, slot, (uint32_t)v, planes);
                    }
                    for (int q = 32 * v; q < 32 * v + 32 && q < half; ++q) {
                        int y = q / hw;
                        int x = 2 * (q % hw) + ((y + c) & 1);
                        int si = s[y * L + x];
                        int h = s[y * L + (x + 1) % L] + s[y * L + (x + L - 1) % L] +
                                s[((y + 1) % L) * L + x] + s[((y + L - 1) % L) * L + x];
                        int k = si * h;
                        int flip;
                        if (r->heatbath) {
                            uint64_t U = hb_threshold(k, U2, U4);
                            uint32_t x = r->lcg ? lcg_u[q & 31] : site_uniform(r, g, c, slot, q, planes);
                            flip = ((uint64_t)x < U);
                        } else if (k <= 0) {
                            flip = 1;
                        } else {
                            uint64_t T = (k == 2) ? T2 : T4;
                            uint32_t x = r->lcg ? lcg_u[q & 31] : site_uniform(r, g, c, slot, q, planes);
                            flip = ((uint64_t)x < T);
                        }
                        if (flip) {
                            s[y * L + x] = (int8_t)(-si);
                            r->E[j] += 2 * k;
                            r->M[j] -= 2 * si;
                        }
                    }
                }
            }
        }
        r->sweeps = g + 1;
    }
}

/* Energy histogram over the current population: n(b), b = (E+2N)/4. */
static void histogram(const orc_run *r, int64_t *n, int *bmin, int *bmax)
{
    int nb = r->N + 1;
    memset(n, 0, sizeof(int64_t) * (size_t)nb);
    int lo = nb, hi = -1;
    for (int j = 0; j < r->Rcur; ++j) {
        int b = bin_of(r, r->E[j]);
        n[b] += 1;
        if (b < lo) lo = b;
        if (b > hi) hi = b;
    }
    *bmin = lo;
    *bmax = hi;
}

/* Weights w(b) = exp(-dbeta (E_b - E_min)) and W = sum_b n(b) w(b), ascending b
 * (Eq. (Q) with the E_min shift of reading R6). */
static double weights(const orc_run *r, const int64_t *n, int bmin, int bmax, double dbeta, double *w)
{
    int32_t Emin = energy_of_bin(r, bmin);
    double W = 0.0;
    for (int b = bmin; b <= bmax; ++b) {
        if (n[b] == 0) continue;
        double d = (double)(energy_of_bin(r, b) - Emin);
        w[b] = exp(-(dbeta * d));
        W += (double)n[b] * w[b];
    }
    return W;
}

/* Step 2: resample from beta_i-1 to beta_next (Eqs. (Q), (resampling factors)).
 * Returns the new population size, or (state unchanged) -1 if it would exceed
 * the capacity and -2 if no replica would survive. */
int orc_resample(orc_run *r, double beta_next, double *lnQ_out, int32_t *Emin_out)
{
    int nb = r->N + 1;
    int64_t *n = (int64_t *)calloc(nb, 8);
    double *w = (double *)calloc(nb, 8);
    uint32_t *base = (uint32_t *)calloc(nb, 4);
    uint32_t *thr = (uint32_t *)calloc(nb, 4);
    int bmin, bmax;
    histogram(r, n, &bmin, &bmax);
    double dbeta = beta_next - r->beta;
    double W = weights(r, n, bmin, bmax, dbeta, w);
    int32_t Emin = energy_of_bin(r, bmin);
    double lnQ = log(W) - log((double)r->Rcur) - dbeta * (double)Emin;
    for (int b = bmin; b <= bmax; ++b) {
        if (n[b] == 0) continue;
        double tau = ((double)r->R * w[b]) / W;
        double fl = floor(tau);
        double frac = tau - fl;
        base[b] = (uint32_t)fl;
        thr[b] = (uint32_t)floor(ldexp(frac, 32));
    }
    int step = r->step + 1;
    int64_t total = 0;
    for (int j = 0; j < r->Rcur; ++j) {
        int b = bin_of(r, r->E[j]);
        uint32_t x = philox_word(r->key0, r->key1, (uint32_t)j >> 2, (uint32_t)step, 0, r->tag | 1, j & 3);
        r->counts[j] = base[b] + (x <= thr[b] ? 1u : 0u);
        total += r->counts[j];
    }
    r->counts_n = r->Rcur;
    free(r->slot);
    r->slot = NULL;
    free(n); free(w); free(base); free(thr);
    if (total > r->capacity) return -1;
    if (total == 0) return -2;
    /* compaction: parents in ascending order, copies contiguous */
    int64_t off = 0;
    for (int j = 0; j < r->Rcur; ++j)
        for (uint32_t cpy = 0; cpy < r->counts[j]; ++cpy) {
            memcpy(spin_at(r, r->spin2, (int)off), spin_at(r, r->spin, j), (size_t)r->N);
            r->E2[off] = r->E[j];
            r->M2[off] = r->M[j];
            ++off;
        }
    int8_t *ts = r->spin; r->spin = r->spin2; r->spin2 = ts;
    int32_t *te = r->E; r->E = r->E2; r->E2 = te;
    int32_t *tm = r->M; r->M = r->M2; r->M2 = tm;
    r->Rcur = (int)total;
    r->step = step;
    r->beta = beta_next;
    r->lnZ += lnQ;
    r->lnQ_last = lnQ;
    if (lnQ_out) *lnQ_out = lnQ;
    if (Emin_out) *Emin_out = Emin;
    return (int)total;
}

/* Histogram overlap alpha(beta_{i-1}, beta') of Sec. 2.3, written over energy
 * bins: alpha = (1/R_{i-1}) sum_b n(b) min(1, tau_hat(b)). */
double orc_alpha(orc_run *r, double beta_prime)
{
    int nb = r->N + 1;
    int64_t *n = (int64_t *)calloc(nb, 8);
    double *w = (double *)calloc(nb, 8);
    int bmin, bmax;
    histogram(r, n, &bmin, &bmax);
    double W = weights(r, n, bmin, bmax, beta_prime - r->beta, w);
    double acc = 0.0;
    for (int b = bmin; b <= bmax; ++b) {
        if (n[b] == 0) continue;
        double tau = ((double)r->R * w[b]) / W;
        acc += (double)n[b] * (tau < 1.0 ? tau : 1.0);
    }
    free(n); free(w);
    return acc / (double)r->Rcur;
}

/* Adaptive temperature step (Sec. 2.3, reading R8).  Returns 0 on success,
 * -1 if no step with alpha >= alpha* exists above the current beta. */
int orc_adapt_beta(orc_run *r, double alpha_star, double beta_f, double *beta_next)
{
    if (orc_alpha(r, beta_f) >= alpha_star) {
        *beta_next = beta_f;
        return 0;
    }
    double lo = r->beta, hi = beta_f;
    for (int it = 0; it < 50; ++it) {
        double mid = lo + 0.5 * (hi - lo);
        if (orc_alpha(r, mid) >= alpha_star)
            lo = mid;
        else
            hi = mid;
    }
    if (lo == r->beta) return -1;
    *beta_next = lo;
    return 0;
}

/* Step 4: population averages (Eq. (observables)), free energy (Eq. (free
 * energy)) and entropy (Eq. (entropy)), from exact integer sums.  The
 * measurement also enters the multi-histogram accumulators (reading R9). */
void orc_measure(orc_run *r, orc_obs *o)
{
    int64_t sE = 0, sE2 = 0, sA = 0, sM2 = 0;
    unsigned __int128 sM4 = 0;
    for (int j = 0; j < r->Rcur; ++j) {
        int64_t e = r->E[j], m = r->M[j];
        int64_t am = m < 0 ? -m : m;
        sE += e;
        sE2 += e * e;
        sA += am;
        sM2 += m * m;
        unsigned __int128 m2 = (unsigned __int128)(m * m);
        sM4 += m2 * m2;
        int b = bin_of(r, r->E[j]);
        r->H[b] += 1;
        r->SA[b] += am;
        r->SM2[b] += m * m;
        r->SM4[b] += m2 * m2;
    }
    double N = (double)r->N, R = (double)r->Rcur, beta = r->beta;
    __int128 D = (__int128)r->Rcur * (__int128)sE2 - (__int128)sE * (__int128)sE;
    o->beta = beta;
    o->e = (double)sE / (R * N);
    o->C = (beta * beta * (double)D) / (N * R * R);
    o->abs_m = (double)sA / (R * N);
    o->m2 = (double)sM2 / (R * N * N);
    o->m4 = (double)sM4 / (R * N * N * N * N);
    o->betaF_per_N = -r->lnZ / N;
    o->S_per_N = beta * o->e + r->lnZ / N;
    o->lnQ = r->lnQ_last;
    o->R = r->Rcur;
    o->sumE = sE;
    o->sumE2 = sE2;
    o->sumAbsM = sA;
    o->sumM2 = sM2;
    o->sumM4_lo = (uint64_t)sM4;
    o->sumM4_hi = (uint64_t)(sM4 >> 64);
    if (r->nmeas == r->meas_cap) {
        r->meas_cap *= 2;
        r->m_beta = (double *)realloc(r->m_beta, 8 * (size_t)r->meas_cap);
        r->m_lnZ = (double *)realloc(r->m_lnZ, 8 * (size_t)r->meas_cap);
        r->m_R = (int64_t *)realloc(r->m_R, 8 * (size_t)r->meas_cap);
    }
    r->m_beta[r->nmeas] = beta;
    r->m_lnZ[r->nmeas] = r->lnZ;
    r->m_R[r->nmeas] = r->Rcur;
    r->nmeas += 1;
}

/* Multi-histogram reweighting (Sec. 2.4, Eq. (MHR)):
 *   Omega(E) = sum_i P_i(E) / sum_i R_i exp(beta_i F_i - beta_i E),
 * with beta_i F_i = -ln Z_i, then canonical averages at any beta from Omega.
 * Magnetisation moments use the per-energy averages sum A(E) / H(E). */
void orc_reweight(orc_run *r, const double *betas, int nb_beta, orc_obs *out)
{
    int nb = r->N + 1;
    double N = (double)r->N;
    double *lnOmega = (double *)malloc(8 * (size_t)nb);
    double *lw = (double *)malloc(8 * (size_t)nb);
    double *terms = (double *)malloc(8 * (size_t)(r->nmeas > 0 ? r->nmeas : 1));
    for (int b = 0; b < nb; ++b) {
        if (r->H[b] == 0) continue;
        double E = (double)energy_of_bin(r, b);
        double mx = -INFINITY;
        for (int i = 0; i < r->nmeas; ++i) {
            terms[i] = log((double)r->m_R[i]) - r->m_lnZ[i] - r->m_beta[i] * E;
            if (terms[i] > mx) mx = terms[i];
        }
        double s = 0.0;
        for (int i = 0; i < r->nmeas; ++i) s += exp(terms[i] - mx);
        lnOmega[b] = log((double)r->H[b]) - (mx + log(s));
    }
    for (int k = 0; k < nb_beta; ++k) {
        double beta = betas[k];
        double mx = -INFINITY;
        for (int b = 0; b < nb; ++b) {
            if (r->H[b] == 0) continue;
            lw[b] = lnOmega[b] - beta * (double)energy_of_bin(r, b);
            if (lw[b] > mx) mx = lw[b];
        }
        double s = 0.0;
        for (int b = 0; b < nb; ++b)
            if (r->H[b] != 0) s += exp(lw[b] - mx);
        double lnZ = mx + log(s);
        double mE = 0.0, mA = 0.0, mM2 = 0.0, mM4 = 0.0;
        for (int b = 0; b < nb; ++b) {
            if (r->H[b] == 0) continue;
            double p = exp(lw[b] - lnZ);
            double h = (double)r->H[b];
            mE += p * (double)energy_of_bin(r, b);
            mA += p * ((double)r->SA[b] / h);
            mM2 += p * ((double)r->SM2[b] / h);
            mM4 += p * ((double)r->SM4[b] / h);
        }
        double var = 0.0;
        for (int b = 0; b < nb; ++b) {
            if (r->H[b] == 0) continue;
            double p = exp(lw[b] - lnZ);
            double d = (double)energy_of_bin(r, b) - mE;
            var += p * d * d;
        }
        orc_obs *o = &out[k];
        memset(o, 0, sizeof(*o));
        o->beta = beta;
        o->e = mE / N;
        o->C = beta * beta * var / N;
        o->abs_m = mA / N;
        o->m2 = mM2 / (N * N);
        o->m4 = mM4 / (N * N * N * N);
        o->betaF_per_N = -lnZ / N;
        o->S_per_N = beta * o->e + lnZ / N;
    }
    free(lnOmega); free(lw); free(terms);
}

/* ------------------------------------------------------------------------- */
/* State access for step-wise comparisons                                     */
/* ------------------------------------------------------------------------- */
int orc_population(const orc_run *r) { return r->Rcur; }
int orc_step(const orc_run *r) { return r->step; }
uint64_t orc_sweeps(const orc_run *r) { return r->sweeps; }
double orc_beta(const orc_run *r) { return r->beta; }
double orc_lnZ(const orc_run *r) { return r->lnZ; }

void orc_get_population(const orc_run *r, int8_t *spins, int32_t *E, int32_t *M)
{
    if (spins) memcpy(spins, r->spin, (size_t)r->Rcur * r->N);
    if (E) memcpy(E, r->E, 4 * (size_t)r->Rcur);
    if (M) memcpy(M, r->M, 4 * (size_t)r->Rcur);
}

int orc_get_counts(const orc_run *r, uint32_t *counts)
{
    if (counts) memcpy(counts, r->counts, 4 * (size_t)r->counts_n);
    return r->counts_n;
}

/* Replace the population (spins given; E and M recounted from the spins) and
 * the counters that key the random streams. */
int orc_set_population(orc_run *r, int Rcur, const int8_t *spins, int step, uint64_t sweeps,
                       double beta, double lnZ)
{
    if (Rcur < 1 || Rcur > r->capacity) return -1;
    memcpy(r->spin, spins, (size_t)Rcur * r->N);
    for (int j = 0; j < Rcur; ++j) count_EM(r, spin_at(r, r->spin, j), &r->E[j], &r->M[j]);
    r->Rcur = Rcur;
    r->step = step;
    r->sweeps = sweeps;
    r->beta = beta;
    r->lnZ = lnZ;
    return 0;
}

/* Give replica j the random-stream slot slots[j] in later sweeps (NULL
 * restores slot j); lets a few sampled replicas of a large population be
 * swept alone.  Resampling clears the table. */
void orc_set_slots(orc_run *r, const int32_t *slots)
{
    free(r->slot);
    r->slot = NULL;
    if (!slots) return;
    r->slot = (int32_t *)malloc(4 * (size_t)r->capacity);
    memcpy(r->slot, slots, 4 * (size_t)r->Rcur);
}

/* The 32-bit uniforms that decide the sites of word v (sites 32 v .. 32 v + 31
 * of colour c) of replica slot j in sweep g (test hook for pins on the
 * streams of reading R3: uniformity and independence between sites). */
void orc_word_uniforms(const orc_run *r, uint64_t g, int c, int j, int v, uint32_t out[32])
{
    if (r->lcg) {
        lcg_uniforms(r, g, c, j, v, out);
        return;
    }
    uint32_t planes[16];
    sweep_planes(r, g, c, j, (uint32_t)v, planes);
    for (int b = 0; b < 32; ++b) out[b] = site_uniform(r, g, c, j, 32 * v + b, planes);
}

/* Full recount of E and M for replica j (invariant check of the incremental
 * bookkeeping in orc_sweep). */
void orc_recount(const orc_run *r, int j, int32_t *E, int32_t *M)
{
    count_EM(r, r->spin + (size_t)j * r->N, E, M);
}

/* Resampling tables for a given histogram, exposed for unit tests. */
double orc_tables(int N, int R, int Rprev, const int64_t *n, double dbeta,
                  uint32_t *base, uint32_t *thr)
{
    orc_run tmp;
    memset(&tmp, 0, sizeof(tmp));
    tmp.N = N;
    tmp.R = R;
    int nb = N + 1, bmin = nb, bmax = -1;
    for (int b = 0; b < nb; ++b)
        if (n[b]) {
            if (b < bmin) bmin = b;
            bmax = b;
        }
    double *w = (double *)calloc(nb, 8);
    double W = weights(&tmp, n, bmin, bmax, dbeta, w);
    for (int b = bmin; b <= bmax; ++b) {
        if (n[b] == 0) continue;
        double tau = ((double)R * w[b]) / W;
        double fl = floor(tau);
        base[b] = (uint32_t)fl;
        thr[b] = (uint32_t)floor(ldexp(tau - fl, 32));
    }
    int32_t Emin = 4 * bmin - 2 * N;
    double lnQ = log(W) - log((double)Rprev) - dbeta * (double)Emin;
    free(w);
    return lnQ;
}

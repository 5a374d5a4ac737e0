// Integer reductions over a population, shared by the single-run kernels
// (pa_kernels.hip) and the batched kernels (pa_batch.hip): 128-bit sums, the
// block prefix sum of the copy counts, and the two passes of the population
// statistics.
#pragma once
#include "pa_internal.h"

namespace pa {
namespace dev {

__device__ __forceinline__ void add_u128(uint64_t& lo, uint64_t& hi, uint64_t blo, uint64_t bhi)
{
    const uint64_t s = lo + blo;
    hi += bhi + (s < lo ? 1u : 0u);
    lo = s;
}

__device__ __forceinline__ void atomic_add_u128(uint64_t* lo_p, uint64_t* hi_p, uint64_t lo, uint64_t hi)
{
    const uint64_t old = atomicAdd((unsigned long long*)lo_p, (unsigned long long)lo);
    const uint64_t carry = (old + lo < old) ? 1u : 0u;
    if (hi + carry) atomicAdd((unsigned long long*)hi_p, (unsigned long long)(hi + carry));
}

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* total)
{
    __shared__ uint32_t wsum[kBlock / 64];
    const int lane = (int)(threadIdx.x & 63u), wid = (int)(threadIdx.x >> 6);
    uint32_t incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, off);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wid) before += wsum[w];
        all += wsum[w];
    }
    __syncthreads();
    *total = all;
    return before + incl - x;
}

// Parent index of every child of one wave: lane L (parent first + L) owns the
// children [off_L, off_L + c_L), and the lanes' ranges follow each other (an
// exclusive scan of the counts).  The wave takes its children 64 at a time;
// each lane finds the owner of its child by a binary search over the lanes'
// range ends, so the cost follows the wave's number of children and not its
// largest count (a parent with many copies no longer holds up the wave).
// Children at or beyond cap are not written.  Called by every lane.
__device__ __forceinline__ void fill_parents(uint32_t* __restrict__ parent, uint32_t off, uint32_t c,
                                             uint32_t first, uint32_t cap)
{
    const int lane = (int)(threadIdx.x & 63u);
    const uint32_t end = off + c;
    const uint32_t w0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)off);
    const uint32_t w1 = (uint32_t)__builtin_amdgcn_readlane((int)end, 63);
    for (uint32_t base = w0; base < w1; base += 64u) {
        const uint32_t q = base + (uint32_t)lane;
        int owner = 0;  // number of lanes whose range ends at or before q
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const uint32_t e = (uint32_t)__shfl((int)end, owner + step - 1);
            if (e <= q) owner += step;
        }
        if (q < w1 && q < cap) parent[q] = first + (uint32_t)owner;
    }
}

// Population statistics, first pass, for the replicas [i0, i0 + kBlock) of// Population statistics, first pass, for the replicas [i0, i0 + kBlock) of
// one block (i < n only): the energy histogram n(b), b = (E + 2N) / 4, and, if
// `record`, the per-energy accumulators of multi-histogram reweighting are
// added to the population's arrays; the energy range and the exact sums of E,
// E^2, |M|, M^2 (int64) and M^4 (128 bit) go to the block's partial `part`
// (summed by stats_final).  Integer arithmetic only, so the result does not
// depend on scheduling order.  Device-wide atomics to one address serialise,
// so the block first histograms its replicas in LDS over its own energy
// window and then adds one atomic per occupied bin; a window wider than the
// LDS table falls back to one atomic per distinct bin of each wave.  Called by
// every thread of the block.
constexpr int kStatsWin = 2048;  // LDS histogram bins per block
constexpr int kMhrWin = 512;     // LDS multi-histogram bins per block

__device__ __forceinline__ void stats_block(const int32_t* __restrict__ E, const int32_t* __restrict__ M, int32_t n,
                                            int32_t N, int32_t i0, uint32_t* hist, int32_t nbins, bool record,
                                            const DevMhr& mhr, StatsPart* part)
{
    __shared__ uint32_t win[kStatsWin];
    __shared__ uint64_t mwin[5][kMhrWin];  // H, sum |M|, sum M^2, sum M^4 (lo, hi)
    __shared__ uint64_t red[kBlock / 64][6];
    __shared__ int32_t red_min[kBlock / 64], red_max[kBlock / 64];
    const int lane = (int)(threadIdx.x & 63u), wid = (int)(threadIdx.x >> 6), t = (int)threadIdx.x;
    const int i = i0 + t;
    uint64_t sE = 0, sE2 = 0, sA = 0, sM2 = 0, m4lo = 0, m4hi = 0;
    int32_t emin = 0x7FFFFFFF, emax = (int32_t)0x80000000;
    int b = -1;
    if (i < n) {
        const int64_t e = E[i], m = M[i];
        const uint64_t am = (uint64_t)(m < 0 ? -m : m);
        const uint64_t m2 = am * am;
        sE = (uint64_t)e;
        sE2 = (uint64_t)(e * e);
        sA = am;
        sM2 = m2;
        m4lo = m2 * m2;
        m4hi = __umul64hi(m2, m2);
        emin = emax = (int32_t)e;
        const int bb = (int)((e + 2 * N) >> 2);
        if (bb >= 0 && bb < nbins) b = bb;
    }
    const uint64_t a1 = sA, q1 = sM2, lo1 = m4lo, hi1 = m4hi;  // this replica's |M|, M^2, M^4
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sE += __shfl_xor(sE, off);
        sE2 += __shfl_xor(sE2, off);
        sA += __shfl_xor(sA, off);
        sM2 += __shfl_xor(sM2, off);
        const uint64_t olo = __shfl_xor(m4lo, off), ohi = __shfl_xor(m4hi, off);
        add_u128(m4lo, m4hi, olo, ohi);
        emin = min(emin, __shfl_xor(emin, off));
        emax = max(emax, __shfl_xor(emax, off));
    }
    if (lane == 0) {
        red[wid][0] = sE;
        red[wid][1] = sE2;
        red[wid][2] = sA;
        red[wid][3] = sM2;
        red[wid][4] = m4lo;
        red[wid][5] = m4hi;
        red_min[wid] = emin;
        red_max[wid] = emax;
    }
    __syncthreads();
    int32_t bemin = red_min[0], bemax = red_max[0];
#pragma unroll
    for (int w = 1; w < kBlock / 64; ++w) {
        bemin = min(bemin, red_min[w]);
        bemax = max(bemax, red_max[w]);
    }
    if (t == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            sE += red[w][0];
            sE2 += red[w][1];
            sA += red[w][2];
            sM2 += red[w][3];
            add_u128(m4lo, m4hi, red[w][4], red[w][5]);
        }
        StatsPart p;
        p.sumE = sE;
        p.sumE2 = sE2;
        p.sumAbsM = sA;
        p.sumM2 = sM2;
        p.sumM4_lo = m4lo;
        p.sumM4_hi = m4hi;
        p.emin = bemin;
        p.emax = bemax;
        p.pad[0] = p.pad[1] = 0u;
        *part = p;
    }
    // the block's energy window [lb, lb + lw); bins lie inside [0, nbins)
    const int lb = max((bemin + 2 * N) >> 2, 0);
    const int lw = min((bemax + 2 * N) >> 2, nbins - 1) - lb + 1;
    if (lw <= kStatsWin) {
        for (int k = t; k < lw; k += kBlock) win[k] = 0u;
        __syncthreads();
        if (b >= 0) atomicAdd(&win[b - lb], 1u);
        __syncthreads();
        for (int k = t; k < lw; k += kBlock)
            if (win[k]) atomicAdd(&hist[lb + k], win[k]);
    } else {
        uint64_t pending = __ballot(b >= 0);
        while (pending) {
            const int leader = __builtin_ctzll(pending);
            const int bv = __builtin_amdgcn_readlane(b, leader);
            const uint64_t same = __ballot(b == bv);
            if (lane == leader) atomicAdd(&hist[bv], (uint32_t)__popcll(same));
            pending &= ~same;
        }
    }
    if (!record) return;
    if (lw <= kMhrWin) {
        for (int k = t; k < lw; k += kBlock)
            for (int c = 0; c < 5; ++c) mwin[c][k] = 0u;
        __syncthreads();
        if (b >= 0) {
            const int k = b - lb;
            atomicAdd((unsigned long long*)&mwin[0][k], 1ull);
            atomicAdd((unsigned long long*)&mwin[1][k], (unsigned long long)a1);
            atomicAdd((unsigned long long*)&mwin[2][k], (unsigned long long)q1);
            atomic_add_u128(&mwin[3][k], &mwin[4][k], lo1, hi1);
        }
        __syncthreads();
        for (int k = t; k < lw; k += kBlock) {
            if (mwin[0][k] == 0u) continue;
            const int bb = lb + k;
            atomicAdd((unsigned long long*)&mhr.H[bb], (unsigned long long)mwin[0][k]);
            atomicAdd((unsigned long long*)&mhr.SA[bb], (unsigned long long)mwin[1][k]);
            atomicAdd((unsigned long long*)&mhr.SM2[bb], (unsigned long long)mwin[2][k]);
            atomic_add_u128(&mhr.SM4[2 * bb], &mhr.SM4[2 * bb + 1], mwin[3][k], mwin[4][k]);
        }
    } else if (b >= 0) {
        atomicAdd((unsigned long long*)&mhr.H[b], 1ull);
        atomicAdd((unsigned long long*)&mhr.SA[b], (unsigned long long)a1);
        atomicAdd((unsigned long long*)&mhr.SM2[b], (unsigned long long)q1);
        atomic_add_u128(&mhr.SM4[2 * b], &mhr.SM4[2 * b + 1], lo1, hi1);
    }
}

// Sums per-thread statistics over one block of NT threads into st (energy
// range and moment sums; r_new and done are left as they are), and into the
// block's LDS copy `sh` if given.  Called by every thread of the block.
template <int NT>
__device__ __forceinline__ void stats_block_total(uint64_t sE, uint64_t sE2, uint64_t sA, uint64_t sM2,
                                                  uint64_t m4lo, uint64_t m4hi, int32_t emin, int32_t emax,
                                                  DevStats* st, DevStats* sh = nullptr)
{
    __shared__ uint64_t red[NT / 64][6];
    __shared__ int32_t red_min[NT / 64], red_max[NT / 64];
    const int lane = (int)(threadIdx.x & 63u), wid = (int)(threadIdx.x >> 6);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sE += __shfl_xor(sE, off);
        sE2 += __shfl_xor(sE2, off);
        sA += __shfl_xor(sA, off);
        sM2 += __shfl_xor(sM2, off);
        const uint64_t olo = __shfl_xor(m4lo, off), ohi = __shfl_xor(m4hi, off);
        add_u128(m4lo, m4hi, olo, ohi);
        emin = min(emin, __shfl_xor(emin, off));
        emax = max(emax, __shfl_xor(emax, off));
    }
    if (lane == 0) {
        red[wid][0] = sE;
        red[wid][1] = sE2;
        red[wid][2] = sA;
        red[wid][3] = sM2;
        red[wid][4] = m4lo;
        red[wid][5] = m4hi;
        red_min[wid] = emin;
        red_max[wid] = emax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NT / 64; ++w) {
            sE += red[w][0];
            sE2 += red[w][1];
            sA += red[w][2];
            sM2 += red[w][3];
            add_u128(m4lo, m4hi, red[w][4], red[w][5]);
            emin = min(emin, red_min[w]);
            emax = max(emax, red_max[w]);
        }
        st->emin = emin;
        st->emax = emax;
        st->sumE = sE;
        st->sumE2 = sE2;
        st->sumAbsM = sA;
        st->sumM2 = sM2;
        st->sumM4_lo = m4lo;
        st->sumM4_hi = m4hi;
        if (sh) {
            sh->emin = emin;
            sh->emax = emax;
            sh->sumE = sE;
            sh->sumE2 = sE2;
            sh->sumAbsM = sA;
            sh->sumM2 = sM2;
            sh->sumM4_lo = m4lo;
            sh->sumM4_hi = m4hi;
        }
    }
}

// Second pass, one block of kBlock threads: sums the nparts partials into st
// (energy range and moment sums; r_new is left as it is).
__device__ __forceinline__ void stats_final(const StatsPart* __restrict__ parts, int32_t nparts, DevStats* st)
{
    uint64_t sE = 0, sE2 = 0, sA = 0, sM2 = 0, m4lo = 0, m4hi = 0;
    int32_t emin = 0x7FFFFFFF, emax = (int32_t)0x80000000;
    for (int p = (int)threadIdx.x; p < nparts; p += kBlock) {
        const StatsPart q = parts[p];
        sE += q.sumE;
        sE2 += q.sumE2;
        sA += q.sumAbsM;
        sM2 += q.sumM2;
        add_u128(m4lo, m4hi, q.sumM4_lo, q.sumM4_hi);
        emin = min(emin, q.emin);
        emax = max(emax, q.emax);
    }
    stats_block_total<kBlock>(sE, sE2, sA, sM2, m4lo, m4hi, emin, emax, st);
}

}  // namespace dev
}  // namespace pa

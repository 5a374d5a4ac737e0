// Device building blocks of the sweep, shared by the single-run kernel
// (pa_sweep.hip) and the batched kernels (pa_batch.hip): Philox4x32-10,
// lattice geometry, the bit-sliced Metropolis sweep cores and the spin stores.
// The population reductions live in pa_reduce.h.
#pragma once
#include "pa_internal.h"


namespace pa {
namespace dev {

constexpr uint32_t kM0 = 0xD2511F53u;
constexpr uint32_t kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u;
constexpr uint32_t kW1 = 0xBB67AE85u;

struct U4 {
    uint32_t x, y, z, w;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64
// multiplies, xor of the high halves with the other words and the round key.
// The three-way xors are single v_bitop3 instructions (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                       uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kM0 * c0;
        const uint64_t p1 = (uint64_t)kM1 * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kW0;
        k1 += kW1;
    }
    return {c0, c1, c2, c3};
}

// The same function for counters whose words 1..3 are equal on every lane of
// the wave (only c0 differs).  In the first three rounds some products and
// xors then involve wave-uniform values only; written as plain xors with the
// uniform operands combined first, those parts compile to scalar
// instructions.  The arithmetic is that of philox10.  (The LDS path gains from
// it; the register path, with its uniform branch per bit plane, measured
// slower with it and keeps philox10.)
__device__ __forceinline__ U4 philox10u(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                        uint32_t k1)
{
    uint64_t p0, p1;
    uint32_t n0, n2;
    // first Philox round: c1, c2, c3 uniform
    p0 = (uint64_t)kM0 * c0;
    p1 = (uint64_t)kM1 * c2;
    n0 = ((uint32_t)(p1 >> 32) ^ c1) ^ k0;
    n2 = (uint32_t)(p0 >> 32) ^ (c3 ^ k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += kW0;
    k1 += kW1;
    // second Philox round: c0, c1 uniform
    p0 = (uint64_t)kM0 * c0;
    p1 = (uint64_t)kM1 * c2;
    n0 = (uint32_t)(p1 >> 32) ^ (c1 ^ k0);
    n2 = c3 ^ ((uint32_t)(p0 >> 32) ^ k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += kW0;
    k1 += kW1;
    // third Philox round: c3 uniform
    p0 = (uint64_t)kM0 * c0;
    p1 = (uint64_t)kM1 * c2;
    n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    n2 = (uint32_t)(p0 >> 32) ^ (c3 ^ k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += kW0;
    k1 += kW1;
#pragma unroll
    for (int r = 3; r < 10; ++r) {
        p0 = (uint64_t)kM0 * c0;
        p1 = (uint64_t)kM1 * c2;
        n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kW0;
        k1 += kW1;
    }
    return {c0, c1, c2, c3};
}

// The register-path sweep evaluates Philox4x32-10 on counters (c0, c1, c2, c3)
// whose words c1 (sweep and colour), c2 (replica) and c3 (stream) are the same
// for every block of a half sweep, and the same on every lane of a wave that
// holds one replica.  The first round's new word 0, hi(M1 c2) ^ c1 ^ k0, then
// depends on none of c0, and so does the second round's product of it: both
// are taken once per half sweep (PhiloxHalf) instead of per block, with plain
// operations that stay scalar when their inputs are.  philox10_h is philox10
// with those values supplied; the arithmetic is the same.
struct PhiloxHalf {
    uint32_t a0;      // round 1: hi(M1 c2) ^ c1 ^ k0
    uint32_t a1;      // round 1: lo(M1 c2)
    uint32_t p0h, p0l;  // round 2: the product M0 a0
};

__device__ __forceinline__ PhiloxHalf philox_half(uint32_t c1, uint32_t c2, uint32_t k0)
{
    const uint64_t P1 = (uint64_t)kM1 * c2;
    PhiloxHalf h;
    h.a0 = ((uint32_t)(P1 >> 32) ^ c1) ^ k0;
    h.a1 = (uint32_t)P1;
    const uint64_t P0 = (uint64_t)kM0 * h.a0;
    h.p0h = (uint32_t)(P0 >> 32);
    h.p0l = (uint32_t)P0;
    return h;
}

__device__ __forceinline__ U4 philox10_h(uint32_t c0, uint32_t c3, const PhiloxHalf& h, uint32_t k0, uint32_t k1)
{
    // round 1 (word 0 and word 1 of its output are h.a0, h.a1)
    const uint64_t P0 = (uint64_t)kM0 * c0;
    const uint32_t a2 = (uint32_t)(P0 >> 32) ^ (c3 ^ k1);
    const uint32_t a3 = (uint32_t)P0;
    k0 += kW0;
    k1 += kW1;
    // round 2 (its product M0 a0 is h.p0h, h.p0l)
    const uint64_t P1 = (uint64_t)kM1 * a2;
    uint32_t x0 = (uint32_t)(P1 >> 32) ^ (h.a1 ^ k0);
    uint32_t x1 = (uint32_t)P1;
    uint32_t x2 = a3 ^ (h.p0h ^ k1);
    uint32_t x3 = h.p0l;
    k0 += kW0;
    k1 += kW1;
    // round 3 (word 3 of its input is h.p0l)
    {
        const uint64_t p0 = (uint64_t)kM0 * x0;
        const uint64_t p1 = (uint64_t)kM1 * x2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), x1, k0);
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ (x3 ^ k1);
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = n0;
        x2 = n2;
        k0 += kW0;
        k1 += kW1;
    }
#pragma unroll
    for (int r = 3; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kM0 * x0;
        const uint64_t p1 = (uint64_t)kM1 * x2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), x1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), x3, k1);
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = n0;
        x2 = n2;
        k0 += kW0;
        k1 += kW1;
    }
    return {x0, x1, x2, x3};
}

// Philox blocks of one half sweep on the register path, counter (c0, 2g + c, j,
// c3): with one replica per wave (Half) the per-half-sweep values of
// philox_half are shared by every block, with several (replicas differ
// between lanes) each block is plain philox10, which measured a few
// instructions cheaper there.
struct HalfBlocks {
    PhiloxHalf h;
    uint32_t k0, k1;
    __device__ __forceinline__ U4 operator()(uint32_t c0, uint32_t c3) const { return philox10_h(c0, c3, h, k0, k1); }
};

struct PlainBlocks {
    uint32_t c1, c2, k0, k1;
    __device__ __forceinline__ U4 operator()(uint32_t c0, uint32_t c3) const
    {
        return philox10(c0, c1, c2, c3, k0, k1);
    }
};

__device__ __forceinline__ uint32_t pick(const U4& v, uint32_t i)
{
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// Random-stream numbers: the low 4 bits of counter word 3, whose upper bits
// hold the run number (SweepArgs::tag = 16 * run), so every (seed, run,
// stream) has streams of its own.
constexpr uint32_t kStreamSweepHigh = 0;
constexpr uint32_t kStreamResample = 1;
constexpr uint32_t kStreamInit = 2;
constexpr uint32_t kStreamSweepLow = 3;
constexpr uint32_t kStreamLcgSeed = 4;

template <int L>
struct Geo {
    static constexpr int N = L * L;
    static constexpr int HW = L / 2;                  // sites per row of one colour
    static constexpr int NW = N / 64;                 // 32-site words per colour
    static constexpr int G = NW < 64 ? NW : 64;       // lanes sharing one replica
    static constexpr int K = NW / G;                  // words per lane per colour
    static constexpr int REPW = 64 / G;               // replicas per wave
    static constexpr bool WIDE = HW >= 32;            // rows made of whole words
    static constexpr int WPR = WIDE ? HW / 32 : 1;    // words per row (wide)
    static constexpr int RL = WIDE ? K / WPR : 1;     // rows per lane (wide)
    static constexpr int RPW = WIDE ? 1 : 32 / HW;    // rows per word (narrow)
    static constexpr size_t BITS_BYTES = N / 8;       // bytes per replica, bit store
    static constexpr int RPWV = (K == 1) ? REPW : 1;  // replicas per wave
    // LDS path: a lane decides up to 8 of its K words before the words with
    // sites still tied are resolved through the wave's tie queue (QCAP entries
    // of four words each).
    static constexpr int SLOTS = (K == 1) ? 1 : (K < 8 ? K : 8);
    static constexpr int QCAP = 128;
    // LDS words of one wave on the LDS path: replica [2][NW], then the queue
    static constexpr int WAVE_LDS_WORDS = (K == 1) ? 0 : 2 * NW + 4 * QCAP;
    static constexpr int lds_words(int wpb) { return wpb * WAVE_LDS_WORDS; }
    static_assert(L % 16 == 0 && L >= 16 && L <= 256, "lattice size");
    static_assert(K >= 1 && NW % G == 0, "lane mapping");
};

// Segment masks for narrow rows (HW < 32): bit 0 / top bit of every row
// segment, and the segments of even rows inside a word.
template <int HW>
struct Seg {
    static constexpr uint32_t seg = (HW >= 32) ? 0xFFFFFFFFu : ((1u << (HW % 32)) - 1u);
    static constexpr uint32_t low()
    {
        uint32_t m = 0;
        for (int o = 0; o < 32; o += HW) m |= 1u << o;
        return m;
    }
    static constexpr uint32_t high() { return low() << (HW - 1); }
    static constexpr uint32_t even()
    {
        uint32_t m = 0;
        for (int o = 0; o < 32; o += 2 * HW) m |= seg << o;
        return m;
    }
};

// Value held by the lane `delta` positions away inside the same G-lane group.
template <int G>
__device__ __forceinline__ uint32_t from_lane(uint32_t v, int lane, int delta)
{
    const int base = lane & ~(G - 1);
    const int src = base + ((lane - base + delta + G) & (G - 1));
    return (uint32_t)__shfl((int)v, src);
}

// Neighbour words (other colour) of one own word of colour C.
struct Nb {
    uint32_t up, dn, same, side;
};

template <int L, int C>
struct Neighbours {
    using Gm = Geo<L>;
    // boundary words fetched from the adjacent lanes, one set per half sweep
    uint32_t upb[Gm::WPR], dnb[Gm::WPR];
    int lane, gl;

    __device__ __forceinline__ Neighbours(const uint32_t (&oth)[Gm::K], int lane_, int gl_) : lane(lane_), gl(gl_)
    {
        if constexpr (Gm::WIDE) {
#pragma unroll
            for (int t = 0; t < Gm::WPR; ++t) {
                upb[t] = from_lane<Gm::G>(oth[(Gm::RL - 1) * Gm::WPR + t], lane, -1);
                dnb[t] = from_lane<Gm::G>(oth[t], lane, +1);
            }
        } else {
            upb[0] = from_lane<Gm::G>(oth[0], lane, -1);
            dnb[0] = from_lane<Gm::G>(oth[0], lane, +1);
        }
    }

    __device__ __forceinline__ Nb get(const uint32_t (&oth)[Gm::K], int k) const
    {
        Nb n;
        if constexpr (Gm::WIDE) {
            const int r = k / Gm::WPR, t = k % Gm::WPR;
            const int tp = (t + Gm::WPR - 1) % Gm::WPR, tn = (t + 1) % Gm::WPR;
            const uint32_t cur = oth[k];
            n.same = cur;
            n.up = (r > 0) ? oth[k - Gm::WPR] : upb[t];
            n.dn = (r < Gm::RL - 1) ? oth[k + Gm::WPR] : dnb[t];
            // (y + C) even: horizontal neighbour at h-1, else at h+1
            const uint32_t hm1 = __builtin_amdgcn_alignbit(cur, oth[r * Gm::WPR + tp], 31);
            const uint32_t hp1 = __builtin_amdgcn_alignbit(oth[r * Gm::WPR + tn], cur, 1);
            if constexpr (Gm::RL % 2 == 0) {
                n.side = (((r + C) & 1) == 0) ? hm1 : hp1;
            } else {
                const int y = gl * Gm::RL + r;
                n.side = (((y + C) & 1) == 0) ? hm1 : hp1;
            }
        } else {
            constexpr int HW = Gm::HW;
            using S = Seg<HW>;
            const uint32_t o = oth[0];
            n.same = o;
            n.up = __builtin_amdgcn_alignbit(o, upb[0], 32 - HW);
            n.dn = __builtin_amdgcn_alignbit(dnb[0], o, HW);
            const uint32_t rotl = ((o << 1) & ~S::low()) | ((o >> (HW - 1)) & S::low());
            const uint32_t rotr = ((o >> 1) & ~S::high()) | ((o << (HW - 1)) & S::high());
            n.side = (C == 0) ? ((rotl & S::even()) | (rotr & ~S::even()))
                              : ((rotr & S::even()) | (rotl & ~S::even()));
        }
        return n;
    }
};

// One bit plane of the bit-serial comparison "uniform < threshold", high bit
// first, for the sites still tied.  k = 2 sites (cls1) compare against T_2,
// k = 4 sites against T_4; `tb` holds the two threshold bits of this plane
// (bit 1: T_2, bit 0: T_4) and is uniform, so each case is straight-line code.
//   threshold bit 1: plane bit 0 -> below (accept), plane bit 1 -> still tied
//   threshold bit 0: plane bit 1 -> above (reject), plane bit 0 -> still tied
__device__ __forceinline__ void compare_plane(uint32_t x, uint32_t tb, uint32_t cls1, uint32_t& eq, uint32_t& acc)
{
    // Every case writes its results with its own three-input operation, so the
    // compiler cannot pull a shared AND/OR out of the branches (which costs
    // extra moves on the merge paths).  Truth tables over (a, b, c) with
    // a = 0xF0, b = 0xCC, c = 0xAA.
    switch (tb) {
    case 0:
        eq = __builtin_amdgcn_bitop3_b32(eq, x, x, 0x30);  // eq & ~x
        break;
    case 3:
        acc = __builtin_amdgcn_bitop3_b32(acc, eq, x, 0xF4);  // acc | (eq & ~x)
        eq = __builtin_amdgcn_bitop3_b32(eq, x, x, 0xC0);     // eq & x
        break;
    case 2:  // T_2 bit set, T_4 bit clear
        acc |= __builtin_amdgcn_bitop3_b32(eq, cls1, x, 0x40);  // eq & cls1 & ~x
        eq = __builtin_amdgcn_bitop3_b32(eq, x, cls1, 0x90);    // eq & ~(x ^ cls1)
        break;
    default:  // T_4 bit set, T_2 bit clear
        acc |= __builtin_amdgcn_bitop3_b32(eq, cls1, x, 0x10);  // eq & ~cls1 & ~x
        eq = __builtin_amdgcn_bitop3_b32(eq, x, cls1, 0x60);    // eq & (x ^ cls1)
        break;
    }
}

// Metropolis acceptance mask of one 32-site word.  A site flips if at least two
// of its four neighbours are anti-aligned (k = s h <= 0), else if its uniform
// x (high 16 bits from the bit planes, low 16 bits drawn on a tie) is below
// the threshold of its class (one anti-aligned neighbour: k = 2; none: k = 4).
template <class BLK>
__device__ __forceinline__ uint32_t accept_mask(uint32_t w, const Nb& n, uint32_t v, const BLK& blk,
                                                const SweepArgs& a)
{
    const uint32_t d1 = w ^ n.up, d2 = w ^ n.dn, d3 = w ^ n.same, d4 = w ^ n.side;
    const uint32_t o12 = d1 | d2, a12 = d1 & d2, o34 = d3 | d4, a34 = d3 & d4;
    const uint32_t ge2 = a12 | a34 | (o12 & o34);
    const uint32_t any = o12 | o34;
    const uint32_t cls1 = any & ~ge2;  // k = 2
    uint32_t eq = ~ge2;                // sites still tied with their threshold
    uint32_t acc = ge2;
    if (__builtin_expect((a.t2h | a.t4h) > 0xFFFFu, 0)) {  // a threshold is 2^32 (beta ~ 0)
        if (a.t2h > 0xFFFFu) {  // T_2 = 2^32: always accepted
            acc |= cls1;
            eq &= ~cls1;
        }
        if (a.t4h > 0xFFFFu) {
            acc |= ~any;
            eq &= any;
        }
    }
    if (__any(eq != 0u)) {
        // blocks 0, 1 and 2 are computed together (three independent chains),
        // since the first eight planes leave some site of the wave tied almost
        // surely (the wave holds about 2000 sites that need a uniform)
        const U4 P0 = blk(4u * v, a.tag | kStreamSweepHigh);
        const U4 P1 = blk(4u * v + 1u, a.tag | kStreamSweepHigh);
        const U4 P2 = blk(4u * v + 2u, a.tag | kStreamSweepHigh);
        const uint32_t pl[12] = {P0.x, P0.y, P0.z, P0.w, P1.x, P1.y, P1.z, P1.w, P2.x, P2.y, P2.z, P2.w};
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            const int bit = 15 - q;
            const uint32_t tb = (((a.t2h >> bit) & 1u) << 1) | ((a.t4h >> bit) & 1u);
            compare_plane(pl[q], tb, cls1, eq, acc);
        }
#pragma unroll
        for (int kk = 3; kk < 4; ++kk) {
            if (!__any(eq != 0u)) break;
            const U4 P = blk(4u * v + (uint32_t)kk, a.tag | kStreamSweepHigh);
            const uint32_t pq[4] = {P.x, P.y, P.z, P.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int bit = 15 - (4 * kk + q);
                const uint32_t tb = (((a.t2h >> bit) & 1u) << 1) | ((a.t4h >> bit) & 1u);
                compare_plane(pq[q], tb, cls1, eq, acc);
            }
        }
    }
    if (__any(eq != 0u)) {
        uint32_t tie = eq;
        while (tie) {
            const int b = __builtin_ctz(tie);
            tie &= tie - 1u;
            const uint32_t q = 32u * v + (uint32_t)b;
            const U4 P = blk(q >> 3, a.tag | kStreamSweepLow);
            const uint32_t word = pick(P, (q >> 1) & 3u);
            const uint32_t lo = (q & 1u) ? (word & 0xFFFFu) : (word >> 16);
            const uint32_t tl = ((cls1 >> b) & 1u) ? a.t2l : a.t4l;
            if (lo < tl) acc |= 1u << b;
        }
    }
    return acc;
}

// Neighbour classes of the heat-bath update.  With a the number of
// anti-aligned neighbours, k = s h = 4 - 2a: neg holds the sites with k < 0
// (a >= 3), zero those with k = 0 (a = 2) and cls1 those with |k| = 2 (a = 1
// or 3); the remaining sites have |k| = 4.
struct HbClass {
    uint32_t neg, zero, cls1;
};

__device__ __forceinline__ HbClass hb_classes(uint32_t w, const Nb& n)
{
    const uint32_t d1 = w ^ n.up, d2 = w ^ n.dn, d3 = w ^ n.same, d4 = w ^ n.side;
    const uint32_t o12 = d1 | d2, a12 = d1 & d2, o34 = d3 | d4, a34 = d3 & d4;
    const uint32_t ge1 = o12 | o34;
    const uint32_t ge2 = a12 | a34 | (o12 & o34);
    const uint32_t ge3 = (a12 & o34) | (a34 & o12);
    const uint32_t all4 = a12 & a34;
    HbClass c;
    c.neg = ge3;
    c.zero = ge2 & ~ge3;
    c.cls1 = (ge1 & ~ge2) | (ge3 & ~all4);
    return c;
}

// Heat-bath flip mask of one 32-site word.  A site flips with probability
// 1 / (1 + e^{2 beta k}): iff its uniform x is below U_k, where U_2 and U_4 (at
// most 2^31) arrive in the threshold arguments, U_0 = 2^31 and
// U_{-k} = 2^32 - U_k.  For k < 0, "x < 2^32 - U_|k|" is "not (~x < U_|k|)",
// so those sites compare the complement of their uniform with U_|k| (the
// planes and the low half xored with neg) and take the opposite result.  The
// k = 0 sites are decided by the top bit of x alone.
template <class BLK>
__device__ __forceinline__ uint32_t heatbath_mask(uint32_t w, const Nb& n, uint32_t v, const BLK& blk,
                                                  const SweepArgs& a)
{
    const HbClass c = hb_classes(w, n);
    uint32_t eq = ~c.zero;
    // blocks 0, 1 and 2 together (three independent chains), as in accept_mask
    const U4 P0 = blk(4u * v, a.tag | kStreamSweepHigh);
    const U4 P1 = blk(4u * v + 1u, a.tag | kStreamSweepHigh);
    const U4 P2 = blk(4u * v + 2u, a.tag | kStreamSweepHigh);
    const uint32_t pl[12] = {P0.x, P0.y, P0.z, P0.w, P1.x, P1.y, P1.z, P1.w, P2.x, P2.y, P2.z, P2.w};
    uint32_t acc = c.zero & ~pl[0];  // U_0 = 2^31: x < U_0 iff its top bit is 0
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        const int bit = 15 - q;
        const uint32_t tb = (((a.t2h >> bit) & 1u) << 1) | ((a.t4h >> bit) & 1u);
        compare_plane(pl[q] ^ c.neg, tb, c.cls1, eq, acc);
    }
#pragma unroll
    for (int kk = 3; kk < 4; ++kk) {
        if (!__any(eq != 0u)) break;
        const U4 P = blk(4u * v + (uint32_t)kk, a.tag | kStreamSweepHigh);
        const uint32_t pq[4] = {P.x, P.y, P.z, P.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int bit = 15 - (4 * kk + q);
            const uint32_t tb = (((a.t2h >> bit) & 1u) << 1) | ((a.t4h >> bit) & 1u);
            compare_plane(pq[q] ^ c.neg, tb, c.cls1, eq, acc);
        }
    }
    if (__any(eq != 0u)) {
        uint32_t tie = eq;
        while (tie) {
            const int b = __builtin_ctz(tie);
            tie &= tie - 1u;
            const uint32_t q = 32u * v + (uint32_t)b;
            const U4 P = blk(q >> 3, a.tag | kStreamSweepLow);
            const uint32_t word = pick(P, (q >> 1) & 3u);
            uint32_t lo = (q & 1u) ? (word & 0xFFFFu) : (word >> 16);
            if ((c.neg >> b) & 1u) lo ^= 0xFFFFu;
            const uint32_t tl = ((c.cls1 >> b) & 1u) ? a.t2l : a.t4l;
            if (lo < tl) acc |= 1u << b;
        }
    }
    return acc ^ c.neg;
}

// In-line LCG variant of the multi-spin-coded sweep (Sec. 4): the generator
// r' = A r + C mod 2^32 (A = 1664525, C = 1013904223), seeded once per word
// and update by the base generator, supplies the 32 uniforms of the word.
// Site b takes the (b+1)-th output after the seed r_0, written in closed form
// as r_{b+1} = A^{b+1} r_0 + C (A^b + ... + 1) mod 2^32, so the 32 outputs
// are independent multiply-adds instead of a chain.
constexpr uint32_t kLcgA = 1664525u;
constexpr uint32_t kLcgC = 1013904223u;

constexpr uint32_t lcg_mul(int n)  // A^n mod 2^32
{
    uint32_t m = 1u;
    for (int i = 0; i < n; ++i) m *= kLcgA;
    return m;
}

constexpr uint32_t lcg_add(int n)  // C (A^{n-1} + ... + A + 1) mod 2^32
{
    uint32_t c = 0u;
    for (int i = 0; i < n; ++i) c = c * kLcgA + kLcgC;
    return c;
}

// acc = 2 acc + [x <= t]: the comparison writes a lane mask that the add
// takes as its carry-in (two VALU instructions; the compiler's own form is a
// compare, a select and a shift-or).  Arithmetic only, no memory access.
__device__ __forceinline__ uint32_t shift_in_le(uint32_t acc, uint32_t x, uint32_t t)
{
    uint64_t le, carry;
    __asm__("v_cmp_ge_u32_e64 %1, %4, %3\n\t"
            "v_addc_co_u32_e64 %0, %2, %0, %0, %1"
            : "+v"(acc), "=&s"(le), "=&s"(carry)
            : "v"(x), "s"(t));
    return acc;
}

// Metropolis acceptance mask of one 32-site word whose uniforms are the LCG
// outputs after `seed`: a site flips if k <= 0, else if its uniform x is below
// T_2 (one anti-aligned neighbour) or T_4 (none), i.e. x <= T - 1 (T >= 1).
__device__ __forceinline__ uint32_t lcg_accept_mask(uint32_t w, const Nb& n, uint32_t seed, const SweepArgs& a)
{
    const uint32_t d1 = w ^ n.up, d2 = w ^ n.dn, d3 = w ^ n.same, d4 = w ^ n.side;
    const uint32_t o12 = d1 | d2, a12 = d1 & d2, o34 = d3 | d4, a34 = d3 & d4;
    const uint32_t ge2 = a12 | a34 | (o12 & o34);
    const uint32_t any = o12 | o34;
    // T - 1 in 32 bits (T = 2^32 gives 2^32 - 1)
    const uint32_t t2m1 = (a.t2h << 16) + a.t2l - 1u;
    const uint32_t t4m1 = (a.t4h << 16) + a.t4l - 1u;
    uint32_t m2 = 0u, m4 = 0u;
#pragma unroll
    for (int b = 31; b >= 0; --b) {
        const uint32_t x = (uint32_t)((uint64_t)lcg_mul(b + 1) * seed + (uint64_t)lcg_add(b + 1));
        m2 = shift_in_le(m2, x, t2m1);
        m4 = shift_in_le(m4, x, t4m1);
    }
    return ge2 | (any & ~ge2 & m2) | (~any & m4);
}

// One colour of the LCG sweep for the lane's one word (register path).
template <int L, int C>
__device__ __forceinline__ void half_sweep_lcg(uint32_t (&own)[1], const uint32_t (&oth)[1], int lane, int gl,
                                               uint32_t seed, const SweepArgs& a)
{
    const Neighbours<L, C> nb(oth, lane, gl);
    own[0] ^= lcg_accept_mask(own[0], nb.get(oth, 0), seed, a);
}

template <int L, int C, bool HB>
__device__ __forceinline__ void half_sweep(uint32_t (&own)[Geo<L>::K], const uint32_t (&oth)[Geo<L>::K], int lane,
                                           int gl, uint32_t g, uint32_t j, const SweepArgs& a)
{
    using Gm = Geo<L>;
    const Neighbours<L, C> nb(oth, lane, gl);
    const uint32_t ctr1 = 2u * g + (uint32_t)C;
    const auto blocks = [&]() {
        if constexpr (Gm::REPW == 1)
            return HalfBlocks{philox_half(ctr1, j, a.key0), a.key0, a.key1};
        else
            return PlainBlocks{ctr1, j, a.key0, a.key1};
    }();
#pragma unroll
    for (int k = 0; k < Gm::K; ++k) {
        const uint32_t v = (uint32_t)(gl * Gm::K + k);
        if constexpr (HB)
            own[k] ^= heatbath_mask(own[k], nb.get(oth, k), v, blocks, a);
        else
            own[k] ^= accept_mask(own[k], nb.get(oth, k), v, blocks, a);
    }
}


// Decisions of the first 8 bit planes (Philox blocks 0 and 1) for NG words of
// one lane together.  A site flips if at least two of its four neighbours are
// anti-aligned (k = s h <= 0); a site with one anti-aligned neighbour (k = 2,
// `cls1`) or none (k = 4) flips if its uniform x is below T_2 or T_4.  The
// planes are compared high bit first with one uniform branch per plane over the
// two threshold bits, shared by the NG words: 2-3 operations per word and
// plane.  The words are updated with their decided flips; `tie` receives the
// sites whose 8 high bits equal the threshold's (probability 2^-8 each),
// decided later by decide_word_tail.  With HB (heat-bath, the update of
// heatbath_mask) every site draws, the k = 0 sites are decided by plane 0, the
// k < 0 sites compare the complemented planes (`ng`) and are flipped
// provisionally, so that the tail's result xored on top gives their decision.
template <int NG, bool HB>
__device__ __forceinline__ void decide8_group(uint32_t (&w)[NG], const Nb (&n)[NG], const uint32_t (&v)[NG],
                                              uint32_t ctr1, uint32_t j, const SweepArgs& a, uint32_t (&tie)[NG],
                                              uint32_t (&cls1)[NG], uint32_t (&ng)[NG])
{
    uint32_t eq[NG], acc[NG], zero[NG];
    uint32_t need = 0u;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if constexpr (HB) {
            const HbClass c = hb_classes(w[g], n[g]);
            cls1[g] = c.cls1;
            ng[g] = c.neg;
            zero[g] = c.zero;
            eq[g] = ~c.zero;
            acc[g] = 0u;
        } else {
            const uint32_t d1 = w[g] ^ n[g].up, d2 = w[g] ^ n[g].dn, d3 = w[g] ^ n[g].same, d4 = w[g] ^ n[g].side;
            const uint32_t o12 = d1 | d2, a12 = d1 & d2, o34 = d3 | d4, a34 = d3 & d4;
            const uint32_t ge2 = a12 | a34 | (o12 & o34);
            const uint32_t any = o12 | o34;
            cls1[g] = any & ~ge2;
            const uint32_t cls2 = ~any;
            const uint32_t all2 = (a.t2h > 0xFFFFu) ? cls1[g] : 0u;  // T = 2^32: always accepted
            const uint32_t all4 = (a.t4h > 0xFFFFu) ? cls2 : 0u;
            eq[g] = (cls1[g] & ~all2) | (cls2 & ~all4);
            acc[g] = ge2 | all2 | all4;
            ng[g] = 0u;
            zero[g] = 0u;
        }
        need |= eq[g];
    }
    // heat-bath draws for every site: its k = 0 sites are decided by plane 0
    // even when no site of the wave is left for the later planes
    if (HB || __any(need != 0u)) {
        uint32_t pl[NG][8];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const U4 P0 = philox10u(4u * v[g], ctr1, j, a.tag | kStreamSweepHigh, a.key0, a.key1);
            const U4 P1 = philox10u(4u * v[g] + 1u, ctr1, j, a.tag | kStreamSweepHigh, a.key0, a.key1);
            pl[g][0] = P0.x, pl[g][1] = P0.y, pl[g][2] = P0.z, pl[g][3] = P0.w;
            pl[g][4] = P1.x, pl[g][5] = P1.y, pl[g][6] = P1.z, pl[g][7] = P1.w;
            if constexpr (HB) {
                acc[g] = zero[g] & ~pl[g][0];  // U_0 = 2^31: x < U_0 iff its top bit is 0
#pragma unroll
                for (int q = 0; q < 8; ++q) pl[g][q] ^= ng[g];
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int bit = 15 - q;
            const uint32_t tb = (((a.t2h >> bit) & 1u) << 1) | ((a.t4h >> bit) & 1u);
            switch (tb) {
            case 0:
#pragma unroll
                for (int g = 0; g < NG; ++g) eq[g] = __builtin_amdgcn_bitop3_b32(eq[g], pl[g][q], pl[g][q], 0x30);
                break;
            case 3:
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    acc[g] = __builtin_amdgcn_bitop3_b32(acc[g], eq[g], pl[g][q], 0xF4);
                    eq[g] = __builtin_amdgcn_bitop3_b32(eq[g], pl[g][q], pl[g][q], 0xC0);
                }
                break;
            case 2:
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    acc[g] |= __builtin_amdgcn_bitop3_b32(eq[g], cls1[g], pl[g][q], 0x40);
                    eq[g] = __builtin_amdgcn_bitop3_b32(eq[g], pl[g][q], cls1[g], 0x90);
                }
                break;
            default:
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    acc[g] |= __builtin_amdgcn_bitop3_b32(eq[g], cls1[g], pl[g][q], 0x10);
                    eq[g] = __builtin_amdgcn_bitop3_b32(eq[g], pl[g][q], cls1[g], 0x60);
                }
                break;
            }
        }
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        w[g] ^= acc[g] ^ ng[g];
        tie[g] = eq[g];
    }
}

// Orders the LDS accesses of one wave: everything before is complete and
// visible to every lane of the wave after.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Remaining comparison of the tied sites `mask` of word v (all tied after 8
// planes): Philox block 2 (planes 8-11) once for the word, block 3 (planes
// 12-15) once if a site is still tied, then the SWEEP-LOW half of each site
// still tied.  k2m marks the sites of class k = 2, ngm those that compare the
// complement of their uniform (heat-bath, k < 0).  Returns the sites whose
// (complemented) uniform is below their threshold, each decided exactly as a
// comparison of its whole 32-bit uniform would decide it.
__device__ __forceinline__ uint32_t decide_word_tail(uint32_t v, uint32_t mask, uint32_t k2m, uint32_t ngm,
                                                     uint32_t ctr1, uint32_t j, const SweepArgs& a)
{
    uint32_t below = 0u;
#pragma unroll
    for (int kk = 2; kk < 4; ++kk) {
        if (mask == 0u) return below;
        const U4 P = philox10u(4u * v + (uint32_t)kk, ctr1, j, a.tag | kStreamSweepHigh, a.key0, a.key1);
        uint32_t rem = mask;
        while (rem) {
            const uint32_t b = (uint32_t)__builtin_ctz(rem);
            rem &= rem - 1u;
            const uint32_t th = ((k2m >> b) & 1u) ? a.t2h : a.t4h;
            const uint32_t x = ((((P.x >> b) & 1u) << 3) | (((P.y >> b) & 1u) << 2) | (((P.z >> b) & 1u) << 1) |
                                ((P.w >> b) & 1u)) ^ (((ngm >> b) & 1u) * 15u);
            const uint32_t t = (th >> (12 - 4 * kk)) & 15u;
            if (x != t) {
                mask &= ~(1u << b);
                if (x < t) below |= 1u << b;
            }
        }
    }
    while (mask) {
        const uint32_t b = (uint32_t)__builtin_ctz(mask);
        mask &= mask - 1u;
        const uint32_t q = 32u * v + b;
        const U4 P = philox10u(q >> 3, ctr1, j, a.tag | kStreamSweepLow, a.key0, a.key1);
        const uint32_t word = pick(P, (q >> 1) & 3u);
        const uint32_t lo = ((q & 1u) ? (word & 0xFFFFu) : (word >> 16)) ^ (((ngm >> b) & 1u) * 0xFFFFu);
        if (lo < (((k2m >> b) & 1u) ? a.t2l : a.t4l)) below |= 1u << b;
    }
    return below;
}

// Tie queue of one wave.  The sites still tied after decide8_group are rare
// (2^-8 each), so instead of evaluating the later Philox blocks for every
// word, every word of the lanes' S words that holds a tied site is queued in
// LDS and decided by one lane, which evaluates the later blocks once for all
// of the word's tied sites.  Entry i of the queue is four words:
//   queue[i]            lane | slot << 6   (slot: which of the lane's S words)
//   queue[Q + i]        the word's tied sites
//   queue[2 Q + i]      the tied sites of class k = 2
//   queue[3 Q + i]      the tied sites that compare the complement of their
//                       uniform (heat-bath, k < 0)
// with Q = QCAP.  Each slot's entries are placed by a wave vote: the lanes with
// a tie in that slot take consecutive entries in lane order.
//
// vj(lane, slot, &v, &j) gives the word and replica of a lane's slot, and
// word(lane, slot) the LDS address of that word, into which the resolving lane
// xors the additional flips (each word is in one entry, so no two lanes touch
// the same word).  If the queue would hold more than min(a.qcap, QCAP)
// entries, every lane decides its own tied sites instead and extra[s] receives
// its additional flips (zero otherwise).
template <int S, int QCAP, class VJ, class WORD>
__device__ __forceinline__ void resolve_ties_wave(const uint32_t (&tie)[S], const uint32_t (&cls1)[S],
                                                  const uint32_t (&ng)[S], int lane, uint32_t ctr1, const SweepArgs& a,
                                                  uint32_t* queue, uint32_t (&extra)[S], const VJ& vj, const WORD& word)
{
    const uint32_t cap = min(a.qcap, (uint32_t)QCAP);
    uint64_t vote[S];
    uint32_t total = 0u;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        extra[s] = 0u;
        vote[s] = __ballot(tie[s] != 0u);
        total += (uint32_t)__popcll(vote[s]);
    }
    if (total == 0u) return;
    if (total > cap) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (tie[s] == 0u) continue;
            uint32_t v, j;
            vj(lane, s, &v, &j);
            extra[s] = decide_word_tail(v, tie[s], cls1[s] & tie[s], ng[s] & tie[s], ctr1, j, a);
        }
        return;
    }
    uint32_t base = 0u;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        if (tie[s] != 0u) {
            const uint32_t lo = (uint32_t)vote[s], hi = (uint32_t)(vote[s] >> 32);
            const uint32_t i = base + __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
            queue[i] = (uint32_t)lane | ((uint32_t)s << 6);
            queue[QCAP + i] = tie[s];
            queue[2 * QCAP + i] = cls1[s] & tie[s];
            queue[3 * QCAP + i] = ng[s] & tie[s];
        }
        base += (uint32_t)__popcll(vote[s]);
    }
    wave_lds_sync();
    for (uint32_t i = (uint32_t)lane; i < total; i += 64u) {
        const uint32_t e = queue[i];
        const int owner = (int)(e & 63u), s = (int)(e >> 6);
        uint32_t v, j;
        vj(owner, s, &v, &j);
        const uint32_t f = decide_word_tail(v, queue[QCAP + i], queue[2 * QCAP + i], queue[3 * QCAP + i], ctr1, j, a);
        if (f) atomicXor(word(owner, s), f);
    }
    wave_lds_sync();
}

// Sign bits of 64 consecutive int8 spins -> (even-x bits, odd-x bits).
__device__ __forceinline__ void pack64(const uint4* src, uint32_t& ev, uint32_t& od)
{
    ev = 0;
    od = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint4 q = src[i];
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int p = 2 * (4 * i + k);
            ev |= ((w[k] >> 7) & 1u) << p;
            ev |= ((w[k] >> 23) & 1u) << (p + 1);
            od |= ((w[k] >> 15) & 1u) << p;
            od |= ((w[k] >> 31) & 1u) << (p + 1);
        }
    }
}

__device__ __forceinline__ void unpack64(uint32_t ev, uint32_t od, uint4* dst)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int p = 2 * (4 * i + k);
            const uint32_t m = ((ev >> p) & 1u) * 0xFEu | ((od >> p) & 1u) * 0xFE00u |
                               ((ev >> (p + 1)) & 1u) * 0xFE0000u | ((od >> (p + 1)) & 1u) * 0xFE000000u;
            w[k] = 0x01010101u | m;
        }
        dst[i] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// Row-parity blend between the even-x / odd-x bits of a 64-site chunk and the
// two colour words: colour 0 holds the even-x sites of even rows.
template <int L>
__device__ __forceinline__ uint32_t even_row_mask(uint32_t v)
{
    using Gm = Geo<L>;
    if constexpr (Gm::WIDE) {
        return (((v / Gm::WPR) & 1u) == 0u) ? 0xFFFFFFFFu : 0u;
    } else {
        return Seg<Gm::HW>::even();
    }
}

// Replica identity of a lane: group of G lanes per replica inside the wave.
struct LaneInfo {
    int lane, gl;
    uint32_t j;
    bool valid;
};

// Initial-state word (stream INIT): the INIT output word p >> 5 with
// p = c N/2 + q is exactly the 32-site word (c, v) of the bit store.
template <int L>
__device__ __forceinline__ uint32_t init_word(int c, uint32_t v, uint32_t j, const SweepArgs& a)
{
    const uint32_t idx = (uint32_t)(c * Geo<L>::NW) + v;
    return pick(philox10(idx >> 2, 0u, j, a.tag | kStreamInit, a.key0, a.key1), idx & 3u);
}

// Bytes of one replica in the spin store.
template <int L, bool INT8>
constexpr size_t replica_bytes()
{
    return INT8 ? (size_t)Geo<L>::N : Geo<L>::BITS_BYTES;
}

// The stored replica a sweep starts from for slot j: slot j of the store, or,
// when the sweep follows a resampling (a.parent set), replica parent[j] of the
// parent store, so that the copy of the resampling and the load of the sweep
// are one pass.
template <int L, bool INT8>
__device__ __forceinline__ const uint8_t* replica_in(const SweepArgs& a, uint32_t j)
{
    if (a.parent) return a.src + (size_t)a.parent[j] * replica_bytes<L, INT8>();
    return a.spin + (size_t)j * replica_bytes<L, INT8>();
}

// Load the colour-0 / colour-1 words of word index v of the replica at rep.
template <int L, bool INT8>
__device__ __forceinline__ void load_word(const uint8_t* rep, uint32_t v, uint32_t& w0, uint32_t& w1)
{
    using Gm = Geo<L>;
    if constexpr (INT8) {
        const uint4* base = reinterpret_cast<const uint4*>(rep);
        uint32_t ev, od;
        pack64(base + 4 * v, ev, od);
        const uint32_t em = even_row_mask<L>(v);
        w0 = (ev & em) | (od & ~em);
        w1 = (od & em) | (ev & ~em);
    } else {
        const uint32_t* base = reinterpret_cast<const uint32_t*>(rep);
        w0 = base[v];
        w1 = base[Gm::NW + v];
    }
}

template <int L, bool INT8>
__device__ __forceinline__ void store_word(const SweepArgs& a, uint32_t j, uint32_t v, uint32_t w0, uint32_t w1)
{
    using Gm = Geo<L>;
    if constexpr (INT8) {
        uint4* base = reinterpret_cast<uint4*>(a.spin + (size_t)j * Gm::N);
        const uint32_t em = even_row_mask<L>(v);
        unpack64((w0 & em) | (w1 & ~em), (w1 & em) | (w0 & ~em), base + 4 * v);
    } else {
        uint32_t* base = reinterpret_cast<uint32_t*>(a.spin + (size_t)j * Gm::BITS_BYTES);
        base[v] = w0;
        base[Gm::NW + v] = w1;
    }
}

// Epilogue of a sweep launched with a.acc: the wave's replicas (E, M on the
// first lane of each valid group) are added to the population statistics,
// slot and histogram copy chosen by the wave's index.  The moment sums are
// summed over the wave first, so one lane issues one atomic per quantity; the
// energies go to the histogram copy with one atomic per distinct bin of the
// wave.  Integer sums, so the result does not depend on the order in which
// waves finish.  Called by every lane of the wave.
template <int L>
__device__ __forceinline__ void accumulate_stats(const SweepArgs& a, const LaneInfo& li, int32_t e, int32_t m)
{
    using Gm = Geo<L>;
    const bool lead = li.valid && li.gl == 0;
    uint64_t sE = 0, sE2 = 0, sA = 0, sM2 = 0, q_lo = 0, q_hi = 0;
    int32_t emin = 0x7FFFFFFF, emax = (int32_t)0x80000000;
    int b = 0;
    if (lead) {
        const int64_t e64 = e;
        const uint64_t am = (uint64_t)(m < 0 ? -(int64_t)m : (int64_t)m);
        const uint64_t m2 = am * am;                 // <= 2^32
        const uint64_t p_lo = m2 * m2, p_hi = __umul64hi(m2, m2);  // M^4 <= 2^64
        sE = (uint64_t)e64;
        sE2 = (uint64_t)(e64 * e64);
        sA = am;
        sM2 = m2;
        q_lo = p_lo & 0xFFFFFFFFull;
        q_hi = (p_lo >> 32) | (p_hi << 32);
        emin = emax = e;
        b = (e + 2 * Gm::N) >> 2;  // in [0, N] for |E| <= 2N
    }
    if constexpr (Gm::REPW > 1) {
#pragma unroll
        for (int off = 32; off >= Gm::G; off >>= 1) {
            sE += __shfl_xor(sE, off);
            sE2 += __shfl_xor(sE2, off);
            sA += __shfl_xor(sA, off);
            sM2 += __shfl_xor(sM2, off);
            q_lo += __shfl_xor(q_lo, off);
            q_hi += __shfl_xor(q_hi, off);
            emin = min(emin, __shfl_xor(emin, off));
            emax = max(emax, __shfl_xor(emax, off));
        }
    }
    const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int)(li.j / (uint32_t)Gm::REPW));
    if (li.lane == 0 && __builtin_amdgcn_readfirstlane((int)(emin <= emax))) {
        AccSlot* s = a.acc + (w % (uint32_t)kAccSlots);
        atomicAdd((unsigned long long*)&s->sumE, (unsigned long long)sE);
        atomicAdd((unsigned long long*)&s->sumE2, (unsigned long long)sE2);
        atomicAdd((unsigned long long*)&s->sumAbsM, (unsigned long long)sA);
        atomicAdd((unsigned long long*)&s->sumM2, (unsigned long long)sM2);
        atomicAdd((unsigned long long*)&s->m4lo, (unsigned long long)q_lo);
        atomicAdd((unsigned long long*)&s->m4hi, (unsigned long long)q_hi);
        atomicMin(&s->emin, emin);
        atomicMax(&s->emax, emax);
    }
    uint32_t* h = a.acc_hist + (size_t)(w % (uint32_t)kAccHists) * (size_t)a.nbins;
    if constexpr (Gm::REPW == 1) {
        if (li.lane == 0 && lead) atomicAdd(&h[b], 1u);
    } else {
        uint64_t pending = __ballot(lead);
        while (pending) {
            const int leader = __builtin_ctzll(pending);
            const int bv = __builtin_amdgcn_readlane(b, leader);
            const uint64_t same = __ballot(lead && b == bv);
            if (li.lane == leader) atomicAdd(&h[bv], (uint32_t)__popcll(same));
            pending &= ~same;
        }
    }
}

// E = 2 (anti-aligned bonds) - 2N and M = N - 2 (down spins), written by the
// first lane of the replica's group; with a.acc the epilogue above follows.
template <int L>
__device__ __forceinline__ void write_EM(const SweepArgs& a, const LaneInfo& li, uint32_t anti, uint32_t downs)
{
    using Gm = Geo<L>;
#pragma unroll
    for (int off = Gm::G / 2; off >= 1; off >>= 1) {
        anti += (uint32_t)__shfl_xor((int)anti, off);
        downs += (uint32_t)__shfl_xor((int)downs, off);
    }
    const int32_t e = 2 * (int32_t)anti - 2 * Gm::N, m = Gm::N - 2 * (int32_t)downs;
    if (li.valid && li.gl == 0) {
        a.E[li.j] = e;
        a.M[li.j] = m;
    }
    if (a.acc) accumulate_stats<L>(a, li, e, m);
}

// Register-resident sweep: each lane owns one word per colour (L <= 64).
// LCG: the in-line LCG variant; the word's seeds for both colours of a sweep
// come from one Philox block (outputs x and y).
template <int L, bool INT8, bool HB, bool LCG>
__device__ __forceinline__ void sweep_regs(const SweepArgs& a, const LaneInfo& li)
{
    using Gm = Geo<L>;
    static_assert(Gm::K == 1, "one word per lane");
    const uint32_t v = (uint32_t)li.gl;
    uint32_t s0[1], s1[1];
    if (a.init) {
        s0[0] = init_word<L>(0, v, li.j, a);
        s1[0] = init_word<L>(1, v, li.j, a);
    } else if (li.valid) {
        load_word<L, INT8>(replica_in<L, INT8>(a, li.j), v, s0[0], s1[0]);
    } else {
        s0[0] = s1[0] = 0u;
    }
    for (int t = 0; t < a.nsweeps; ++t) {
        const uint32_t g = a.g0 + (uint32_t)t;
        if constexpr (LCG) {
            const U4 P = philox10(v, g, li.j, a.tag | kStreamLcgSeed, a.key0, a.key1);
            half_sweep_lcg<L, 0>(s0, s1, li.lane, li.gl, P.x, a);
            half_sweep_lcg<L, 1>(s1, s0, li.lane, li.gl, P.y, a);
        } else {
            half_sweep<L, 0, HB>(s0, s1, li.lane, li.gl, g, li.j, a);
            half_sweep<L, 1, HB>(s1, s0, li.lane, li.gl, g, li.j, a);
        }
    }
    const Neighbours<L, 0> nb(s1, li.lane, li.gl);
    const Nb n = nb.get(s1, 0);
    const uint32_t anti = __popc(s0[0] ^ n.up) + __popc(s0[0] ^ n.dn) + __popc(s0[0] ^ n.same) + __popc(s0[0] ^ n.side);
    const uint32_t downs = __popc(s0[0]) + __popc(s1[0]);
    write_EM<L>(a, li, anti, downs);
    if (li.valid) store_word<L, INT8>(a, li.j, v, s0[0], s1[0]);
}


// LDS-resident sweep for rows of whole words (L >= 128): one wave owns one
// replica; word (k, lane) of a colour sits at k * 64 + lane, so the 64 lanes
// touch 64 consecutive words for every k.
template <int L>
struct LdsRep {
    using Gm = Geo<L>;
    static constexpr int K = Gm::K, WPR = Gm::WPR, RL = Gm::RL;
    uint32_t* w;  // [2][NW]
    __device__ __forceinline__ uint32_t& at(int c, int k, int gl) const { return w[c * Gm::NW + k * 64 + gl]; }
    // neighbour words (other colour 1 - C) of own word k of lane gl
    template <int C>
    __device__ __forceinline__ Nb nb(int k, int gl) const
    {
        constexpr int O = 1 - C;
        const int r = k / WPR, t = k - (k / WPR) * WPR;
        Nb n;
        n.same = at(O, k, gl);
        n.up = (r > 0) ? at(O, k - WPR, gl) : at(O, (RL - 1) * WPR + t, (gl + 63) & 63);
        n.dn = (r < RL - 1) ? at(O, k + WPR, gl) : at(O, t, (gl + 1) & 63);
        if (((r + C) & 1) == 0) {  // RL is even: row parity is the parity of r
            const int tp = (t == 0) ? WPR - 1 : t - 1;
            n.side = __builtin_amdgcn_alignbit(n.same, at(O, r * WPR + tp, gl), 31);
        } else {
            const int tn = (t == WPR - 1) ? 0 : t + 1;
            n.side = __builtin_amdgcn_alignbit(at(O, r * WPR + tn, gl), n.same, 1);
        }
        return n;
    }
};

// One colour of a sweep on the LDS path: the lane's K words in chunks of
// SLOTS, each chunk followed by the wave's tie resolution.
template <int L, int C, bool HB>
__device__ __forceinline__ void half_sweep_lds(const LdsRep<L>& rep, int gl, uint32_t g, uint32_t j,
                                               const SweepArgs& a, uint32_t* queue)
{
    using Gm = Geo<L>;
    constexpr int S = Gm::SLOTS;
    static_assert(Gm::K % S == 0, "slots divide the words of a lane");
    const uint32_t ctr1 = 2u * g + (uint32_t)C;
#pragma unroll 1
    for (int k0 = 0; k0 < Gm::K; k0 += S) {
        uint32_t tie[S], k2[S], ng[S], extra[S];
        // groups of four words share the per-plane branches of decide8_group
        // (L = 128: one group, L = 256: two)
        constexpr int NG = 4;
        static_assert(S % NG == 0, "slot groups");
#pragma unroll
        for (int s0 = 0; s0 < S; s0 += NG) {
            uint32_t w[NG], v[NG], tg[NG], cg[NG], ngg[NG];
            Nb n[NG];
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int k = k0 + s0 + g;
                n[g] = rep.template nb<C>(k, gl);
                w[g] = rep.at(C, k, gl);
                v[g] = (uint32_t)(gl * Gm::K + k);
            }
            decide8_group<NG, HB>(w, n, v, ctr1, j, a, tg, cg, ngg);
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                rep.at(C, k0 + s0 + g, gl) = w[g];
                tie[s0 + g] = tg[g];
                k2[s0 + g] = cg[g];
                ng[s0 + g] = ngg[g];
            }
        }
        const auto vj = [&](int owner, int s, uint32_t* vo, uint32_t* jo) {
            *vo = (uint32_t)(owner * Gm::K + k0 + s);
            *jo = j;
        };
        const auto word = [&](int owner, int s) { return &rep.at(C, k0 + s, owner); };
        resolve_ties_wave<S, Gm::QCAP>(tie, k2, ng, gl, ctr1, a, queue, extra, vj, word);
#pragma unroll
        for (int s = 0; s < S; ++s)
            if (extra[s]) rep.at(C, k0 + s, gl) ^= extra[s];
    }
    wave_lds_sync();
}

// One colour of an LCG sweep on the LDS path: every word of the lane in turn,
// its seed from the word's Philox block of this sweep (x: colour 0, y:
// colour 1).  The uniforms are whole 32-bit numbers, so there are no ties.
template <int L, int C>
__device__ __forceinline__ void half_sweep_lds_lcg(const LdsRep<L>& rep, int gl, uint32_t g, uint32_t j,
                                                   const SweepArgs& a)
{
    using Gm = Geo<L>;
#pragma unroll 1
    for (int k = 0; k < Gm::K; ++k) {
        const Nb n = rep.template nb<C>(k, gl);
        const uint32_t w = rep.at(C, k, gl);
        const U4 P = philox10u((uint32_t)(gl * Gm::K + k), g, j, a.tag | kStreamLcgSeed, a.key0, a.key1);
        rep.at(C, k, gl) = w ^ lcg_accept_mask(w, n, C == 0 ? P.x : P.y, a);
    }
    wave_lds_sync();
}

// The wave's LDS: replica [2][NW], then the tie queue and the slot results.
template <int L, bool INT8, bool HB, bool LCG>
__device__ __forceinline__ void sweep_lds(const SweepArgs& a, uint32_t j, uint32_t* lds)
{
    using Gm = Geo<L>;
    static_assert(Gm::WIDE && Gm::RL % 2 == 0 && Gm::G == 64, "LDS path layout");
    const LdsRep<L> rep{lds};
    uint32_t* queue = lds + 2 * Gm::NW;
    const int gl = (int)(threadIdx.x & 63u);
    const uint8_t* in = a.init ? nullptr : replica_in<L, INT8>(a, j);
#pragma unroll 1
    for (int k = 0; k < Gm::K; ++k) {
        const uint32_t v = (uint32_t)(gl * Gm::K + k);
        uint32_t w0, w1;
        if (a.init) {
            w0 = init_word<L>(0, v, j, a);
            w1 = init_word<L>(1, v, j, a);
        } else {
            load_word<L, INT8>(in, v, w0, w1);
        }
        rep.at(0, k, gl) = w0;
        rep.at(1, k, gl) = w1;
    }
    wave_lds_sync();
    for (int t = 0; t < a.nsweeps; ++t) {
        const uint32_t g = a.g0 + (uint32_t)t;
        if constexpr (LCG) {
            half_sweep_lds_lcg<L, 0>(rep, gl, g, j, a);
            half_sweep_lds_lcg<L, 1>(rep, gl, g, j, a);
        } else {
            half_sweep_lds<L, 0, HB>(rep, gl, g, j, a, queue);
            half_sweep_lds<L, 1, HB>(rep, gl, g, j, a, queue);
        }
    }
    uint32_t anti = 0, downs = 0;
#pragma unroll 1
    for (int k = 0; k < Gm::K; ++k) {
        const Nb n = rep.template nb<0>(k, gl);
        const uint32_t w0 = rep.at(0, k, gl), w1 = rep.at(1, k, gl);
        anti += __popc(w0 ^ n.up) + __popc(w0 ^ n.dn) + __popc(w0 ^ n.same) + __popc(w0 ^ n.side);
        downs += __popc(w0) + __popc(w1);
        store_word<L, INT8>(a, j, (uint32_t)(gl * Gm::K + k), w0, w1);
    }
    LaneInfo li;
    li.lane = gl;
    li.gl = gl;
    li.j = j;
    li.valid = true;
    write_EM<L>(a, li, anti, downs);
}

// Minimum waves per SIMD the sweep kernels are compiled for.  At L = 128 the
// grouped decision needs a few more registers than fit three waves per SIMD;
// holding the kernel to three (a few values go to scratch outside the inner
// loops) is faster than two waves without the cap.
template <int L>
constexpr int sweep_min_waves()
{
    return L == 128 ? 3 : 1;
}

// Threads per block of the single-run sweep kernel.
template <int L>
constexpr int sweep_block()
{
    return Geo<L>::K == 1 ? kBlock : 64;
}

// Sweep entry shared by the single-run and batched kernels, for the block
// holding waves [wave0, wave0 + wpb) of a run (wpb = blockDim.x / 64); lds is
// the block's Geo<L>::lds_words(wpb) words (none on the register path).
// Waves share no barrier: each returns as soon as it holds no replica.  HB
// selects the heat-bath update instead of Metropolis; LCG the in-line LCG
// variant of the Metropolis sweep.
template <int L, bool INT8, bool HB, bool LCG = false>
__device__ __forceinline__ void sweep_waves(const SweepArgs& a, int wave0, int wpb, uint32_t* lds)
{
    using Gm = Geo<L>;
    const int lane = (int)(threadIdx.x & 63u), wib = (int)(threadIdx.x >> 6);
    const int wave = wave0 + wib;
    if (wave * Gm::RPWV >= a.n_rep) return;  // uniform per wave
    if constexpr (Gm::K == 1) {
        LaneInfo li;
        li.lane = lane;
        li.gl = lane % Gm::G;
        int jj = wave * Gm::REPW + lane / Gm::G;
        if constexpr (Gm::REPW == 1) jj = __builtin_amdgcn_readfirstlane(jj);
        li.j = (uint32_t)jj;
        li.valid = jj < a.n_rep;
        sweep_regs<L, INT8, HB, LCG>(a, li);
    } else {
        sweep_lds<L, INT8, HB, LCG>(a, (uint32_t)__builtin_amdgcn_readfirstlane(wave),
                                    lds + wib * Gm::WAVE_LDS_WORDS);
    }
}

}  // namespace dev
}  // namespace pa

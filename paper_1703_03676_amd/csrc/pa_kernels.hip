// Device kernels of the population-annealing hot path for gfx950 (CDNA4).
//
//   sweep_kernel   checkerboard Metropolis sweeps (Sec. 3 spin updates), also
//                  draws the initial state (Sec. 2.1 step 1) and recounts E, M
//   stats_kernel   energy histogram, energy range and exact moment sums
//                  (inputs of Eq. (Q), Eq. (observables), multi-histogram)
//   counts_kernel  integer copy counts, Eq. (resampling factors)
//   scan / scatter prefix sum of the counts -> parent index of every child
//   copy_kernel    replica copy into the other half of the ping-pong store
//
// Spin representation inside the sweep: each colour of a replica is a set of
// 32-site words (canonical within-colour index q = (y L + x) >> 1, bit q & 31
// of word q >> 5; bit set = spin -1).  A wave owns whole replicas and keeps
// them in VGPRs for all requested sweeps; vertical neighbours cross lanes by
// shuffle, horizontal neighbours are funnel shifts.  The Metropolis decision
// for all 32 sites of a word is bit-sliced: the uniform of each site is
// compared to the integer threshold one bit plane at a time (16 planes from
// four Philox blocks, high bit first), and the planes stop as soon as no site
// in the wave is still undecided.
#include "pa_internal.h"

namespace pa {
namespace {

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

__device__ __forceinline__ uint32_t pick(const U4& v, uint32_t i)
{
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// Random-stream tags (counter word 3).
constexpr uint32_t kStreamSweepHigh = 0;
constexpr uint32_t kStreamResample = 1;
constexpr uint32_t kStreamInit = 2;
constexpr uint32_t kStreamSweepLow = 3;

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
    switch (tb) {
    case 0:
        eq &= ~x;
        break;
    case 3:
        acc |= eq & ~x;
        eq &= x;
        break;
    case 2:  // T_2 bit set, T_4 bit clear
        acc |= eq & cls1 & ~x;
        eq &= ~(x ^ cls1);
        break;
    default:  // T_4 bit set, T_2 bit clear
        acc |= eq & ~cls1 & ~x;
        eq &= x ^ cls1;
        break;
    }
}

// Metropolis acceptance mask of one 32-site word.  A site flips if at least two
// of its four neighbours are anti-aligned (k = s h <= 0), else if its uniform
// x (high 16 bits from the bit planes, low 16 bits drawn on a tie) is below
// the threshold of its class (one anti-aligned neighbour: k = 2; none: k = 4).
__device__ __forceinline__ uint32_t accept_mask(uint32_t w, const Nb& n, uint32_t v, uint32_t ctr1, uint32_t j,
                                                const SweepArgs& a)
{
    const uint32_t d1 = w ^ n.up, d2 = w ^ n.dn, d3 = w ^ n.same, d4 = w ^ n.side;
    const uint32_t o12 = d1 | d2, a12 = d1 & d2, o34 = d3 | d4, a34 = d3 & d4;
    const uint32_t ge2 = a12 | a34 | (o12 & o34);
    const uint32_t any = o12 | o34;
    const uint32_t cls1 = any & ~ge2;  // k = 2
    uint32_t eq = ~ge2;                // sites still tied with their threshold
    uint32_t acc = ge2;
    if (a.t2h > 0xFFFFu) {             // T_2 = 2^32: always accepted
        acc |= cls1;
        eq &= ~cls1;
    }
    if (a.t4h > 0xFFFFu) {
        acc |= ~any;
        eq &= any;
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        if (!__any(eq != 0u)) break;
        const U4 P = philox10(4u * v + (uint32_t)kk, ctr1, j, kStreamSweepHigh, a.key0, a.key1);
        const uint32_t pl[4] = {P.x, P.y, P.z, P.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int bit = 15 - (4 * kk + q);
            const uint32_t tb = (((a.t2h >> bit) & 1u) << 1) | ((a.t4h >> bit) & 1u);
            compare_plane(pl[q], tb, cls1, eq, acc);
        }
    }
    if (__any(eq != 0u)) {
        uint32_t tie = eq;
        while (tie) {
            const int b = __builtin_ctz(tie);
            tie &= tie - 1u;
            const uint32_t q = 32u * v + (uint32_t)b;
            const U4 P = philox10(q >> 3, ctr1, j, kStreamSweepLow, a.key0, a.key1);
            const uint32_t word = pick(P, (q >> 1) & 3u);
            const uint32_t lo = (q & 1u) ? (word & 0xFFFFu) : (word >> 16);
            const uint32_t tl = ((cls1 >> b) & 1u) ? a.t2l : a.t4l;
            if (lo < tl) acc |= 1u << b;
        }
    }
    return acc;
}

template <int L, int C>
__device__ __forceinline__ void half_sweep(uint32_t (&own)[Geo<L>::K], const uint32_t (&oth)[Geo<L>::K], int lane,
                                           int gl, uint32_t g, uint32_t j, const SweepArgs& a)
{
    using Gm = Geo<L>;
    const Neighbours<L, C> nb(oth, lane, gl);
    const uint32_t ctr1 = 2u * g + (uint32_t)C;
#pragma unroll
    for (int k = 0; k < Gm::K; ++k) {
        const uint32_t v = (uint32_t)(gl * Gm::K + k);
        own[k] ^= accept_mask(own[k], nb.get(oth, k), v, ctr1, j, a);
    }
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
    return pick(philox10(idx >> 2, 0u, j, kStreamInit, a.key0, a.key1), idx & 3u);
}

// Load the colour-0 / colour-1 words of word index v of replica j.
template <int L, bool INT8>
__device__ __forceinline__ void load_word(const SweepArgs& a, uint32_t j, uint32_t v, uint32_t& w0, uint32_t& w1)
{
    using Gm = Geo<L>;
    if constexpr (INT8) {
        const uint4* base = reinterpret_cast<const uint4*>(a.spin + (size_t)j * Gm::N);
        uint32_t ev, od;
        pack64(base + 4 * v, ev, od);
        const uint32_t em = even_row_mask<L>(v);
        w0 = (ev & em) | (od & ~em);
        w1 = (od & em) | (ev & ~em);
    } else {
        const uint32_t* base = reinterpret_cast<const uint32_t*>(a.spin + (size_t)j * Gm::BITS_BYTES);
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

// E = 2 (anti-aligned bonds) - 2N and M = N - 2 (down spins), written by the
// first lane of the replica's group.
template <int L>
__device__ __forceinline__ void write_EM(const SweepArgs& a, const LaneInfo& li, uint32_t anti, uint32_t downs)
{
    using Gm = Geo<L>;
#pragma unroll
    for (int off = Gm::G / 2; off >= 1; off >>= 1) {
        anti += (uint32_t)__shfl_xor((int)anti, off);
        downs += (uint32_t)__shfl_xor((int)downs, off);
    }
    if (li.valid && li.gl == 0) {
        a.E[li.j] = 2 * (int32_t)anti - 2 * Gm::N;
        a.M[li.j] = Gm::N - 2 * (int32_t)downs;
    }
}

// Register-resident sweep: each lane owns one word per colour (L <= 64).
template <int L, bool INT8>
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
        load_word<L, INT8>(a, li.j, v, s0[0], s1[0]);
    } else {
        s0[0] = s1[0] = 0u;
    }
    for (int t = 0; t < a.nsweeps; ++t) {
        const uint32_t g = a.g0 + (uint32_t)t;
        half_sweep<L, 0>(s0, s1, li.lane, li.gl, g, li.j, a);
        half_sweep<L, 1>(s1, s0, li.lane, li.gl, g, li.j, a);
    }
    const Neighbours<L, 0> nb(s1, li.lane, li.gl);
    const Nb n = nb.get(s1, 0);
    const uint32_t anti = __popc(s0[0] ^ n.up) + __popc(s0[0] ^ n.dn) + __popc(s0[0] ^ n.same) + __popc(s0[0] ^ n.side);
    const uint32_t downs = __popc(s0[0]) + __popc(s1[0]);
    write_EM<L>(a, li, anti, downs);
    if (li.valid) store_word<L, INT8>(a, li.j, v, s0[0], s1[0]);
}

// LDS-resident sweep for rows of whole words (L >= 128): one wave per block
// owns one replica; word (k, lane) of a colour sits at k * 64 + lane, so the
// 64 lanes touch 64 consecutive words for every k.
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

template <int L, bool INT8, int C>
__device__ __forceinline__ void half_sweep_lds(const LdsRep<L>& rep, int gl, uint32_t g, uint32_t j, const SweepArgs& a)
{
    const uint32_t ctr1 = 2u * g + (uint32_t)C;
#pragma unroll 1
    for (int k = 0; k < Geo<L>::K; ++k) {
        const uint32_t v = (uint32_t)(gl * Geo<L>::K + k);
        const Nb n = rep.template nb<C>(k, gl);
        uint32_t& own = rep.at(C, k, gl);
        own ^= accept_mask(own, n, v, ctr1, j, a);
    }
    __syncthreads();
}

template <int L, bool INT8>
__device__ __forceinline__ void sweep_lds(const SweepArgs& a, const LaneInfo& li, uint32_t* lds)
{
    using Gm = Geo<L>;
    static_assert(Gm::WIDE && Gm::RL % 2 == 0 && Gm::G == 64, "LDS path layout");
    const LdsRep<L> rep{lds};
    const int gl = li.gl;
#pragma unroll 1
    for (int k = 0; k < Gm::K; ++k) {
        const uint32_t v = (uint32_t)(gl * Gm::K + k);
        uint32_t w0, w1;
        if (a.init) {
            w0 = init_word<L>(0, v, li.j, a);
            w1 = init_word<L>(1, v, li.j, a);
        } else {
            load_word<L, INT8>(a, li.j, v, w0, w1);
        }
        rep.at(0, k, gl) = w0;
        rep.at(1, k, gl) = w1;
    }
    __syncthreads();
    for (int t = 0; t < a.nsweeps; ++t) {
        const uint32_t g = a.g0 + (uint32_t)t;
        half_sweep_lds<L, INT8, 0>(rep, gl, g, li.j, a);
        half_sweep_lds<L, INT8, 1>(rep, gl, g, li.j, a);
    }
    uint32_t anti = 0, downs = 0;
#pragma unroll 1
    for (int k = 0; k < Gm::K; ++k) {
        const Nb n = rep.template nb<0>(k, gl);
        const uint32_t w0 = rep.at(0, k, gl), w1 = rep.at(1, k, gl);
        anti += __popc(w0 ^ n.up) + __popc(w0 ^ n.dn) + __popc(w0 ^ n.same) + __popc(w0 ^ n.side);
        downs += __popc(w0) + __popc(w1);
        store_word<L, INT8>(a, li.j, (uint32_t)(gl * Gm::K + k), w0, w1);
    }
    write_EM<L>(a, li, anti, downs);
}

template <int L>
constexpr int sweep_block()
{
    return Geo<L>::K == 1 ? kBlock : 64;
}

template <int L, bool INT8>
__global__ __launch_bounds__(sweep_block<L>()) void sweep_kernel(SweepArgs a)
{
    using Gm = Geo<L>;
    LaneInfo li;
    li.lane = (int)(threadIdx.x & 63u);
    li.gl = li.lane % Gm::G;
    const int wave = (int)((blockIdx.x * sweep_block<L>() + threadIdx.x) >> 6);
    if (wave * Gm::REPW >= a.n_rep) return;  // uniform per wave (per block on the LDS path)
    int jj = wave * Gm::REPW + li.lane / Gm::G;
    if constexpr (Gm::REPW == 1) jj = __builtin_amdgcn_readfirstlane(jj);
    li.j = (uint32_t)jj;
    li.valid = jj < a.n_rep;
    if constexpr (Gm::K == 1) {
        sweep_regs<L, INT8>(a, li);
    } else {
        __shared__ uint32_t lds[2 * Gm::NW];
        sweep_lds<L, INT8>(a, li, lds);
    }
}

// ---------------------------------------------------------------------------
// Population statistics: histogram n(b), b = (E + 2N) / 4, energy range, and
// the exact sums of E, E^2, |M|, M^2 (int64) and M^4 (128 bit).  Integer
// atomics only, so the result does not depend on scheduling order.
// ---------------------------------------------------------------------------
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

__global__ __launch_bounds__(kBlock) void stats_kernel(const int32_t* __restrict__ E, const int32_t* __restrict__ M,
                                                       int32_t n, int32_t N, DevStats* st, uint32_t* hist,
                                                       int32_t nbins, int record, DevMhr mhr)
{
    const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
    uint64_t sE = 0, sE2 = 0, sA = 0, sM2 = 0, m4lo = 0, m4hi = 0;
    int32_t emin = 0x7FFFFFFF, emax = (int32_t)0x80000000;
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
        const int b = (int)((e + 2 * N) >> 2);
        if (b >= 0 && b < nbins) atomicAdd(&hist[b], 1u);
        if (record && b >= 0 && b < nbins) {
            atomicAdd((unsigned long long*)&mhr.H[b], 1ull);
            atomicAdd((unsigned long long*)&mhr.SA[b], (unsigned long long)am);
            atomicAdd((unsigned long long*)&mhr.SM2[b], (unsigned long long)m2);
            atomic_add_u128(&mhr.SM4[2 * b], &mhr.SM4[2 * b + 1], m4lo, m4hi);
        }
    }
    // wave reduction
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
    if ((threadIdx.x & 63u) == 0u && (int)(blockIdx.x * kBlock + (threadIdx.x & ~63u)) < n) {
        atomicAdd((unsigned long long*)&st->sumE, (unsigned long long)sE);
        atomicAdd((unsigned long long*)&st->sumE2, (unsigned long long)sE2);
        atomicAdd((unsigned long long*)&st->sumAbsM, (unsigned long long)sA);
        atomicAdd((unsigned long long*)&st->sumM2, (unsigned long long)sM2);
        atomic_add_u128(&st->sumM4_lo, &st->sumM4_hi, m4lo, m4hi);
        atomicMin(&st->emin, emin);
        atomicMax(&st->emax, emax);
    }
}

__global__ void stats_reset_kernel(DevStats* st, uint32_t* hist, int32_t nbins)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i == 0) {
        st->emin = 0x7FFFFFFF;
        st->emax = (int32_t)0x80000000;
        st->r_new = 0;
        st->pad = 0;
        st->sumE = st->sumE2 = st->sumAbsM = st->sumM2 = st->sumM4_lo = st->sumM4_hi = 0;
    }
    for (int b = i; b < nbins; b += (int)(gridDim.x * blockDim.x)) hist[b] = 0;
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t value, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// ---------------------------------------------------------------------------
// Resampling: copy counts (one RESAMPLE uniform per parent), block sums,
// exclusive scan, parent index per child, replica copy.
// ---------------------------------------------------------------------------
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

__global__ __launch_bounds__(kBlock) void counts_kernel(const int32_t* __restrict__ E, int32_t n, int32_t N,
                                                        int32_t bmin, int32_t nwin, const uint32_t* __restrict__ tbl,
                                                        uint32_t step, uint32_t key0, uint32_t key1,
                                                        uint32_t* __restrict__ counts, uint32_t* __restrict__ bsum)
{
    const int j = (int)(blockIdx.x * kBlock + threadIdx.x);
    uint32_t c = 0;
    if (j < n) {
        const int b = ((E[j] + 2 * N) >> 2) - bmin;
        const uint32_t x = pick(philox10((uint32_t)j >> 2, step, 0u, kStreamResample, key0, key1), (uint32_t)j & 3u);
        if (b >= 0 && b < nwin) {  // always true for the population the tables were built from
            const uint32_t base = tbl[2 * b], thr = tbl[2 * b + 1];
            c = base + (x <= thr ? 1u : 0u);
        }
        counts[j] = c;
    }
    uint32_t total;
    block_exclusive_scan(c, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Single block: exclusive scan of the block sums in place; total -> st->r_new.
__global__ __launch_bounds__(1024) void scan_blocks_kernel(uint32_t* bsum, int32_t nblk, DevStats* st)
{
    __shared__ uint32_t part[1024];
    const int t = (int)threadIdx.x;
    const int per = (nblk + 1023) / 1024;
    const int lo = t * per, hi = min(nblk, lo + per);
    uint32_t s = 0;
    for (int i = lo; i < hi; ++i) s += bsum[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t y = (t >= off) ? part[t - off] : 0u;
        __syncthreads();
        part[t] += y;
        __syncthreads();
    }
    uint32_t run = part[t] - s;  // exclusive prefix of this thread's chunk
    for (int i = lo; i < hi; ++i) {
        const uint32_t v = bsum[i];
        bsum[i] = run;
        run += v;
    }
    if (t == 1023) st->r_new = part[1023];
}

__global__ __launch_bounds__(kBlock) void scatter_kernel(const uint32_t* __restrict__ counts,
                                                         const uint32_t* __restrict__ bsum, int32_t n,
                                                         uint32_t* __restrict__ parent)
{
    const int j = (int)(blockIdx.x * kBlock + threadIdx.x);
    const uint32_t c = (j < n) ? counts[j] : 0u;
    uint32_t total;
    const uint32_t off = bsum[blockIdx.x] + block_exclusive_scan(c, &total);
    for (uint32_t k = 0; k < c; ++k) parent[off + k] = (uint32_t)j;
}

__global__ __launch_bounds__(kBlock) void copy_kernel(const uint4* __restrict__ src, const int32_t* __restrict__ Es,
                                                      const int32_t* __restrict__ Ms,
                                                      const uint32_t* __restrict__ parent, int32_t n_new,
                                                      uint32_t chunks, uint4* __restrict__ dst,
                                                      int32_t* __restrict__ Ed, int32_t* __restrict__ Md)
{
    const size_t total = (size_t)n_new * chunks;
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < total; i += (size_t)gridDim.x * kBlock) {
        const uint32_t child = (uint32_t)(i / chunks), ch = (uint32_t)(i % chunks);
        const uint32_t p = parent[child];
        dst[i] = src[(size_t)p * chunks + ch];
        if (ch == 0) {
            Ed[child] = Es[p];
            Md[child] = Ms[p];
        }
    }
}

template <int L, bool INT8>
hipError_t launch_sweep_t(const SweepArgs& a, hipStream_t s)
{
    using Gm = Geo<L>;
    const int reps_per_block = (sweep_block<L>() / 64) * Gm::REPW;
    const int blocks = (a.n_rep + reps_per_block - 1) / reps_per_block;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((sweep_kernel<L, INT8>), dim3(blocks), dim3(sweep_block<L>()), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep(int L, int layout, const SweepArgs& a, hipStream_t s)
{
    const bool i8 = layout == 0;
    switch (L) {
    case 16: return i8 ? launch_sweep_t<16, true>(a, s) : launch_sweep_t<16, false>(a, s);
    case 32: return i8 ? launch_sweep_t<32, true>(a, s) : launch_sweep_t<32, false>(a, s);
    case 64: return i8 ? launch_sweep_t<64, true>(a, s) : launch_sweep_t<64, false>(a, s);
    case 128: return i8 ? launch_sweep_t<128, true>(a, s) : launch_sweep_t<128, false>(a, s);
    case 256: return i8 ? launch_sweep_t<256, true>(a, s) : launch_sweep_t<256, false>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stats(const int32_t* E, const int32_t* M, int32_t n, int32_t N, DevStats* st, uint32_t* hist,
                        int32_t nbins, int record, DevMhr mhr, hipStream_t s)
{
    const int blocks = (n + kBlock - 1) / kBlock;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(stats_kernel, dim3(blocks), dim3(kBlock), 0, s, E, M, n, N, st, hist, nbins, record, mhr);
    return hipGetLastError();
}

hipError_t launch_stats_reset(DevStats* st, uint32_t* hist, int32_t nbins, hipStream_t s)
{
    const int blocks = std::min((nbins + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL(stats_reset_kernel, dim3(std::max(blocks, 1)), dim3(kBlock), 0, s, st, hist, nbins);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, p, value, n);
    return hipGetLastError();
}

hipError_t launch_counts(const int32_t* E, int32_t n, int32_t N, int32_t bmin, int32_t nwin, const uint32_t* tbl,
                         uint32_t step, uint32_t key0, uint32_t key1, uint32_t* counts, uint32_t* bsum, hipStream_t s)
{
    const int blocks = (n + kBlock - 1) / kBlock;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(counts_kernel, dim3(blocks), dim3(kBlock), 0, s, E, n, N, bmin, nwin, tbl, step, key0, key1,
                       counts, bsum);
    return hipGetLastError();
}

hipError_t launch_scan_blocks(uint32_t* bsum, int32_t nblk, DevStats* st, hipStream_t s)
{
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(1024), 0, s, bsum, nblk, st);
    return hipGetLastError();
}

hipError_t launch_scatter(const uint32_t* counts, const uint32_t* bsum, int32_t n, uint32_t* parent, hipStream_t s)
{
    const int blocks = (n + kBlock - 1) / kBlock;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_kernel, dim3(blocks), dim3(kBlock), 0, s, counts, bsum, n, parent);
    return hipGetLastError();
}

hipError_t launch_copy(const uint8_t* src, const int32_t* Esrc, const int32_t* Msrc, const uint32_t* parent,
                       int32_t n_new, size_t rep_bytes, uint8_t* dst, int32_t* Edst, int32_t* Mdst, hipStream_t s)
{
    const uint32_t chunks = (uint32_t)(rep_bytes / 16);
    const size_t total = (size_t)n_new * chunks;
    if (total == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((total + kBlock - 1) / kBlock, 8192);
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, reinterpret_cast<const uint4*>(src),
                       Esrc, Msrc, parent, n_new, chunks, reinterpret_cast<uint4*>(dst), Edst, Mdst);
    return hipGetLastError();
}

}  // namespace pa

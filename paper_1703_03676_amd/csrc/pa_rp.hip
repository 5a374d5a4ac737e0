// Replica-parallel kernels for the interleaved spin store (PA_SPIN_INTERLEAVED):
// each replica is swept by its own thread, site by site (Sec. 3, spin updates:
// the replica-parallel setup, with the same spin of all replicas next to each
// other in memory so that the threads of a wave read and write adjacent bytes);
// from L = 64 on, four lanes share a replica's sites of one colour.  The scheme
// needs nothing of the model but a site's neighbours and the energy change of
// its update, so it serves as the general fall-back the paper describes; its
// parallelism is a few threads per replica, too little to fill the GPU for
// small populations.
//
// Store: spin (x, y) of replica j is the signed byte at (y L + x) * stride + j,
// stride = the capacity rounded up to 64.
//
// The chain is the one of the other kernels: the same update order (colour
// (x + y) even, then odd), the same per-site uniform (Philox SWEEP-HIGH bit
// planes for its high 16 bits, SWEEP-LOW for the low 16; or the in-line LCG
// variant's outputs) and the same thresholds, so the populations are
// bit-identical to those of the bit-sliced kernels and of the oracle.
#include "pa_device.h"
#include "pa_launch.h"

namespace pa {
namespace {

using namespace pa::dev;

// The 2D Ising model on an L x L torus, seen by the generic sweep: sites in
// update order (colour c, within-colour index q), their neighbours, and the
// energy term of a site.
template <int L>
struct Ising2D {
    static constexpr int N = L * L;
    static constexpr int HALF = N / 2;  // sites per colour
    // site of within-colour index q of colour c: row y = q / (L/2), column
    // x = 2 (q mod L/2) + ((y + c) & 1)
    __device__ __forceinline__ static int site(int c, int q)
    {
        const int y = q / (L / 2), h = q - y * (L / 2);
        return y * L + 2 * h + ((y + c) & 1);
    }
    // sum of the four neighbours of site s (periodic), each spin read at
    // byte s' * stride + j of the store
    __device__ __forceinline__ static int field(const int8_t* sp, size_t stride, int s)
    {
        const int y = s / L, x = s - y * L;
        const int l = y * L + ((x + L - 1) & (L - 1)), r = y * L + ((x + 1) & (L - 1));
        const int u = ((y + L - 1) & (L - 1)) * L + x, d = ((y + 1) & (L - 1)) * L + x;
        return (int)sp[(size_t)l * stride] + (int)sp[(size_t)r * stride] + (int)sp[(size_t)u * stride] +
               (int)sp[(size_t)d * stride];
    }
};

// Bit-plane uniform of one 32-site word (the sites q = 32 v .. 32 v + 31 of one
// colour of one replica), evaluated lazily: blocks 0 and 1 (planes 0-7) when a
// site first needs a uniform, blocks 2 and 3 (planes 8-15) when a site's high
// byte ties with its threshold's, the SWEEP-LOW half when the high 16 bits tie.
struct WordUniform {
    uint32_t v, ctr1, j, tag, key0, key1;
    uint32_t pl[16];
    int have;  // planes computed: 0, 8 or 16

    __device__ __forceinline__ void block(int b)
    {
        const U4 P = philox10(4u * v + (uint32_t)b, ctr1, j, tag | kStreamSweepHigh, key0, key1);
        pl[4 * b] = P.x;
        pl[4 * b + 1] = P.y;
        pl[4 * b + 2] = P.z;
        pl[4 * b + 3] = P.w;
    }
    // 8 bits of the site's uniform from planes F .. F + 7 (plane 0 = bit 31)
    template <int F>
    __device__ __forceinline__ uint32_t byte(uint32_t b) const
    {
        uint32_t x = 0;
#pragma unroll
        for (int p = F; p < F + 8; ++p) x = (x << 1) | ((pl[p] >> b) & 1u);
        return x;
    }
    // x < T for the uniform x of site bit b of the word, 0 <= T <= 2^32
    __device__ __forceinline__ bool below(uint32_t b, uint64_t T)
    {
        if (T >= ((uint64_t)1 << 32)) return true;
        if (T == 0) return false;
        const uint32_t t = (uint32_t)T;
        if (have < 8) {
            block(0);
            block(1);
            have = 8;
        }
        const uint32_t x8 = byte<0>(b), t8 = t >> 24;
        if (x8 != t8) return x8 < t8;
        if (have < 16) {
            block(2);
            block(3);
            have = 16;
        }
        const uint32_t x16 = byte<8>(b), t16 = (t >> 16) & 0xFFu;
        if (x16 != t16) return x16 < t16;
        const uint32_t q = 32u * v + b;
        const U4 P = philox10(q >> 3, ctr1, j, tag | kStreamSweepLow, key0, key1);
        const uint32_t word = pick(P, (q >> 1) & 3u);
        const uint32_t lo = (q & 1u) ? (word & 0xFFFFu) : (word >> 16);
        return lo < (t & 0xFFFFu);
    }
};

// The in-line LCG variant's uniforms of one word: site b takes the (b+1)-th
// output after the word's seed.
__device__ __forceinline__ uint32_t lcg_uniform(uint32_t seed, uint32_t b)
{
    uint32_t x = seed;
    for (uint32_t i = 0; i <= b; ++i) x = kLcgA * x + kLcgC;
    return x;
}

// Acceptance threshold (T <= 2^32: flip iff the uniform x < T) of a site with
// k = s h; Metropolis: k <= 0 flips without a draw (returned as 2^32).
template <bool HB>
__device__ __forceinline__ uint64_t flip_threshold(int k, uint64_t T2, uint64_t T4)
{
    const uint64_t two32 = (uint64_t)1 << 32;
    if constexpr (HB) {
        switch (k) {
        case 4: return T4;
        case 2: return T2;
        case 0: return two32 / 2;
        case -2: return two32 - T2;
        default: return two32 - T4;
        }
    } else {
        return k <= 0 ? two32 : (k == 2 ? T2 : T4);
    }
}

// E = -sum over the 2N bonds, M = sum of spins, of replica j.
template <int L>
__device__ __forceinline__ void recount(const int8_t* sp, size_t stride, int32_t* E, int32_t* M)
{
    int e = 0, m = 0;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            const int s = sp[(size_t)(y * L + x) * stride];
            const int r = sp[(size_t)(y * L + ((x + 1) & (L - 1))) * stride];
            const int d = sp[(size_t)(((y + 1) & (L - 1)) * L + x) * stride];
            e -= s * (r + d);
            m += s;
        }
    *E = e;
    *M = m;
}

// Lanes per replica: from L = 64 on, the words of one colour are shared out
// among four lanes of one wave (lane = part * 16 + r holds replica 16 w + r of
// wave w), so a launch has four times as many threads as replicas; within a
// half sweep the parts' sites do not neighbour each other, and the block waits
// for all of them before the other colour.  Below, one lane per replica (the
// kernels then need more registers per lane than four parts leave).
template <int L>
struct RpShape {
    static constexpr int PARTS = L >= 64 ? 4 : 1;
    static constexpr int REPS_PER_WAVE = 64 / PARTS;
    static constexpr int REPS_PER_BLOCK = (kBlock / 64) * REPS_PER_WAVE;
    static constexpr int BATCH = L >= 64 ? 16 : 32;  // sites whose spins and fields are read together
};

template <int L, int U>
__global__ __launch_bounds__(kBlock) void rp_sweep_kernel(SweepArgs a)
{
    using Model = Ising2D<L>;
    using Sh = RpShape<L>;
    constexpr bool HB = U == kHeatbath, LCG = U == kLcg;
    constexpr int WORDS = Model::HALF / 32;  // 32-site words per colour
    constexpr int kRpParts = Sh::PARTS, kRpRepsPerWave = Sh::REPS_PER_WAVE, kRpBatch = Sh::BATCH;
    int32_t n = a.n_rep;
    if (a.n_dev) n = min(n, (int32_t)*a.n_dev);
    const int lane = (int)(threadIdx.x & 63u), part = lane / kRpRepsPerWave;
    const int j = (int)(blockIdx.x * Sh::REPS_PER_BLOCK + (threadIdx.x >> 6) * kRpRepsPerWave) +
                  (lane & (kRpRepsPerWave - 1));
    const bool valid = j < n;
    const size_t stride = a.stride;
    int8_t* sp = reinterpret_cast<int8_t*>(a.spin) + j;
    if (a.init || a.nsweeps == 0) {  // initial state or recount: one lane per replica
        if (!valid || part != 0) return;
        if (a.init) {
            // initial state: INIT output word p >> 5 (p = c N/2 + q), bit p & 31 set = spin -1
            for (int pb = 0; pb < Model::N / 128; ++pb) {
                const U4 P = philox10((uint32_t)pb, 0u, (uint32_t)j, a.tag | kStreamInit, a.key0, a.key1);
                const uint32_t w[4] = {P.x, P.y, P.z, P.w};
                for (int k = 0; k < 128; ++k) {
                    const int p = pb * 128 + k, c = p / Model::HALF, q = p - c * Model::HALF;
                    sp[(size_t)Model::site(c, q) * stride] = ((w[k >> 5] >> (k & 31)) & 1u) ? (int8_t)-1 : (int8_t)1;
                }
            }
        }
        recount<L>(sp, stride, &a.E[j], &a.M[j]);
        return;
    }
    // every lane of the block takes part in the barriers; lanes beyond the
    // population do no work
    int32_t dE = 0, dM = 0;
    const uint64_t T2 = ((uint64_t)a.t2h << 16) + a.t2l, T4 = ((uint64_t)a.t4h << 16) + a.t4l;
    for (int t = 0; t < a.nsweeps; ++t) {
        const uint32_t g = a.g0 + (uint32_t)t;
#pragma unroll 1
        for (int c = 0; c < 2; ++c) {
#pragma unroll 1
            for (int v = part; valid && v < WORDS; v += kRpParts) {
                WordUniform wu;
                wu.v = (uint32_t)v;
                wu.ctr1 = 2u * g + (uint32_t)c;
                wu.j = (uint32_t)j;
                wu.tag = a.tag;
                wu.key0 = a.key0;
                wu.key1 = a.key1;
                wu.have = 0;
                uint32_t seed = 0;  // LCG: the seed of this word and colour
                if constexpr (LCG) {
                    const U4 P = philox10((uint32_t)v, g, (uint32_t)j, a.tag | kStreamLcgSeed, a.key0, a.key1);
                    seed = c == 0 ? P.x : P.y;
                }
                // The spins and local fields of kRpBatch sites are all read
                // before any of them is updated: the neighbours of a site are
                // of the other colour, which this half sweep does not change,
                // so the result is the one of the site-by-site order, and the
                // loads are in flight together instead of one site at a time.
#pragma unroll
                for (int b0 = 0; b0 < 32; b0 += kRpBatch) {
                int si[kRpBatch], k[kRpBatch];
#pragma unroll
                for (int i = 0; i < kRpBatch; ++i) {
                    const int s = Model::site(c, 32 * v + b0 + i);
                    si[i] = sp[(size_t)s * stride];
                    k[i] = Model::field(sp, stride, s);
                }
#pragma unroll
                for (int i = 0; i < kRpBatch; ++i) {
                    const int b = b0 + i;
                    const int kb = si[i] * k[i];
                    const uint64_t T = flip_threshold<HB>(kb, T2, T4);
                    bool flip;
                    if constexpr (LCG) {
                        flip = T >= ((uint64_t)1 << 32) || (uint64_t)lcg_uniform(seed, (uint32_t)b) < T;
                    } else {
                        flip = wu.below((uint32_t)b, T);
                    }
                    if (flip) {
                        sp[(size_t)Model::site(c, 32 * v + b) * stride] = (int8_t)-si[i];
                        dE += 2 * kb;
                        dM -= 2 * si[i];
                    }
                }
                }
            }
            if constexpr (kRpParts > 1) __syncthreads();  // this colour's updates, before the other colour reads them
        }
    }
    // the parts' energy and magnetisation changes, summed over the replica's lanes
#pragma unroll
    for (int off = kRpRepsPerWave; off < 64; off <<= 1) {
        dE += __shfl_xor(dE, off);
        dM += __shfl_xor(dM, off);
    }
    if (valid && part == 0) {
        a.E[j] += dE;
        a.M[j] += dM;
    }
}

// Replica copy child <- parent[child] of the interleaved store, for child <
// min(*n_new, cap): threads take consecutive children of one chunk of sites,
// so each site row is read near the parents' columns and written as one
// contiguous run of bytes.
constexpr int kRpCopySites = 256;

__global__ __launch_bounds__(kBlock) void rp_copy_kernel(const int8_t* __restrict__ src, const int32_t* __restrict__ Es,
                                                         const int32_t* __restrict__ Ms,
                                                         const uint32_t* __restrict__ parent,
                                                         const uint32_t* __restrict__ n_new, uint32_t cap, int32_t N,
                                                         uint32_t stride, int8_t* __restrict__ dst,
                                                         int32_t* __restrict__ Ed, int32_t* __restrict__ Md)
{
    const uint32_t nn = min(*n_new, cap);
    const uint32_t child = blockIdx.x * kBlock + threadIdx.x;
    if (child >= nn) return;
    const uint32_t p = parent[child];
    const int s0 = (int)blockIdx.y * kRpCopySites, s1 = min(s0 + kRpCopySites, N);
    for (int s = s0; s < s1; ++s) dst[(size_t)s * stride + child] = src[(size_t)s * stride + p];
    if (blockIdx.y == 0) {
        Ed[child] = Es[p];
        Md[child] = Ms[p];
    }
}

template <int L, int U>
hipError_t launch_rp_t(const SweepArgs& a, hipStream_t s)
{
    const int blocks = (a.n_rep + RpShape<L>::REPS_PER_BLOCK - 1) / RpShape<L>::REPS_PER_BLOCK;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((rp_sweep_kernel<L, U>), dim3(blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int L>
hipError_t launch_rp_l(int update, const SweepArgs& a, hipStream_t s)
{
    switch (update) {
    case kMetropolis: return launch_rp_t<L, kMetropolis>(a, s);
    case kHeatbath: return launch_rp_t<L, kHeatbath>(a, s);
    case kLcg: return launch_rp_t<L, kLcg>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_sweep_rp(int L, int update, const SweepArgs& a, hipStream_t s)
{
    // no fused gather and no statistics epilogue on this store
    if (a.parent || a.acc || a.stride == 0) return hipErrorInvalidValue;
    switch (L) {
    case 16: return launch_rp_l<16>(update, a, s);
    case 32: return launch_rp_l<32>(update, a, s);
    case 64: return launch_rp_l<64>(update, a, s);
    case 128: return launch_rp_l<128>(update, a, s);
    case 256: return launch_rp_l<256>(update, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_copy_rp(const uint8_t* src, const int32_t* Esrc, const int32_t* Msrc, const uint32_t* parent,
                          const uint32_t* n_new, int32_t cap, int32_t N, uint32_t stride, uint8_t* dst, int32_t* Edst,
                          int32_t* Mdst, hipStream_t s)
{
    if (cap <= 0) return hipSuccess;
    const dim3 grid((unsigned)((cap + kBlock - 1) / kBlock), (unsigned)((N + kRpCopySites - 1) / kRpCopySites));
    hipLaunchKernelGGL(rp_copy_kernel, grid, dim3(kBlock), 0, s, reinterpret_cast<const int8_t*>(src), Esrc, Msrc,
                       parent, n_new, (uint32_t)cap, N, stride, reinterpret_cast<int8_t*>(dst), Edst, Mdst);
    return hipGetLastError();
}

}  // namespace pa

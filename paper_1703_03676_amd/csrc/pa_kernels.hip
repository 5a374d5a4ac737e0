// Population kernels of the single-run path for gfx950 (CDNA4); the sweep
// kernel is in pa_sweep.hip.
//
//   stats_kernel   energy histogram, energy range and exact moment sums
//                  (inputs of Eq. (Q), Eq. (observables), multi-histogram)
//   stats_gather   the same statistics from the sweep epilogue's accumulators
//   counts_kernel  integer copy counts, Eq. (resampling factors), block totals
//   scatter        prefix sum of the counts -> parent index of every child
//   copy_kernel    replica copy into the other half of the ping-pong store
//
#include "pa_device.h"
#include "pa_launch.h"
#include "pa_reduce.h"

namespace pa {
namespace {

using namespace pa::dev;

// ---------------------------------------------------------------------------
// Population statistics (histogram, energy range, exact moment sums).  Each
// chunk of kBlock replicas is added to the histogram and gets its partial sums,
// by the workgroups in turn; the workgroup that finishes last (counted in
// st->done) sums the partials into *st.
// With `host` (pinned host memory, device view) that block also writes the
// statistics block and the occupied window [emin, emax] of the histogram there
// (bin b at byte 64 + 4 b), so the host reads them after the kernel without a
// separate copy.
// ---------------------------------------------------------------------------
// Sums the partials into *st, clears the block counter and, with `host`,
// publishes the statistics block and the histogram window there.  Called by
// every thread of the one block that finalises.
__device__ __forceinline__ void stats_publish(const StatsPart* parts, int nparts, DevStats* st, const uint32_t* hist,
                                              int32_t N, uint32_t* host)
{
    stats_final(parts, nparts, st);
    __syncthreads();  // *st written by thread 0 is visible to the block
    if (threadIdx.x == 0) st->done = 0u;
    if (!host) return;
    const uint32_t* sw = reinterpret_cast<const uint32_t*>(st);
    if (threadIdx.x < sizeof(DevStats) / 4) host[threadIdx.x] = (threadIdx.x == 3) ? 0u : sw[threadIdx.x];
    const int32_t emin = st->emin, emax = st->emax;
    if (emin > emax || emin < -2 * N || emax > 2 * N) return;  // empty or invalid: the host uses no bins
    uint32_t* h = host + sizeof(DevStats) / 4;
    for (int b = (emin + 2 * N) / 4 + (int)threadIdx.x; b <= (emax + 2 * N) / 4; b += kBlock) h[b] = hist[b];
}

__global__ __launch_bounds__(kBlock) void stats_kernel(const int32_t* __restrict__ E, const int32_t* __restrict__ M,
                                                       int32_t n, const uint32_t* n_dev, int32_t N, uint32_t* hist,
                                                       int32_t nbins, int record, DevMhr mhr, StatsPart* parts,
                                                       DevStats* st, uint32_t* __restrict__ host)
{
    __shared__ uint32_t last;
    if (n_dev) n = min(n, (int32_t)*n_dev);
    const int nparts = (n + kBlock - 1) / kBlock;
    if (nparts == 0) {  // empty population (a refused step): block 0 publishes the empty statistics
        if (blockIdx.x == 0) stats_publish(parts, 0, st, hist, N, host);
        return;
    }
    // chunks of kBlock replicas, strided over the grid; the blocks that hold
    // at least one chunk count themselves in st->done
    const int nblk = min(nparts, (int)gridDim.x);
    if ((int)blockIdx.x >= nblk) return;  // uniform per block
    for (int c = (int)blockIdx.x; c < nparts; c += (int)gridDim.x) {
        stats_block(E, M, n, N, c * kBlock, hist, nbins, record != 0, mhr, &parts[c]);
        __syncthreads();  // the LDS tables are reused by the next chunk
    }
    __threadfence();  // this block's partials and histogram updates, device-wide
    __syncthreads();
    if (threadIdx.x == 0) last = (atomicAdd(&st->done, 1u) == (uint32_t)(nblk - 1)) ? 1u : 0u;
    __syncthreads();
    if (!last) return;  // uniform per block
    __threadfence();    // every other block's updates are visible to this one
    stats_publish(parts, nparts, st, hist, N, host);
}

__global__ void stats_reset_kernel(DevStats* st, uint32_t* hist, int32_t nbins)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i == 0) {
        st->emin = 0x7FFFFFFF;
        st->emax = (int32_t)0x80000000;
        st->done = 0u;
        st->sumE = st->sumE2 = st->sumAbsM = st->sumM2 = st->sumM4_lo = st->sumM4_hi = 0;
    }
    for (int b = i; b < nbins; b += (int)(gridDim.x * blockDim.x)) hist[b] = 0;
}

// ---------------------------------------------------------------------------
// Statistics accumulated by the sweep's epilogue (AccSlot): one block sums the
// kAccSlots slots into *st (M^4 rebuilt as a 128-bit sum), then the
// kAccHists histogram copies over the occupied window [emin, emax] into hist,
// resetting every slot and bin it reads (sums 0, empty range, bins 0) for the
// next sweep.  hist has been cleared before (by the scatter) and r_new is
// kept.  With `host` the statistics block and the window are published there
// as stats_kernel does.
// ---------------------------------------------------------------------------
constexpr int kGatherThreads = 1024;
static_assert(kAccSlots <= kGatherThreads, "one slot per thread");

__device__ __forceinline__ void reset_slot(AccSlot* s)
{
    s->sumE = s->sumE2 = s->sumAbsM = s->sumM2 = s->m4lo = s->m4hi = 0;
    s->emin = 0x7FFFFFFF;
    s->emax = (int32_t)0x80000000;
}

__global__ __launch_bounds__(kGatherThreads) void stats_gather_kernel(AccSlot* __restrict__ acc,
                                                                      uint32_t* __restrict__ acc_hist, int32_t nbins,
                                                                      int32_t N, DevStats* st,
                                                                      uint32_t* __restrict__ hist,
                                                                      uint32_t* __restrict__ host)
{
    __shared__ DevStats sh;
    const int t = (int)threadIdx.x;
    const uint32_t r_new = st->r_new;  // from the scatter
    uint64_t sE = 0, sE2 = 0, sA = 0, sM2 = 0, m4lo = 0, m4hi = 0;
    int32_t emin = 0x7FFFFFFF, emax = (int32_t)0x80000000;
    if (t < kAccSlots) {
        AccSlot* s = acc + t;
        sE = s->sumE;
        sE2 = s->sumE2;
        sA = s->sumAbsM;
        sM2 = s->sumM2;
        const uint64_t low32 = s->m4lo, rest = s->m4hi;  // M^4 sum = rest * 2^32 + low32
        m4lo = rest << 32;
        m4hi = rest >> 32;
        add_u128(m4lo, m4hi, low32, 0u);
        emin = s->emin;
        emax = s->emax;
        reset_slot(s);
    }
    stats_block_total<kGatherThreads>(sE, sE2, sA, sM2, m4lo, m4hi, emin, emax, st, &sh);
    __syncthreads();  // the totals in sh, written by thread 0, are visible to the block
    const int32_t lo = sh.emin, hi = sh.emax;
    if (host && t < (int)(sizeof(DevStats) / 4)) {
        const uint32_t* sw = reinterpret_cast<const uint32_t*>(&sh);
        host[t] = (t == 2) ? r_new : (t == 3) ? 0u : sw[t];
    }
    if (lo > hi || lo < -2 * N || hi > 2 * N) return;  // empty: no bins were added
    uint32_t* hh = host ? host + sizeof(DevStats) / 4 : nullptr;
    for (int b = (lo + 2 * N) / 4 + t; b <= (hi + 2 * N) / 4; b += kGatherThreads) {
        uint32_t c[kAccHists];
#pragma unroll
        for (int k = 0; k < kAccHists; ++k) c[k] = acc_hist[(size_t)k * nbins + b];
        uint32_t v = 0;
#pragma unroll
        for (int k = 0; k < kAccHists; ++k) {
            v += c[k];
            acc_hist[(size_t)k * nbins + b] = 0u;
        }
        hist[b] = v;
        if (hh) hh[b] = v;
    }
}

// Every slot to the empty state and every histogram copy to zero.
__global__ void acc_reset_kernel(AccSlot* acc, uint32_t* acc_hist, size_t nh)
{
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < (size_t)kAccSlots) reset_slot(acc + i);
    for (size_t k = i; k < nh; k += (size_t)gridDim.x * blockDim.x) acc_hist[k] = 0u;
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
__global__ __launch_bounds__(kBlock) void counts_kernel(const int32_t* __restrict__ E, int32_t n, int32_t N,
                                                        int32_t bmin, int32_t nwin, const uint32_t* __restrict__ tbl,
                                                        uint32_t step, uint32_t key0, uint32_t key1, uint32_t tag,
                                                        uint32_t* __restrict__ counts, uint32_t* __restrict__ bsum)
{
    const int j = (int)(blockIdx.x * kBlock + threadIdx.x);
    uint32_t c = 0;
    if (j < n) {
        const int b = ((E[j] + 2 * N) >> 2) - bmin;
        const uint32_t x = pick(philox10((uint32_t)j >> 2, step, 0u, tag | kStreamResample, key0, key1), (uint32_t)j & 3u);
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

// Single block: exclusive scan of the block totals in place; the grand total
// goes to st->r_new.  Used when there are more than kScanFreeBlocks blocks.
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

// Parent index of every child; children beyond `cap` are not written (the
// caller rejects such a population).  Without `scanned`, the offset of the
// block's first child is the sum of the totals of the blocks before it (bsum,
// from counts_kernel), so no separate scan pass is needed, and the last block
// writes the grand total to st->r_new; with `scanned`, bsum already holds the
// exclusive prefix (scan_blocks_kernel, for many blocks, where summing would
// grow with the square of their number).  The kernel also clears the rest of
// the statistics block and the histogram, ready for the statistics of the
// resampled population (the host has read the previous ones).
__global__ __launch_bounds__(kBlock) void scatter_kernel(const uint32_t* __restrict__ counts,
                                                         const uint32_t* __restrict__ bsum, int32_t n, uint32_t cap,
                                                         uint32_t* __restrict__ parent, DevStats* st,
                                                         uint32_t* __restrict__ hist, int32_t nbins, int scanned)
{
    __shared__ uint32_t wpart[kBlock / 64];
    const int lane = (int)(threadIdx.x & 63u), wid = (int)(threadIdx.x >> 6);
    uint32_t base = 0;
    if (scanned) {
        base = bsum[blockIdx.x];
    } else {
        uint32_t before = 0;
        for (int i = (int)threadIdx.x; i < (int)blockIdx.x; i += kBlock) before += bsum[i];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) before += (uint32_t)__shfl_xor((int)before, off);
        if (lane == 0) wpart[wid] = before;
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) base += wpart[w];
    }
    const int j = (int)(blockIdx.x * kBlock + threadIdx.x);
    const uint32_t c = (j < n) ? counts[j] : 0u;
    uint32_t total;
    const uint32_t off = base + block_exclusive_scan(c, &total);
    fill_parents(parent, off, c, (uint32_t)(j - lane), cap);
    if (threadIdx.x == 0) {
        if (!scanned && blockIdx.x == gridDim.x - 1) st->r_new = base + total;
        if (blockIdx.x == 0) {
            st->emin = 0x7FFFFFFF;
            st->emax = (int32_t)0x80000000;
            st->done = 0u;
            st->sumE = st->sumE2 = st->sumAbsM = st->sumM2 = st->sumM4_lo = st->sumM4_hi = 0;
        }
    }
    for (int b = j; b < nbins; b += (int)(gridDim.x * kBlock)) hist[b] = 0;
}

// Replica copy child <- parent[child] for child < min(*n_new, cap); the size
// of the new population is read on the device, so the copy can be queued
// before the host has seen it.  A team of T threads (T divides the block, at
// most the 16-byte chunks of a replica) moves one child at a time: one parent
// index per team, contiguous coalesced 16-byte chunks, no per-chunk index
// arithmetic; four chunks per thread are in flight.  Plain HBM streaming.
template <int T>
__global__ __launch_bounds__(kBlock) void copy_kernel(const uint4* __restrict__ src, const int32_t* __restrict__ Es,
                                                      const int32_t* __restrict__ Ms,
                                                      const uint32_t* __restrict__ parent,
                                                      const uint32_t* __restrict__ n_new, uint32_t cap,
                                                      uint32_t chunks, uint4* __restrict__ dst,
                                                      int32_t* __restrict__ Ed, int32_t* __restrict__ Md)
{
    constexpr int TEAMS = kBlock / T;
    const uint32_t nn = min(*n_new, cap);
    const int t = (int)(threadIdx.x % T), team = (int)(threadIdx.x / T);
    for (uint32_t child = blockIdx.x * TEAMS + (uint32_t)team; child < nn; child += gridDim.x * TEAMS) {
        const uint32_t p = parent[child];
        // E and M are loaded first so that their latency overlaps the spins
        int32_t e = 0, m = 0;
        if (t == 0) {
            e = Es[p];
            m = Ms[p];
        }
        const uint4* s = src + (size_t)p * chunks;
        uint4* d = dst + (size_t)child * chunks;
        uint32_t c = (uint32_t)t;
        for (; c + 3u * T < chunks; c += 4u * T) {
            const uint4 v0 = s[c], v1 = s[c + T], v2 = s[c + 2 * T], v3 = s[c + 3 * T];
            d[c] = v0;
            d[c + T] = v1;
            d[c + 2 * T] = v2;
            d[c + 3 * T] = v3;
        }
        for (; c < chunks; c += T) d[c] = s[c];
        if (t == 0) {
            Ed[child] = e;
            Md[child] = m;
        }
    }
}


}  // namespace


hipError_t launch_stats(const int32_t* E, const int32_t* M, int32_t n, const uint32_t* n_dev, int32_t N,
                        DevStats* st, uint32_t* hist, int32_t nbins, int record, DevMhr mhr, StatsPart* parts,
                        void* host, hipStream_t s)
{
    // at most kStatsBlocks blocks: each block's device-wide fence before it is
    // counted costs more than the chunks it saves beyond that
    const int blocks = std::min((n + kBlock - 1) / kBlock, kStatsBlocks);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(stats_kernel, dim3(blocks), dim3(kBlock), 0, s, E, M, n, n_dev, N, hist, nbins, record, mhr,
                       parts, st, (uint32_t*)host);
    return hipGetLastError();
}

hipError_t launch_stats_reset(DevStats* st, uint32_t* hist, int32_t nbins, hipStream_t s)
{
    const int blocks = std::min((nbins + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL(stats_reset_kernel, dim3(std::max(blocks, 1)), dim3(kBlock), 0, s, st, hist, nbins);
    return hipGetLastError();
}

hipError_t launch_stats_gather(AccSlot* acc, uint32_t* acc_hist, int32_t nbins, int32_t N, DevStats* st,
                               uint32_t* hist, void* host, hipStream_t s)
{
    hipLaunchKernelGGL(stats_gather_kernel, dim3(1), dim3(kGatherThreads), 0, s, acc, acc_hist, nbins, N, st, hist,
                       (uint32_t*)host);
    return hipGetLastError();
}

hipError_t launch_acc_reset(AccSlot* acc, uint32_t* acc_hist, int32_t nbins, hipStream_t s)
{
    const size_t nh = (size_t)kAccHists * (size_t)nbins;
    const size_t blocks = std::min<size_t>((nh + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(acc_reset_kernel, dim3((unsigned)std::max<size_t>(blocks, 1)), dim3(kBlock), 0, s, acc,
                       acc_hist, nh);
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
                         uint32_t step, uint32_t key0, uint32_t key1, uint32_t tag, uint32_t* counts, uint32_t* bsum,
                         hipStream_t s)
{
    const int blocks = (n + kBlock - 1) / kBlock;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(counts_kernel, dim3(blocks), dim3(kBlock), 0, s, E, n, N, bmin, nwin, tbl, step, key0, key1,
                       tag, counts, bsum);
    return hipGetLastError();
}

hipError_t launch_scatter(const uint32_t* counts, uint32_t* bsum, int32_t n, int32_t cap, uint32_t* parent,
                          DevStats* st, uint32_t* hist, int32_t nbins, hipStream_t s)
{
    const int blocks = std::max((n + kBlock - 1) / kBlock, 1);
    const int scanned = blocks > kScanFreeBlocks ? 1 : 0;
    if (scanned) hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(1024), 0, s, bsum, blocks, st);
    hipLaunchKernelGGL(scatter_kernel, dim3(blocks), dim3(kBlock), 0, s, counts, (const uint32_t*)bsum, n,
                       (uint32_t)cap, parent, st, hist, nbins, scanned);
    return hipGetLastError();
}

hipError_t launch_copy(const uint8_t* src, const int32_t* Esrc, const int32_t* Msrc, const uint32_t* parent,
                       const uint32_t* n_new, int32_t cap, size_t rep_bytes, uint8_t* dst, int32_t* Edst,
                       int32_t* Mdst, hipStream_t s)
{
    const uint32_t chunks = (uint32_t)(rep_bytes / 16);  // 32 (L = 64, bits) ... 4096 (L = 256, int8)
    if (cap <= 0 || chunks == 0) return hipSuccess;
    const uint4* sp = reinterpret_cast<const uint4*>(src);
    uint4* dp = reinterpret_cast<uint4*>(dst);
    // one child per team; enough blocks to cover the population up to 8192
    // blocks (32 per CU), the rest by the grid-stride loop
    auto grid = [&](int teams) { return (unsigned)std::min<int64_t>(((int64_t)cap + teams - 1) / teams, 8192); };
    if (chunks >= 256) {
        hipLaunchKernelGGL((copy_kernel<256>), dim3(grid(1)), dim3(kBlock), 0, s, sp, Esrc, Msrc, parent, n_new,
                           (uint32_t)cap, chunks, dp, Edst, Mdst);
    } else if (chunks >= 64) {
        hipLaunchKernelGGL((copy_kernel<64>), dim3(grid(4)), dim3(kBlock), 0, s, sp, Esrc, Msrc, parent, n_new,
                           (uint32_t)cap, chunks, dp, Edst, Mdst);
    } else {
        hipLaunchKernelGGL((copy_kernel<16>), dim3(grid(16)), dim3(kBlock), 0, s, sp, Esrc, Msrc, parent, n_new,
                           (uint32_t)cap, chunks, dp, Edst, Mdst);
    }
    return hipGetLastError();
}

}  // namespace pa

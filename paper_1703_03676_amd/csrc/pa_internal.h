// Internal interface between the C-ABI host layer (pa_api.hip) and the
// device kernels (pa_kernels.hip).  Not installed; not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

// Device-side statistics block; the energy histogram follows it directly in
// the workspace so one copy brings both back to the host.
struct DevStats {
    int32_t emin, emax;     // energy range of the population
    uint32_t r_new;         // total of the copy counts (resampling)
    uint32_t pad;
    uint64_t sumE, sumE2, sumAbsM, sumM2, sumM4_lo, sumM4_hi;  // two's complement sums
};
static_assert(sizeof(DevStats) == 64, "stats block layout");

// Partial statistics of one block of kBlock replicas; the partials of a
// population are summed by a second kernel into its DevStats.
struct StatsPart {
    uint64_t sumE, sumE2, sumAbsM, sumM2, sumM4_lo, sumM4_hi;
    int32_t emin, emax;
    uint32_t pad[2];
};
static_assert(sizeof(StatsPart) == 64, "partial statistics layout");

// Per-energy accumulators for multi-histogram reweighting (device resident).
struct DevMhr {
    uint64_t* H;        // [nbins] number of measured replicas per energy
    uint64_t* SA;       // [nbins] sum |M|
    uint64_t* SM2;      // [nbins] sum M^2
    uint64_t* SM4;      // [2*nbins] sum M^4 as (lo, hi) pairs
};

struct SweepArgs {
    uint8_t* spin;          // population spin store (layout-specific)
    int32_t* E;
    int32_t* M;
    int32_t n_rep;          // number of replicas to process
    int32_t nsweeps;
    uint32_t g0;            // global sweep number of the first sweep
    uint32_t key0, key1;    // Philox key
    uint32_t t2h, t2l;      // threshold T_2 = t2h * 2^16 + t2l  (t2h <= 65536)
    uint32_t t4h, t4l;      // threshold T_4  (heat-bath: U_2, U_4, each <= 2^31)
    int32_t init;           // 1: draw the initial state instead of loading spins
    const uint32_t* n_dev;  // if set: the population size is min(*n_dev, n_rep), read on the device
    const uint8_t* src;     // with parent: replica j starts from replica parent[j] of this store
    const uint32_t* parent; // (the resampling copy fused into the sweep's load); else NULL
};

// Kernel launchers; each returns the launch status.
// heatbath selects the heat-bath update (thresholds U_2, U_4 in t2*/t4*)
// instead of Metropolis (T_2, T_4).
hipError_t launch_sweep(int L, int layout, bool heatbath, const SweepArgs& a, hipStream_t s);
// Statistics of a population (after launch_stats_reset): histogram, range,
// moment sums; parts holds ceil(n / kBlock) partials.  With n_dev the size is
// min(*n_dev, n), read on the device.
hipError_t launch_stats(const int32_t* E, const int32_t* M, int32_t n, const uint32_t* n_dev, int32_t N,
                        DevStats* st, uint32_t* hist, int32_t nbins, int record, DevMhr mhr, StatsPart* parts,
                        hipStream_t s);
hipError_t launch_counts(const int32_t* E, int32_t n, int32_t N, int32_t bmin, int32_t nwin, const uint32_t* tbl,
                         uint32_t step, uint32_t key0, uint32_t key1, uint32_t* counts, uint32_t* bsum,
                         hipStream_t s);
hipError_t launch_scan_blocks(uint32_t* bsum, int32_t nblk, DevStats* st, hipStream_t s);
// Parent indices (children beyond cap are dropped) and the replica copy of
// min(*n_new, cap) children, n_new read on the device.
hipError_t launch_scatter(const uint32_t* counts, const uint32_t* bsum, int32_t n, int32_t cap, uint32_t* parent,
                          hipStream_t s);
hipError_t launch_copy(const uint8_t* src, const int32_t* Esrc, const int32_t* Msrc, const uint32_t* parent,
                       const uint32_t* n_new, int32_t cap, size_t rep_bytes, uint8_t* dst, int32_t* Edst,
                       int32_t* Mdst, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t s);
// Clears the range, the sums and the histogram (not r_new).
hipError_t launch_stats_reset(DevStats* st, uint32_t* hist, int32_t nbins, hipStream_t s);

constexpr int kBlock = 256;     // threads per block of the population kernels

}  // namespace pa

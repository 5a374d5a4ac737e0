// Data structures shared by the C-ABI host layer (pa_api.hip) and the device
// code (pa_device.h, pa_reduce.h and the kernels); the kernel launchers are
// declared in pa_launch.h.  Not installed; not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

// Device-side statistics block; the energy histogram follows it directly in
// the workspace so one copy brings both back to the host.
struct DevStats {
    int32_t emin, emax;     // energy range of the population
    uint32_t r_new;         // total of the copy counts (resampling)
    uint32_t done;          // blocks of the statistics pass finished (zero between passes)
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

// Statistics taken in the sweep's epilogue: every wave adds the moment sums
// and the energy range of its replicas to slot (w mod kAccSlots) and their
// energies to histogram copy (w mod kAccHists), w being the wave's index in
// the launch, with device atomics spread over that many addresses so that
// they seldom meet; a gather pass sums slots and copies into the DevStats
// block and the histogram and leaves them cleared for the next sweep.  M^4
// (up to 2^64) is split so that both of its sums fit 64 bits: m4lo adds its
// low 32 bits, m4hi the rest (M^4 >> 32).
constexpr int kAccSlots = 256;
constexpr int kAccHists = 16;
struct AccSlot {
    uint64_t sumE, sumE2, sumAbsM, sumM2, m4lo, m4hi;
    int32_t emin, emax;
    uint64_t pad[9];  // one 128-byte cache line per slot
};
static_assert(sizeof(AccSlot) == 128, "accumulator slot layout");

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
    uint32_t key0, key1;    // Philox key: the run's seed
    uint32_t tag;           // 16 * run number: counter word 3 without the stream number
    uint32_t t2h, t2l;      // threshold T_2 = t2h * 2^16 + t2l  (t2h <= 65536)
    uint32_t t4h, t4l;      // threshold T_4  (heat-bath: U_2, U_4, each <= 2^31)
    uint32_t qcap;          // LDS path: tie-queue entries a wave may use before every lane decides its
                            // own ties (values at or above the queue size: the whole queue)
    int32_t init;           // 1: draw the initial state instead of loading spins
    const uint32_t* n_dev;  // if set: the population size is min(*n_dev, n_rep), read on the device
    const uint8_t* src;     // with parent: replica j starts from replica parent[j] of this store
    const uint32_t* parent; // (the resampling copy fused into the sweep's load); else NULL
    uint32_t stride;        // interleaved store: bytes from one site's row of spins (one byte per
                            // replica) to the next, the capacity rounded up to 64; 0 for the other stores
    AccSlot* acc;           // if set: the sweep's epilogue adds the population statistics to these
    uint32_t* acc_hist;     // kAccSlots slots and kAccHists histogram copies of nbins bins each
    int32_t nbins;          // (bit-sliced kernels only)
};

constexpr int kBlock = 256;     // threads per block of the population kernels

// Update rule of the sweep kernels.
enum Update : int {
    kMetropolis = 0,  // Metropolis with the bit-sliced Philox uniforms
    kHeatbath = 1,    // heat-bath with the same uniforms
    kLcg = 2          // Metropolis with uniforms from the in-line LCG variant
};

}  // namespace pa

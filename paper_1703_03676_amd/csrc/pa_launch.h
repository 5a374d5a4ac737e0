// Kernel launchers of the single-run path (defined in pa_sweep.hip and
// pa_kernels.hip, called by pa_api.hip).  Not installed; not part of the ABI.
#pragma once
#include "pa_internal.h"

namespace pa {

// Kernel launchers; each returns the launch status.
// `update` (pa::Update) selects Metropolis (thresholds T_2, T_4 in t2*/t4*),
// heat-bath (U_2, U_4) or the in-line LCG variant of Metropolis.
hipError_t launch_sweep(int L, int layout, int update, const SweepArgs& a, hipStream_t s);
// Statistics of a population (after the statistics block and the histogram
// have been cleared, by launch_stats_reset or launch_scatter): histogram,
// range, moment sums; parts holds ceil(n / kBlock) partials.  With n_dev the
// size is min(*n_dev, n), read on the device.  At most kStatsBlocks blocks,
// each taking chunks of kBlock replicas in turn.
constexpr int kStatsBlocks = 128;
hipError_t launch_stats(const int32_t* E, const int32_t* M, int32_t n, const uint32_t* n_dev, int32_t N,
                        DevStats* st, uint32_t* hist, int32_t nbins, int record, DevMhr mhr, StatsPart* parts,
                        void* host, hipStream_t s);
// With `host` (device view of pinned host memory of at least 64 + 4 nbins
// bytes) the statistics block and the histogram window [emin, emax] are also
// written there (bin b at byte 64 + 4 b).
hipError_t launch_counts(const int32_t* E, int32_t n, int32_t N, int32_t bmin, int32_t nwin, const uint32_t* tbl,
                         uint32_t step, uint32_t key0, uint32_t key1, uint32_t tag, uint32_t* counts, uint32_t* bsum,
                         hipStream_t s);
// Parent indices (children beyond cap are dropped), the total of the counts in
// st->r_new, and the statistics block and histogram cleared for the next
// statistics; then the replica copy of min(*n_new, cap) children, n_new read
// on the device.
// Up to kScanFreeBlocks blocks of counts, each scatter block sums the totals
// before it; beyond, a single-block scan of the totals runs first.
constexpr int kScanFreeBlocks = 1024;
hipError_t launch_scatter(const uint32_t* counts, uint32_t* bsum, int32_t n, int32_t cap, uint32_t* parent,
                          DevStats* st, uint32_t* hist, int32_t nbins, hipStream_t s);
hipError_t launch_copy(const uint8_t* src, const int32_t* Esrc, const int32_t* Msrc, const uint32_t* parent,
                       const uint32_t* n_new, int32_t cap, size_t rep_bytes, uint8_t* dst, int32_t* Edst,
                       int32_t* Mdst, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t s);
// Interleaved store (pa_rp.hip): the replica-parallel sweep (a.stride set, no
// fused gather), and the replica copy of resampling for that store.
hipError_t launch_sweep_rp(int L, int update, const SweepArgs& a, hipStream_t s);
hipError_t launch_copy_rp(const uint8_t* src, const int32_t* Esrc, const int32_t* Msrc, const uint32_t* parent,
                          const uint32_t* n_new, int32_t cap, int32_t N, uint32_t stride, uint8_t* dst, int32_t* Edst,
                          int32_t* Mdst, hipStream_t s);
// Statistics of the population a sweep launched with SweepArgs::acc has just
// swept: the epilogue's accumulators summed into st and the histogram window
// (hist cleared before, r_new kept), published to `host` as by launch_stats,
// and the accumulators left cleared.  launch_acc_reset clears them once.
hipError_t launch_stats_gather(AccSlot* acc, uint32_t* acc_hist, int32_t nbins, int32_t N, DevStats* st,
                               uint32_t* hist, void* host, hipStream_t s);
hipError_t launch_acc_reset(AccSlot* acc, uint32_t* acc_hist, int32_t nbins, hipStream_t s);
// Clears the range, the sums and the histogram (not r_new).
hipError_t launch_stats_reset(DevStats* st, uint32_t* hist, int32_t nbins, hipStream_t s);

}  // namespace pa

// C ABI of libpa (declared in include/pa.h): run state, validation, workspace
// layout, and the FP64 host arithmetic of the method (Metropolis thresholds,
// Eq. (Q) weights and resampling tables, observables, adaptive step,
// multi-histogram reweighting).  Everything per replica runs in the kernels of
// pa_kernels.hip; the host works only on energy bins and a few scalars.
//
// FP64 results that decide integers (thresholds, copy-count tables, the
// bisection) are computed with a fixed operation order, ascending energy bins,
// and without contraction (-ffp-contract=off), so a run is reproducible bit for
// bit from its seed and schedule.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pa.h"
#include "pa_host.h"
#include "pa_internal.h"
#include "pa_launch.h"

using pa::DevMhr;
using pa::DevStats;
namespace host = pa::host;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool lattice_supported(int L) { return L == 16 || L == 32 || L == 64 || L == 128 || L == 256; }

int32_t default_capacity(int32_t R)
{
    return R + (int32_t)std::ceil(10.0 * std::sqrt((double)R)) + 64;
}

struct Layout {
    size_t spin[2], E[2], M[2], counts, parent, bsum, tbl, stats, parts, acc, mhr, total;
    size_t rep_bytes;   // bytes of one replica
    uint32_t stride;    // interleaved store: bytes per site row (capacity rounded up to 64); else 0
    int32_t capacity, nbins, nblk;
};

// Validates the parameters and places every device array in the workspace.
bool make_layout(const pa_params* p, Layout* lo)
{
    if (!p || !lattice_supported(p->L) || p->R < 1) return false;
    if (p->layout != PA_SPIN_INT8 && p->layout != PA_SPIN_BITS && p->layout != PA_SPIN_INTERLEAVED) return false;
    if (p->flags & ~(uint32_t)(PA_FLAG_MHR | PA_FLAG_HEATBATH | PA_FLAG_LCG)) return false;
    if ((p->flags & PA_FLAG_HEATBATH) && (p->flags & PA_FLAG_LCG)) return false;
    if (p->run_id >= (1u << 28)) return false;
    const int64_t cap = p->capacity ? p->capacity : default_capacity(p->R);
    if (cap < p->R || cap > (int64_t)1 << 30) return false;
    const int64_t N = (int64_t)p->L * p->L;
    lo->capacity = (int32_t)cap;
    lo->nbins = (int32_t)N + 1;
    lo->rep_bytes = (p->layout == PA_SPIN_BITS) ? (size_t)N / 8 : (size_t)N;
    lo->stride = (p->layout == PA_SPIN_INTERLEAVED) ? (uint32_t)((cap + 63) / 64 * 64) : 0u;
    lo->nblk = (int32_t)((cap + pa::kBlock - 1) / pa::kBlock);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    for (int b = 0; b < 2; ++b) {
        lo->spin[b] = take(lo->stride ? (size_t)N * lo->stride : (size_t)cap * lo->rep_bytes);
        lo->E[b] = take((size_t)cap * 4);
        lo->M[b] = take((size_t)cap * 4);
    }
    lo->counts = take((size_t)cap * 4);
    lo->parent = take((size_t)cap * 4);
    lo->bsum = take((size_t)lo->nblk * 4 + 4);
    lo->tbl = take((size_t)lo->nbins * 8);
    lo->stats = take(sizeof(DevStats) + (size_t)lo->nbins * 4);
    lo->parts = take(sizeof(pa::StatsPart) * (size_t)lo->nblk);
    lo->acc = take(sizeof(pa::AccSlot) * pa::kAccSlots + (size_t)pa::kAccHists * (size_t)lo->nbins * 4);
    lo->mhr = (p->flags & PA_FLAG_MHR) ? take((size_t)lo->nbins * 40) : o;
    lo->total = o;
    return true;
}

// Per-call device scratch of the resampling path: copy counts and parent
// indices (one per replica of the capacity), block totals, the copy-count
// tables of the occupied energy window and the statistics partials, kept in
// the run's workspace.
struct Scratch {
    uint32_t *counts, *parent, *bsum, *tbl;
    pa::StatsPart* parts;
};

}  // namespace

struct pa_run {
    pa_params p;
    Layout lo;
    int L, N, nbins;
    hipStream_t stream;
    uint8_t* ws;
    uint8_t* spin[2];
    int32_t* E[2];
    int32_t* M[2];
    int cur;
    uint32_t *counts, *parent, *bsum, *tbl, *hist;
    DevStats* stats;
    pa::StatsPart* parts;
    pa::AccSlot* acc;      // statistics accumulated by the sweep's epilogue (pa_anneal)
    uint32_t* acc_hist;    // kAccHists histogram copies of nbins bins
    DevMhr mhr;
    // host-side run state
    int64_t R_cur;
    int32_t step;
    uint64_t sweeps;
    double beta, lnZ, lnQ_last;
    int32_t counts_n;
    bool broken;
    std::string last_error;
    uint64_t version, stats_version;
    uint64_t gathered_version = 0;  // population whose statistics the last sweep's epilogue publishes to hstats
    DevStats h_stats;
    std::vector<uint32_t> h_hist;
    uint8_t* pinned;
    size_t pinned_bytes;
    uint32_t* hstats = nullptr;  // pinned: statistics block + histogram window, written by the statistics kernel or gather
    void* hstats_dev = nullptr;  // device view of hstats
    hipEvent_t ev_rnew = nullptr;  // marks the resampling total in host memory
    hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;  // sweep timing in pa_anneal (created on first use)
    std::vector<double> m_beta, m_lnZ;
    std::vector<int64_t> m_R;
    std::vector<double> w;  // host scratch: weights per energy bin
    host::WeightTable wpre; // weights of the next fixed step, filled while the GPU sweeps
    uint32_t qcap = 0xFFFFFFFFu;  // tie-queue limit of the LDS-path sweeps (test hook)
    int32_t stats_path = PA_STATS_AUTO;  // where the statistics of a swept population are taken
};

namespace {

int update_of(const pa_params& p)
{
    if (p.flags & PA_FLAG_HEATBATH) return pa::kHeatbath;
    if (p.flags & PA_FLAG_LCG) return pa::kLcg;
    return pa::kMetropolis;
}

pa_status fail_hip(pa_run* r, hipError_t e, const char* what)
{
    r->broken = true;
    r->last_error = std::string(what) + ": " + hipGetErrorString(e);
    return PA_EHIP;
}

#define HIPCHK(expr)                                        \
    do {                                                    \
        const hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return fail_hip(r, e_, #expr); \
    } while (0)

pa_status usable(const pa_run* r)
{
    if (!r) return PA_EINVAL;
    return r->broken ? PA_ESTATE : PA_OK;
}

// Philox key (the seed) and the run's part of counter word 3 (16 * run_id),
// so that distinct (seed, run_id) pairs never share a random stream.
void key_of(const pa_run* r, uint32_t* k0, uint32_t* k1, uint32_t* tag)
{
    *k0 = (uint32_t)r->p.seed;
    *k1 = (uint32_t)(r->p.seed >> 32);
    *tag = r->p.run_id << 4;
}

// Whether the sweeps of this run take the statistics of the population they
// make in their epilogue (else a separate pass, stats_kernel, takes them).
// Measured per temperature step at theta = 1 (where the difference shows most),
// against the separate pass: faster with one replica per wave up to about
// 32768 replicas (L = 64: 1.6 us less at R = 20000; L = 128 within 1 us up to
// R = 30000) and at L = 256 at every R (15-100 us less); slower beyond (L =
// 128, R = 100000: 13 us more) and when a wave holds several replicas (L = 16,
// 32: 2-13 us more), where the epilogue's reductions cost as much as a short
// sweep.
bool stats_in_epilogue(const pa_run* r)
{
    if (r->p.layout == PA_SPIN_INTERLEAVED) return false;
    if (r->stats_path != PA_STATS_AUTO) return r->stats_path == PA_STATS_EPILOGUE;
    return r->L == 256 || (r->L >= 64 && r->p.R <= 32768);
}

// The sweep kernel of the run's spin store: bit-sliced (int8 and bit stores)
// or replica-parallel (interleaved store).
hipError_t launch_sweep_of(const pa_run* r, pa::SweepArgs& a)
{
    if (r->p.layout == PA_SPIN_INTERLEAVED) {
        a.stride = r->lo.stride;
        return pa::launch_sweep_rp(r->L, update_of(r->p), a, r->stream);
    }
    return pa::launch_sweep(r->L, r->p.layout, update_of(r->p), a, r->stream);
}

// Queues nsweeps sweeps of the current population (or, with `init`, the
// initial state; with neither, the recount of E and M).  Where the run takes
// statistics in the epilogue (stats_in_epilogue), the gather publishes those
// of population version `ver` to hstats, so they need no separate pass
// (refresh_stats).
pa_status launch_sweeps(pa_run* r, int32_t nsweeps, bool init, uint64_t ver)
{
    pa::SweepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.spin = r->spin[r->cur];
    a.E = r->E[r->cur];
    a.M = r->M[r->cur];
    a.n_rep = (int32_t)r->R_cur;
    a.nsweeps = nsweeps;
    a.g0 = (uint32_t)r->sweeps;
    key_of(r, &a.key0, &a.key1, &a.tag);
    const bool hb = (r->p.flags & PA_FLAG_HEATBATH) != 0;
    host::sweep_thresholds(hb, r->beta, &a.t2h, &a.t2l, &a.t4h, &a.t4l);
    a.init = init ? 1 : 0;
    a.qcap = r->qcap;
    const bool epilogue = stats_in_epilogue(r);
    if (epilogue) {
        a.acc = r->acc;
        a.acc_hist = r->acc_hist;
        a.nbins = r->nbins;
    }
    r->gathered_version = 0;
    HIPCHK(launch_sweep_of(r, a));
    if (epilogue) {
        HIPCHK(pa::launch_stats_gather(r->acc, r->acc_hist, r->nbins, r->N, r->stats, r->hist, r->hstats_dev,
                                       r->stream));
        r->gathered_version = ver;
    }
    return PA_OK;
}

// Reads the statistics block and the histogram window that the statistics
// kernel or the gather of a sweep's epilogue wrote to pinned host memory
// (after the stream has been synchronised); bins outside [emin, emax] of
// h_hist are not used.
pa_status read_host_stats(pa_run* r, DevStats* out)
{
    std::memcpy(out, r->hstats, sizeof(DevStats));
    if (out->emin < -2 * r->N || out->emax > 2 * r->N || out->emin > out->emax) {
        r->broken = true;
        r->last_error = "population energies out of range";
        return PA_ESTATE;
    }
    const int b0 = (out->emin + 2 * r->N) / 4, b1 = (out->emax + 2 * r->N) / 4;
    std::memcpy(r->h_hist.data() + b0, r->hstats + sizeof(DevStats) / 4 + b0, (size_t)(b1 - b0 + 1) * 4);
    return PA_OK;
}

Scratch run_scratch(const pa_run* r) { return Scratch{r->counts, r->parent, r->bsum, r->tbl, r->parts}; }

// Brings the histogram and the integer sums of the current population to the
// host: from the host copy if it is current, else from the gather that the
// epilogue of the sweep which made this population queued, else from the
// statistics kernel.  With `record` the measurement is also added to the
// multi-histogram accumulators (only then is a cached result not reused).
pa_status refresh_stats(pa_run* r, bool record, pa::StatsPart* parts)
{
    if (!record && r->stats_version == r->version) return PA_OK;
    if (record || r->gathered_version != r->version) {
        HIPCHK(pa::launch_stats_reset(r->stats, r->hist, r->nbins, r->stream));
        HIPCHK(pa::launch_stats(r->E[r->cur], r->M[r->cur], (int32_t)r->R_cur, nullptr, r->N, r->stats, r->hist,
                                r->nbins, record ? 1 : 0, r->mhr, parts, r->hstats_dev, r->stream));
    }  // else the epilogue of the sweep that made this population has queued them
    HIPCHK(hipStreamSynchronize(r->stream));
    const pa_status st = read_host_stats(r, &r->h_stats);
    if (st != PA_OK) return st;
    r->stats_version = r->version;
    return PA_OK;
}

host::Hist window(const pa_run* r) { return host::hist_window(r->h_hist.data(), r->h_stats, r->N); }

// Queues the resampling of the current population to beta_next into the
// other ping-pong buffer: Eq. (Q) with the E_min shift and the tables of Eq.
// (resampling factors) on the host (from the host copy of the statistics),
// then copy counts, their prefix sum (the total goes to stats->r_new), parent
// indices and (with `copy`) the replica copy.  The scatter and the copy read
// the total on the device and are clamped to the capacity, so they can run
// before the host has checked it; nothing of the current buffer changes.
// Without `copy` the caller's next sweep gathers the parents itself.  The
// scatter also clears the statistics block and the histogram, so the
// statistics of the resampled population need no separate reset.
pa_status queue_resample(pa_run* r, double beta_next, bool copy, double* lnQ, int32_t* Emin, const Scratch& sc)
{
    const host::Hist h = window(r);
    const int bmin = h.bmin, nwin = h.bmax - h.bmin + 1;
    *Emin = h.energy(bmin);
    uint32_t* tab = (uint32_t*)r->pinned;
    *lnQ = host::resample_tables(h, r->p.R, r->R_cur, beta_next - r->beta, tab, r->w, &r->wpre);
    HIPCHK(hipMemcpyAsync(sc.tbl, tab, (size_t)nwin * 8, hipMemcpyHostToDevice, r->stream));
    uint32_t k0, k1, tag;
    key_of(r, &k0, &k1, &tag);
    const int32_t n = (int32_t)r->R_cur;
    const int nxt = r->cur ^ 1;
    HIPCHK(pa::launch_counts(r->E[r->cur], n, r->N, bmin, nwin, sc.tbl, (uint32_t)(r->step + 1), k0, k1, tag,
                             sc.counts, sc.bsum, r->stream));
    HIPCHK(pa::launch_scatter(sc.counts, sc.bsum, n, r->lo.capacity, sc.parent, r->stats, r->hist, r->nbins,
                              r->stream));
    if (copy && r->p.layout == PA_SPIN_INTERLEAVED)
        HIPCHK(pa::launch_copy_rp(r->spin[r->cur], r->E[r->cur], r->M[r->cur], sc.parent, &r->stats->r_new,
                                  r->lo.capacity, r->N, r->lo.stride, r->spin[nxt], r->E[nxt], r->M[nxt],
                                  r->stream));
    else if (copy)
        HIPCHK(pa::launch_copy(r->spin[r->cur], r->E[r->cur], r->M[r->cur], sc.parent, &r->stats->r_new,
                               r->lo.capacity, r->lo.rep_bytes, r->spin[nxt], r->E[nxt], r->M[nxt], r->stream));
    r->counts_n = n;
    return PA_OK;
}

// Makes the resampled population current (after its total has been checked).
void commit_resample(pa_run* r, double beta_next, double lnQ, int64_t R_new)
{
    r->cur ^= 1;
    r->R_cur = R_new;
    r->step += 1;
    r->beta = beta_next;
    r->lnZ += lnQ;
    r->lnQ_last = lnQ;
    r->version += 1;
}

}  // namespace

extern "C" {

size_t pa_workspace_bytes(const pa_params* p)
{
    Layout lo;
    return make_layout(p, &lo) ? lo.total : 0;
}

const char* pa_strerror(pa_status s)
{
    switch (s) {
    case PA_OK: return "success";
    case PA_EINVAL: return "invalid argument";
    case PA_ENOMEM: return "workspace too small or host allocation failed";
    case PA_ECAPACITY: return "population exceeds capacity";
    case PA_EHIP: return "HIP runtime error";
    case PA_ESTATE: return "run unusable or call out of order";
    case PA_EEXTINCT: return "resampling would leave no replica";
    }
    return "unknown status";
}

const char* pa_last_error(const pa_run* r) { return r ? r->last_error.c_str() : ""; }

pa_status pa_init(const pa_params* p, void* d_workspace, size_t bytes, void* hip_stream, pa_run** out)
{
    if (!out) return PA_EINVAL;
    *out = nullptr;
    Layout lo;
    if (!make_layout(p, &lo) || !d_workspace) return PA_EINVAL;
    if (((uintptr_t)d_workspace) % kAlign != 0) return PA_EINVAL;
    if (bytes < lo.total) return PA_ENOMEM;
    pa_run* r = new (std::nothrow) pa_run();
    if (!r) return PA_ENOMEM;
    r->p = *p;
    r->p.capacity = lo.capacity;
    r->lo = lo;
    r->L = p->L;
    r->N = p->L * p->L;
    r->nbins = lo.nbins;
    r->stream = (hipStream_t)hip_stream;
    uint8_t* ws = (uint8_t*)d_workspace;
    r->ws = ws;
    for (int b = 0; b < 2; ++b) {
        r->spin[b] = ws + lo.spin[b];
        r->E[b] = (int32_t*)(ws + lo.E[b]);
        r->M[b] = (int32_t*)(ws + lo.M[b]);
    }
    r->counts = (uint32_t*)(ws + lo.counts);
    r->parent = (uint32_t*)(ws + lo.parent);
    r->bsum = (uint32_t*)(ws + lo.bsum);
    r->tbl = (uint32_t*)(ws + lo.tbl);
    r->stats = (DevStats*)(ws + lo.stats);
    r->hist = (uint32_t*)(ws + lo.stats + sizeof(DevStats));
    r->parts = (pa::StatsPart*)(ws + lo.parts);
    r->acc = (pa::AccSlot*)(ws + lo.acc);
    r->acc_hist = (uint32_t*)(ws + lo.acc + sizeof(pa::AccSlot) * pa::kAccSlots);
    if (p->flags & PA_FLAG_MHR) {
        uint64_t* m = (uint64_t*)(ws + lo.mhr);
        r->mhr.H = m;
        r->mhr.SA = m + r->nbins;
        r->mhr.SM2 = m + 2 * (size_t)r->nbins;
        r->mhr.SM4 = m + 3 * (size_t)r->nbins;
    } else {
        r->mhr = DevMhr{nullptr, nullptr, nullptr, nullptr};
    }
    r->h_hist.assign((size_t)r->nbins, 0u);
    r->pinned_bytes = sizeof(DevStats) + (size_t)r->nbins * 8;
    if (hipHostMalloc((void**)&r->pinned, r->pinned_bytes, hipHostMallocDefault) != hipSuccess) {
        delete r;
        return PA_ENOMEM;
    }
    if (hipHostMalloc((void**)&r->hstats, sizeof(DevStats) + (size_t)r->nbins * 4, hipHostMallocMapped) !=
        hipSuccess) {
        (void)hipHostFree(r->pinned);
        delete r;
        return PA_ENOMEM;
    }
    if (hipHostGetDevicePointer(&r->hstats_dev, r->hstats, 0) != hipSuccess ||
        hipEventCreateWithFlags(&r->ev_rnew, hipEventDisableTiming) != hipSuccess) {
        (void)hipHostFree(r->hstats);
        (void)hipHostFree(r->pinned);
        delete r;
        return PA_EHIP;
    }
    r->cur = 0;
    r->R_cur = p->R;
    r->step = 0;
    r->sweeps = 0;
    r->beta = 0.0;
    r->lnZ = (double)r->N * std::log(2.0);
    r->lnQ_last = 0.0;
    r->counts_n = 0;
    r->version = 1;
    r->stats_version = 0;
    *out = r;
    {
        const hipError_t e = pa::launch_acc_reset(r->acc, r->acc_hist, r->nbins, r->stream);
        if (e != hipSuccess) return fail_hip(r, e, "clear the sweep's statistics accumulators");
    }
    if (p->flags & PA_FLAG_MHR) {
        pa_status st = PA_OK;
        const hipError_t e = pa::launch_fill_u32((uint32_t*)r->mhr.H, 0u, (size_t)r->nbins * 10, r->stream);
        if (e != hipSuccess) st = fail_hip(r, e, "zero multi-histogram accumulators");
        if (st != PA_OK) return st;
    }
    return launch_sweeps(r, 0, true, r->version);
}

pa_status pa_sweep(pa_run* r, int32_t nsweeps)
{
    pa_status st = usable(r);
    if (st != PA_OK) return st;
    if (nsweeps < 0 || r->sweeps + (uint64_t)nsweeps >= ((uint64_t)1 << 31)) return PA_EINVAL;
    if (nsweeps == 0) return PA_OK;
    st = launch_sweeps(r, nsweeps, false, r->version + 1);
    if (st != PA_OK) return st;
    r->sweeps += (uint64_t)nsweeps;
    r->version += 1;
    return PA_OK;
}

// pa_resample: the statistics, the copy counts, their prefix sum, the parent
// indices and the replica copy, with the per-call device scratch `sc`.
static pa_status resample_with(pa_run* r, double beta_next, pa_resample_info* out, const Scratch& sc)
{
    pa_status st = usable(r);
    if (st != PA_OK) return st;
    if (!std::isfinite(beta_next) || beta_next < r->beta) return PA_EINVAL;
    st = refresh_stats(r, false, sc.parts);
    if (st != PA_OK) return st;

    double lnQ;
    int32_t Emin;
    st = queue_resample(r, beta_next, true, &lnQ, &Emin, sc);
    if (st != PA_OK) return st;
    // the host waits only for the total; the copy runs on meanwhile
    uint32_t* rn = (uint32_t*)(r->pinned + r->pinned_bytes - 8);
    HIPCHK(hipMemcpyAsync(rn, &r->stats->r_new, 4, hipMemcpyDeviceToHost, r->stream));
    HIPCHK(hipEventRecord(r->ev_rnew, r->stream));
    HIPCHK(hipEventSynchronize(r->ev_rnew));
    const int64_t R_new = *rn;
    r->stats_version = 0;  // the stats block now holds the resampling total
    if (R_new > r->lo.capacity) return PA_ECAPACITY;
    if (R_new == 0) return PA_EEXTINCT;
    commit_resample(r, beta_next, lnQ, R_new);
    if (out) {
        out->lnQ = lnQ;
        out->R_new = R_new;
        out->E_min = Emin;
    }
    return PA_OK;
}

pa_status pa_resample(pa_run* r, double beta_next, pa_resample_info* out)
{
    const pa_status st = usable(r);
    if (st != PA_OK) return st;
    return resample_with(r, beta_next, out, run_scratch(r));
}

pa_status pa_anneal(pa_run* r, const pa_schedule* sc, int32_t max_steps, pa_obs* out, float* sweep_ms, int32_t cap,
                    int32_t* nsteps)
{
    if (nsteps) *nsteps = 0;
    pa_status st = usable(r);
    if (st != PA_OK) return st;
    if (!sc || max_steps < 0 || cap < 0 || (cap > 0 && !out) || sc->theta < 0 || !std::isfinite(sc->beta_f) ||
        sc->beta_f < r->beta)
        return PA_EINVAL;
    if (sc->mode == PA_STEP_FIXED) {
        if (!(sc->dbeta > 0.0) || !std::isfinite(sc->dbeta)) return PA_EINVAL;
    } else if (sc->mode == PA_STEP_ADAPTIVE) {
        if (!(sc->alpha_star > 0.0 && sc->alpha_star < 1.0)) return PA_EINVAL;
    } else {
        return PA_EINVAL;
    }
    const bool record = (r->p.flags & PA_FLAG_MHR) != 0;
    st = refresh_stats(r, false, r->parts);
    if (st != PA_OK) return st;
    if (sweep_ms && cap > 0 && !r->ev_t0) {
        HIPCHK(hipEventCreate(&r->ev_t0));
        HIPCHK(hipEventCreate(&r->ev_t1));
    }
    uint32_t k0, k1, tag;
    key_of(r, &k0, &k1, &tag);
    int32_t done = 0;
    // fixed schedule: inverse temperature of step i, not below the one before
    auto fixed_beta = [&](int64_t i, double prev) {
        const int64_t nb = std::max<int64_t>(1, std::llround(sc->beta_f / sc->dbeta));
        double b = (i >= nb) ? sc->beta_f : (double)i * sc->dbeta;
        if (b > sc->beta_f) b = sc->beta_f;
        return b < prev ? prev : b;
    };
    while (done < max_steps && r->beta < sc->beta_f) {
        if (r->sweeps + (uint64_t)sc->theta >= ((uint64_t)1 << 31)) return PA_EINVAL;
        // next inverse temperature from the host copy of the current statistics
        const host::Hist h = window(r);
        double bn;
        if (sc->mode == PA_STEP_FIXED) {
            bn = fixed_beta((int64_t)r->step + 1, r->beta);
        } else if (!host::adapt_beta(h, r->p.R, r->R_cur, r->beta, sc->beta_f, sc->alpha_star, &bn, nullptr, r->w)) {
            return PA_EINVAL;
        }
        // Resampling into the other buffer, the sweeps and the statistics
        // there are all queued before the host sees the new population size,
        // which the kernels read on the device; a refused step leaves `cur`.
        double lnQ;
        int32_t Emin;
        // with sweeps, the sweep kernel loads every child from its parent: the
        // replica copy and the sweep's load are one pass over the store (the
        // replica-parallel sweep of the interleaved store works in place and
        // takes the copy first)
        const bool gather = sc->theta > 0 && r->p.layout != PA_SPIN_INTERLEAVED;
        const bool epilogue = sc->theta > 0 && stats_in_epilogue(r);
        st = queue_resample(r, bn, !gather, &lnQ, &Emin, run_scratch(r));
        if (st != PA_OK) return st;
        const int nxt = r->cur ^ 1;
        const uint32_t* n_dev = &r->stats->r_new;
        if (sc->theta > 0) {
            pa::SweepArgs a;
            std::memset(&a, 0, sizeof(a));
            a.spin = r->spin[nxt];
            a.E = r->E[nxt];
            a.M = r->M[nxt];
            a.n_rep = r->lo.capacity;
            a.n_dev = n_dev;
            a.src = gather ? r->spin[r->cur] : nullptr;
            a.parent = gather ? r->parent : nullptr;
            a.nsweeps = sc->theta;
            a.g0 = (uint32_t)r->sweeps;
            a.key0 = k0;
            a.key1 = k1;
            a.tag = tag;
            a.qcap = r->qcap;
            if (epilogue) {  // the statistics of the new population in the sweep's epilogue
                a.acc = r->acc;
                a.acc_hist = r->acc_hist;
                a.nbins = r->nbins;
            }
            const bool hb = (r->p.flags & PA_FLAG_HEATBATH) != 0;
            host::sweep_thresholds(hb, bn, &a.t2h, &a.t2l, &a.t4h, &a.t4l);
            const bool timed = sweep_ms && done < cap;
            if (timed) HIPCHK(hipEventRecord(r->ev_t0, r->stream));
            HIPCHK(launch_sweep_of(r, a));
            if (timed) HIPCHK(hipEventRecord(r->ev_t1, r->stream));
        }
        // (the scatter of queue_resample has cleared the statistics); they are
        // published to hstats, which then no longer holds those of the current
        // population, even if this step is refused
        r->gathered_version = 0;
        if (epilogue)
            HIPCHK(pa::launch_stats_gather(r->acc, r->acc_hist, r->nbins, r->N, r->stats, r->hist, r->hstats_dev,
                                           r->stream));
        else
            HIPCHK(pa::launch_stats(r->E[nxt], r->M[nxt], r->lo.capacity, n_dev, r->N, r->stats, r->hist, r->nbins,
                                    0, r->mhr, r->parts, r->hstats_dev, r->stream));
        if (sc->mode == PA_STEP_FIXED && bn < sc->beta_f) {
            // while the GPU sweeps: the weights of the next step (its dbeta is
            // known in advance), over the current window plus a margin
            const double db = fixed_beta((int64_t)r->step + 2, bn) - bn;
            const size_t want = (size_t)(h.bmax - h.bmin + 1) * 5 / 4 + 16;
            if (!r->wpre.covers(db, (int)want)) r->wpre.fill(db, want);
        }
        HIPCHK(hipStreamSynchronize(r->stream));
        const int64_t R_new = reinterpret_cast<const DevStats*>(r->hstats)->r_new;
        if (R_new > r->lo.capacity || R_new == 0) {
            r->stats_version = 0;  // the statistics block holds the refused population
            return R_new == 0 ? PA_EEXTINCT : PA_ECAPACITY;
        }
        commit_resample(r, bn, lnQ, R_new);
        r->sweeps += (uint64_t)sc->theta;
        r->version += 1;
        st = read_host_stats(r, &r->h_stats);
        if (st != PA_OK) return st;
        r->stats_version = r->version;
        // measurement (Eq. (observables)); the multi-histogram record is queued
        // without a wait, since its statistics equal the ones just read
        if (record) {
            HIPCHK(pa::launch_stats_reset(r->stats, r->hist, r->nbins, r->stream));
            HIPCHK(pa::launch_stats(r->E[r->cur], r->M[r->cur], (int32_t)r->R_cur, nullptr, r->N, r->stats, r->hist,
                                    r->nbins, 1, r->mhr, r->parts, nullptr, r->stream));
            r->m_beta.push_back(r->beta);
            r->m_lnZ.push_back(r->lnZ);
            r->m_R.push_back(r->R_cur);
        }
        if (done < cap) host::observables(r->h_stats, r->R_cur, r->N, r->beta, r->lnZ, r->lnQ_last, &out[done]);
        if (sweep_ms && done < cap) {
            float ms = 0.0f;
            if (sc->theta > 0) HIPCHK(hipEventElapsedTime(&ms, r->ev_t0, r->ev_t1));
            sweep_ms[done] = ms;
        }
        ++done;
        if (nsteps) *nsteps = done;
    }
    return PA_OK;
}

pa_status pa_alpha(pa_run* r, double beta_prime, double* alpha)
{
    pa_status st = usable(r);
    if (st != PA_OK) return st;
    if (!alpha || !std::isfinite(beta_prime)) return PA_EINVAL;
    st = refresh_stats(r, false, r->parts);
    if (st != PA_OK) return st;
    std::vector<double> w;
    *alpha = host::overlap(window(r), r->p.R, r->R_cur, beta_prime - r->beta, w);
    return PA_OK;
}

pa_status pa_adapt_beta(pa_run* r, double alpha_star, double beta_f, double* beta_next, double* alpha_at_next)
{
    pa_status st = usable(r);
    if (st != PA_OK) return st;
    if (!beta_next || !(alpha_star > 0.0 && alpha_star < 1.0) || !std::isfinite(beta_f) || beta_f < r->beta)
        return PA_EINVAL;
    st = refresh_stats(r, false, r->parts);
    if (st != PA_OK) return st;
    std::vector<double> w;
    if (!host::adapt_beta(window(r), r->p.R, r->R_cur, r->beta, beta_f, alpha_star, beta_next, alpha_at_next, w))
        return PA_EINVAL;
    return PA_OK;
}

pa_status pa_observables(pa_run* r, pa_obs* o)
{
    pa_status st = usable(r);
    if (st != PA_OK) return st;
    if (!o) return PA_EINVAL;
    const bool record = (r->p.flags & PA_FLAG_MHR) != 0;
    st = refresh_stats(r, record, r->parts);
    if (st != PA_OK) return st;
    host::observables(r->h_stats, r->R_cur, r->N, r->beta, r->lnZ, r->lnQ_last, o);
    if (record) {
        r->m_beta.push_back(r->beta);
        r->m_lnZ.push_back(r->lnZ);
        r->m_R.push_back(r->R_cur);
    }
    return PA_OK;
}

pa_status pa_reweight(pa_run* r, const double* betas, int32_t nb, pa_obs* out)
{
    pa_status st = usable(r);
    if (st != PA_OK) return st;
    if (!(r->p.flags & PA_FLAG_MHR) || nb < 0 || (nb > 0 && (!betas || !out)) || r->m_beta.empty())
        return PA_EINVAL;
    const size_t nbins = (size_t)r->nbins;
    std::vector<uint64_t> acc(5 * nbins);
    HIPCHK(hipMemcpyAsync(acc.data(), r->mhr.H, acc.size() * 8, hipMemcpyDeviceToHost, r->stream));
    HIPCHK(hipStreamSynchronize(r->stream));
    const uint64_t* H = acc.data();
    host::reweight(r->N, H, H + nbins, H + 2 * nbins, H + 3 * nbins, r->m_beta, r->m_lnZ, r->m_R, betas, nb, out);
    return PA_OK;
}

pa_status pa_weighted_average(int32_t N, int32_t nruns, int32_t nb, const pa_obs* obs, pa_obs* out)
{
    if (N < 1 || nruns < 1 || nb < 0 || (nb > 0 && (!obs || !out))) return PA_EINVAL;
    return host::weighted_average(N, nruns, nb, obs, out) ? PA_OK : PA_EINVAL;
}

pa_status pa_set_tie_queue_cap(pa_run* r, int32_t cap)
{
    pa_status st = usable(r);
    if (st != PA_OK) return st;
    if (cap < 0) return PA_EINVAL;
    r->qcap = (uint32_t)cap;
    return PA_OK;
}

pa_status pa_set_stats_path(pa_run* r, int32_t mode)
{
    pa_status st = usable(r);
    if (st != PA_OK) return st;
    if (mode != PA_STATS_AUTO && mode != PA_STATS_EPILOGUE && mode != PA_STATS_PASS) return PA_EINVAL;
    r->stats_path = mode;
    return PA_OK;
}

pa_status pa_state(const pa_run* r, pa_state_info* out)
{
    if (!r || !out) return PA_EINVAL;
    out->R = r->R_cur;
    out->step = r->step;
    out->sweeps = r->sweeps;
    out->beta = r->beta;
    out->lnZ = r->lnZ;
    return PA_OK;
}

pa_status pa_free(pa_run* r)
{
    if (!r) return PA_OK;
    if (r->ev_rnew) (void)hipEventDestroy(r->ev_rnew);
    if (r->ev_t0) (void)hipEventDestroy(r->ev_t0);
    if (r->ev_t1) (void)hipEventDestroy(r->ev_t1);
    if (r->pinned) (void)hipHostFree(r->pinned);
    if (r->hstats) (void)hipHostFree(r->hstats);
    delete r;
    return PA_OK;
}

pa_status pa_download_population(pa_run* r, int8_t* spins, int32_t* E, int32_t* M)
{
    pa_status st = usable(r);
    if (st != PA_OK) return st;
    const size_t n = (size_t)r->R_cur;
    if (E) HIPCHK(hipMemcpyAsync(E, r->E[r->cur], n * 4, hipMemcpyDeviceToHost, r->stream));
    if (M) HIPCHK(hipMemcpyAsync(M, r->M[r->cur], n * 4, hipMemcpyDeviceToHost, r->stream));
    if (spins) {
        if (r->p.layout == PA_SPIN_INT8) {
            HIPCHK(hipMemcpyAsync(spins, r->spin[r->cur], n * (size_t)r->N, hipMemcpyDeviceToHost, r->stream));
        } else if (r->p.layout == PA_SPIN_INTERLEAVED) {
            // site rows of the first n replicas, then [site][replica] -> [replica][site]
            std::vector<int8_t> rows(n * (size_t)r->N);
            HIPCHK(hipMemcpy2DAsync(rows.data(), n, r->spin[r->cur], r->lo.stride, n, (size_t)r->N,
                                    hipMemcpyDeviceToHost, r->stream));
            HIPCHK(hipStreamSynchronize(r->stream));
            host::interleaved_to_int8(rows.data(), (size_t)r->N, n, spins);
        } else {
            std::vector<uint32_t> words(n * (size_t)r->N / 32);
            HIPCHK(hipMemcpyAsync(words.data(), r->spin[r->cur], words.size() * 4, hipMemcpyDeviceToHost, r->stream));
            HIPCHK(hipStreamSynchronize(r->stream));
            host::bits_to_int8(words.data(), r->L, n, spins);
        }
    }
    HIPCHK(hipStreamSynchronize(r->stream));
    return PA_OK;
}

pa_status pa_download_replicas(pa_run* r, const int32_t* idx, int32_t n, int8_t* spins, int32_t* E, int32_t* M)
{
    pa_status st = usable(r);
    if (st != PA_OK) return st;
    if (n < 0 || (n > 0 && (!idx || !spins))) return PA_EINVAL;
    for (int32_t k = 0; k < n; ++k)
        if (idx[k] < 0 || idx[k] >= r->R_cur) return PA_EINVAL;
    const size_t rb = r->lo.rep_bytes;
    std::vector<uint8_t> raw((size_t)n * rb);
    std::vector<int32_t> e((size_t)n), m((size_t)n);
    for (int32_t k = 0; k < n; ++k) {
        const size_t j = (size_t)idx[k];
        if (r->p.layout == PA_SPIN_INTERLEAVED)  // byte j of every site row
            HIPCHK(hipMemcpy2DAsync(raw.data() + (size_t)k * rb, 1, r->spin[r->cur] + j, r->lo.stride, 1,
                                    (size_t)r->N, hipMemcpyDeviceToHost, r->stream));
        else
            HIPCHK(hipMemcpyAsync(raw.data() + (size_t)k * rb, r->spin[r->cur] + j * rb, rb, hipMemcpyDeviceToHost,
                                  r->stream));
        HIPCHK(hipMemcpyAsync(&e[(size_t)k], r->E[r->cur] + j, 4, hipMemcpyDeviceToHost, r->stream));
        HIPCHK(hipMemcpyAsync(&m[(size_t)k], r->M[r->cur] + j, 4, hipMemcpyDeviceToHost, r->stream));
    }
    HIPCHK(hipStreamSynchronize(r->stream));
    if (r->p.layout != PA_SPIN_BITS)
        std::memcpy(spins, raw.data(), raw.size());
    else
        host::bits_to_int8(reinterpret_cast<const uint32_t*>(raw.data()), r->L, (size_t)n, spins);
    if (E) std::memcpy(E, e.data(), e.size() * 4);
    if (M) std::memcpy(M, m.data(), m.size() * 4);
    return PA_OK;
}

pa_status pa_upload_population(pa_run* r, int32_t R_cur, const int8_t* spins, int32_t step, uint64_t sweeps,
                               double beta, double lnZ)
{
    pa_status st = usable(r);
    if (st != PA_OK) return st;
    if (!spins || R_cur < 1 || R_cur > r->lo.capacity || step < 0 || !std::isfinite(beta) || beta < 0.0 ||
        sweeps >= ((uint64_t)1 << 31))
        return PA_EINVAL;
    const size_t n = (size_t)R_cur, N = (size_t)r->N;
    for (size_t i = 0; i < n * N; ++i)
        if (spins[i] != 1 && spins[i] != -1) return PA_EINVAL;
    if (r->p.layout == PA_SPIN_INT8) {
        HIPCHK(hipMemcpyAsync(r->spin[r->cur], spins, n * N, hipMemcpyHostToDevice, r->stream));
        HIPCHK(hipStreamSynchronize(r->stream));
    } else if (r->p.layout == PA_SPIN_INTERLEAVED) {
        std::vector<int8_t> rows(n * N);
        host::int8_to_interleaved(spins, N, n, rows.data());
        HIPCHK(hipMemcpy2DAsync(r->spin[r->cur], r->lo.stride, rows.data(), n, n, N, hipMemcpyHostToDevice,
                                r->stream));
        HIPCHK(hipStreamSynchronize(r->stream));
    } else {
        std::vector<uint32_t> words(n * N / 32, 0u);
        host::int8_to_bits(spins, r->L, n, words.data());
        HIPCHK(hipMemcpyAsync(r->spin[r->cur], words.data(), words.size() * 4, hipMemcpyHostToDevice, r->stream));
        HIPCHK(hipStreamSynchronize(r->stream));
    }
    r->R_cur = R_cur;
    r->step = step;
    r->sweeps = sweeps;
    r->beta = beta;
    r->lnZ = lnZ;
    r->lnQ_last = 0.0;
    r->version += 1;
    return launch_sweeps(r, 0, false, r->version);  // recount E and M on the device
}

pa_status pa_download_counts(pa_run* r, uint32_t* counts, int32_t* n)
{
    pa_status st = usable(r);
    if (st != PA_OK) return st;
    if (!counts || !n) return PA_EINVAL;
    *n = r->counts_n;
    if (r->counts_n > 0) {
        HIPCHK(hipMemcpyAsync(counts, r->counts, (size_t)r->counts_n * 4, hipMemcpyDeviceToHost, r->stream));
        HIPCHK(hipStreamSynchronize(r->stream));
    }
    return PA_OK;
}

}  // extern "C"

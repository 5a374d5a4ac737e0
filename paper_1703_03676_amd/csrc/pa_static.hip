// Population statistics for callers that cannot allocate memory: the
// observables of Eq. (observables), (free energy) and (entropy) of a population
// held in caller buffers, with the statistics kernel's partial sums, its
// statistics block and the energy histogram in a statically allocated device
// array instead of a run's workspace.
//
// The array lives in this translation unit.  Host code never passes its name
// to a kernel: on the host the name is only a stand-in for the symbol.  The
// device address of each GPU's copy comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that address reaches the
// kernels and the copies.
#include <mutex>

#include "pa.h"
#include "pa_host.h"
#include "pa_internal.h"
#include "pa_launch.h"

namespace {

using pa::DevStats;
using pa::StatsPart;

// Layout of the array: statistics block, partials of up to kMaxParts chunks of
// kBlock replicas, energy histogram of up to kMaxBins bins (L = 256).
constexpr int kMaxParts = PA_STATIC_MAX_R / pa::kBlock;
constexpr int kMaxBins = 256 * 256 + 1;
constexpr size_t kOffParts = 256;
constexpr size_t kOffHist = kOffParts + (size_t)kMaxParts * sizeof(StatsPart);
constexpr size_t kScratchBytes = kOffHist + (((size_t)kMaxBins * 4 + 255) / 256) * 256;
static_assert(PA_STATIC_MAX_R % pa::kBlock == 0, "whole chunks");
static_assert(kOffHist % 256 == 0, "histogram alignment");

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t* g_ptr[kMaxDevices];  // device address of `scratch` on each GPU (null until looked up)

// Device address of this GPU's scratch, looked up on first use with the device
// current (the caller's current device is the one the stream belongs to).
hipError_t scratch_ptr(uint8_t** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = static_cast<uint8_t*>(p);
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" size_t pa_static_scratch_bytes(void) { return kScratchBytes; }

extern "C" pa_status pa_observables_static(int32_t L, int32_t R, const int32_t* d_E, const int32_t* d_M, double beta,
                                           double lnZ, double lnQ, void* hip_stream, pa_obs* out)
{
    if (!(L == 16 || L == 32 || L == 64 || L == 128 || L == 256)) return PA_EINVAL;
    if (R < 1 || R > PA_STATIC_MAX_R || !d_E || !d_M || !out) return PA_EINVAL;
    if (!std::isfinite(beta) || !std::isfinite(lnZ)) return PA_EINVAL;
    const int32_t N = L * L, nbins = N + 1;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    uint8_t* base = nullptr;
    if (scratch_ptr(&base) != hipSuccess) return PA_EHIP;
    DevStats* st = reinterpret_cast<DevStats*>(base);
    StatsPart* parts = reinterpret_cast<StatsPart*>(base + kOffParts);
    uint32_t* hist = reinterpret_cast<uint32_t*>(base + kOffHist);
    // the statistics block and the histogram start from zero (a fill kernel;
    // the array keeps whatever the previous call on this GPU left in it)
    if (pa::launch_stats_reset(st, hist, nbins, s) != hipSuccess) return PA_EHIP;
    if (pa::launch_stats(d_E, d_M, R, nullptr, N, st, hist, nbins, 0, pa::DevMhr{}, parts, nullptr, s) != hipSuccess)
        return PA_EHIP;
    DevStats h;
    if (hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return PA_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return PA_EHIP;
    pa::host::observables(h, R, N, beta, lnZ, lnQ, out);
    return PA_OK;
}

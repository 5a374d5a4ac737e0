// Checkerboard Metropolis sweep kernel of the single-run path for gfx950
// (CDNA4): sweeps (Sec. 3 spin updates), the initial state (Sec. 2.1 step 1)
// and the recount of E and M.
//
// Spin representation inside the sweep: each colour of a replica is a set of
// 32-site words (canonical within-colour index q = (y L + x) >> 1, bit q & 31
// of word q >> 5; bit set = spin -1).  A wave owns whole replicas and keeps
// them on chip for all requested sweeps: in VGPRs for L <= 64 (vertical
// neighbours cross lanes by shuffle, horizontal ones are funnel shifts), in
// LDS for L >= 128.  The Metropolis decision for all 32 sites of a word is
// bit-sliced: the uniform of each site is compared to the integer threshold
// one bit plane at a time (16 planes from four Philox blocks, high bit first).
// For L <= 64 the planes stop as soon as no site of the wave is undecided; for
// L >= 128 a lane decides 8 planes for several words and queues the sites
// still tied, which the wave then decides one per lane (pa_device.h).  A run
// created with PA_FLAG_HEATBATH uses the heat-bath update in the same scheme,
// one created with PA_FLAG_LCG the in-line LCG variant of the multi-spin-coded
// sweep (Sec. 4), each with its own kernel instantiations.
#include "pa_device.h"
#include "pa_launch.h"

namespace pa {
namespace {

using namespace pa::dev;

template <int L, bool INT8, int U>
__global__ __launch_bounds__(sweep_block<L>())
__attribute__((amdgpu_waves_per_eu(sweep_min_waves<L>(), 8))) void sweep_kernel(SweepArgs a)
{
    using Gm = Geo<L>;
    constexpr int WPB = sweep_block<L>() / 64;
    __shared__ uint32_t lds[Gm::lds_words(WPB) > 0 ? Gm::lds_words(WPB) : 1];
    if (a.n_dev) a.n_rep = min(a.n_rep, (int32_t)*a.n_dev);
    sweep_waves<L, INT8, U == kHeatbath, U == kLcg>(a, (int)blockIdx.x * WPB, WPB, lds);
}

template <int L, bool INT8, int U>
hipError_t launch_sweep_t(const SweepArgs& a, hipStream_t s)
{
    using Gm = Geo<L>;
    const int reps_per_block = (sweep_block<L>() / 64) * Gm::RPWV;
    const int blocks = (a.n_rep + reps_per_block - 1) / reps_per_block;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((sweep_kernel<L, INT8, U>), dim3(blocks), dim3(sweep_block<L>()), 0, s, a);
    return hipGetLastError();
}

template <int L, bool INT8>
hipError_t launch_sweep_u(int update, const SweepArgs& a, hipStream_t s)
{
    switch (update) {
    case kMetropolis: return launch_sweep_t<L, INT8, kMetropolis>(a, s);
    case kHeatbath: return launch_sweep_t<L, INT8, kHeatbath>(a, s);
    case kLcg: return launch_sweep_t<L, INT8, kLcg>(a, s);
    default: return hipErrorInvalidValue;
    }
}

template <int L>
hipError_t launch_sweep_l(bool i8, int update, const SweepArgs& a, hipStream_t s)
{
    return i8 ? launch_sweep_u<L, true>(update, a, s) : launch_sweep_u<L, false>(update, a, s);
}

}  // namespace

hipError_t launch_sweep(int L, int layout, int update, const SweepArgs& a, hipStream_t s)
{
    const bool i8 = layout == 0;
    switch (L) {
    case 16: return launch_sweep_l<16>(i8, update, a, s);
    case 32: return launch_sweep_l<32>(i8, update, a, s);
    case 64: return launch_sweep_l<64>(i8, update, a, s);
    case 128: return launch_sweep_l<128>(i8, update, a, s);
    case 256: return launch_sweep_l<256>(i8, update, a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace pa

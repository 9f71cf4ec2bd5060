// gfx950 phase kernel of the colour-phase schedule: one launch set per colour phase, one
// wavefront per domain.  Built twice: for tethers, and with ECMC_SPRING_TU=1 for harmonic
// springs (Eq. (2)), whose kernels carry the spring energy draws.  The device code of the EC
// move is in ecmc_device.h.
#include "ecmc_device.h"

#ifndef ECMC_SPRING_TU
#define ECMC_SPRING_TU 0
#endif
#if ECMC_SPRING_TU
#define K_PHASE k_phase_spring
#define PHASE_LAUNCHER launch_phase_spring
#else
#define K_PHASE k_phase
#define PHASE_LAUNCHER launch_phase
#endif

namespace ecmc {

namespace {

constexpr bool SPRING = ECMC_SPRING_TU != 0;

// ------------------------------------------------------------------ phase kernel
// One colour phase: one wavefront per domain of the colour, for the domains whose bead count
// (from k_count) falls in this launch's staging tier (stage_lo, stage_hi].
template <int BPL, bool LOG, bool EXACT, bool WHOLE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(phase_waves(BPL)))) void K_PHASE(const PhaseArgs a) {
    constexpr int SMAX = 64 * BPL;
    __shared__ double s_pos[3][SMAX];
    __shared__ int32_t s_id[SMAX], s_meta[SMAX], s_part[SMAX], s_mot[motile_list(BPL, false) ? SMAX : 1];
    __shared__ unsigned long long s_motm[motile_list(BPL, false) ? 1 : BPL];
    // this sweep's number and partition, from the device-side sweep counter
    PhaseArgs b = a;
    b.sweep = a.dstate[0];
    int off[3];
    partition_offsets(b, b.joint ? b.D + 1 : b.D, b.sweep, 0u, off);
    Frame f;
    int F;
    bool wraps;
    if (b.joint) frame_of<WHOLE, true>(b, b.colour, blockIdx.x, off, 0, f, F, wraps);
    else frame_of<WHOLE>(b, b.colour, blockIdx.x, off, 0, f, F, wraps);
    // The count comes from k_count, taken before any tier of this phase ran: a block of
    // another tier may be rewriting this domain's cell lists, so a count read here could be
    // a half-updated one.  A domain outside this launch's tier belongs to another launch.
    const int S0 = __builtin_amdgcn_readfirstlane(a.dstage[blockIdx.x]);
    if (S0 <= a.stage_lo || S0 > a.stage_hi) return;
    if (S0 > SMAX) {
        if (lane_id() == 0) atomicOr(a.err, ERR_STAGE);
        return;
    }
    const StageMem m = {&s_pos[0][0], s_id, s_meta, s_part, s_motm, s_mot, SMAX};
    domain_body<BPL, LOG, EXACT, WHOLE, SPRING>(b, f, F, wraps, S0, m);
}

}  // namespace

// EXACT: the plain FP64 search (every staged bead evaluated at every event); otherwise the
// single-precision screen with FP64 evaluation of the beads that can come first.
template <int BPL, bool WHOLE>
static hipError_t launch_bpl(const PhaseArgs &a, bool log, int grid, hipStream_t s) {
    if (log && a.exact_search) hipLaunchKernelGGL((K_PHASE<BPL, true, true, WHOLE>), dim3(grid), dim3(64), 0, s, a);
    else if (log) hipLaunchKernelGGL((K_PHASE<BPL, true, false, WHOLE>), dim3(grid), dim3(64), 0, s, a);
    else if (a.exact_search) hipLaunchKernelGGL((K_PHASE<BPL, false, true, WHOLE>), dim3(grid), dim3(64), 0, s, a);
    else hipLaunchKernelGGL((K_PHASE<BPL, false, false, WHOLE>), dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <int BPL>
static hipError_t launch_bpl(const PhaseArgs &a, bool log, int grid, hipStream_t s) {
    return a.whole ? launch_bpl<BPL, true>(a, log, grid, s) : launch_bpl<BPL, false>(a, log, grid, s);
}

hipError_t PHASE_LAUNCHER(const PhaseArgs &a, int bpl, bool log, int grid, hipStream_t s) {
    switch (bpl) {
        case 1: return launch_bpl<1>(a, log, grid, s);
        case 2: return launch_bpl<2>(a, log, grid, s);
        case 3: return launch_bpl<3>(a, log, grid, s);
        case 4: return launch_bpl<4>(a, log, grid, s);
        case 6: return launch_bpl<6>(a, log, grid, s);
        case 7: return launch_bpl<7>(a, log, grid, s);
        case 8: return launch_bpl<8>(a, log, grid, s);
        case 12: return launch_bpl<12>(a, log, grid, s);
        case 16: return launch_bpl<16>(a, log, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ecmc

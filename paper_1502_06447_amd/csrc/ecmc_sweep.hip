// gfx950 kernel of the dependency-ordered sweep: all eight colour phases of a checkerboard
// sweep in one launch, without a device-wide barrier between the phases.
//
// The sweep's result is defined by running the colours 0..7 one after the other, the domains
// of one colour in any order (they never touch each other's frames).  A domain reads the cells
// of its frame (its own cells and a one-cell halo, which belongs to the 26 surrounding
// domains) and writes only its own cells.  Two domains therefore conflict only when they are
// neighbours in the periodic domain grid, and neighbours always differ in colour.  So a domain
// may start as soon as its neighbours of earlier colours are finished: by then its frame holds
// exactly what the colour-by-colour order would give it, and its neighbours of later colours
// wait for it in turn.
//
// Persistent waves take tickets from one counter in colour-major order.  A wave only waits on
// domains of smaller tickets, which running waves hold and finish without waiting on larger
// ones, so the waits always end.  As a guard against a broken invariant every wait gives up
// after a fixed wall-clock time (far beyond any domain's run time) and flags ERR_WAIT.  Completion is published with an
// agent-scope release (the per-XCD L2 caches are written back) and observed with an
// agent-scope acquire.
//
// A domain whose frame holds more beads than the LDS staging area is staged in a slot of the
// device workspace instead and run with the plain FP64 search (identical results).
#include "ecmc_device.h"

// Built three times: for tethers, with ECMC_SPRING_TU=1 for harmonic springs (Eq. (2)), and
// with ECMC_PUSH_TU=1 for the push-off of overlapping starts (Sec. II.B, FP64 search only).
#ifndef ECMC_SPRING_TU
#define ECMC_SPRING_TU 0
#endif
#ifndef ECMC_PUSH_TU
#define ECMC_PUSH_TU 0
#endif
#if ECMC_PUSH_TU
#define K_SWEEP k_sweep_push
#define SWEEP_LAUNCHER launch_sweep_push
#elif ECMC_SPRING_TU
#define K_SWEEP k_sweep_spring
#define SWEEP_LAUNCHER launch_sweep_spring
#else
#define K_SWEEP k_sweep
#define SWEEP_LAUNCHER launch_sweep
#endif

namespace ecmc {

namespace {

constexpr bool SPRING = ECMC_SPRING_TU != 0;
constexpr bool PUSH = ECMC_PUSH_TU != 0;

// Whether a wait that started at t0 (steady-counter ticks) has run out of time: a.wait_ticks
// ticks of the constant-rate counter, set on the host to many seconds.  A bound in time rather
// than in polls: a domain's run time varies by orders of magnitude with the bond model and the
// event log (a spring domain runs ~45 times the events of a tether domain), a poll's latency
// with the memory system.
__device__ __forceinline__ bool out_of_time(const PhaseArgs &a, unsigned long long t0) {
    return (unsigned long long)wall_clock64() - t0 > a.wait_ticks;
}

// Wait until this launch has finished every neighbour of domain f whose colour comes earlier,
// then acquire what they wrote.  Returns false if the wait ran out of time (ERR_WAIT flagged):
// a neighbour may then still be writing the shared halo, so the caller leaves the domain as it
// is.
__device__ __forceinline__ bool wait_for_earlier(const PhaseArgs &a, const Frame &f) {
    const int lane = lane_id();
    const int nd = a.nd;
    const uint32_t *done = a.done;  // the melt's stamps
    const uint32_t epoch = a.epoch;
    bool need = false;
    int nb = 0;
    if (lane < 27 && lane != 13) {
        const int ox = lane % 3 - 1, oy = (lane / 3) % 3 - 1, oz = lane / 9 - 1;
        // a step of one domain along an axis flips that axis' parity bit (nd is even)
        const int col = f.colour ^ ((ox != 0) | ((oy != 0) << 1) | ((oz != 0) << 2));
        need = col < f.colour;
        nb = (f.dom[0] + ox + nd) % nd + nd * ((f.dom[1] + oy + nd) % nd + nd * ((f.dom[2] + oz + nd) % nd));
    }
    const unsigned long long t0 = (unsigned long long)wall_clock64();
    bool ok = true;
    for (;;) {
        need = need && __hip_atomic_load(&done[nb], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch;
        if (!__ballot(need)) break;
        if (__builtin_amdgcn_readfirstlane((int)out_of_time(a, t0))) {
            if (lane == 0) atomicOr(a.err, ERR_WAIT);
            ok = false;
            break;
        }
        __builtin_amdgcn_s_sleep(8);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok;
}

// A free staging slot, searched from `start`; -1 (and ERR_WAIT) if none came free in time.
// Called after the dependency wait: a wave holding a slot never waits on another domain, so
// every slot is given back.
__device__ __forceinline__ int take_slot(const PhaseArgs &a, uint32_t start) {
    int got = -1;
    if (lane_id() == 0) {
        const unsigned long long t0 = (unsigned long long)wall_clock64();
        while (got < 0) {
            const int nslow = a.nslow;
            uint32_t *lock = a.slow_lock;
            for (int i = 0; i < nslow && got < 0; ++i) {
                const int s = (int)((start + (uint32_t)i) % (uint32_t)nslow);
                if (atomicCAS(&lock[s], 0u, 1u) == 0u) got = s;
            }
            if (got >= 0) break;
            if (out_of_time(a, t0)) {
                atomicOr(a.err, ERR_WAIT);
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
    }
    return __builtin_amdgcn_readfirstlane(got);
}

// The melt of ticket r (its index within a colour): the last melt whose first ticket is at
// or below r.
__device__ __forceinline__ int melt_of(const PhaseArgs &a, int r) {
    int lo = 0, hi = a.n_melts - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.melts[mid].tick0 <= r) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int BPL, bool LOG, bool EXACT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(phase_waves(BPL)))) void K_SWEEP(const PhaseArgs a) {
    constexpr int SMAX = 64 * BPL;
    __shared__ double s_pos[3][SMAX];
    __shared__ int32_t s_id[SMAX], s_meta[SMAX], s_part[SMAX], s_mot[motile_list(BPL, PUSH) ? SMAX : 1];
    __shared__ unsigned long long s_motm[motile_list(BPL, PUSH) ? 1 : BPL];
    const int lane = lane_id();
    // one ticket per workgroup, taken when the workgroup runs: ticket order, not launch order,
    // is the order of the waits.  Tickets run colour by colour, melt by melt within a colour.
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(&a.queue[0], 1u);
    t = __builtin_amdgcn_readfirstlane(t);
    const int colour = (int)(t / (uint32_t)a.tickets);
    const int r = (int)(t % (uint32_t)a.tickets);
    const int mi = melt_of(a, r);
    const MeltDev &M = a.melts[mi];
    // the melt's view of the arguments; the sweep number and this launch's stamp come from
    // device memory, so that a replayed graph of sweep launches moves on by itself
    PhaseArgs b = a;
    b.L = M.L;
    b.h = M.h;
    b.halfL = M.halfL;
    b.in_lo = M.in_lo;
    b.in_hi = M.in_hi;
    b.p_sure = M.p_sure;
    b.err_f = M.err_f;
    b.n = M.n;
    b.D = M.D;
    b.nd = M.nd;
    b.ccount = a.ccount + M.cell0;
    b.cids = a.cids + M.cell0 * a.cap;
    b.done = a.done + M.dom0;
    b.sweep = a.dstate[0];
    b.epoch = a.dstate[1] + 1u;
    b.stream = (uint32_t)mi;
    int off[3];
    partition_offsets(b, b.D, b.sweep, b.stream, off);
    Frame f;
    int F;
    bool wraps;
    frame_of<false>(b, colour, r - M.tick0, off, M.dom0, f, F, wraps);
    // after a wait that ran out of time the domain is left untouched; its stamp is still
    // published below, so that the waits of later colours end and the error reaches the host
    const bool ready = wait_for_earlier(b, f);
    const int S = ready ? frame_count(b, f, F) : 0;
    int slot = -1;
    if (!ready) {
        // nothing to do
    } else if (S <= SMAX) {
        const StageMem m = {&s_pos[0][0], s_id, s_meta, s_part, s_motm, s_mot, SMAX};
        domain_body<BPL, LOG, EXACT, false, SPRING, PUSH>(b, f, F, wraps, S, m);
    } else if (S <= a.slow_cap) {
        slot = take_slot(a, t);
        if (slot >= 0) {
            // slot layout: three rows of positions, then id, meta, part and motile-list rows
            const int cap = a.slow_cap;
            double *base = a.slow + (size_t)slot * (size_t)cap * (SLOW_SLOT_BYTES_PER_BEAD / 8);
            int32_t *ib = reinterpret_cast<int32_t *>(base + 3 * (size_t)cap);
            const StageMem m = {base, ib, ib + cap, ib + 2 * cap, nullptr, ib + 3 * cap, cap};
            domain_body<16, LOG, true, false, SPRING, PUSH>(b, f, F, wraps, S, m);
        }
    } else if (lane == 0) {
        atomicOr(a.err, ERR_STAGE);
    }
    // publish: every write of this domain is visible device-wide before its stamp (the stamp
    // and the arrays are read again here rather than held through the ECs)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) {
        uint32_t *st = late(a.dstate);
        __hip_atomic_store(&late(a.done)[f.gdomain], st[1] + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (slot >= 0)
            __hip_atomic_store(&late(a.slow_lock)[slot], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the last workgroup to finish resets the ticket counter and advances the sweep
        // counter and the stamp for the next launch
        uint32_t *q = late(a.queue);
        const uint32_t left = atomicAdd(&q[1], 1u);
        if (left == gridDim.x - 1) {
            __hip_atomic_store(&q[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&q[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&st[0], st[0] + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&st[1], st[1] + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int BPL, bool LOG, bool EXACT>
hipError_t launch_sweep_v(const PhaseArgs &a, int *grid, hipStream_t s) {
    const int g = 8 * a.tickets;  // one workgroup per domain of the sweep
    *grid = g;
    hipLaunchKernelGGL((K_SWEEP<BPL, LOG, EXACT>), dim3(g), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <int BPL>
hipError_t launch_sweep_b(const PhaseArgs &a, bool log, int *grid, hipStream_t s) {
    if constexpr (PUSH) {
        // the push-off runs the plain FP64 search only
        return log ? launch_sweep_v<BPL, true, true>(a, grid, s) : launch_sweep_v<BPL, false, true>(a, grid, s);
    }
    if (log) return a.exact_search ? launch_sweep_v<BPL, true, true>(a, grid, s) : launch_sweep_v<BPL, true, false>(a, grid, s);
    return a.exact_search ? launch_sweep_v<BPL, false, true>(a, grid, s) : launch_sweep_v<BPL, false, false>(a, grid, s);
}

}  // namespace

#if !ECMC_SPRING_TU && !ECMC_PUSH_TU
bool sweep_bpl_supported(int bpl) {
    switch (bpl) {
        case 1: case 2: case 3: case 4: case 6: case 7: case 8: return true;
        default: return false;
    }
}
#endif

hipError_t SWEEP_LAUNCHER(const PhaseArgs &a, int bpl, bool log, int *grid, hipStream_t s) {
    switch (bpl) {
        case 1: return launch_sweep_b<1>(a, log, grid, s);
        case 2: return launch_sweep_b<2>(a, log, grid, s);
        case 3: return launch_sweep_b<3>(a, log, grid, s);
        case 4: return launch_sweep_b<4>(a, log, grid, s);
        case 6: return launch_sweep_b<6>(a, log, grid, s);
        case 7: return launch_sweep_b<7>(a, log, grid, s);
        case 8: return launch_sweep_b<8>(a, log, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ecmc

// gfx950 kernels of the colour-phase schedule (one launch set per colour phase), the
// observables and the shape analysis.  The device code of the EC move is in ecmc_device.h.
#include "ecmc_device.h"

namespace ecmc {

namespace {

// Beads in the frame of every domain of the phase, one wavefront per domain, taken before
// the phase's tier launches start: they run concurrently and pick their domains by it.
template <bool WHOLE>
__global__ __launch_bounds__(64) void k_count(const PhaseArgs a) {
    int off[3];
    partition_offsets(a, a.D, a.dstate[0], 0u, off);
    Frame f;
    int F;
    bool wraps;
    frame_of<WHOLE>(a, a.colour, blockIdx.x, off, 0, f, F, wraps);
    const int S = frame_count(a, f, F);
    if (lane_id() == 0) a.dstage[blockIdx.x] = S;
}

// The end of a sweep by colour phases: the sweep counter (in device memory, where the
// dependency-ordered sweep advances it too) moves on.
__global__ void k_advance(const PhaseArgs a) {
    if (threadIdx.x == 0) a.dstate[0] += 1u;
}

// ------------------------------------------------------------------ phase kernel
// One colour phase: one wavefront per domain of the colour, for the domains whose bead count
// (from k_count) falls in this launch's staging tier (stage_lo, stage_hi].
template <int BPL, bool LOG, bool EXACT, bool WHOLE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(phase_waves(BPL)))) void k_phase(const PhaseArgs a) {
    constexpr int SMAX = 64 * BPL;
    __shared__ double s_pos[3][SMAX];
    __shared__ int32_t s_id[SMAX], s_meta[SMAX], s_part[SMAX], s_mot[SMAX];
    // this sweep's number and partition, from the device-side sweep counter
    PhaseArgs b = a;
    b.sweep = a.dstate[0];
    int off[3];
    partition_offsets(b, b.D, b.sweep, 0u, off);
    Frame f;
    int F;
    bool wraps;
    frame_of<WHOLE>(b, b.colour, blockIdx.x, off, 0, f, F, wraps);
    // The count comes from k_count, taken before any tier of this phase ran: a block of
    // another tier may be rewriting this domain's cell lists, so a count read here could be
    // a half-updated one.  A domain outside this launch's tier belongs to another launch.
    const int S0 = __builtin_amdgcn_readfirstlane(a.dstage[blockIdx.x]);
    if (S0 <= a.stage_lo || S0 > a.stage_hi) return;
    if (S0 > SMAX) {
        if (lane_id() == 0) atomicOr(a.err, ERR_STAGE);
        return;
    }
    const StageMem m = {&s_pos[0][0], s_id, s_meta, s_part, s_mot, SMAX};
    domain_body<BPL, LOG, EXACT, WHOLE>(b, f, F, wraps, S0, m);
}

// ------------------------------------------------------------------ observables
// sum over the wavefront, returned to every lane (fixed order, so reproducible)
__device__ __forceinline__ double wave_sum_f64(double v) {
    v = v + dpp_f64<0xB1>(v);
    v = v + dpp_f64<0x4E>(v);
    v = v + dpp_f64<0x141>(v);
    v = v + dpp_f64<0x140>(v);
    const double r0 = rdlane(v, 0), r1 = rdlane(v, 16), r2 = rdlane(v, 32), r3 = rdlane(v, 48);
    return (r0 + r1) + (r2 + r3);
}

// inclusive prefix sum of doubles over the wavefront
__device__ __forceinline__ double wave_scan_f64(double v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// One wavefront per polymer (observables of Sec. IV.A and the appendix).  Lane t of a chunk holds chain position
// base + t: its minimum-image bond vector to the previous bead, prefix-summed over the wave
// (plus the carry of the earlier chunks), is the bead's unwrapped position u relative to the
// first bead.  R is the last u; R_g^2 = N^-1 sum u^2 - |N^-1 sum u|^2 (positions relative to
// the first bead keep the cancellation small); the middle bead floor(N/2) is unwrapped with
// its image counters; bond lengths are binned in LDS, one global add per bin and block.
constexpr int OBS_WAVES = 4;
constexpr int OBS_MAX_BINS = 1024;

__global__ __launch_bounds__(64 * OBS_WAVES) void k_observables(const ObsArgs a) {
    __shared__ unsigned s_hist[OBS_MAX_BINS];
    const int lane = lane_id();
    const int w = (int)threadIdx.x >> 6;
    for (int i = (int)threadIdx.x; i < a.nbins; i += 64 * OBS_WAVES) s_hist[i] = 0u;
    __syncthreads();
    for (int64_t q = (int64_t)blockIdx.x * OBS_WAVES + w; q < a.npoly; q += (int64_t)gridDim.x * OBS_WAVES) {
        // the box of this polymer's melt
        const double L = a.polyL[q], halfL = 0.5 * L;
        auto mi = [&](double d) { return d > halfL ? d - L : (d < -halfL ? d + L : d); };
        const int64_t s = a.pstart[q];
        const int N = (int)(a.pstart[q + 1] - s);
        double c0 = 0.0, c1 = 0.0, c2 = 0.0;  // u of the last bead of the previous chunk
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, sq = 0.0;
        for (int base = 0; base < N; base += 64) {
            const int t = base + lane;
            double d0 = 0.0, d1 = 0.0, d2 = 0.0;
            if (t < N) {
                const int ib = a.porder[s + t];
                if (t > 0) {
                    const int ia = a.porder[s + t - 1];
                    d0 = mi(a.px[ib] - a.px[ia]);
                    d1 = mi(a.py[ib] - a.py[ia]);
                    d2 = mi(a.pz[ib] - a.pz[ia]);
                    if (a.hist) {
                        const double q0 = d0 * d0;
                        const double q1 = d1 * d1;
                        const double q2 = d2 * d2;
                        const double len = __builtin_sqrt(q0 + q1 + q2);
                        int bin = (int)__builtin_floor((len - a.sigma) / (a.bmax - a.sigma) * a.nbins);
                        if (bin < 0) bin = 0;
                        if (bin > a.nbins - 1) bin = a.nbins - 1;
                        atomicAdd(&s_hist[bin], 1u);
                    }
                }
                if (t == N / 2) {
                    a.mid[3 * q + 0] = a.px[ib] + (double)a.img[3 * ib + 0] * L;
                    a.mid[3 * q + 1] = a.py[ib] + (double)a.img[3 * ib + 1] * L;
                    a.mid[3 * q + 2] = a.pz[ib] + (double)a.img[3 * ib + 2] * L;
                }
            }
            const double u0 = c0 + wave_scan_f64(d0);
            const double u1 = c1 + wave_scan_f64(d1);
            const double u2 = c2 + wave_scan_f64(d2);
            if (t < N) {
                s0 += u0;
                s1 += u1;
                s2 += u2;
                const double w0 = u0 * u0;
                const double w1 = u1 * u1;
                const double w2 = u2 * u2;
                sq += (w0 + w1) + w2;
            }
            c0 = rdlane(u0, 63);  // lanes past the chain end add zero bonds
            c1 = rdlane(u1, 63);
            c2 = rdlane(u2, 63);
        }
        const double m0 = wave_sum_f64(s0) / (double)N;
        const double m1 = wave_sum_f64(s1) / (double)N;
        const double m2 = wave_sum_f64(s2) / (double)N;
        const double qq = wave_sum_f64(sq) / (double)N;
        if (lane == 0) {
            const double r0 = c0 * c0;
            const double r1 = c1 * c1;
            const double r2 = c2 * c2;
            a.r2[q] = (r0 + r1) + r2;
            const double g0 = m0 * m0;
            const double g1 = m1 * m1;
            const double g2 = m2 * m2;
            a.rg2[q] = qq - ((g0 + g1) + g2);
        }
    }
    __syncthreads();
    if (a.hist)
        for (int i = (int)threadIdx.x; i < a.nbins; i += 64 * OBS_WAVES)
            if (s_hist[i]) atomicAdd(&a.hist[i], (unsigned long long)s_hist[i]);
}

// Eigenvalues, descending, of a symmetric 3 x 3 matrix (xx, yy, zz, xy, xz, yz): the
// trigonometric closed form of the characteristic cubic.  With q = tr/3 and
// B = (G - q 1) / p, p = sqrt(tr((G - q 1)^2) / 6), the eigenvalues are
// q + 2 p cos(phi + 2 pi k / 3) with phi = acos(det(B) / 2) / 3.
__device__ void sym3_eigenvalues(const double g[6], double e[3]) {
    const double xx = g[0], yy = g[1], zz = g[2], xy = g[3], xz = g[4], yz = g[5];
    const double p1 = (xy * xy + xz * xz) + yz * yz;
    const double q = ((xx + yy) + zz) / 3.0;
    const double dx = xx - q, dy = yy - q, dz = zz - q;
    const double p2 = ((dx * dx + dy * dy) + dz * dz) + 2.0 * p1;
    if (!(p2 > 0.0)) {
        e[0] = e[1] = e[2] = q;
        return;
    }
    const double p = sqrt(p2 / 6.0);
    const double bxx = dx / p, byy = dy / p, bzz = dz / p, bxy = xy / p, bxz = xz / p, byz = yz / p;
    const double det = bxx * (byy * bzz - byz * byz) - bxy * (bxy * bzz - byz * bxz) + bxz * (bxy * byz - byy * bxz);
    double r = 0.5 * det;
    r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
    const double phi = acos(r) / 3.0;
    const double two_pi_3 = 2.0943951023931954923;  // 2 pi / 3
    e[0] = q + 2.0 * p * cos(phi);
    e[2] = q + 2.0 * p * cos(phi + two_pi_3);
    e[1] = 3.0 * q - e[0] - e[2];
}

// Shape analysis (appendix, moment of inertia tensor; the centre of mass for g2 of
// Sec. IV.A): one wavefront per polymer.  As in k_observables the chain is unwrapped from its
// first bead by prefix sums of minimum-image bond vectors; the sums of u and of u_a u_b give
// the gyration tensor G = N^-1 sum u u^T - u_cm u_cm^T (positions relative to the first bead
// keep the cancellation small), its eigenvalues, and the centre of mass in image-unwrapped
// coordinates.
__global__ __launch_bounds__(64 * OBS_WAVES) void k_shape(const ObsArgs a) {
    const int lane = lane_id();
    const int w = (int)threadIdx.x >> 6;
    for (int64_t q = (int64_t)blockIdx.x * OBS_WAVES + w; q < a.npoly; q += (int64_t)gridDim.x * OBS_WAVES) {
        // the box of this polymer's melt
        const double L = a.polyL[q], halfL = 0.5 * L;
        auto mi = [&](double d) { return d > halfL ? d - L : (d < -halfL ? d + L : d); };
        const int64_t s = a.pstart[q];
        const int N = (int)(a.pstart[q + 1] - s);
        double c0 = 0.0, c1 = 0.0, c2 = 0.0;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, sxx = 0.0, syy = 0.0, szz = 0.0, sxy = 0.0, sxz = 0.0, syz = 0.0;
        for (int base = 0; base < N; base += 64) {
            const int t = base + lane;
            double d0 = 0.0, d1 = 0.0, d2 = 0.0;
            if (t < N && t > 0) {
                const int ia = a.porder[s + t - 1], ib = a.porder[s + t];
                d0 = mi(a.px[ib] - a.px[ia]);
                d1 = mi(a.py[ib] - a.py[ia]);
                d2 = mi(a.pz[ib] - a.pz[ia]);
            }
            const double u0 = c0 + wave_scan_f64(d0);
            const double u1 = c1 + wave_scan_f64(d1);
            const double u2 = c2 + wave_scan_f64(d2);
            if (t < N) {
                s0 += u0;
                s1 += u1;
                s2 += u2;
                sxx += u0 * u0;
                syy += u1 * u1;
                szz += u2 * u2;
                sxy += u0 * u1;
                sxz += u0 * u2;
                syz += u1 * u2;
            }
            c0 = rdlane(u0, 63);
            c1 = rdlane(u1, 63);
            c2 = rdlane(u2, 63);
        }
        const double inv = 1.0 / (double)N;
        const double m0 = wave_sum_f64(s0) * inv, m1 = wave_sum_f64(s1) * inv, m2 = wave_sum_f64(s2) * inv;
        double g[6];
        g[0] = wave_sum_f64(sxx) * inv - m0 * m0;
        g[1] = wave_sum_f64(syy) * inv - m1 * m1;
        g[2] = wave_sum_f64(szz) * inv - m2 * m2;
        g[3] = wave_sum_f64(sxy) * inv - m0 * m1;
        g[4] = wave_sum_f64(sxz) * inv - m0 * m2;
        g[5] = wave_sum_f64(syz) * inv - m1 * m2;
        if (lane == 0) {
            double e[3];
            sym3_eigenvalues(g, e);
#pragma unroll
            for (int k = 0; k < 6; ++k) a.gyr[6 * q + k] = g[k];
#pragma unroll
            for (int k = 0; k < 3; ++k) a.eig[3 * q + k] = e[k];
            const int i0 = a.porder[s];
            a.com[3 * q + 0] = a.px[i0] + (double)a.img[3 * i0 + 0] * L + m0;
            a.com[3 * q + 1] = a.py[i0] + (double)a.img[3 * i0 + 1] * L + m1;
            a.com[3 * q + 2] = a.pz[i0] + (double)a.img[3 * i0 + 2] * L + m2;
        }
    }
}

}  // namespace

bool bpl_supported(int bpl) {
    switch (bpl) {
        case 1: case 2: case 3: case 4: case 6: case 8: case 12: case 16: return true;
        default: return false;
    }
}

// EXACT: the plain FP64 search (every staged bead evaluated at every event); otherwise the
// single-precision screen with FP64 evaluation of the beads that can come first.
template <int BPL, bool WHOLE>
static hipError_t launch_bpl(const PhaseArgs &a, bool log, int grid, hipStream_t s) {
    if (log && a.exact_search) hipLaunchKernelGGL((k_phase<BPL, true, true, WHOLE>), dim3(grid), dim3(64), 0, s, a);
    else if (log) hipLaunchKernelGGL((k_phase<BPL, true, false, WHOLE>), dim3(grid), dim3(64), 0, s, a);
    else if (a.exact_search) hipLaunchKernelGGL((k_phase<BPL, false, true, WHOLE>), dim3(grid), dim3(64), 0, s, a);
    else hipLaunchKernelGGL((k_phase<BPL, false, false, WHOLE>), dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <int BPL>
static hipError_t launch_bpl(const PhaseArgs &a, bool log, int grid, hipStream_t s) {
    return a.whole ? launch_bpl<BPL, true>(a, log, grid, s) : launch_bpl<BPL, false>(a, log, grid, s);
}

hipError_t launch_phase(const PhaseArgs &a, int bpl, bool log, int grid, hipStream_t s) {
    switch (bpl) {
        case 1: return launch_bpl<1>(a, log, grid, s);
        case 2: return launch_bpl<2>(a, log, grid, s);
        case 3: return launch_bpl<3>(a, log, grid, s);
        case 4: return launch_bpl<4>(a, log, grid, s);
        case 6: return launch_bpl<6>(a, log, grid, s);
        case 8: return launch_bpl<8>(a, log, grid, s);
        case 12: return launch_bpl<12>(a, log, grid, s);
        case 16: return launch_bpl<16>(a, log, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_advance(const PhaseArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_count(const PhaseArgs &a, int grid, hipStream_t s) {
    if (a.whole) hipLaunchKernelGGL(k_count<true>, dim3(grid), dim3(64), 0, s, a);
    else hipLaunchKernelGGL(k_count<false>, dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_shape(const ObsArgs &a, hipStream_t s) {
    if (a.npoly <= 0) return hipSuccess;
    int64_t grid = (a.npoly + OBS_WAVES - 1) / OBS_WAVES;
    if (grid > 16384) grid = 16384;
    hipLaunchKernelGGL(k_shape, dim3((unsigned)grid), dim3(64 * OBS_WAVES), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_observables(const ObsArgs &a, hipStream_t s) {
    if (a.npoly <= 0) return hipSuccess;
    if (a.nbins < 1 || a.nbins > OBS_MAX_BINS) return hipErrorInvalidValue;
    int64_t grid = (a.npoly + OBS_WAVES - 1) / OBS_WAVES;
    if (grid > 16384) grid = 16384;
    hipLaunchKernelGGL(k_observables, dim3((unsigned)grid), dim3(64 * OBS_WAVES), 0, s, a);
    return hipGetLastError();
}

}  // namespace ecmc

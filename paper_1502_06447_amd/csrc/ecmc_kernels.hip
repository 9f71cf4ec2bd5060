// gfx950 kernels around the colour-phase schedule (the per-phase bead counts, the sweep
// counter), the observables and the shape analysis.  The device code of the EC move is in
// ecmc_device.h, the phase kernel itself in ecmc_phase.hip.
#include "ecmc_device.h"

namespace ecmc {

namespace {

// Beads in the frame of every domain of the phase, one wavefront per domain, taken before
// the phase's tier launches start: they run concurrently and pick their domains by it.
template <bool WHOLE>
__global__ __launch_bounds__(64) void k_count(const PhaseArgs a) {
    int off[3];
    partition_offsets(a, a.joint ? a.D + 1 : a.D, a.dstate[0], 0u, off);
    Frame f;
    int F;
    bool wraps;
    if (a.joint) frame_of<WHOLE, true>(a, a.colour, blockIdx.x, off, 0, f, F, wraps);
    else frame_of<WHOLE>(a, a.colour, blockIdx.x, off, 0, f, F, wraps);
    const int S = frame_count(a, f, F);
    if (lane_id() == 0) a.dstage[blockIdx.x] = S;
}

// The end of a sweep by colour phases: the sweep counter (in device memory, where the
// dependency-ordered sweep advances it too) moves on.
__global__ void k_advance(const PhaseArgs a) {
    if (threadIdx.x == 0) a.dstate[0] += 1u;
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
    __shared__ double s_acc[2][OBS_WAVES];
    const int lane = lane_id();
    const int w = (int)threadIdx.x >> 6;
    double acc_r2 = 0.0, acc_rg2 = 0.0;  // this wavefront's polymers (lane 0)
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
            const double e2 = (r0 + r1) + r2;
            a.r2[q] = e2;
            const double g0 = m0 * m0;
            const double g1 = m1 * m1;
            const double g2 = m2 * m2;
            const double gy2 = qq - ((g0 + g1) + g2);
            a.rg2[q] = gy2;
            acc_r2 += e2;
            acc_rg2 += gy2;
            if (a.rhist) {
                // W(R): |R| binned from 0 in rbins bins of width rmax / rbins, the rest in the last
                int bin = (int)__builtin_floor(__builtin_sqrt(e2) / a.rmax * (double)a.rbins);
                if (bin > a.rbins - 1) bin = a.rbins - 1;
                atomicAdd(&a.rhist[bin], 1ull);
            }
        }
    }
    if (lane == 0) {
        s_acc[0][w] = acc_r2;
        s_acc[1][w] = acc_rg2;
    }
    __syncthreads();
    if (a.hist)
        for (int i = (int)threadIdx.x; i < a.nbins; i += 64 * OBS_WAVES)
            if (s_hist[i]) atomicAdd(&a.hist[i], (unsigned long long)s_hist[i]);
    if (a.acc && threadIdx.x == 0) {
        double t0 = 0.0, t1 = 0.0;
        for (int i = 0; i < OBS_WAVES; ++i) {
            t0 += s_acc[0][i];
            t1 += s_acc[1][i];
        }
        const int slot = (int)(blockIdx.x % OBS_ACC_SLOTS);
        atomicAdd(&a.acc[slot], t0);
        atomicAdd(&a.acc[OBS_ACC_SLOTS + slot], t1);
    }
}

// Clears n 8-byte words (a kernel rather than a memset node, so that the call can be captured
// in a HIP graph).
__global__ void k_zero_u64(unsigned long long *p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0ull;
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
            if (a.snap && t == N / 2) {
                // the middle bead, unwrapped with its image counters (as the observables do)
                const int ib = a.porder[s + t];
                a.snap[6 * q + 0] = a.px[ib] + (double)a.img[3 * ib + 0] * L;
                a.snap[6 * q + 1] = a.py[ib] + (double)a.img[3 * ib + 1] * L;
                a.snap[6 * q + 2] = a.pz[ib] + (double)a.img[3 * ib + 2] * L;
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
            if (a.snap) {
                a.snap[6 * q + 3] = a.com[3 * q + 0];
                a.snap[6 * q + 4] = a.com[3 * q + 1];
                a.snap[6 * q + 5] = a.com[3 * q + 2];
            }
        }
    }
}

// ------------------------------------------------------------------ pair distances
// Pair counts behind g(r): one thread per cell (all melts' cells in one grid).  Each bead of the
// cell meets the beads of the 27 cells around it (n >= 4, so these are distinct) with a larger
// id: every pair closer than rmax <= the cell edge lies in neighbouring cells and is met once.
// The displacement is (r_j - r_i) plus the box edge where the neighbour cell wraps, which is
// the minimum image for such pairs; bins are counted in LDS, one global add per bin and block.
constexpr int PAIR_THREADS = 256;

__global__ __launch_bounds__(PAIR_THREADS) void k_pairs(const PairArgs a) {
    __shared__ unsigned s_hist[OBS_MAX_BINS];
    for (int i = (int)threadIdx.x; i < a.nbins; i += PAIR_THREADS) s_hist[i] = 0u;
    __syncthreads();
    const double r2max = a.rmax * a.rmax;
    for (long long c = (long long)blockIdx.x * PAIR_THREADS + threadIdx.x; c < a.cells;
         c += (long long)gridDim.x * PAIR_THREADS) {
        int lo = 0, hi = a.n_melts - 1;  // the melt of cell c: the last whose first cell is <= c
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.melts[mid].cell0 <= c) lo = mid;
            else hi = mid - 1;
        }
        const MeltDev &M = a.melts[lo];
        const int n = M.n;
        const double L = M.L;
        const int lc = (int)(c - M.cell0);
        const int cx = lc % n, cy = (lc / n) % n, cz = lc / (n * n);
        const int ni = a.ccount[c];
        for (int ii = 0; ii < ni; ++ii) {
            const int i = a.cids[c * a.cap + ii];
            const double xi = a.px[i], yi = a.py[i], zi = a.pz[i];
            for (int nb = 0; nb < 27; ++nb) {
                const int rx = cx + nb % 3 - 1, ry = cy + (nb / 3) % 3 - 1, rz = cz + nb / 9 - 1;
                const double sx = rx < 0 ? -L : (rx >= n ? L : 0.0);
                const double sy = ry < 0 ? -L : (ry >= n ? L : 0.0);
                const double sz = rz < 0 ? -L : (rz >= n ? L : 0.0);
                const long long cn = M.cell0 + (rx + n) % n + n * ((ry + n) % n + n * ((rz + n) % n));
                const int nj = a.ccount[cn];
                for (int jj = 0; jj < nj; ++jj) {
                    const int j = a.cids[cn * a.cap + jj];
                    if (j <= i) continue;
                    const double d0 = (a.px[j] - xi) + sx;
                    const double d1 = (a.py[j] - yi) + sy;
                    const double d2 = (a.pz[j] - zi) + sz;
                    const double q0 = d0 * d0;
                    const double q1 = d1 * d1;
                    const double q2 = d2 * d2;
                    const double dd = (q0 + q1) + q2;
                    if (a.q_lim > 0.0) {
                        // overlap count of the push-off: squared distance below q_lim
                        if (dd < a.q_lim) atomicAdd(&s_hist[0], 1u);
                        continue;
                    }
                    if (!(dd < r2max * 1.0000001)) continue;  // cheap pre-test; the exact one below
                    const double r = __builtin_sqrt(dd);
                    if (!(r < a.rmax)) continue;
                    int bin = (int)__builtin_floor(r / a.rmax * (double)a.nbins);
                    if (bin > a.nbins - 1) bin = a.nbins - 1;
                    atomicAdd(&s_hist[bin], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < a.nbins; i += PAIR_THREADS)
        if (s_hist[i]) atomicAdd(&a.hist[i], (unsigned long long)s_hist[i]);
}

// ------------------------------------------------------------------ state check
// The conditions every EC keeps, checked on the device: one thread per cell of all melts.  Each
// bead the cell lists must lie in the cell's closed interval [k h, face(k + 1)] on every axis and
// carry the cell's index in its cell word; each bond (i, j > i) must be at most the limit in
// minimum image.  Counts go to LDS, then one global add per counter and block.
__global__ __launch_bounds__(PAIR_THREADS) void k_check(const PairArgs a) {
    __shared__ unsigned s_cnt[3];
    if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0u;
    __syncthreads();
    unsigned stretched = 0, misplaced = 0, listed = 0;
    for (long long c = (long long)blockIdx.x * PAIR_THREADS + threadIdx.x; c < a.cells;
         c += (long long)gridDim.x * PAIR_THREADS) {
        int lo = 0, hi = a.n_melts - 1;  // the melt of cell c: the last whose first cell is <= c
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.melts[mid].cell0 <= c) lo = mid;
            else hi = mid - 1;
        }
        const MeltDev &M = a.melts[lo];
        const int n = M.n;
        const double L = M.L, h = M.h, halfL = M.halfL;
        const int lc = (int)(c - M.cell0);
        const int k[3] = {lc % n, (lc / n) % n, lc / (n * n)};
        double blo[3], bhi[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            blo[ax] = (double)k[ax] * h;
            bhi[ax] = k[ax] + 1 < n ? (double)(k[ax] + 1) * h : L;
        }
        int ni = a.ccount[c];
        if (ni > a.cap) {  // an overflowing list: the beads it could not hold are misplaced
            misplaced += (unsigned)(ni - a.cap);
            ni = a.cap;
        }
        for (int ii = 0; ii < ni; ++ii) {
            const int i = a.cids[c * a.cap + ii];
            ++listed;
            const double r[3] = {a.px[i], a.py[i], a.pz[i]};
            const int32_t w = a.cellp[i];
            bool bad = false;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax)
                bad = bad || !(r[ax] >= blo[ax] && r[ax] <= bhi[ax]) || ((w >> (ax * CELL_BITS)) & CELL_MASK) != k[ax];
            misplaced += bad ? 1u : 0u;
            for (int t = 0; t < 2; ++t) {
                const int j = a.part[2 * i + t];
                if (j <= i) continue;  // no partner (-1), or the pair is checked from j
                double d0 = a.px[j] - r[0], d1 = a.py[j] - r[1], d2 = a.pz[j] - r[2];
                d0 = d0 > halfL ? d0 - L : (d0 < -halfL ? d0 + L : d0);
                d1 = d1 > halfL ? d1 - L : (d1 < -halfL ? d1 + L : d1);
                d2 = d2 > halfL ? d2 - L : (d2 < -halfL ? d2 + L : d2);
                const double q0 = d0 * d0;
                const double q1 = d1 * d1;
                const double q2 = d2 * d2;
                stretched += ((q0 + q1) + q2) > a.b2lim ? 1u : 0u;
            }
        }
    }
    if (stretched) atomicAdd(&s_cnt[0], stretched);
    if (misplaced) atomicAdd(&s_cnt[1], misplaced);
    if (listed) atomicAdd(&s_cnt[2], listed);
    __syncthreads();
    if (threadIdx.x < 3 && s_cnt[threadIdx.x]) atomicAdd(&a.hist[threadIdx.x], (unsigned long long)s_cnt[threadIdx.x]);
}

// ------------------------------------------------------------------ mean-square displacements
// g1 and g2 of Sec. IV.A from T snapshots [T][P][6] (middle bead, centre of mass): one block
// per lag d, its threads over the (T - d) P pairs of snapshots d apart, summed in FP64 and
// reduced in a fixed tree; out[d] = g1(d), out[T + d] = g2(d) (0 at d = 0).
constexpr int MSD_THREADS = 256;

__global__ __launch_bounds__(MSD_THREADS) void k_msd(const double *snaps, long long T, long long P, double *out) {
    __shared__ double s1[MSD_THREADS], s2[MSD_THREADS];
    const long long d = blockIdx.x;
    double a1 = 0.0, a2 = 0.0;
    const long long m = d > 0 ? (T - d) * P : 0;
    for (long long k = threadIdx.x; k < m; k += MSD_THREADS) {
        const double *u = snaps + 6 * k;            // snapshot t, polymer q (k = t P + q)
        const double *v = snaps + 6 * (k + d * P);  // snapshot t + d, same polymer
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const double x = v[e] - u[e];
            const double y = (v[e] - v[3 + e]) - (u[e] - u[3 + e]);
            a1 += x * x;
            a2 += y * y;
        }
    }
    s1[threadIdx.x] = a1;
    s2[threadIdx.x] = a2;
    __syncthreads();
    for (int w = MSD_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[d] = m > 0 ? s1[0] / (double)m : 0.0;
        out[T + d] = m > 0 ? s2[0] / (double)m : 0.0;
    }
}

// ------------------------------------------------------------------ internal distances
// R^2(n) of the start-configuration check (Sec. II.B): block b takes polymers b, b + G, ... in
// turn.  Wave 0 unwraps the chain into LDS (sized for the longest chain) as prefix sums of
// minimum-image bond vectors, as k_observables does; thread t then owns the lags t + 1 + T j
// (T threads, a multiple of 64 covering the lags) and adds |u_{i+n} - u_i|^2 over i for each
// into its own LDS slot (lanes read consecutive u_{i+n}, u_i is a broadcast).  Block b writes
// its sum for lag n to lagsum[n G + b]; k_lag_total then adds each lag's G partial sums in a
// fixed tree, so the result does not depend on timing.
constexpr int LAG_THREADS = 256;

__global__ __launch_bounds__(LAG_THREADS) void k_internal(const ObsArgs a, int stride) {
    extern __shared__ double lag_lds[];
    double *ux = lag_lds, *uy = lag_lds + stride, *uz = lag_lds + 2 * stride, *acc = lag_lds + 3 * stride;
    const int tid = (int)threadIdx.x, T = (int)blockDim.x;
    for (int n = tid; n < a.nlag; n += T) acc[n] = 0.0;
    for (int64_t q = blockIdx.x; q < a.npoly; q += gridDim.x) {
        const double L = a.polyL[q], halfL = 0.5 * L;
        auto mi = [&](double d) { return d > halfL ? d - L : (d < -halfL ? d + L : d); };
        const int64_t s = a.pstart[q];
        const int N = (int)(a.pstart[q + 1] - s);  // at most stride (checked by the host)
        if (tid < 64) {
            double c0 = 0.0, c1 = 0.0, c2 = 0.0;
            for (int base = 0; base < N; base += 64) {
                const int t = base + tid;
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
                    ux[t] = u0;
                    uy[t] = u1;
                    uz[t] = u2;
                }
                c0 = rdlane(u0, 63);
                c1 = rdlane(u1, 63);
                c2 = rdlane(u2, 63);
            }
        }
        __syncthreads();
        const int nend = N < a.nlag ? N : a.nlag;
        for (int n = tid + 1; n < nend; n += T) {
            double sum = 0.0;
            for (int i = 0; i + n < N; ++i) {
                const double d0 = ux[i + n] - ux[i];
                const double d1 = uy[i + n] - uy[i];
                const double d2 = uz[i + n] - uz[i];
                const double q0 = d0 * d0;
                const double q1 = d1 * d1;
                const double q2 = d2 * d2;
                sum += (q0 + q1) + q2;
            }
            acc[n] += sum;
        }
        __syncthreads();
    }
    const int64_t G = gridDim.x;
    for (int n = tid; n < a.nlag; n += T) a.lagsum[n * G + blockIdx.x] = acc[n];
}

// one block per lag: thread t adds the partial sums t, t + 256, ... in order, then a fixed tree
__global__ __launch_bounds__(LAG_THREADS) void k_lag_total(double *lagsum, int rows, int nlag) {
    __shared__ double red[LAG_THREADS];
    const int n = (int)blockIdx.x, tid = (int)threadIdx.x;
    const double *row = lagsum + (int64_t)n * rows;
    double sum = 0.0;
    for (int b = tid; b < rows; b += LAG_THREADS) sum += row[b];
    red[tid] = sum;
    __syncthreads();
    for (int w = LAG_THREADS / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) lagsum[(int64_t)nlag * rows + n] = red[0];
}

}  // namespace

bool bpl_supported(int bpl) {
    switch (bpl) {
        case 1: case 2: case 3: case 4: case 6: case 8: case 12: case 16: return true;
        default: return false;
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

hipError_t launch_pairs(const PairArgs &a, hipStream_t s) {
    if (a.cells <= 0) return hipSuccess;
    if (a.nbins < 1 || a.nbins > OBS_MAX_BINS) return hipErrorInvalidValue;
    long long grid = (a.cells + PAIR_THREADS - 1) / PAIR_THREADS;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_pairs, dim3((unsigned)grid), dim3(PAIR_THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_check(const PairArgs &a, hipStream_t s) {
    if (a.cells <= 0) return hipSuccess;
    long long grid = (a.cells + PAIR_THREADS - 1) / PAIR_THREADS;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_check, dim3((unsigned)grid), dim3(PAIR_THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_msd(const double *snaps, int64_t T, int64_t npoly, double *out, hipStream_t s) {
    if (T <= 0) return hipSuccess;
    if (T > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_msd, dim3((unsigned)T), dim3(MSD_THREADS), 0, s, snaps, (long long)T, (long long)npoly, out);
    return hipGetLastError();
}

hipError_t launch_internal(const ObsArgs &a, int rows, int longest, hipStream_t s) {
    if (a.npoly <= 0 || a.nlag < 1) return hipSuccess;
    if (longest < 1 || longest > LAG_MAX_BEADS || a.nlag > longest || rows < 1 || rows > a.npoly ||
        (int64_t)rows * a.nlag > LAG_SLOTS)
        return hipErrorInvalidValue;
    // threads: a multiple of 64 covering the lags 1..nlag-1, at most 256
    int threads = 64 * ((a.nlag - 1 + 63) / 64);
    if (threads < 64) threads = 64;
    if (threads > LAG_THREADS) threads = LAG_THREADS;
    hipLaunchKernelGGL(k_internal, dim3((unsigned)rows), dim3((unsigned)threads), (size_t)(24 * longest + 8 * a.nlag), s, a,
                       longest);
    hipLaunchKernelGGL(k_lag_total, dim3((unsigned)a.nlag), dim3(LAG_THREADS), 0, s, a.lagsum, rows, a.nlag);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long grid = (n + 255) / 256;
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)grid), dim3(256), 0, s, p, n);
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

// gfx950 kernels of the event-chain (EC) move for tethered hard-sphere melts
// (Kampmann, Boltz, Kierfeld, arXiv:1502.06447, Sec. II and II.A).
//
// One wavefront (64 lanes) owns one active domain of a colour phase.  At the start
// of the phase it stages the domain and its one-cell halo from the cell lists:
// the staged beads are sorted by id and dealt out to the lanes, BPL beads per
// lane, with positions, cell words and tether partners held in VGPRs.  Every
// event then costs one pass over the lane's BPL beads (one candidate each: a
// hard-sphere contact, or for a tethered partner of the pivot that is not hit,
// the tether limit), a wavefront min-reduction through DPP, and a uniform update
// of the pivot.  Nothing in the event loop touches HBM; the phase ends by writing
// back the motile beads and rebuilding the domain's cell lists.
//
// Floating point: binary64, round to nearest, no contraction (built with
// -ffp-contract=off), correctly rounded sqrt; the operation order of every
// candidate distance, face distance and position update is fixed so that results
// are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include "ecmc_internal.h"

namespace ecmc {

namespace {

constexpr double INF = __builtin_huge_val();

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ double rdlane(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int rdlane(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned v) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ double fmin_(double a, double b) { return b < a ? b : a; }

// minimum over the wavefront, returned to every lane: butterfly inside each row of 16
// lanes (quad_perm 1032, quad_perm 2301, half-row mirror, row mirror), then the four
// row results read out and combined uniformly.
__device__ __forceinline__ double wave_min_f64(double v) {
    v = fmin_(v, dpp_f64<0xB1>(v));
    v = fmin_(v, dpp_f64<0x4E>(v));
    v = fmin_(v, dpp_f64<0x141>(v));
    v = fmin_(v, dpp_f64<0x140>(v));
    const double r0 = rdlane(v, 0), r1 = rdlane(v, 16), r2 = rdlane(v, 32), r3 = rdlane(v, 48);
    return fmin_(fmin_(r0, r1), fmin_(r2, r3));
}

__device__ __forceinline__ unsigned umin_(unsigned a, unsigned b) { return b < a ? b : a; }

__device__ __forceinline__ unsigned wave_min_u32(unsigned v) {
    v = umin_(v, dpp_u32<0xB1>(v));
    v = umin_(v, dpp_u32<0x4E>(v));
    v = umin_(v, dpp_u32<0x141>(v));
    v = umin_(v, dpp_u32<0x140>(v));
    const unsigned r0 = (unsigned)rdlane((int)v, 0), r1 = (unsigned)rdlane((int)v, 16);
    const unsigned r2 = (unsigned)rdlane((int)v, 32), r3 = (unsigned)rdlane((int)v, 48);
    return umin_(umin_(r0, r1), umin_(r2, r3));
}

// inclusive prefix sum over the wavefront (staging only)
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

__device__ __forceinline__ int mbcnt(unsigned long long m) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ int cell_of(int32_t m, int ax) { return (m >> (ax * CELL_BITS)) & CELL_MASK; }

// cell faces: bnd(k) = k h for k < n, bnd(n) = L
__device__ __forceinline__ double face(int k, int n, double h, double L) { return k < n ? (double)k * h : L; }

// ------------------------------------------------------------------ candidates
// Every lane holds BPL staged beads in a frame rotated to the current axis of motion:
// A = coordinate along the axis, B and C = the other two (cyclic order).  For each
// staged bead: the displacement from the pivot (periodic shift from the cell-index
// difference, added after the subtraction), its component along the motion d_par and
// the squared distance from the line of motion d_perp^2; then one candidate:
//   hard sphere, if d_par > 0 and d_perp^2 < sigma^2:  x = d_par - sqrt(sigma^2 - d_perp^2)
//   tether, for a partner of the pivot that is not hit:  x = d_par + sqrt(max(b^2 - d_perp^2, 0))
// (for a partner that is hit the contact always comes first: x_hs <= d_par <= x_tether),
// clamped at 0.  The lane keeps the smallest (x, staged index); staged indices follow
// bead ids, so this is the order by id.
template <int BPL>
struct Lanes {
    double A[BPL], B[BPL], C[BPL];
    int32_t META[BPL], PART[BPL];
};

struct Pivot {
    int P, slot, owner;
    int32_t meta, part;
    double a, b, c;
};

template <int BPL, bool WRAP>
__device__ __forceinline__ void candidates(const Lanes<BPL> &R, const Pivot &pv, int sha, int shb, int shc,
                                           double sgnd, double sig2, double b2, double L, double &bx,
                                           unsigned &bkey) {
    const int lane = lane_id();
    const int q0 = pv.part & 0xFFFF, q1 = (pv.part >> 16) & 0xFFFF;
    bx = INF;
    bkey = 0xFFFFFFFFu;
#pragma unroll
    for (int k = 0; k < BPL; ++k) {
        const int idx = k * 64 + lane;
        double da = R.A[k] - pv.a;
        double db = R.B[k] - pv.b;
        double dc = R.C[k] - pv.c;
        if (WRAP) {
            const int ea = (int)((R.META[k] >> sha) & CELL_MASK) - (int)((pv.meta >> sha) & CELL_MASK);
            const int eb = (int)((R.META[k] >> shb) & CELL_MASK) - (int)((pv.meta >> shb) & CELL_MASK);
            const int ec = (int)((R.META[k] >> shc) & CELL_MASK) - (int)((pv.meta >> shc) & CELL_MASK);
            da = da + (ea > 1 ? -L : (ea < -1 ? L : 0.0));
            db = db + (eb > 1 ? -L : (eb < -1 ? L : 0.0));
            dc = dc + (ec > 1 ? -L : (ec < -1 ? L : 0.0));
        }
        const double dpar = da * sgnd;
        const double pb = db * db;
        const double pc = dc * dc;
        const double dperp2 = pb + pc;
        const bool hs = (dpar > 0.0) && (dperp2 < sig2);
        const bool partner = (idx == q0) || (idx == q1);
        double arg = (hs ? sig2 : b2) - dperp2;
        if (!(arg > 0.0)) arg = 0.0;
        const double sq = __builtin_sqrt(arg);
        double x = hs ? dpar - sq : dpar + sq;
        if (!(x > 0.0)) x = 0.0;
        const bool ok = (idx != pv.P) && (hs || partner);
        if (ok && x < bx) {
            bx = x;
            bkey = (unsigned)(idx * 2 + (hs ? 0 : 1));
        }
    }
}

// Select element `slot` (uniform) of a lane's register array.  Written as a masked OR so
// that the compiler cannot turn it into an indexed load, which would move the array out
// of VGPRs into scratch memory.
template <int BPL>
__device__ __forceinline__ double pick(const double (&V)[BPL], int slot) {
    unsigned long long acc = 0;
#pragma unroll
    for (int k = 0; k < BPL; ++k) {
        const unsigned long long m = 0ull - (unsigned long long)(slot == k);
        acc |= (unsigned long long)__double_as_longlong(V[k]) & m;
    }
    return __longlong_as_double((long long)acc);
}

template <int BPL>
__device__ __forceinline__ int32_t pick(const int32_t (&V)[BPL], int slot) {
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < BPL; ++k) acc |= (uint32_t)V[k] & (0u - (uint32_t)(slot == k));
    return (int32_t)acc;
}

template <int BPL>
__device__ __forceinline__ void put(double (&V)[BPL], int slot, int owner, double v) {
    const bool me = lane_id() == owner;
#pragma unroll
    for (int k = 0; k < BPL; ++k)
        if (slot == k && me) V[k] = v;
}

template <int BPL>
__device__ __forceinline__ void put(int32_t (&V)[BPL], int slot, int owner, int32_t v) {
    const bool me = lane_id() == owner;
#pragma unroll
    for (int k = 0; k < BPL; ++k)
        if (slot == k && me) V[k] = v;
}

template <int BPL>
__device__ __forceinline__ Pivot load_pivot(int P, const Lanes<BPL> &R) {
    Pivot v;
    v.P = P;
    v.slot = P >> 6;
    v.owner = P & 63;
    v.a = rdlane(pick(R.A, v.slot), v.owner);
    v.b = rdlane(pick(R.B, v.slot), v.owner);
    v.c = rdlane(pick(R.C, v.slot), v.owner);
    v.meta = rdlane(pick(R.META, v.slot), v.owner);
    v.part = rdlane(pick(R.PART, v.slot), v.owner);
    return v;
}

// the pivot only moves along A, so only that coordinate and the cell word change
template <int BPL>
__device__ __forceinline__ void store_pivot(const Pivot &v, Lanes<BPL> &R) {
    put(R.A, v.slot, v.owner, v.a);
    put(R.META, v.slot, v.owner, v.meta);
}

__device__ __forceinline__ double blend(unsigned long long m, double x, double y) {
    const unsigned long long bx = (unsigned long long)__double_as_longlong(x);
    const unsigned long long by = (unsigned long long)__double_as_longlong(y);
    return __longlong_as_double((long long)((bx & m) | (by & ~m)));
}

// cyclic change of the frame: (A, B, C) = (r[ax], r[ax+1], r[ax+2]) for the new axis.
// A bitwise blend rather than two branches, so that the arrays stay in VGPRs.
template <int BPL>
__device__ __forceinline__ void rotate(Lanes<BPL> &R, int from, int to) {
    const int r = (to - from + 3) % 3;
    if (r == 0) return;
    const unsigned long long m = 0ull - (unsigned long long)(r == 1);
#pragma unroll
    for (int k = 0; k < BPL; ++k) {
        const double a = R.A[k], b = R.B[k], c = R.C[k];
        R.A[k] = blend(m, b, c);
        R.B[k] = blend(m, c, a);
        R.C[k] = blend(m, a, b);
    }
}

struct Tally {
    unsigned long long hs, tl, hr, tr, wall, cross, ec, steps;
    double dsum;
};

struct Frame {
    int ds[3];      // first cell of the domain per axis
    int S;          // staged beads
    uint32_t domain;
};

__device__ __forceinline__ void log_event(const PhaseArgs &a, const Frame &f, long long k, long long step, int p,
                                          int t, int kind) {
    if (lane_id() == 0) {
        const unsigned long long s = atomicAdd(a.log_n, 1ull);
        if ((long long)s < a.log_cap)
            a.log[s] = ecmc_event{a.sweep, f.domain, (uint32_t)k, (uint32_t)step, p, t, (uint32_t)kind,
                                  (uint32_t)a.colour};
        else
            atomicOr(a.err, ERR_LOG);
    }
}

// One EC along axis ax (the lanes' frame is already rotated to it), direction sign
// sgn, from staged pivot P0, x_max = ell.  Returns false if the iteration cap was hit.
template <int BPL, bool LOG>
__device__ __forceinline__ bool run_ec(const PhaseArgs &a, const Frame &f, const int32_t *s_id, Lanes<BPL> &R,
                                       int P0, int ax, int sgn, bool wr, long long k, Tally &t) {
    const int n = a.n;
    const double L = a.L, h = a.h;
    const int sha = ax * CELL_BITS, shb = ((ax + 1) % 3) * CELL_BITS, shc = ((ax + 2) % 3) * CELL_BITS;
    const int dsa = f.ds[0] * (ax == 0) + f.ds[1] * (ax == 1) + f.ds[2] * (ax == 2);
    Pivot pv = load_pivot(P0, R);
    double xmax = a.ell;
    long long step = 0;
    ++t.ec;
    for (;;) {
        if (step >= a.event_cap) {
            store_pivot(pv, R);
            return false;
        }
        ++step;
        ++t.steps;
        const double sgnd = sgn > 0 ? 1.0 : -1.0;
        double bx;
        unsigned bkey;
        if (wr) candidates<BPL, true>(R, pv, sha, shb, shc, sgnd, a.sig2, a.b2, L, bx, bkey);
        else candidates<BPL, false>(R, pv, sha, shb, shc, sgnd, a.sig2, a.b2, L, bx, bkey);
        const double xint = wave_min_f64(bx);
        unsigned key = 0xFFFFFFFFu;
        if (xint < INF) {
            const unsigned long long tie = __ballot(bx == xint);
            if (__popcll(tie) == 1) key = (unsigned)rdlane((int)bkey, (int)(__ffsll((long long)tie) - 1));
            else key = wave_min_u32(bx == xint ? bkey : 0xFFFFFFFFu);
        }
        const int c = (pv.meta >> sha) & CELL_MASK;
        const double r_old = pv.a;
        double xc = sgn > 0 ? face(c + 1, n, h, L) - r_old : r_old - face(c, n, h, L);
        if (!(xc > 0.0)) xc = 0.0;
        const double mlim = xint < xc ? xint : xc;
        if (xmax <= mlim) {
            // END: the pivot takes the rest of the displacement
            pv.a = sgn > 0 ? r_old + xmax : r_old - xmax;
            store_pivot(pv, R);
            if (LOG) log_event(a, f, k, step, s_id[pv.P], -1, ECMC_EV_END);
            return true;
        }
        if (xint <= xc) {
            // interaction event: move to contact / tether limit
            pv.a = sgn > 0 ? r_old + xint : r_old - xint;
            xmax = xmax - xint;
            const int j = (int)(key >> 1);
            const int kind = (int)(key & 1u);
            const int jslot = j >> 6, jown = j & 63;
            const int32_t jmeta = rdlane(pick(R.META, jslot), jown);
            if (jmeta & MOTILE_BIT) {
                // lift: the struck bead continues the chain; accumulate (d_par - x)
                const double jr = rdlane(pick(R.A, jslot), jown);
                double da = jr - r_old;
                if (wr) {
                    const int e = (int)((jmeta >> sha) & CELL_MASK) - c;
                    da = da + (e > 1 ? -L : (e < -1 ? L : 0.0));
                }
                const double dpar = da * sgnd;
                t.dsum += dpar - xint;
                if (kind == 0) ++t.hs;
                else ++t.tl;
                if (LOG) log_event(a, f, k, step, s_id[pv.P], s_id[j], kind == 0 ? ECMC_EV_HS_LIFT : ECMC_EV_TETHER_LIFT);
                store_pivot(pv, R);
                pv = load_pivot(j, R);
            } else {
                if (kind == 0) ++t.hr;
                else ++t.tr;
                if (LOG)
                    log_event(a, f, k, step, s_id[pv.P], s_id[j], kind == 0 ? ECMC_EV_HS_REFLECT : ECMC_EV_TETHER_REFLECT);
                sgn = -sgn;
            }
            continue;
        }
        // cell-face event: the pivot is set onto the face
        pv.a = sgn > 0 ? face(c + 1, n, h, L) : face(c, n, h, L);
        xmax = xmax - xc;
        int nc = c + sgn;
        int wrapped = 0;
        if (nc >= n) {
            nc = 0;
            wrapped = 1;
        } else if (nc < 0) {
            nc = n - 1;
            wrapped = -1;
        }
        const bool inside = a.whole || ((nc - dsa + n) % n) < a.D;
        if (inside) {
            pv.meta = (pv.meta & ~(CELL_MASK << sha)) | (nc << sha);
            if (wrapped > 0) {
                pv.a = 0.0;
                if (lane_id() == 0) a.img[3 * s_id[pv.P] + ax] += 1;
            } else if (wrapped < 0) {
                pv.a = L;
                if (lane_id() == 0) a.img[3 * s_id[pv.P] + ax] -= 1;
            }
            ++t.cross;
        } else {
            ++t.wall;
            if (LOG) log_event(a, f, k, step, s_id[pv.P], -1, ECMC_EV_WALL);
            sgn = -sgn;
        }
    }
}

// ------------------------------------------------------------------ phase kernel
template <int BPL, bool LOG>
__global__ __launch_bounds__(64) void k_phase(const PhaseArgs a) {
    constexpr int SMAX = 64 * BPL;
    __shared__ int32_t s_id[SMAX];    // staged bead ids, ascending
    __shared__ int32_t s_meta[SMAX];
    __shared__ int32_t t_id[SMAX];    // unsorted ids, then the motile list
    __shared__ int32_t t_meta[SMAX];  // unsorted cell words, then write-back counters

    const int lane = lane_id();
    const int n = a.n;

    // ---- which domain
    Frame f;
    int dom[3] = {0, 0, 0};
    f.domain = 0;
    if (!a.whole) {
        const int nd2 = a.nd >> 1;
        const int b = blockIdx.x;
        dom[0] = 2 * (b % nd2) + (a.colour & 1);
        dom[1] = 2 * ((b / nd2) % nd2) + ((a.colour >> 1) & 1);
        dom[2] = 2 * (b / (nd2 * nd2)) + ((a.colour >> 2) & 1);
        f.domain = (uint32_t)(dom[0] + a.nd * (dom[1] + a.nd * dom[2]));
    }
    const int F = a.whole ? n : a.D + 2;
    int fs[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        f.ds[ax] = a.whole ? 0 : (a.off[ax] + dom[ax] * a.D) % n;
        fs[ax] = a.whole ? 0 : (f.ds[ax] - 1 + n) % n;
    }
    // the frame (domain + halo) wraps the periodic box on some axis
    const bool wraps = a.whole || fs[0] + F > n || fs[1] + F > n || fs[2] + F > n;

    // ---- stage the frame's beads: cell counts, prefix sum, ids and cell words
    const int nfc = F * F * F;
    int S = 0;
    for (int base = 0; base < nfc; base += 64) {
        const int c = base + lane;
        int cnt = 0, flat = 0;
        int32_t word = 0;
        if (c < nfc) {
            const int fx = c % F, fy = (c / F) % F, fz = c / (F * F);
            const int cx = (fs[0] + fx) % n, cy = (fs[1] + fy) % n, cz = (fs[2] + fz) % n;
            flat = cx + n * (cy + n * cz);
            const bool mot = a.whole || (fx >= 1 && fx <= a.D && fy >= 1 && fy <= a.D && fz >= 1 && fz <= a.D);
            word = pack_cell(cx, cy, cz) | (mot ? MOTILE_BIT : 0);
            cnt = a.ccount[flat];
        }
        const int incl = wave_incl_scan(cnt);
        const int excl = incl - cnt;
        const int tot = rdlane(incl, 63);
        if (S + incl <= SMAX) {
            for (int i = 0; i < cnt; ++i) {
                t_id[S + excl + i] = a.cids[(long long)flat * a.cap + i];
                t_meta[S + excl + i] = word;
            }
        }
        S += tot;
    }
    if (S > SMAX) {
        if (lane == 0) atomicOr(a.err, ERR_STAGE);
        return;
    }
    f.S = S;
    __syncthreads();
    // rank sort by bead id
    for (int e = lane; e < S; e += 64) {
        const int my = t_id[e];
        int r = 0;
        for (int i = 0; i < S; ++i) r += (t_id[i] < my) ? 1 : 0;
        s_id[r] = my;
        s_meta[r] = t_meta[e];
    }
    __syncthreads();

    // lanes' beads in frame (x, y, z); empty slots far away so they never yield a candidate
    Lanes<BPL> R;
#pragma unroll
    for (int k = 0; k < BPL; ++k) {
        const int idx = k * 64 + lane;
        R.A[k] = R.B[k] = R.C[k] = 1.0e30;
        R.META[k] = 0;
        R.PART[k] = -1;
        if (idx < S) {
            const int id = s_id[idx];
            R.META[k] = s_meta[idx];
            R.A[k] = a.px[id];
            R.B[k] = a.py[id];
            R.C[k] = a.pz[id];
            if (R.META[k] & MOTILE_BIT) {
                int packed = 0;
                for (int tt = 0; tt < 2; ++tt) {
                    const int g = a.part[2 * id + tt];
                    int found = 0xFFFF;
                    if (g >= 0) {
                        int lo = 0, hi = S - 1;
                        while (lo <= hi) {
                            const int mid = (lo + hi) >> 1;
                            const int v = s_id[mid];
                            if (v == g) {
                                found = mid;
                                break;
                            }
                            if (v < g) lo = mid + 1;
                            else hi = mid - 1;
                        }
                    }
                    packed |= found << (16 * tt);
                }
                R.PART[k] = packed;
            }
        }
    }
    // motile list in ascending id (reuses t_id)
    int nmot = 0;
#pragma unroll
    for (int k = 0; k < BPL; ++k) {
        const int idx = k * 64 + lane;
        const bool m = idx < S && (R.META[k] & MOTILE_BIT);
        const unsigned long long bal = __ballot(m);
        if (m) t_id[nmot + mbcnt(bal)] = idx;
        nmot += __popcll(bal);
    }
    __syncthreads();

    // ---- ECs
    Tally t = {0, 0, 0, 0, 0, 0, 0, 0, 0.0};
    bool ok = true;
    int cur = 0;  // axis the lanes' frame is rotated to
    for (long long k = 0; k < a.K && nmot > 0 && ok; ++k) {
        uint32_t ctr[4] = {(uint32_t)k, f.domain, a.sweep, 0u};
        philox4x32_10(ctr, a.key0, a.key1);
        const int P0 = __builtin_amdgcn_readfirstlane(t_id[scale_u32(ctr[0], (uint32_t)nmot)]);
        const uint32_t dir = scale_u32(ctr[1], 6u);
        const int ax = __builtin_amdgcn_readfirstlane((int)(dir >> 1));
        const int sgn = (dir & 1u) ? -1 : 1;
        rotate(R, cur, ax);
        cur = ax;
        ok = run_ec<BPL, LOG>(a, f, s_id, R, P0, ax, sgn, wraps, k, t);
    }
    rotate(R, cur, 0);

    // ---- write back the motile beads and the domain's cell lists
    const int ndc = a.whole ? n * n * n : a.D * a.D * a.D;
    for (int i = lane; i < ndc; i += 64) t_meta[i] = 0;
    __syncthreads();
    bool overflow = false;
#pragma unroll
    for (int k = 0; k < BPL; ++k) {
        const int idx = k * 64 + lane;
        if (idx < S && (R.META[k] & MOTILE_BIT)) {
            const int id = s_id[idx];
            a.px[id] = R.A[k];
            a.py[id] = R.B[k];
            a.pz[id] = R.C[k];
            const int32_t w = R.META[k] & ~MOTILE_BIT;
            a.cellp[id] = w;
            const int cx = cell_of(w, 0), cy = cell_of(w, 1), cz = cell_of(w, 2);
            int lc;
            if (a.whole) {
                lc = cx + n * (cy + n * cz);
            } else {
                const int tx = (cx - f.ds[0] + n) % n, ty = (cy - f.ds[1] + n) % n, tz = (cz - f.ds[2] + n) % n;
                lc = tx + a.D * (ty + a.D * tz);
            }
            const int slot = atomicAdd(&t_meta[lc], 1);
            if (slot < a.cap) a.cids[(long long)(cx + n * (cy + n * cz)) * a.cap + slot] = id;
            else overflow = true;
        }
    }
    __syncthreads();
    for (int i = lane; i < ndc; i += 64) {
        int cx, cy, cz;
        if (a.whole) {
            cx = i % n;
            cy = (i / n) % n;
            cz = i / (n * n);
        } else {
            cx = (f.ds[0] + i % a.D) % n;
            cy = (f.ds[1] + (i / a.D) % a.D) % n;
            cz = (f.ds[2] + i / (a.D * a.D)) % n;
        }
        const int v = t_meta[i];
        a.ccount[cx + n * (cy + n * cz)] = v < a.cap ? v : a.cap;
    }
    if (__ballot(overflow) && lane == 0) atomicOr(a.err, ERR_CELL);
    if (lane == 0) {
        if (!ok) atomicOr(a.err, ERR_STUCK);
        if (t.hs) atomicAdd(&a.cnt[C_HS_LIFT], t.hs);
        if (t.tl) atomicAdd(&a.cnt[C_TETHER_LIFT], t.tl);
        if (t.hr) atomicAdd(&a.cnt[C_HS_REFLECT], t.hr);
        if (t.tr) atomicAdd(&a.cnt[C_TETHER_REFLECT], t.tr);
        if (t.wall) atomicAdd(&a.cnt[C_WALL], t.wall);
        if (t.cross) atomicAdd(&a.cnt[C_CROSS], t.cross);
        if (t.ec) atomicAdd(&a.cnt[C_EC], t.ec);
        if (t.steps) atomicAdd(&a.cnt[C_STEPS], t.steps);
        if (t.dsum != 0.0) atomicAdd(a.sum_delta, t.dsum);
    }
}

// ------------------------------------------------------------------ observables
// One thread per polymer: R = sum of minimum-image bonds, unwrapped positions u for the
// centre of mass and R_g^2 = N^-1 sum (u - u_cm)^2, the middle bead unwrapped with its
// image counters, bond lengths binned on [sigma, b_max].
__global__ void k_observables(const ObsArgs a) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < a.npoly;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = a.pstart[q], e = a.pstart[q + 1];
        const int64_t N = e - s;
        auto mi = [&](double d) { return d > a.halfL ? d - a.L : (d < -a.halfL ? d + a.L : d); };
        const int i0 = a.porder[s];
        double u0 = a.px[i0], u1 = a.py[i0], u2 = a.pz[i0];
        double R0 = 0.0, R1 = 0.0, R2 = 0.0;
        double s0 = u0, s1 = u1, s2 = u2;
        for (int64_t t = s + 1; t < e; ++t) {
            const int ia = a.porder[t - 1], ib = a.porder[t];
            const double d0 = mi(a.px[ib] - a.px[ia]);
            const double d1 = mi(a.py[ib] - a.py[ia]);
            const double d2 = mi(a.pz[ib] - a.pz[ia]);
            R0 += d0;
            u0 += d0;
            s0 += u0;
            R1 += d1;
            u1 += d1;
            s1 += u1;
            R2 += d2;
            u2 += d2;
            s2 += u2;
            if (a.hist) {
                const double q0 = d0 * d0;
                const double q1 = d1 * d1;
                const double q2 = d2 * d2;
                const double len = __builtin_sqrt(q0 + q1 + q2);
                int bin = (int)__builtin_floor((len - a.sigma) / (a.bmax - a.sigma) * a.nbins);
                if (bin < 0) bin = 0;
                if (bin > a.nbins - 1) bin = a.nbins - 1;
                atomicAdd(&a.hist[bin], 1ull);
            }
        }
        const double c0 = s0 / (double)N, c1 = s1 / (double)N, c2 = s2 / (double)N;
        const double r0 = R0 * R0;
        const double r1 = R1 * R1;
        const double r2 = R2 * R2;
        a.r2[q] = r0 + r1 + r2;
        double g = 0.0;
        double v0 = a.px[i0], v1 = a.py[i0], v2 = a.pz[i0];
        for (int64_t t = s; t < e; ++t) {
            if (t > s) {
                const int ia = a.porder[t - 1], ib = a.porder[t];
                v0 += mi(a.px[ib] - a.px[ia]);
                v1 += mi(a.py[ib] - a.py[ia]);
                v2 += mi(a.pz[ib] - a.pz[ia]);
            }
            const double w0 = (v0 - c0) * (v0 - c0);
            g += w0;
            const double w1 = (v1 - c1) * (v1 - c1);
            g += w1;
            const double w2 = (v2 - c2) * (v2 - c2);
            g += w2;
        }
        a.rg2[q] = g / (double)N;
        const int im = a.porder[s + N / 2];
        a.mid[3 * q + 0] = a.px[im] + (double)a.img[3 * im + 0] * a.L;
        a.mid[3 * q + 1] = a.py[im] + (double)a.img[3 * im + 1] * a.L;
        a.mid[3 * q + 2] = a.pz[im] + (double)a.img[3 * im + 2] * a.L;
    }
}

}  // namespace

bool bpl_supported(int bpl) {
    switch (bpl) {
        case 1: case 2: case 3: case 4: case 6: case 8: case 12: case 16: return true;
        default: return false;
    }
}

template <int BPL>
static hipError_t launch_bpl(const PhaseArgs &a, bool log, int grid, hipStream_t s) {
    if (log) hipLaunchKernelGGL((k_phase<BPL, true>), dim3(grid), dim3(64), 0, s, a);
    else hipLaunchKernelGGL((k_phase<BPL, false>), dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
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

hipError_t launch_observables(const ObsArgs &a, hipStream_t s) {
    if (a.npoly <= 0) return hipSuccess;
    const int block = 256;
    int64_t grid = (a.npoly + block - 1) / block;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_observables, dim3((unsigned)grid), dim3(block), 0, s, a);
    return hipGetLastError();
}

}  // namespace ecmc

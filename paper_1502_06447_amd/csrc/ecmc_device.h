// Device code of the event-chain (EC) move for tethered hard-sphere melts on gfx950
// (Kampmann, Boltz, Kierfeld, arXiv:1502.06447, Sec. II and II.A), shared by the two
// schedules of a sweep: one launch per colour phase (ecmc_kernels.hip) and one
// dependency-ordered launch per sweep (ecmc_sweep.hip).
//
// One wavefront (64 lanes) owns one active domain at a time.  It stages the domain and its
// one-cell halo from the cell lists: the staged beads are sorted by id and dealt out to the
// lanes, BPL beads per lane, with single-precision screening copies of the positions in
// VGPRs and the FP64 positions, cell words and tether partners in LDS.  Every event then
// costs one pass over the lane's BPL beads (one candidate each: a hard-sphere contact, or
// for a tethered partner of the pivot that is not hit, the tether limit), a wavefront
// min-reduction through DPP, an FP64 evaluation of the few beads the screen cannot rule
// out, and a uniform update of the pivot.  Nothing in the event loop touches HBM; the
// domain ends by writing back its motile beads and rebuilding its cell lists.
//
// Floating point: binary64, round to nearest, no contraction (built with
// -ffp-contract=off), correctly rounded sqrt; the operation order of every candidate
// distance, face distance and position update is fixed so that results are reproducible
// bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include "ecmc_internal.h"

namespace ecmc {

namespace {

constexpr double INF = __builtin_huge_val();

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// A kernel argument read again where it is used.  Arguments needed only before and after the
// EC loop (the staging and write-back pointers, the sweep's own state) would otherwise stay
// in scalar registers through the loop and push its constants out to VGPR lanes, to be
// reloaded at every step.
template <class T>
__device__ __forceinline__ T late(const T &arg) {
    return *(const volatile T *)&arg;
}

__device__ __forceinline__ double rdlane(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int rdlane(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// DPP lane move within a row of 16 lanes (a full permutation: every lane has a source; the
// lane's own value is the fallback a disabled source would give).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int l = __double2loint(v), u = __double2hiint(v);
    const int lo = __builtin_amdgcn_update_dpp(l, l, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(u, u, CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}


__device__ __forceinline__ unsigned umin_(unsigned a, unsigned b) { return b < a ? b : a; }

// One step of a wavefront min-reduction of unsigned words: the lane's value against the one
// the DPP control brings in; lanes outside row_mask, or with no source, keep their own (the
// identity 0xFFFFFFFF stands in).  The compiler folds the move into v_min_u32_dpp.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned umin_dpp(unsigned v) {
    return umin_(v, (unsigned)__builtin_amdgcn_update_dpp((int)0xFFFFFFFFu, (int)v, CTRL, ROWS, 0xF, false));
}

// Minimum over the wavefront, returned to every lane.  Within each row of 16 lanes a
// butterfly (quad_perm 1032, quad_perm 2301, half-row mirror, row mirror), then row 1 takes
// row 0 (row_bcast:15), row 3 takes row 2, and rows 2-3 take row 1 (row_bcast:31): lane 63
// holds the minimum of all 64 lanes.
__device__ __forceinline__ unsigned wave_min_u32(unsigned v) {
    v = umin_dpp<0xB1, 0xF>(v);
    v = umin_dpp<0x4E, 0xF>(v);
    v = umin_dpp<0x141, 0xF>(v);
    v = umin_dpp<0x140, 0xF>(v);
    v = umin_dpp<0x142, 0xA>(v);
    v = umin_dpp<0x143, 0xC>(v);
    return (unsigned)rdlane((int)v, 63);
}

// two such reductions interleaved (they share the latency of the DPP steps)
__device__ __forceinline__ void wave_min2_u32(unsigned &u, unsigned &v) {
    u = umin_dpp<0xB1, 0xF>(u);
    v = umin_dpp<0xB1, 0xF>(v);
    u = umin_dpp<0x4E, 0xF>(u);
    v = umin_dpp<0x4E, 0xF>(v);
    u = umin_dpp<0x141, 0xF>(u);
    v = umin_dpp<0x141, 0xF>(v);
    u = umin_dpp<0x140, 0xF>(u);
    v = umin_dpp<0x140, 0xF>(v);
    u = umin_dpp<0x142, 0xA>(u);
    v = umin_dpp<0x142, 0xA>(v);
    u = umin_dpp<0x143, 0xC>(u);
    v = umin_dpp<0x143, 0xC>(v);
    u = (unsigned)rdlane((int)u, 63);
    v = (unsigned)rdlane((int)v, 63);
}

// Minimum over the wavefront of a value that is >= 0 or +inf.  For such doubles the bit
// patterns order like the numbers, so the high words are reduced first and then the low
// words of the lanes that hold the smallest high word.
__device__ __forceinline__ double wave_min_nonneg_f64(double v) {
    const unsigned hi = (unsigned)__double2hiint(v), lo = (unsigned)__double2loint(v);
    const unsigned mh = wave_min_u32(hi);
    const unsigned ml = wave_min_u32(hi == mh ? lo : 0xFFFFFFFFu);
    return __hiloint2double((int)mh, (int)ml);
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

// ------------------------------------------------------------------ event search
// Every lane holds single-precision screening copies of its BPL staged beads, in the
// domain frame (coordinates relative to the frame's lower corner, unwrapped across the
// periodic boundary) rotated to the current axis of motion: A along the axis, B and C
// the other two in cyclic order.  The exact FP64 positions, cell words and tether
// partners of the staged beads live in LDS and are read only for the few beads the
// screen cannot rule out.
template <int NS, bool WHOLE>
struct Lanes {
    float A[NS], B[NS], C[NS];
    int32_t META[WHOLE ? NS : 1];  // whole box: cell words for the periodic shift of the screen
};

// Register slots of the screening copies: the plain FP64 search (EXACT) screens nothing and
// keeps a single unused slot.
constexpr int lane_slots(int bpl, bool exact) { return exact ? 1 : bpl; }

// the current pivot, uniform across the wavefront
struct Pivot {
    int P;            // staged index
    int32_t meta;     // cell word
    int32_t part;     // staged indices of the tethered partners (16 bits each, 0xFFFF = none)
    double a, b, c;   // FP64 position in the rotated frame
    float fa, fb, fc; // screening copy
};

// the staged data in LDS
struct Stage {
    double *pos;           // FP64 x, y, z: three rows of `stride` doubles
    int stride;
    int32_t *meta;
    int32_t *part;
    int32_t *id;
    // address arithmetic rather than a select of three pointers, which the compiler turns
    // into a pointer table in scratch memory
    __device__ __forceinline__ double *axis(int ax) const { return pos + ax * stride; }
};

// Correctly rounded square root of an x that is 0 or at least 2^-767 (every argument here:
// a difference of squares of lengths near sigma, or 0 after the clamp).  A hardware estimate
// of 1/sqrt(x) refined by coupled Newton steps on g ~ sqrt(x) and h ~ 1/(2 sqrt(x)), with a
// final residual correction (Markstein); the general square root adds a rescaling for
// x < 2^-767 and a fix-up for 0 and infinity around the same steps, which for these
// arguments change nothing: the results are the same bits.
__device__ __forceinline__ double sqrt_nonneg(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    double d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    return x > 0.0 ? g : 0.0;
}

// Exact FP64 candidate of one staged bead: displacement from the pivot (periodic shift
// from the cell-index difference, added after the subtraction), d_par and d_perp^2, then
//   hard sphere, if d_par > 0 and d_perp^2 < sigma^2:  x = d_par - sqrt(sigma^2 - d_perp^2)
//   tether, for a partner of the pivot that is not hit:  x = d_par + sqrt(max(b^2 - d_perp^2, 0))
// (for a partner that is hit the contact always comes first: x_hs <= d_par <= x_tether),
// clamped at 0.  Returns whether the bead is a candidate at all.
//
// Springs (Eq. (2), SPRING): a partner that is not hit takes the tether formula with b^2
// replaced by the square of the bond length at which the drawn energy dE is used up, capped
// at b^2.  The bond shortens at no cost until the pivot passes the partner's foot on its
// line and lengthens after it; from the shortest length still ahead, b0 = d_perp if
// d_par > 0 and the present length otherwise, (k/2)(b - sigma)^2 grows by dE at
// b_end = sigma + sqrt((b0 - sigma)^2 + g) with g = 2 dE / k.  The general correctly
// rounded square root is used there: its arguments are not bounded away from 0.
//
// Push-off (Sec. II.B, PUSH): a bead closer to the pivot than the working diameter (squared
// distance below ov2 = d^2 (1 - 1e-9)) is no hard-sphere event; sig2 is then d^2.
// d_par and d_perp^2 of a staged bead relative to the pivot: the displacement in the rotated
// frame (with the periodic shift from the cell-index difference added after the subtraction
// when the frame wraps), d_par along the direction of motion.  Every search computes them
// with this one sequence of operations, so that they agree on every bit.
template <bool WRAP>
__device__ __forceinline__ void rel_to_pivot(double A, double B, double C, int32_t meta, const Pivot &pv, int sha,
                                             int shb, int shc, double sgnd, double L, double &dpar, double &dperp2) {
    double da = A - pv.a;
    double db = B - pv.b;
    double dc = C - pv.c;
    if (WRAP) {
        const int ea = (int)((meta >> sha) & CELL_MASK) - (int)((pv.meta >> sha) & CELL_MASK);
        const int eb = (int)((meta >> shb) & CELL_MASK) - (int)((pv.meta >> shb) & CELL_MASK);
        const int ec = (int)((meta >> shc) & CELL_MASK) - (int)((pv.meta >> shc) & CELL_MASK);
        da = da + (ea > 1 ? -L : (ea < -1 ? L : 0.0));
        db = db + (eb > 1 ? -L : (eb < -1 ? L : 0.0));
        dc = dc + (ec > 1 ? -L : (ec < -1 ? L : 0.0));
    }
    dpar = da * sgnd;
    const double pb = db * db;
    const double pc = dc * dc;
    dperp2 = pb + pc;
}

template <bool WRAP, bool SPRING = false, bool PUSH = false>
__device__ __forceinline__ bool exact_candidate(double A, double B, double C, int32_t meta, const Pivot &pv, int sha,
                                                int shb, int shc, double sgnd, double sig2, double b2, double L,
                                                bool partner, double &x, bool &hs, double gterm = 0.0,
                                                double sigma = 0.0, double ov2 = 0.0) {
    double dpar, dperp2;
    rel_to_pivot<WRAP>(A, B, C, meta, pv, sha, shb, shc, sgnd, L, dpar, dperp2);
    hs = (dpar > 0.0) && (dperp2 < sig2);
    if (PUSH && hs && dpar * dpar + dperp2 < ov2) hs = false;
    double bb2 = b2;
    if (SPRING && partner && !hs) {
        const double b0 = __builtin_sqrt(dpar > 0.0 ? dperp2 : dpar * dpar + dperp2);
        const double e = b0 - sigma;
        const double be = sigma + __builtin_sqrt(e * e + gterm);
        const double be2 = be * be;
        bb2 = be2 > b2 ? b2 : be2;
    }
    double arg = (hs ? sig2 : bb2) - dperp2;
    if (!(arg > 0.0)) arg = 0.0;
    const double sq = sqrt_nonneg(arg);
    double v = hs ? dpar - sq : dpar + sq;
    if (!(v > 0.0)) v = 0.0;
    x = v;
    return hs || partner;
}

// Single-precision screen constants (derived on the host, see ecmc_api.cpp).
struct ScreenK {
    float sig2f, b2f;    // sigma^2, b^2 in float
    float in_lo, in_hi;  // float d_perp^2 below in_lo: surely inside sigma; not below in_hi: surely not
    float p_sure;        // float d_par above it: surely ahead; d_par ahead implies float d_par > -p_sure
    float err;           // bound on |x_float - x_exact| for every candidate
    float Lf;
};

// The winner of the event search and the data the pivot needs if it is lifted to it.
struct Hit {
    double x;
    unsigned key;       // staged index * 2 + kind (0 hard sphere, 1 tether)
    double a, b, c;     // FP64 position of the struck bead (rotated frame)
    int32_t meta, part;
};

// The single-precision screen of one event search.  For every staged bead the lane holding
// it computes a float estimate of the bead's x and an interval [lo, hi] that provably holds
// the exact x of each bead that is a candidate at all (lo = +inf for beads that cannot be).
// t = min hi and l = min lo over the wavefront: the exact interaction distance x_int lies in
// [l, t] whenever a candidate exists (x_int = +inf, l = t = +inf otherwise).
template <int BPL>
struct Screen {
    float lo[BPL];
    float t, l;
};

template <int BPL, bool WHOLE, bool SPRING = false>
__device__ __forceinline__ void screen(Screen<BPL> &sc, const Lanes<BPL, WHOLE> &R, const Pivot &pv, int sha, int shb,
                                       int shc, double sgnd, const ScreenK &K) {
    const int q0 = pv.part & 0xFFFF, q1 = (pv.part >> 16) & 0xFFFF;
    const float sgnf = sgnd > 0.0 ? 1.0f : -1.0f;
    // minima of hi and lo as bit patterns: both are >= 0 (or +inf), where the unsigned order of
    // the patterns is the order of the numbers
    constexpr unsigned INFB = 0x7F800000u;
    unsigned hmin = INFB, lmin = INFB;
#pragma unroll
    for (int k = 0; k < BPL; ++k) {
        // the lanes of this slot holding the pivot and its partners, as scalar lane masks
        const unsigned long long mme = (pv.P >> 6) == k ? 1ull << (pv.P & 63) : 0ull;
        const unsigned long long mpart =
            ((q0 >> 6) == k ? 1ull << (q0 & 63) : 0ull) | ((q1 >> 6) == k ? 1ull << (q1 & 63) : 0ull);
        float da = R.A[k] - pv.fa;
        float db = R.B[k] - pv.fb;
        float dc = R.C[k] - pv.fc;
        if (WHOLE) {
            const int ea = (int)((R.META[k] >> sha) & CELL_MASK) - (int)((pv.meta >> sha) & CELL_MASK);
            const int eb = (int)((R.META[k] >> shb) & CELL_MASK) - (int)((pv.meta >> shb) & CELL_MASK);
            const int ec = (int)((R.META[k] >> shc) & CELL_MASK) - (int)((pv.meta >> shc) & CELL_MASK);
            da = da + (ea > 1 ? -K.Lf : (ea < -1 ? K.Lf : 0.0f));
            db = db + (eb > 1 ? -K.Lf : (eb < -1 ? K.Lf : 0.0f));
            dc = dc + (ec > 1 ? -K.Lf : (ec < -1 ? K.Lf : 0.0f));
        }
        const float p = da * sgnf;
        // one rounding fewer than db * db + dc * dc, so within the same error bound
        const float q = __builtin_fmaf(db, db, dc * dc);
        // lane masks (one ballot per comparison, combined in scalar registers): a hard-sphere
        // contact surely / possibly ahead
        const unsigned long long m_sure = __ballot(p > K.p_sure) & __ballot(q < K.in_lo);
        const unsigned long long m_maybe = __ballot(p > -K.p_sure) & __ballot(q < K.in_hi);
        const bool hs_maybe = __builtin_amdgcn_inverse_ballot_w64(m_maybe);
        // the estimate follows the hard-sphere formula whenever a contact is possible; a
        // partner that may or may not be hit gets the interval spanning both formulas.  The
        // exact x is >= 0, so lo is clamped there: still a lower bound, and the membership
        // test lo <= t (t >= 0) is unchanged.
        const float sr = __builtin_amdgcn_sqrtf(fmaxf(hs_maybe ? K.sig2f - q : K.b2f - q, 0.0f));
        const float est = fmaxf(hs_maybe ? p - sr : p + sr, 0.0f);
        float l = fmaxf(est - K.err, 0.0f), hg = est + K.err;
        const unsigned long long m_amb = mpart & m_maybe & ~m_sure;
        if (__builtin_expect(m_amb != 0, 0)) {
            if (__builtin_amdgcn_inverse_ballot_w64(m_amb)) {
                const float st2 = __builtin_amdgcn_sqrtf(fmaxf(K.b2f - q, 0.0f));
                const float et = fmaxf(p + st2, 0.0f);
                l = fminf(l, fmaxf(et - K.err, 0.0f));
                hg = fmaxf(hg, et + K.err);
            }
        }
        if constexpr (SPRING) {
            // a spring partner not hit has d_par <= x <= x_tether (its bond length at the event
            // is at most b_max and at least the shortest one ahead): the tether estimate stays
            // an upper bound, and the float d_par (within K.err of the exact one) a lower one
            if (__builtin_amdgcn_inverse_ballot_w64(mpart)) l = fminf(l, fmaxf(p - K.err, 0.0f));
        }
        // candidates: possible contacts and the partners, never the pivot itself
        const bool cand = __builtin_amdgcn_inverse_ballot_w64(~mme & (m_maybe | mpart));
        sc.lo[k] = cand ? l : __builtin_huge_valf();
        hmin = umin_(hmin, cand ? __float_as_uint(hg) : INFB);
        lmin = umin_(lmin, __float_as_uint(sc.lo[k]));
    }
    wave_min2_u32(hmin, lmin);
    sc.t = __uint_as_float(hmin);
    sc.l = __uint_as_float(lmin);
}

// Exact first interaction event after the screen: the minimum over all staged beads of
// (x, staged index, kind), evaluated in FP64 from LDS only for the beads whose interval
// starts at or below the threshold t (normally one bead).  Their exact minimum x* is
// certified when x* <= t; otherwise t is raised to x* and the step repeats.  A bead left
// out has exact x >= lo > t >= x*, so the result is exact.  When a single bead passes,
// it is evaluated on its own lane and broadcast without a wavefront reduction.
//
// Every branch below depends on wavefront-uniform values only (ballots, readlanes and
// readfirstlane'd flags), so the wavefront never splits: the DPP reductions need all lanes.
struct Best {
    double x, A, B, C;
    unsigned key;
    int32_t meta, part;
};

// evaluate in FP64 the beads of this lane that are members (lo <= thr, not yet done).  The
// first pass has thr = t, a float: lo <= t is then compared in single precision, which is
// the same comparison.
template <int BPL, bool FIRST, bool SPRING = false>
__device__ __forceinline__ void search_pass(const Screen<BPL> &sc, double thr, unsigned &done, Best &b,
                                            const Stage &st, const Pivot &pv, const double *pA, const double *pB,
                                            const double *pC, int q0, int q1, int sha, int shb, int shc,
                                            double sgnd, double sig2, double b2, double L, bool wr,
                                            double g0 = 0.0, double g1 = 0.0, double sigma = 0.0) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < BPL; ++k) {
        const bool mem = FIRST ? sc.lo[k] <= sc.t
                               : !((done >> k) & 1u) && sc.lo[k] < __builtin_huge_valf() && (double)sc.lo[k] <= thr;
        if (__ballot(mem)) {
            if (mem) {
                const int idx = k * 64 + lane;
                const double A = pA[idx], B = pB[idx], C = pC[idx];
                const int32_t m = st.meta[idx];
                const bool partner = (idx == q0) || (idx == q1);
                const double gt = idx == q0 ? g0 : g1;
                double x;
                bool hs;
                const bool ok = (idx != pv.P) &&
                                (wr ? exact_candidate<true, SPRING>(A, B, C, m, pv, sha, shb, shc, sgnd, sig2, b2, L,
                                                                    partner, x, hs, gt, sigma)
                                    : exact_candidate<false, SPRING>(A, B, C, m, pv, sha, shb, shc, sgnd, sig2, b2, L,
                                                                     partner, x, hs, gt, sigma));
                const unsigned kk = (unsigned)(idx * 2 + (hs ? 0 : 1));
                if (ok && (x < b.x || (x == b.x && kk < b.key))) {
                    b.x = x;
                    b.key = kk;
                    b.A = A;
                    b.B = B;
                    b.C = C;
                    b.meta = m;
                    b.part = st.part[idx];
                }
            }
        }
        if (mem) done |= 1u << k;
    }
}

__device__ __forceinline__ void take(Hit &h, const Best &b, int wl) {
    h.x = rdlane(b.x, wl);
    h.key = (unsigned)rdlane((int)b.key, wl);
    h.a = rdlane(b.A, wl);
    h.b = rdlane(b.B, wl);
    h.c = rdlane(b.C, wl);
    h.meta = rdlane((int)b.meta, wl);
    h.part = rdlane((int)b.part, wl);
}

template <int BPL, bool SPRING = false>
__device__ __forceinline__ Hit search(const Screen<BPL> &sc, const Stage &st, const Pivot &pv, int ax, int sha,
                                      int shb, int shc, double sgnd, double sig2, double b2, double L, bool wr,
                                      double g0 = 0.0, double g1 = 0.0, double sigma = 0.0) {
    const int q0 = pv.part & 0xFFFF, q1 = (pv.part >> 16) & 0xFFFF;
    const double *pA = st.axis(ax);
    const double *pB = st.axis(ax == 2 ? 0 : ax + 1);
    const double *pC = st.axis(ax == 0 ? 2 : ax - 1);
    Hit h;
    h.x = INF;
    h.key = 0xFFFFFFFFu;
    h.a = h.b = h.c = 0.0;
    h.meta = 0;
    h.part = -1;
    if (!(sc.l < __builtin_huge_valf())) return h;
    double thr = (double)sc.t;
    Best b;  // the position, cell word and partners are read only after a candidate is stored
    b.x = INF;
    b.key = 0xFFFFFFFFu;
    unsigned done = 0;
    int nmem = 0;
#pragma unroll
    for (int k = 0; k < BPL; ++k) nmem += __popcll(__ballot(sc.lo[k] <= sc.t));
    search_pass<BPL, true, SPRING>(sc, thr, done, b, st, pv, pA, pB, pC, q0, q1, sha, shb, shc, sgnd, sig2, b2, L, wr,
                                   g0, g1, sigma);
    if (nmem == 1) {
        // one bead passed the screen: it set the threshold (its own hi is t), so when it is
        // a candidate its exact x <= t is the certified minimum
        const unsigned long long own = __ballot(b.x < INF);
        if (own) {
            const int wl = (int)(__ffsll((long long)own) - 1);
            const double x1 = rdlane(b.x, wl);
            if (__builtin_amdgcn_readfirstlane((int)(x1 <= thr))) {
                take(h, b, wl);
                return h;
            }
        }
    }
    double xs = wave_min_nonneg_f64(b.x);
    while (!__builtin_amdgcn_readfirstlane((int)(xs <= thr))) {
        // the threshold came from a screened bead that is no candidate after all: widen
        thr = xs;
        bool more = false;
#pragma unroll
        for (int k = 0; k < BPL; ++k)
            more = more || (!((done >> k) & 1u) && sc.lo[k] < __builtin_huge_valf() && (double)sc.lo[k] <= thr);
        if (!__ballot(more)) break;
        search_pass<BPL, false, SPRING>(sc, thr, done, b, st, pv, pA, pB, pC, q0, q1, sha, shb, shc, sgnd, sig2, b2,
                                        L, wr, g0, g1, sigma);
        xs = wave_min_nonneg_f64(b.x);
    }
    if (!(xs < INF)) return h;
    const unsigned long long tie = __ballot(b.x == xs);
    int wl;
    if (__popcll(tie) == 1) {
        wl = (int)(__ffsll((long long)tie) - 1);
    } else {
        const unsigned key = wave_min_u32(b.x == xs ? b.key : 0xFFFFFFFFu);
        wl = (int)((key >> 1) & 63u);
    }
    take(h, b, wl);
    return h;
}

// The plain FP64 search: every staged bead other than the pivot evaluated exactly, lane by
// lane in chunks of 64 staged indices, then the wavefront minimum by (x, staged index, kind).
// A loop over the staging area rather than over register slots, so that its register needs
// do not grow with the staging capacity.
template <bool SPRING = false, bool PUSH = false>
__device__ __forceinline__ Hit search_all(const Stage &st, const Pivot &pv, int S, int ax, int sha, int shb, int shc,
                                          double sgnd, double sig2, double b2, double L, bool wr, double g0 = 0.0,
                                          double g1 = 0.0, double sigma = 0.0, double ov2 = 0.0) {
    const int lane = lane_id();
    const int q0 = pv.part & 0xFFFF, q1 = (pv.part >> 16) & 0xFFFF;
    const double *pA = st.axis(ax);
    const double *pB = st.axis(ax == 2 ? 0 : ax + 1);
    const double *pC = st.axis(ax == 0 ? 2 : ax - 1);
    Best b;  // the position, cell word and partners are read only after a candidate is stored
    b.x = INF;
    b.key = 0xFFFFFFFFu;
    for (int base = 0; base < S; base += 64) {
        const int idx = base + lane;
        if (idx < S && idx != pv.P) {
            const double A = pA[idx], B = pB[idx], C = pC[idx];
            const int32_t m = st.meta[idx];
            const bool partner = (idx == q0) || (idx == q1);
            const double gt = idx == q0 ? g0 : g1;
            double x;
            bool hs;
            const bool ok =
                wr ? exact_candidate<true, SPRING, PUSH>(A, B, C, m, pv, sha, shb, shc, sgnd, sig2, b2, L, partner, x,
                                                         hs, gt, sigma, ov2)
                   : exact_candidate<false, SPRING, PUSH>(A, B, C, m, pv, sha, shb, shc, sgnd, sig2, b2, L, partner, x,
                                                          hs, gt, sigma, ov2);
            // a lane's indices increase, so on equal x the earlier bead keeps its place
            const unsigned kk = (unsigned)(idx * 2 + (hs ? 0 : 1));
            if (ok && (x < b.x || (x == b.x && kk < b.key))) {
                b.x = x;
                b.key = kk;
                b.A = A;
                b.B = B;
                b.C = C;
                b.meta = m;
                b.part = st.part[idx];
            }
        }
    }
    Hit h;
    h.x = INF;
    h.key = 0xFFFFFFFFu;
    h.a = h.b = h.c = 0.0;
    h.meta = 0;
    h.part = -1;
    const double xs = wave_min_nonneg_f64(b.x);
    if (!(xs < INF)) return h;
    const unsigned long long tie = __ballot(b.x == xs);
    int wl;
    if (__popcll(tie) == 1) {
        wl = (int)(__ffsll((long long)tie) - 1);
    } else {
        const unsigned key = wave_min_u32(b.x == xs ? b.key : 0xFFFFFFFFu);
        wl = (int)((key >> 1) & 63u);
    }
    take(h, b, wl);
    return h;
}

// The wavefront minimum by (x, key) of the lanes' best candidates (bx = +inf where a lane has
// none), and the winner's record read from the staging area.  One wavefront reduction as a
// rule: rounding to single precision keeps the order (x1 <= x2 gives fl(x1) <= fl(x2), and
// the bit patterns of non-negative floats order like the numbers), so the winner is among the
// lanes whose fl(x) is the smallest; only when several lanes share it is the FP64 (x, key)
// minimum taken over those lanes.
__device__ __forceinline__ Hit winner(double bx, unsigned bkey, const Stage &st, const double *pA, const double *pB,
                                      const double *pC) {
    Hit h;
    h.x = INF;
    h.key = 0xFFFFFFFFu;
    h.a = h.b = h.c = 0.0;
    h.meta = 0;
    h.part = -1;
    const unsigned fb = (unsigned)__float_as_int((float)bx);
    const unsigned fm = wave_min_u32(fb);
    if (fm == 0x7F800000u) return h;  // +inf: no candidate in the wavefront
    const unsigned long long tie = __ballot(fb == fm);
    double xs;
    unsigned key;
    if (__popcll(tie) == 1) {
        const int wl = (int)(__ffsll((long long)tie) - 1);
        xs = rdlane(bx, wl);
        key = (unsigned)rdlane((int)bkey, wl);
    } else {
        xs = wave_min_nonneg_f64(fb == fm ? bx : INF);
        key = wave_min_u32(fb == fm && bx == xs ? bkey : 0xFFFFFFFFu);
    }
    const int j = (int)(key >> 1);
    h.x = xs;
    h.key = key;
    h.a = pA[j];
    h.b = pB[j];
    h.c = pC[j];
    h.meta = __builtin_amdgcn_readfirstlane(st.meta[j]);
    h.part = __builtin_amdgcn_readfirstlane(st.part[j]);
    return h;
}

// The plain FP64 search of tethered chains with the square roots deferred.  Pass A takes every
// staged bead of the lane's slots (staged index 64 k + lane) through the cheap part of
// exact_candidate: the displacement, d_par, d_perp^2, whether it is a contact or a partner, and
// the argument of the square root, kept in registers.  Pass B then evaluates x for the lane's
// candidates only, one per pass in slot order, with the same operations as exact_candidate, so
// that every x has the same bits; a pass runs while any lane has a candidate left (about 7
// candidates among ~150 staged beads: usually one or two passes instead of one square root
// per 64 staged beads).  The winner is the minimum by (x, staged index, kind), as in
// search_all, and its record is read from LDS.
template <int BPL>
__device__ __forceinline__ Hit search_deferred(const Stage &st, const Pivot &pv, int S, int ax, int sha, int shb,
                                               int shc, double sgnd, double sig2, double b2, double L, bool wr) {
    const int lane = lane_id();
    const int q0 = pv.part & 0xFFFF, q1 = (pv.part >> 16) & 0xFFFF;
    const double *pA = st.axis(ax);
    const double *pB = st.axis(ax == 2 ? 0 : ax + 1);
    const double *pC = st.axis(ax == 0 ? 2 : ax - 1);
    double dpar[BPL], arg[BPL];
    unsigned cand = 0u, hsm = 0u;
#pragma unroll
    for (int k = 0; k < BPL; ++k) {
        dpar[k] = 0.0;
        arg[k] = 0.0;
        const int idx = k * 64 + lane;
        if (k * 64 < S && idx < S && idx != pv.P) {
            const int32_t meta = st.meta[idx];
            double da = pA[idx] - pv.a;
            double db = pB[idx] - pv.b;
            double dc = pC[idx] - pv.c;
            if (wr) {
                const int ea = (int)((meta >> sha) & CELL_MASK) - (int)((pv.meta >> sha) & CELL_MASK);
                const int eb = (int)((meta >> shb) & CELL_MASK) - (int)((pv.meta >> shb) & CELL_MASK);
                const int ec = (int)((meta >> shc) & CELL_MASK) - (int)((pv.meta >> shc) & CELL_MASK);
                da = da + (ea > 1 ? -L : (ea < -1 ? L : 0.0));
                db = db + (eb > 1 ? -L : (eb < -1 ? L : 0.0));
                dc = dc + (ec > 1 ? -L : (ec < -1 ? L : 0.0));
            }
            const double dp = da * sgnd;
            const double pb = db * db;
            const double pc = dc * dc;
            const double dperp2 = pb + pc;
            const bool hs = (dp > 0.0) && (dperp2 < sig2);
            const bool partner = (idx == q0) || (idx == q1);
            dpar[k] = dp;
            arg[k] = (hs ? sig2 : b2) - dperp2;
            cand |= (hs || partner) ? (1u << k) : 0u;
            hsm |= hs ? (1u << k) : 0u;
        }
    }
    double bx = INF;
    unsigned bkey = 0xFFFFFFFFu;
    while (__ballot(cand != 0u)) {
        const int k = cand ? __builtin_ctz(cand) : 0;
        double dp = dpar[0], a = arg[0];
#pragma unroll
        for (int j = 1; j < BPL; ++j)
            if (k == j) {
                dp = dpar[j];
                a = arg[j];
            }
        if (cand) {
            const bool hs = (hsm >> k) & 1u;
            if (!(a > 0.0)) a = 0.0;
            const double sq = sqrt_nonneg(a);
            double v = hs ? dp - sq : dp + sq;
            if (!(v > 0.0)) v = 0.0;
            const unsigned kk = (unsigned)((k * 64 + lane) * 2 + (hs ? 0 : 1));
            if (v < bx || (v == bx && kk < bkey)) {
                bx = v;
                bkey = kk;
            }
            cand &= cand - 1u;
        }
    }
    return winner(bx, bkey, st, pA, pB, pC);
}

// The plain FP64 search with the square roots deferred for every bond model (springs and the
// push-off as well as tethers).  Pass A takes every staged bead of the lane's slots through
// the displacement only and marks the beads that can be candidates at all: ahead within sigma
// of the line of motion, or a partner of the pivot (a superset of what exact_candidate
// accepts: the push-off drops some of the contacts).  Pass B runs exact_candidate itself on
// the marked beads, one per pass in slot order, and keeps the lane's minimum by (x, staged
// index, kind) as search_all does; so the winner is the same bead with the same x, and the
// square roots (for springs also the bond-energy square roots of the partners) are taken for
// about a dozen beads instead of every staged one.
template <int BPL, bool SPRING, bool PUSH>
__device__ __forceinline__ Hit search_filtered(const Stage &st, const Pivot &pv, int S, int ax, int sha, int shb,
                                               int shc, double sgnd, double sig2, double b2, double L, bool wr,
                                               double g0, double g1, double sigma, double ov2) {
    const int lane = lane_id();
    const int q0 = pv.part & 0xFFFF, q1 = (pv.part >> 16) & 0xFFFF;
    const double *pA = st.axis(ax);
    const double *pB = st.axis(ax == 2 ? 0 : ax + 1);
    const double *pC = st.axis(ax == 0 ? 2 : ax - 1);
    unsigned cand = 0u;
#pragma unroll
    for (int k = 0; k < BPL; ++k) {
        const int idx = k * 64 + lane;
        if (k * 64 < S && idx < S && idx != pv.P) {
            const int32_t meta = st.meta[idx];
            double dp, dperp2;
            if (wr) rel_to_pivot<true>(pA[idx], pB[idx], pC[idx], meta, pv, sha, shb, shc, sgnd, L, dp, dperp2);
            else rel_to_pivot<false>(pA[idx], pB[idx], pC[idx], meta, pv, sha, shb, shc, sgnd, L, dp, dperp2);
            const bool ahead = (dp > 0.0) && (dperp2 < sig2);
            const bool partner = (idx == q0) || (idx == q1);
            cand |= (ahead || partner) ? (1u << k) : 0u;
        }
    }
    double bx = INF;
    unsigned bkey = 0xFFFFFFFFu;
    while (__ballot(cand != 0u)) {
        if (cand) {
            const int idx = __builtin_ctz(cand) * 64 + lane;
            const double A = pA[idx], B = pB[idx], C = pC[idx];
            const int32_t m = st.meta[idx];
            const bool partner = (idx == q0) || (idx == q1);
            const double gt = idx == q0 ? g0 : g1;
            double x;
            bool hs;
            const bool ok =
                wr ? exact_candidate<true, SPRING, PUSH>(A, B, C, m, pv, sha, shb, shc, sgnd, sig2, b2, L, partner, x,
                                                         hs, gt, sigma, ov2)
                   : exact_candidate<false, SPRING, PUSH>(A, B, C, m, pv, sha, shb, shc, sgnd, sig2, b2, L, partner, x,
                                                          hs, gt, sigma, ov2);
            const unsigned kk = (unsigned)(idx * 2 + (hs ? 0 : 1));
            if (ok && (x < bx || (x == bx && kk < bkey))) {
                bx = x;
                bkey = kk;
            }
            cand &= cand - 1u;
        }
    }
    return winner(bx, bkey, st, pA, pB, pC);
}

// Select element `slot` (uniform) of a lane's register array.  Written as a masked OR so
// that the compiler cannot turn it into an indexed load, which would move the array out
// of VGPRs into scratch memory.
template <int BPL>
__device__ __forceinline__ float pick(const float (&V)[BPL], int slot) {
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < BPL; ++k) acc |= (uint32_t)__float_as_int(V[k]) & (0u - (uint32_t)(slot == k));
    return __int_as_float((int)acc);
}

template <int BPL>
__device__ __forceinline__ void put(float (&V)[BPL], int slot, int owner, float v) {
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

__device__ __forceinline__ float fblend(uint32_t m, float x, float y) {
    return __int_as_float((int)(((uint32_t)__float_as_int(x) & m) | ((uint32_t)__float_as_int(y) & ~m)));
}

// cyclic change of the frame: (A, B, C) = (r[ax], r[ax+1], r[ax+2]) for the new axis.
// A bitwise blend rather than two branches, so that the arrays stay in VGPRs.
template <int BPL, bool WHOLE>
__device__ __forceinline__ void rotate(Lanes<BPL, WHOLE> &R, int from, int to) {
    const int r = (to - from + 3) % 3;
    if (r == 0) return;
    const uint32_t m = 0u - (uint32_t)(r == 1);
#pragma unroll
    for (int k = 0; k < BPL; ++k) {
        const float a = R.A[k], b = R.B[k], c = R.C[k];
        R.A[k] = fblend(m, b, c);
        R.B[k] = fblend(m, c, a);
        R.C[k] = fblend(m, a, b);
    }
}

// Per-wave event counters: lane C_* of one VGPR holds counter C_* (32 bits suffice for
// one phase of one domain), so that they do not occupy scalar registers.
struct Tally {
    uint32_t v;
    double dsum;
    __device__ __forceinline__ void inc(int which) { v += (lane_id() == which) ? 1u : 0u; }
};

struct Frame {
    int ds[3];      // first cell of the domain per axis
    int fs[3];      // first cell of the frame (domain plus halo) per axis
    double O[3];    // lower corner of the frame (screening origin)
    int S;          // staged beads
    int dom[3];     // domain coordinates in the domain grid
    int colour;
    uint32_t domain;   // index in the melt's domain grid (the random-number counter)
    uint32_t gdomain;  // index among all domains of a batch (the event log)
};

// screening coordinate of a bead at r in cell c along an axis with frame start fs, origin O
__device__ __forceinline__ float frame_u(double r, int c, int fs, double L, double O) {
    const double w = c < fs ? r + L : r;
    return (float)(w - O);
}

__device__ __forceinline__ void log_event(const PhaseArgs &a, const Frame &f, int k, int step, int p,
                                          int t, int kind) {
    if (lane_id() == 0) {
        const unsigned long long s = atomicAdd(a.log_n, 1ull);
        if ((long long)s < a.log_cap)
            a.log[s] = ecmc_event{a.sweep, f.gdomain, (uint32_t)k, (uint32_t)step, p, t, (uint32_t)kind,
                                  (uint32_t)f.colour};
        else
            atomicOr(a.err, ERR_LOG);
    }
}

// ------------------------------------------------------------------ spring energies
// Natural logarithm of u > 0 by fixed steps, so that every IEEE binary64 evaluation of them
// gives the same bits: u = f 2^e with f in [sqrt(1/2), sqrt(2)); z = (f - 1)/(f + 1);
// ln f = 2 artanh z = 2 z (1 + z^2/3 + z^4/5 + ... + z^22/23) by Horner's rule (|z| <= 0.1716:
// the first term left out is below 2^-60 of the bracket); ln u = e ln 2 + ln f.
__device__ __forceinline__ double ln_artanh(double u) {
    int e;
    double f = frexp(u, &e);  // f in [1/2, 1)
    if (f < 0.70710678118654752440) {
        f = f + f;
        e = e - 1;
    }
    const double z = (f - 1.0) / (f + 1.0);
    const double z2 = z * z;
    double s = 1.0 / 23.0;
#pragma unroll
    for (int n = 10; n >= 0; --n) s = 1.0 / (double)(2 * n + 1) + z2 * s;
    return (double)e * 0.69314718055994530942 + (z + z) * s;
}

// Key of the spring energy draws of random stream `stream`: words 0-1 of the Philox draw at
// counter (2^32 - 1, 2^32 - 1, stream, 0x53505247), a counter the EC and offset draws never use.
__device__ __forceinline__ void spring_key(const PhaseArgs &a, uint32_t stream, uint32_t &k0, uint32_t &k1) {
    uint32_t c[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, stream, 0x53505247u};
    philox4x32_10(c, a.key0, a.key1);
    k0 = c[0];
    k1 = c[1];
}

// The energies of step `step` of EC k of a domain, one per bond slot of the pivot, as
// g = 2 dE / k with dE = -ln u, u uniform in (0, 1] from 53 bits of the Philox draw at
// counter (step, k, domain, sweep) under the spring key: slot t takes words 2t (its upper 21
// bits) and 2t + 1.  A fresh draw per step is exact for an exponential energy budget, which
// has no memory.
__device__ __forceinline__ void spring_terms(const PhaseArgs &a, const Frame &f, int k, int step, uint32_t sk0,
                                             uint32_t sk1, double &g0, double &g1) {
    uint32_t c[4] = {(uint32_t)step, (uint32_t)k, f.domain, a.sweep};
    philox4x32_10(c, sk0, sk1);
    const unsigned long long m0 = ((unsigned long long)c[1] << 21) | (unsigned long long)(c[0] >> 11);
    const unsigned long long m1 = ((unsigned long long)c[3] << 21) | (unsigned long long)(c[2] >> 11);
    // both logarithms in one instruction stream: lane 0 takes slot 0's draw, lane 1 slot 1's
    // (the same operations on each lane's own value; called with every lane active)
    const unsigned long long m = (lane_id() & 1) ? m1 : m0;
    const double g = -ln_artanh((double)(m + 1ull) * 0x1p-53) * a.two_over_k;
    g0 = rdlane(g, 0);
    g1 = rdlane(g, 1);
}

// A reflection after an earlier one in the same EC.  Between two reflections every move is
// reversible (a lift is undone by the reverse lift, a stop sends the pivot back), so after
// the second one the EC runs back to the first and then repeats: whatever is left of x_max
// only matters modulo twice the length W used between them.  Whole periods are dropped
// (logged PERIOD); W == 0 means nothing can move and ends the EC (CYCLE, returns true).
template <bool LOG>
__device__ __forceinline__ bool repeat_reflection(const PhaseArgs &a, const Frame &f, int k, int step,
                                                  int id, double xref, double &xmax, Tally &t) {
    const double w = xref - xmax;
    if (!__builtin_amdgcn_readfirstlane((int)(w > 0.0))) {
        t.inc(C_CYCLE);
        if (LOG) log_event(a, f, k, step, id, -1, ECMC_EV_CYCLE);
        return true;
    }
    const double r = fmod(xmax, w + w);
    if (__builtin_amdgcn_readfirstlane((int)(r < xmax))) {
        xmax = r;
        t.inc(C_PERIOD);
        if (LOG) log_event(a, f, k, step, id, -1, ECMC_EV_PERIOD);
    }
    return false;
}

// ------------------------------------------------------------------ swap move (Sec. II.C)
__device__ __forceinline__ double min_image(double d, double L, double hL) { return d > hL ? d - L : (d < -hL ? d + L : d); }

// Squared minimum-image distance from u to v, both given in the frame rotated to axis ax
// (components along ax, ax+1, ax+2), summed over x, y, z in that order.
__device__ __forceinline__ double dist2_rot(int ax, double ua, double ub, double uc, double va, double vb, double vc,
                                            double L, double hL) {
    const double da = min_image(ua - va, L, hL), db = min_image(ub - vb, L, hL), dc = min_image(uc - vc, L, hL);
    const double qa = da * da, qb = db * db, qc = dc * dc;
    return ax == 0 ? (qa + qb) + qc : (ax == 1 ? (qc + qa) + qb : (qb + qc) + qa);
}

// The exchange of pivot p (now at its contact point) and the struck bead j is accepted when
// every tether of p (measured from j's place) and of j (from p's place) is within b_max: the
// Metropolis acceptance of a tethered chain, whose energy is 0 or infinite.  Partners are
// staged indices (0xFFFF: none); the pivot's own LDS entry is stale during an EC, so a
// partner that is the other bead of the pair is measured at its new place.
__device__ __forceinline__ bool swap_allowed(const Stage &st, const Pivot &pv, const Hit &hit, int J, int ax,
                                             double L, double hL, double b2) {
    const double *pA = st.axis(ax);
    const double *pB = st.axis(ax == 2 ? 0 : ax + 1);
    const double *pC = st.axis(ax == 0 ? 2 : ax - 1);
    bool ok = true;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int q = (pv.part >> (16 * t)) & 0xFFFF;  // p moves to j's place
        if (q != 0xFFFF) {
            const bool qj = q == J;
            const double va = qj ? pv.a : pA[q], vb = qj ? pv.b : pB[q], vc = qj ? pv.c : pC[q];
            ok = ok && !(dist2_rot(ax, hit.a, hit.b, hit.c, va, vb, vc, L, hL) > b2);
        }
        const int u = (hit.part >> (16 * t)) & 0xFFFF;  // j moves to p's place
        if (u != 0xFFFF) {
            const bool up = u == pv.P;
            const double va = up ? hit.a : pA[u], vb = up ? hit.b : pB[u], vc = up ? hit.c : pC[u];
            ok = ok && !(dist2_rot(ax, pv.a, pv.b, pv.c, va, vb, vc, L, hL) > b2);
        }
    }
    return __builtin_amdgcn_readfirstlane((int)ok) != 0;
}

// Write the pivot's position along the axis and its cell word back to LDS, and its
// screening coordinate to the owner lane.
template <int BPL, bool WHOLE>
__device__ __forceinline__ void store_pivot(const Pivot &pv, const Stage &st, double *pA, Lanes<BPL, WHOLE> &R) {
    if (lane_id() == 0) {
        pA[pv.P] = pv.a;
        st.meta[pv.P] = pv.meta;
    }
    put(R.A, pv.P >> 6, pv.P & 63, pv.fa);
    if (WHOLE) put(R.META, pv.P >> 6, pv.P & 63, pv.meta);
}

// One EC along axis ax (the lanes' frame is already rotated to it), direction sign sgn,
// from staged pivot P0, x_max = ell.  Returns false if the iteration cap was hit.
//
// With springs (SPRING) the bond energies of every step are drawn from the key (sk0, sk1), and
// an EC never retraces its path after a reflection (its draws differ), so whole periods are
// not dropped.  The push-off (PUSH, plain FP64 search only) keeps the shortcut: it prepares a
// start and samples nothing, and where a pair that stopped overlapping changes the way back the
// shortcut merely shortens that EC.
template <int BPL, bool LOG, bool EXACT, bool WHOLE, bool SPRING = false, bool PUSH = false>
__device__ __forceinline__ bool run_ec(const PhaseArgs &a, const Frame &f, const Stage &st,
                                       Lanes<lane_slots(BPL, EXACT), WHOLE> &R,
                                       int P0, int ax, int sgn, bool wr, int k, const ScreenK &K, Tally &t,
                                       uint32_t sk0 = 0u, uint32_t sk1 = 0u) {
    const int n = a.n;
    const double L = a.L, h = a.h;
    const int axb = ax == 2 ? 0 : ax + 1, axc = ax == 0 ? 2 : ax - 1;
    const int sha = ax * CELL_BITS, shb = axb * CELL_BITS, shc = axc * CELL_BITS;
    const int dsa = f.ds[0] * (ax == 0) + f.ds[1] * (ax == 1) + f.ds[2] * (ax == 2);
    const int fsa = f.fs[0] * (ax == 0) + f.fs[1] * (ax == 1) + f.fs[2] * (ax == 2);
    const double Oa = f.O[0] * (ax == 0) + f.O[1] * (ax == 1) + f.O[2] * (ax == 2);
    double *pA = st.axis(ax);
    Pivot pv;
    pv.P = P0;
    pv.a = pA[P0];
    pv.b = st.axis(axb)[P0];
    pv.c = st.axis(axc)[P0];
    pv.meta = __builtin_amdgcn_readfirstlane(st.meta[P0]);
    pv.part = __builtin_amdgcn_readfirstlane(st.part[P0]);
    pv.fa = __int_as_float(rdlane(__float_as_int(pick(R.A, P0 >> 6)), P0 & 63));
    pv.fb = __int_as_float(rdlane(__float_as_int(pick(R.B, P0 >> 6)), P0 & 63));
    pv.fc = __int_as_float(rdlane(__float_as_int(pick(R.C, P0 >> 6)), P0 & 63));
    double xmax = a.ell;
    int step = 0;
    bool reflected = false;  // a reflection happened in this EC ...
    double xref = 0.0;       // ... with this much displacement left after it
    unsigned run = 0;      // consecutive zero-length events
    int saved_p = -1, saved_sgn = 0, saved_c = -1;
    t.inc(C_EC);
    for (;;) {
        if (run > 0) {
            // zero-length run: the state (pivot, direction, pivot cell) repeating is a cycle
            const int cc = (pv.meta >> sha) & CELL_MASK;
            if (pv.P == saved_p && sgn == saved_sgn && cc == saved_c) {
                store_pivot(pv, st, pA, R);
                t.inc(C_CYCLE);
                if (LOG) log_event(a, f, k, step, st.id[pv.P], -1, ECMC_EV_CYCLE);
                return true;
            }
            if ((run & (run - 1)) == 0) {
                saved_p = pv.P;
                saved_sgn = sgn;
                saved_c = cc;
            }
        }
        if (step >= a.event_cap) {
            store_pivot(pv, st, pA, R);
            return false;
        }
        ++step;
        t.inc(C_STEPS);
        const double sgnd = sgn > 0 ? 1.0 : -1.0;
        const int c = (pv.meta >> sha) & CELL_MASK;
        const double r_old = pv.a;
        double xc = sgn > 0 ? face(c + 1, n, h, L) - r_old : r_old - face(c, n, h, L);
        if (!(xc > 0.0)) xc = 0.0;
        Hit hit;
        if constexpr (EXACT) {
            double g0 = 0.0, g1 = 0.0;
            if constexpr (SPRING) spring_terms(a, f, k, step, sk0, sk1, g0, g1);
            if constexpr (!SPRING && !PUSH && BPL <= 8)
                hit = search_deferred<BPL>(st, pv, f.S, ax, sha, shb, shc, sgnd, a.sig2, a.b2, L, wr);
            else if constexpr (BPL <= 8)
                hit = search_filtered<BPL, SPRING, PUSH>(st, pv, f.S, ax, sha, shb, shc, sgnd, a.sig2, a.b2, L, wr, g0,
                                                         g1, a.sigma, a.ov2);
            else
                hit = search_all<SPRING, PUSH>(st, pv, f.S, ax, sha, shb, shc, sgnd, a.sig2, a.b2, L, wr, g0, g1,
                                               a.sigma, a.ov2);
        } else {
            Screen<BPL> sc;
            screen<BPL, WHOLE, SPRING>(sc, R, pv, sha, shb, shc, sgnd, K);
            // the exact interaction distance is at least sc.l: when the end of the EC or the
            // cell face comes strictly first (end: at or before), no exact search is needed
            const double lbound = (double)sc.l;
            const bool skip =
                __builtin_amdgcn_readfirstlane((int)((xmax <= xc && xmax <= lbound) || xc < lbound)) != 0;
            if (skip) {
                hit.x = INF;
                hit.key = 0xFFFFFFFFu;
                hit.a = hit.b = hit.c = 0.0;
                hit.meta = 0;
                hit.part = -1;
            } else {
                double g0 = 0.0, g1 = 0.0;
                if constexpr (SPRING) spring_terms(a, f, k, step, sk0, sk1, g0, g1);
                hit = search<BPL, SPRING>(sc, st, pv, ax, sha, shb, shc, sgnd, a.sig2, a.b2, L, wr, g0, g1, a.sigma);
            }
        }
        const double xint = hit.x;
        const double mlim = xint < xc ? xint : xc;
        // the event (0 end, 1 interaction, 2 cell face) as a wavefront-uniform value: the
        // FP64 values compared are the same in every lane, and a uniform branch keeps the
        // whole step in scalar control flow
        const int ev = __builtin_amdgcn_readfirstlane(xmax <= mlim ? 0 : (xint <= xc ? 1 : 2));
        if (ev == 0) {
            // END: the pivot takes the rest of the displacement
            pv.a = sgn > 0 ? r_old + xmax : r_old - xmax;
            pv.fa = frame_u(pv.a, c, fsa, L, Oa);
            store_pivot(pv, st, pA, R);
            if (LOG) log_event(a, f, k, step, st.id[pv.P], -1, ECMC_EV_END);
            return true;
        }
        if (ev == 1) {
            // interaction event: move to contact / tether limit
            if (__builtin_amdgcn_readfirstlane((int)(xint > 0.0))) {
                run = 0;
                saved_p = -1;
            } else {
                ++run;
            }
            pv.a = sgn > 0 ? r_old + xint : r_old - xint;
            pv.fa = frame_u(pv.a, c, fsa, L, Oa);
            xmax = xmax - xint;
            const int j = (int)(hit.key >> 1);
            const int kind = (int)(hit.key & 1u);
            if (hit.meta & MOTILE_BIT) {
                // lift: the struck bead continues the chain; accumulate (d_par - x)
                double da = hit.a - r_old;
                if (wr) {
                    const int e = (int)((hit.meta >> sha) & CELL_MASK) - c;
                    da = da + (e > 1 ? -L : (e < -1 ? L : 0.0));
                }
                const double dpar = da * sgnd;
                t.dsum += dpar - xint;
                if (a.swap && kind == 0 && swap_allowed(st, pv, hit, j, ax, L, a.halfL, a.b2)) {
                    // swap (Sec. II.C): p and j exchange places, p goes on from j's; p's
                    // identity advanced by d_par > 0, so a zero-length run is over
                    t.inc(C_SWAP);
                    if (LOG) log_event(a, f, k, step, st.id[pv.P], st.id[j], ECMC_EV_SWAP);
                    const float ja = __int_as_float(rdlane(__float_as_int(pick(R.A, j >> 6)), j & 63));
                    const float jb = __int_as_float(rdlane(__float_as_int(pick(R.B, j >> 6)), j & 63));
                    const float jc = __int_as_float(rdlane(__float_as_int(pick(R.C, j >> 6)), j & 63));
                    double *pB = st.axis(axb), *pC = st.axis(axc);
                    if (lane_id() == 0) {
                        // image counters: p moves by the minimum-image vector to j, j back
                        const int ip = st.id[pv.P], ij = st.id[j];
                        const double ra[3] = {hit.a - pv.a, hit.b - pv.b, hit.c - pv.c};
                        const int gx[3] = {ax, axb, axc};
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            const int sh = ra[q] > a.halfL ? -1 : (ra[q] < -a.halfL ? 1 : 0);
                            if (sh) {
                                a.img[3 * ip + gx[q]] += sh;
                                a.img[3 * ij + gx[q]] -= sh;
                            }
                        }
                        pA[j] = pv.a;
                        pB[j] = pv.b;
                        pC[j] = pv.c;
                        st.meta[j] = pv.meta;
                        pA[pv.P] = hit.a;
                        pB[pv.P] = hit.b;
                        pC[pv.P] = hit.c;
                        st.meta[pv.P] = hit.meta;
                    }
                    put(R.A, j >> 6, j & 63, pv.fa);
                    put(R.B, j >> 6, j & 63, pv.fb);
                    put(R.C, j >> 6, j & 63, pv.fc);
                    put(R.A, pv.P >> 6, pv.P & 63, ja);
                    put(R.B, pv.P >> 6, pv.P & 63, jb);
                    put(R.C, pv.P >> 6, pv.P & 63, jc);
                    if (WHOLE) {
                        put(R.META, j >> 6, j & 63, pv.meta);
                        put(R.META, pv.P >> 6, pv.P & 63, hit.meta);
                    }
                    pv.a = hit.a;
                    pv.b = hit.b;
                    pv.c = hit.c;
                    pv.meta = hit.meta;
                    pv.fa = ja;
                    pv.fb = jb;
                    pv.fc = jc;
                    run = 0;
                    saved_p = -1;
                    continue;
                }
                t.inc(kind == 0 ? C_HS_LIFT : C_TETHER_LIFT);
                if (LOG) log_event(a, f, k, step, st.id[pv.P], st.id[j], kind == 0 ? ECMC_EV_HS_LIFT : ECMC_EV_TETHER_LIFT);
                store_pivot(pv, st, pA, R);
                pv.P = j;
                pv.a = hit.a;
                pv.b = hit.b;
                pv.c = hit.c;
                pv.meta = hit.meta;
                pv.part = hit.part;
                pv.fa = __int_as_float(rdlane(__float_as_int(pick(R.A, j >> 6)), j & 63));
                pv.fb = __int_as_float(rdlane(__float_as_int(pick(R.B, j >> 6)), j & 63));
                pv.fc = __int_as_float(rdlane(__float_as_int(pick(R.C, j >> 6)), j & 63));
            } else {
                t.inc(kind == 0 ? C_HS_REFLECT : C_TETHER_REFLECT);
                if (LOG)
                    log_event(a, f, k, step, st.id[pv.P], st.id[j], kind == 0 ? ECMC_EV_HS_REFLECT : ECMC_EV_TETHER_REFLECT);
                if (!SPRING && reflected && repeat_reflection<LOG>(a, f, k, step, st.id[pv.P], xref, xmax, t)) {
                    store_pivot(pv, st, pA, R);
                    return true;
                }
                reflected = true;
                xref = xmax;
                sgn = -sgn;
            }
            continue;
        }
        // cell-face event: the pivot is set onto the face
        if (__builtin_amdgcn_readfirstlane((int)(xc > 0.0))) {
            run = 0;
            saved_p = -1;
        } else {
            ++run;
        }
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
        const bool inside = WHOLE || ((nc - dsa + n) % n) < a.D;
        if (inside) {
            pv.meta = (pv.meta & ~(CELL_MASK << sha)) | (nc << sha);
            if (wrapped > 0) {
                pv.a = 0.0;
                if (lane_id() == 0) a.img[3 * st.id[pv.P] + ax] += 1;
            } else if (wrapped < 0) {
                pv.a = L;
                if (lane_id() == 0) a.img[3 * st.id[pv.P] + ax] -= 1;
            }
            pv.fa = frame_u(pv.a, nc, fsa, L, Oa);
            t.inc(C_CROSS);
        } else {
            pv.fa = frame_u(pv.a, c, fsa, L, Oa);
            t.inc(C_WALL);
            if (LOG) log_event(a, f, k, step, st.id[pv.P], -1, ECMC_EV_WALL);
            if (!SPRING && reflected && repeat_reflection<LOG>(a, f, k, step, st.id[pv.P], xref, xmax, t)) {
                store_pivot(pv, st, pA, R);
                return true;
            }
            reflected = true;
            xref = xmax;
            sgn = -sgn;
        }
    }
}

// ------------------------------------------------------------------ domain frames
// Domain b of a colour: its first cell per axis (ds), the frame of domain plus one-cell halo
// (fs, origin O, edge F cells), and whether that frame wraps the box.  The colour of a
// domain is the parity of its grid coordinates, (d_x & 1) | (d_y & 1) << 1 | (d_z & 1) << 2.
//
// Tile-joint (JOINT, Sec. II.A): domain b of the single phase is tile (b mod nd, ...) and the
// tiles sit at pitch D + 1, so that the cell after each tile along every axis is a joint that no
// tile moves (it is in the halo of the tiles on either side).
template <bool WHOLE, bool JOINT = false>
__device__ __forceinline__ void frame_of(const PhaseArgs &a, int colour, int b, const int off[3], int dom0, Frame &f,
                                         int &F, bool &wraps) {
    const int n = a.n;
    int *dom = f.dom;
    dom[0] = dom[1] = dom[2] = 0;
    f.domain = 0;
    f.colour = colour;
    if (!WHOLE && JOINT) {
        dom[0] = b % a.nd;
        dom[1] = (b / a.nd) % a.nd;
        dom[2] = b / (a.nd * a.nd);
        f.domain = (uint32_t)b;
    } else if (!WHOLE) {
        const int nd2 = a.nd >> 1;
        dom[0] = 2 * (b % nd2) + (colour & 1);
        dom[1] = 2 * ((b / nd2) % nd2) + ((colour >> 1) & 1);
        dom[2] = 2 * (b / (nd2 * nd2)) + ((colour >> 2) & 1);
        f.domain = (uint32_t)(dom[0] + a.nd * (dom[1] + a.nd * dom[2]));
    }
    const int pitch = JOINT ? a.D + 1 : a.D;
    f.gdomain = (uint32_t)dom0 + f.domain;
    F = WHOLE ? n : a.D + 2;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        f.ds[ax] = WHOLE ? 0 : (off[ax] + dom[ax] * pitch) % n;
        f.fs[ax] = WHOLE ? 0 : (f.ds[ax] - 1 + n) % n;
        f.O[ax] = WHOLE ? 0.0 : face(f.fs[ax], n, a.h, a.L);
    }
    wraps = WHOLE || f.fs[0] + F > n || f.fs[1] + F > n || f.fs[2] + F > n;
}

// Occupancy the register allocation of the phase kernel aims at (waves per SIMD), for the
// staging tiers of up to 3 beads per lane (the tier that carries almost every domain of a
// dense melt): 5 waves (96 VGPRs) measured faster than the 4 the compiler picks by itself.
// A build-time tuning knob; 0 leaves the choice to the compiler.
#ifndef ECMC_PHASE_WAVES_PER_EU
#define ECMC_PHASE_WAVES_PER_EU 5
#endif
constexpr int phase_waves(int bpl) { return (ECMC_PHASE_WAVES_PER_EU > 0 && bpl <= 3) ? ECMC_PHASE_WAVES_PER_EU : 1; }

// The partition offsets of a sweep (Sec. II.A: the decomposition moves every sweep): one
// integer per axis, uniform in [0, D), from the Philox counter (0, 0, sweep, 2 stream + 1).
__device__ __forceinline__ void partition_offsets(const PhaseArgs &a, int D, uint32_t sweep, uint32_t stream,
                                                  int off[3]) {
    uint32_t ctr[4] = {0u, 0u, sweep, 2u * stream + 1u};
    philox4x32_10(ctr, a.key0, a.key1);
    off[0] = (int)scale_u32(ctr[0], (uint32_t)D);
    off[1] = (int)scale_u32(ctr[1], (uint32_t)D);
    off[2] = (int)scale_u32(ctr[2], (uint32_t)D);
}

// Beads in the frame (domain plus halo) of a domain: the sum of its F^3 cell counts.
__device__ __forceinline__ int frame_count(const PhaseArgs &a, const Frame &f, int F) {
    const int n = a.n, lane = lane_id();
    const int nfc = F * F * F;
    int S = 0;
    for (int base = 0; base < nfc; base += 64) {
        const int c = base + lane;
        int cnt = 0;
        if (c < nfc) {
            const int fx = c % F, fy = (c / F) % F, fz = c / (F * F);
            cnt = a.ccount[(f.fs[0] + fx) % n + n * ((f.fs[1] + fy) % n + n * ((f.fs[2] + fz) % n))];
        }
        S += rdlane(wave_incl_scan(cnt), 63);
    }
    return __builtin_amdgcn_readfirstlane(S);
}

// Where a domain is staged: LDS arrays of the kernel, or a slot of the device workspace
// for a domain above the LDS capacity.  `cap` is the row length of every array.
struct StageMem {
    double *pos;     // three rows of cap doubles; row 2 first holds the unsorted staging lists
    int32_t *id;     // staged bead ids, ascending
    int32_t *meta;   // cell words (+ motile bit)
    int32_t *part;   // tethered partners as staged indices; then the write-back counters
    unsigned long long *motm;  // one word per 64 staged indices: which of them are motile
    int32_t *mot;    // the motile staged indices, ascending (push-off and small tiers only)
    int cap;
};

// Whether a domain body keeps its motile beads as a list of staged indices (4 B per staged bead)
// or only as mask words (8 B per 64): the push-off scans the list; the LDS tiers of up to 4 beads
// per lane keep it because their occupancy is bound by registers, not LDS, and the list's EC start
// is the shorter, and so do the workspace slots (16 per lane, global memory); the LDS tiers of 6
// to 8 beads per lane, whose occupancy LDS bounds, keep the mask words only.
constexpr bool motile_list(int bpl, bool push) { return push || bpl <= 4 || bpl > 8; }

// One domain from its cell lists to the written-back result: stage its S0 beads (the count
// the caller took, S0 <= min(cap, 64 BPL)), run its K ECs, write back the motile beads and
// the domain's cell lists, flush the counters.
// Push-off: whether staged bead i overlaps another staged bead (minimum image of the raw
// coordinates, squared distance summed over x, y, z in that order, below ov2).  Every bead within
// the working diameter of a motile bead is staged.
__device__ __forceinline__ bool overlaps_staged(const PhaseArgs &a, const double *P0r, const double *P1r,
                                                const double *P2r, int S, int i) {
    const double xi = P0r[i], yi = P1r[i], zi = P2r[i];
    for (int j = 0; j < S; ++j) {
        if (j == i) continue;
        const double d0 = min_image(P0r[j] - xi, a.L, a.halfL);
        const double d1 = min_image(P1r[j] - yi, a.L, a.halfL);
        const double d2 = min_image(P2r[j] - zi, a.L, a.halfL);
        const double q0 = d0 * d0, q1 = d1 * d1, q2 = d2 * d2;
        if ((q0 + q1) + q2 < a.ov2) return true;
    }
    return false;
}

template <int BPL, bool LOG, bool EXACT, bool WHOLE, bool SPRING = false, bool PUSH = false>
__device__ __forceinline__ void domain_body(const PhaseArgs &a, Frame &f, int F, bool wraps, int S0,
                                            const StageMem &m) {
    constexpr int NS = lane_slots(BPL, EXACT);
    // the loops over a lane's staged beads are unrolled where they fill register slots
    constexpr int UNR = (EXACT && BPL > 4) ? 1 : BPL;
    const int lane = lane_id();
    const int n = a.n;
    const double L = a.L;
    const int SM = m.cap;
    int32_t *t_id = reinterpret_cast<int32_t *>(m.pos + 2 * SM);
    int32_t *t_meta = t_id + SM;
    double *const P0r = m.pos, *const P1r = m.pos + SM, *const P2r = m.pos + 2 * SM;

    // ---- stage the frame's beads in cell order, checking the caller's count
    const int nfc = F * F * F;
    int S = 0;
    for (int base = 0; base < nfc; base += 64) {
        const int c = base + lane;
        int cnt = 0, flat = 0;
        int32_t word = 0;
        if (c < nfc) {
            const int fx = c % F, fy = (c / F) % F, fz = c / (F * F);
            const int cx = (f.fs[0] + fx) % n, cy = (f.fs[1] + fy) % n, cz = (f.fs[2] + fz) % n;
            flat = cx + n * (cy + n * cz);
            const bool mot = WHOLE || (fx >= 1 && fx <= a.D && fy >= 1 && fy <= a.D && fz >= 1 && fz <= a.D);
            word = pack_cell(cx, cy, cz) | (mot ? MOTILE_BIT : 0);
            cnt = a.ccount[flat];
        }
        const int incl = wave_incl_scan(cnt);
        const int excl = incl - cnt;
        const int tot = rdlane(incl, 63);
        // four list entries per round, their loads in flight together
        for (int i0 = 0; i0 < cnt; i0 += 4) {
            int v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = i0 + j < cnt ? a.cids[(long long)flat * a.cap + i0 + j] : 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int at = S + excl + i0 + j;
                if (i0 + j < cnt && at < S0) {
                    t_id[at] = v[j];
                    t_meta[at] = word;
                }
            }
        }
        S += tot;
    }
    if (S != S0) {
        // the cell lists changed since the count: nothing of this domain is touched
        if (lane == 0) atomicOr(a.err, ERR_RECOUNT);
        return;
    }
    f.S = S;
    __syncthreads();
    // rank sort by bead id (ids are distinct: a bead's rank is the number of smaller ids)
    if constexpr (BPL <= 4) {
        // the lane's ids in registers, every other id read lane by lane from them (no LDS
        // round trip per comparison); past S an id larger than any
        int my[BPL], r[BPL];
#pragma unroll
        for (int k = 0; k < BPL; ++k) {
            const int e = k * 64 + lane;
            my[k] = e < S ? t_id[e] : 0x7FFFFFFF;
            r[k] = 0;
        }
#pragma unroll
        for (int k2 = 0; k2 < BPL; ++k2) {
            if (k2 * 64 < S) {
#pragma unroll
                for (int j = 0; j < 64; ++j) {
                    const int v = __builtin_amdgcn_readlane(my[k2], j);
#pragma unroll
                    for (int k = 0; k < BPL; ++k) r[k] += v < my[k] ? 1 : 0;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < BPL; ++k) {
            const int e = k * 64 + lane;
            if (e < S) {
                m.id[r[k]] = my[k];
                m.meta[r[k]] = t_meta[e];
            }
        }
    } else {
        for (int e = lane; e < S; e += 64) {
            const int my = t_id[e];
            int r = 0;
            for (int i = 0; i < S; ++i) r += (t_id[i] < my) ? 1 : 0;
            m.id[r] = my;
            m.meta[r] = t_meta[e];
        }
    }
    __syncthreads();

    // FP64 positions and partners into the staging area; screening copies into the lanes
    // (empty slots far away, so that they never pass the screen)
    Lanes<NS, WHOLE> R;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        R.A[k] = R.B[k] = R.C[k] = 1.0e30f;
        if (WHOLE) R.META[k] = 0;
    }
    // a partner's staged index by binary search over the ascending ids (0xFFFF: not staged)
    auto staged_index = [&](int g) {
        int found = 0xFFFF;
        if (g >= 0) {
            int lo = 0, hi = S - 1;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int v = m.id[mid];
                if (v == g) {
                    found = mid;
                    break;
                }
                if (v < g) lo = mid + 1;
                else hi = mid - 1;
            }
        }
        return found;
    };
    // one staged bead into LDS (and its screening copy into slot k)
    auto stage_one = [&](int k, int idx, int32_t w, double x, double y, double z, int g0, int g1) {
        P0r[idx] = x;
        P1r[idx] = y;
        P2r[idx] = z;
        if constexpr (!EXACT) {
            R.A[k] = frame_u(x, cell_of(w, 0), f.fs[0], L, f.O[0]);
            R.B[k] = frame_u(y, cell_of(w, 1), f.fs[1], L, f.O[1]);
            R.C[k] = frame_u(z, cell_of(w, 2), f.fs[2], L, f.O[2]);
            if (WHOLE) R.META[k] = w;
        }
        m.part[idx] = (w & MOTILE_BIT) ? (staged_index(g0) | (staged_index(g1) << 16)) : -1;
    };
    if constexpr (BPL <= 4) {
        // every slot's global loads first, so that they are in flight together
        int32_t wk[BPL];
        double xk[BPL], yk[BPL], zk[BPL];
        int g0k[BPL], g1k[BPL];
#pragma unroll
        for (int k = 0; k < BPL; ++k) {
            const int idx = k * 64 + lane;
            wk[k] = 0;
            xk[k] = yk[k] = zk[k] = 0.0;
            g0k[k] = g1k[k] = -1;
            if (idx < S) {
                const int id = m.id[idx];
                wk[k] = m.meta[idx];
                xk[k] = a.px[id];
                yk[k] = a.py[id];
                zk[k] = a.pz[id];
                if (wk[k] & MOTILE_BIT) {
                    g0k[k] = a.part[2 * id];
                    g1k[k] = a.part[2 * id + 1];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < BPL; ++k) {
            const int idx = k * 64 + lane;
            if (idx < S) stage_one(k, idx, wk[k], xk[k], yk[k], zk[k], g0k[k], g1k[k]);
        }
    } else {
#pragma unroll UNR
        for (int k = 0; k < BPL; ++k) {
            const int idx = k * 64 + lane;
            if (idx < S) {
                const int id = m.id[idx];
                const int32_t w = m.meta[idx];
                const bool mt = (w & MOTILE_BIT) != 0;
                stage_one(k, idx, w, a.px[id], a.py[id], a.pz[id], mt ? a.part[2 * id] : -1,
                          mt ? a.part[2 * id + 1] : -1);
            }
        }
    }
    // the motile beads (the domain's own; fixed while the domain runs: a bead never leaves the
    // domain, and a swap exchanges two motile beads) as a list in ascending staged index
    // (= ascending id), or as one mask word per 64 staged indices
    constexpr bool LIST = motile_list(BPL, PUSH);
    int nmot = 0;
#pragma unroll UNR
    for (int k = 0; k < BPL; ++k) {
        const int idx = k * 64 + lane;
        const bool mt = idx < S && (m.meta[idx] & MOTILE_BIT);
        const unsigned long long bal = __ballot(mt);
        if constexpr (LIST) {
            if (mt) m.mot[nmot + mbcnt(bal)] = idx;
        } else if (lane == 0) {
            m.motm[k] = bal;
        }
        nmot += __popcll(bal);
    }
    __syncthreads();

    // ---- ECs
    const Stage st = {m.pos, SM, m.meta, m.part, m.id};
    const ScreenK K = {a.sig2f, a.b2f, a.in_lo, a.in_hi, a.p_sure, a.err_f, (float)L};
    Tally t = {0u, 0.0};
    bool ok = true;
    int cur = 0;  // axis the lanes' frame is rotated to
    uint32_t sk0 = 0u, sk1 = 0u;
    if constexpr (SPRING) spring_key(a, a.stream, sk0, sk1);
    for (int k = 0; k < a.K && nmot > 0 && ok; ++k) {
        uint32_t ctr[4] = {(uint32_t)k, f.domain, a.sweep, 2u * a.stream};
        philox4x32_10(ctr, a.key0, a.key1);
        int P0;
        if constexpr (PUSH) {
            // the EC starts at the r-th motile bead (ascending id) that overlaps some bead, r drawn
            // among them; none left: the domain is done.  Counted, then found by a second pass.
            int nst = 0;
            for (int base = 0; base < nmot; base += 64) {
                const bool ov = base + lane < nmot && overlaps_staged(a, P0r, P1r, P2r, S, m.mot[base + lane]);
                nst += __popcll(__ballot(ov));
            }
            if (nst == 0) break;
            int r = (int)scale_u32(ctr[0], (uint32_t)nst);
            P0 = -1;
            for (int base = 0; base < nmot && P0 < 0; base += 64) {
                const bool ov = base + lane < nmot && overlaps_staged(a, P0r, P1r, P2r, S, m.mot[base + lane]);
                const unsigned long long bal = __ballot(ov);
                const int c = __popcll(bal);
                if (r < c) {
                    const unsigned long long hit = __ballot(ov && mbcnt(bal) == r);
                    const int wl = (int)(__ffsll((long long)hit) - 1);
                    P0 = __builtin_amdgcn_readfirstlane(m.mot[base + wl]);
                }
                r -= c;
            }
        } else if constexpr (LIST) {
            P0 = __builtin_amdgcn_readfirstlane(m.mot[scale_u32(ctr[0], (uint32_t)nmot)]);
        } else {
            // the r-th motile bead in ascending staged index: the mask word that holds it, then
            // the lane whose rank among that word's motile lanes is what is left of r
            int r = (int)scale_u32(ctr[0], (uint32_t)nmot);
            P0 = 0;
            for (int q = 0; q < BPL; ++q) {
                const unsigned long long w = m.motm[q];
                const unsigned long long mk =
                    ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(w >> 32)) << 32) |
                    (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)w);
                const int c = __popcll(mk);
                if (r < c) {
                    const bool mine = ((mk >> lane) & 1ull) && mbcnt(mk) == r;
                    P0 = q * 64 + (int)(__ffsll((long long)__ballot(mine)) - 1);
                    break;
                }
                r -= c;
            }
        }
        const uint32_t dir = scale_u32(ctr[1], 6u);
        const int ax = __builtin_amdgcn_readfirstlane((int)(dir >> 1));
        const int sgn = __builtin_amdgcn_readfirstlane((dir & 1u) ? -1 : 1);
        if constexpr (!EXACT) rotate(R, cur, ax);
        cur = ax;
        ok = run_ec<BPL, LOG, EXACT, WHOLE, SPRING, PUSH>(a, f, st, R, P0, ax, sgn, wraps, k, K, t, sk0, sk1);
    }
    __syncthreads();

    // ---- write back the motile beads and the domain's cell lists
    const int ndc = WHOLE ? n * n * n : a.D * a.D * a.D;
    for (int i = lane; i < ndc; i += 64) m.part[i] = 0;
    __syncthreads();
    bool overflow = false;
#pragma unroll UNR
    for (int k = 0; k < BPL; ++k) {
        const int idx = k * 64 + lane;
        const int32_t w0 = idx < S ? m.meta[idx] : 0;
        if (idx < S && (w0 & MOTILE_BIT)) {
            const int id = m.id[idx];
            late(a.px)[id] = P0r[idx];
            late(a.py)[id] = P1r[idx];
            late(a.pz)[id] = P2r[idx];
            const int32_t w = w0 & ~MOTILE_BIT;
            late(a.cellp)[id] = w;
            const int cx = cell_of(w, 0), cy = cell_of(w, 1), cz = cell_of(w, 2);
            int lc;
            if (WHOLE) {
                lc = cx + n * (cy + n * cz);
            } else {
                const int tx = (cx - f.ds[0] + n) % n, ty = (cy - f.ds[1] + n) % n, tz = (cz - f.ds[2] + n) % n;
                lc = tx + a.D * (ty + a.D * tz);
            }
            const int slot = atomicAdd(&m.part[lc], 1);
            if (slot < a.cap) late(a.cids)[(long long)(cx + n * (cy + n * cz)) * a.cap + slot] = id;
            else overflow = true;
        }
    }
    __syncthreads();
    for (int i = lane; i < ndc; i += 64) {
        int cx, cy, cz;
        if (WHOLE) {
            cx = i % n;
            cy = (i / n) % n;
            cz = i / (n * n);
        } else {
            cx = (f.ds[0] + i % a.D) % n;
            cy = (f.ds[1] + (i / a.D) % a.D) % n;
            cz = (f.ds[2] + i / (a.D * a.D)) % n;
        }
        const int v = m.part[i];
        late(a.ccount)[cx + n * (cy + n * cz)] = v < a.cap ? v : a.cap;
    }
    if (__ballot(overflow) && lane == 0) atomicOr(late(a.err), ERR_CELL);
    if (lane < NCNT && t.v) atomicAdd(&late(a.cnt)[lane], (unsigned long long)t.v);
    if (lane == 0) {
        if (!ok) atomicOr(late(a.err), ERR_STUCK);
        if (t.dsum != 0.0) atomicAdd(late(a.sum_delta), t.dsum);
    }
}

}  // namespace
}  // namespace ecmc

// Host side of the C ABI declared in include/ecmc.h: validation of the start
// configurations, cell binning, workspace layout, launches of the gfx950 kernels.
//
// A context holds one melt or a batch of independent melts.  Their beads, polymers, cells
// and domains are consecutive ranges of shared arrays, in melt order; a per-melt table on
// the device gives each melt's box, cell grid, domain grid and ranges.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ecmc_internal.h"

using namespace ecmc;

// Device memory of ecmc_internal_distances_noalloc: the per-block partial sums of R^2(n), as many
// as the internal-distance area of a workspace can hold (LAG_SLOTS) plus the lag totals, 8 MiB
// on each device.  Host code never names the array in a launch or a copy: its name there is a
// host-side stand-in, and the device address comes from hipGetSymbolAddress at init.
static constexpr int64_t NOALLOC_LAG_SLOTS = LAG_SLOTS;
static __device__ __align__(256) double scratch[NOALLOC_LAG_SLOTS + LAG_MAX_BEADS];

namespace {

// per device: the address of scratch, resolved once with that device current
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch[MAX_DEVICES] = {};

hipError_t resolve_scratch(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch[dev] = (double *)ptr;
    return hipSuccess;
}

constexpr int64_t DEFAULT_EVENT_CAP = 10000000;
constexpr int DEFAULT_CAP = 16;
constexpr int MAX_BINS = 1024;
// time limit of one dependency wait of the sweep kernel, far beyond any domain's run time (a
// guard against a broken invariant, so that every wait ends)
constexpr int WAIT_SECONDS = 30;
constexpr int SLOW_SLOTS = 512;  // workspace staging slots of the dependency-ordered sweep

// ---------------------------------------------------------------- plan
struct MeltPlan {
    double L = 0, h = 0;
    int n = 0, D = 1, nd = 1, ndpc = 0;
    int64_t nb = 0, bead0 = 0, poly0 = 0, npoly = 0;
    int64_t cell0 = 0, dom0 = 0;
    int tick0 = 0;
    float in_lo = 0, in_hi = 0, p_sure = 0, err_f = 0;  // screen constants
};

struct Plan {
    std::vector<MeltPlan> melts;
    bool whole = false;
    int64_t nb = 0, cells = 0, domains = 0;
    int tickets = 0;       // domains per colour, summed over the melts
    int bpl = 0;           // beads per lane of the first staging tier
    int stage = 0;
    int bpl2 = 0;          // second tier for the rare domains above 64 * bpl (by phases; 0 = none)
    int bpl3 = 0;          // third tier above 64 * bpl2 (0 = none)
    bool sweep = false;    // one dependency-ordered launch per sweep
    int nslow = 0;         // its workspace staging slots for domains above 64 * bpl
    int slow_cap = 0;      // beads per slot
};

struct Layout {
    size_t px, py, pz, cellp, img, part, ccount, cids, dstage, done, queue, dstate, slow_lock, slow, melts, porder,
        pstart, polyL, r2, rg2, mid, shape, hist, acc, lags, cnt, dsum, err, log_n, log;
    size_t total;
    int64_t lag_slots;  // partial sums the internal-distance area holds (blocks x lags)
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(const Plan &p, int64_t npoly_max, int cap, int64_t log_cap) {
    Layout l{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t nb = (size_t)p.nb, nc = (size_t)p.cells, np = (size_t)npoly_max;
    l.px = take(8 * nb);
    l.py = take(8 * nb);
    l.pz = take(8 * nb);
    l.cellp = take(4 * nb);
    l.img = take(12 * nb);
    l.part = take(8 * nb);
    l.ccount = take(4 * nc);
    l.cids = take(4 * nc * cap);
    l.dstage = take(4 * (nc / 8 + 1));  // one count per domain of a colour phase (single melt)
    l.done = take(4 * (size_t)(p.domains + 1));
    l.queue = take(8);
    l.dstate = take(8);
    l.slow_lock = take(4 * (size_t)std::max(p.nslow, 0));
    l.slow = take((size_t)std::max(p.nslow, 0) * (size_t)std::max(p.slow_cap, 0) * SLOW_SLOT_BYTES_PER_BEAD);
    l.melts = take(sizeof(MeltDev) * p.melts.size());
    l.porder = take(4 * nb);
    l.pstart = take(4 * (np + 1));
    l.polyL = take(8 * np);
    l.r2 = take(8 * np);
    l.rg2 = take(8 * np);
    l.mid = take(24 * np);
    l.shape = take(96 * np);  // gyration tensor, eigenvalues, centre of mass: 12 doubles per polymer
    l.hist = take(8 * MAX_BINS);
    l.acc = take(8 * (2 * OBS_ACC_SLOTS + MAX_BINS));  // running sums of r2 and rg2, then a histogram
    // internal distances: per-block partial sums of every lag, then the totals
    const int64_t lag_max = std::min<int64_t>(std::max<int64_t>(p.nb, 1), LAG_MAX_BEADS);
    l.lag_slots = std::min<int64_t>(LAG_SLOTS, std::max<int64_t>(npoly_max, 1) * lag_max);
    l.lags = take(8 * (size_t)(l.lag_slots + lag_max));
    l.cnt = take(8 * NCNT);
    l.dsum = take(8);
    l.err = take(4);
    l.log_n = take(8);
    l.log = take(sizeof(ecmc_event) * (size_t)std::max<int64_t>(log_cap, 0));
    l.total = o;
    return l;
}

}  // namespace

struct ecmc_ctx {
    ecmc_options opt;
    int device = -1;                  // the device current at init
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;       // the caller's second stream for the larger staging tiers (or none)
    hipEvent_t fork = nullptr, join = nullptr;
    double sigma = 0, lmax = 0, sig2 = 0, b2 = 0;
    int64_t nb = 0, npoly = 0;
    std::vector<int64_t> chain_count;  // polymers per chain length (index = beads)
    Plan p;
    int cap = DEFAULT_CAP;
    Layout lay{};
    char *ws = nullptr;
    uint32_t sweep_ctr = 0;           // host count of sweeps (the device holds the authoritative one)
    int64_t acc_samples = 0;          // observable samples in the running sums, and their bins
    int32_t acc_nbins = 0;
    unsigned long long wait_ticks = 0;  // limit of one dependency wait, in steady-counter ticks
    std::string err;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timing;
    template <class T>
    T *dev(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

namespace {

thread_local std::string g_err;

ecmc_status fail(ecmc_ctx *c, ecmc_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    g_err = buf;
    return s;
}

#define HIP_OK(ctx, call)                                                                              \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) return fail(ctx, ECMC_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Cells and domains of one melt.  n_req = 0: the largest n with L/n > l_max.  D_req = 0
// (checkerboard): D = 2, with n the largest multiple of 4 below that bound unless n_req fixes
// it (then the smallest D >= 2 that fits).
ecmc_status plan_melt(double L, int64_t nb, double lmax, int n_req, int D_req, int tiling, MeltPlan &mp,
                      ecmc_ctx *c, int m) {
    if (!(std::isfinite(L) && L > 0)) return fail(c, ECMC_E_ARG, "melt %d: need a finite box > 0", m);
    if (nb < 1 || nb > 0x7fffffffLL)
        return fail(c, ECMC_E_ARG, "melt %d: bead count %lld out of range", m, (long long)nb);
    int nmax = (int)std::min(std::floor(L / lmax), (double)MAX_CELLS_PER_AXIS);
    while (nmax > 0 && !(L / nmax > lmax)) --nmax;
    int n = n_req > 0 ? n_req : nmax;
    int D = D_req;
    if (tiling == ECMC_TILING_JOINT) {
        // tiles of D^3 cells at pitch D + 1: n a multiple of the pitch, at least two tiles per axis
        if (D < 1) D = 2;
        if (n_req <= 0) n = nmax - nmax % (D + 1);
    }
    if (tiling == ECMC_TILING_CHECKER && D_req == 0) {
        if (n_req > 0) {
            for (D = 2; D <= n && !(n % D == 0 && (n / D) % 2 == 0); ++D) {
            }
            if (D > n) return fail(c, ECMC_E_BOX, "melt %d: no domain edge D >= 2 with n/D even (n = %d)", m, n);
        } else {
            D = 2;
            n = nmax - nmax % 4;
        }
    }
    if (n < 4 || n > MAX_CELLS_PER_AXIS || !(L / n > lmax))
        return fail(c, ECMC_E_BOX, "cells per axis n = %d: need 4 <= n <= %d and L/n > l_max (melt %d)", n,
                    MAX_CELLS_PER_AXIS, m);
    mp.L = L;
    mp.n = n;
    mp.h = L / n;
    mp.nb = nb;
    if (tiling == ECMC_TILING_WHOLE) {
        mp.D = n;
        mp.nd = 1;
        if (nb > MAX_STAGE) return fail(c, ECMC_E_ARG, "whole-box tiling holds at most %d beads", MAX_STAGE);
        if ((int64_t)n * n * n > 64 * 16)
            return fail(c, ECMC_E_BOX, "whole-box tiling needs n^3 <= 1024 cells (n = %d)", n);
    } else if (tiling == ECMC_TILING_CHECKER) {
        // D >= 2: the integer offset drawn from [0, D) is what moves the partition between
        // sweeps; with D = 1 it is always 0 and every bead stays in its cell for good.
        if (D < 2 || n % D != 0 || (n / D) % 2 != 0)
            return fail(c, ECMC_E_BOX, "checkerboard needs D >= 2, n %% D == 0 and n/D even (melt %d: n = %d, D = %d)",
                        m, n, D);
        mp.D = D;
        mp.nd = n / D;
        mp.ndpc = (mp.nd / 2) * (mp.nd / 2) * (mp.nd / 2);
    } else if (tiling == ECMC_TILING_JOINT) {
        // D >= 2: a 1-cell tile has a wall at every face, so no bead could ever leave the cell
        // it started in, whatever the offset (the partition must let every bead move, Sec. II.A)
        if (D < 2 || n % (D + 1) != 0 || n / (D + 1) < 2)
            return fail(c, ECMC_E_BOX, "tile-joint needs D >= 2, n %% (D + 1) == 0 and n/(D + 1) >= 2 (melt %d: n = %d, D = %d)",
                        m, n, D);
        mp.D = D;
        mp.nd = n / (D + 1);
        mp.ndpc = mp.nd * mp.nd * mp.nd;  // every tile in the one phase
    } else {
        return fail(c, ECMC_E_ARG, "unknown tiling %d", tiling);
    }
    return ECMC_OK;
}

// Single-precision screen constants of a melt (see screen() in the kernels).  Screening
// coordinates are frame coordinates rounded once to float, so every float displacement is
// within delta = 6 u X of the FP64 one (u = 2^-24, X the largest coordinate or displacement:
// the frame edge, or L for the whole box).  For |d_perp| <= b the float d_perp^2 (a product
// and one fused multiply-add, at most 3 u b^2 of rounding) is then within
// m = 4 b delta + 2 delta^2 + 8 u b^2 of the FP64 value, the argument of the square root
// within m + 4 u b^2, the square root within the square root of that (the ill-conditioned
// grazing case), and the estimate of x within delta + sqrt(m + 4 u b^2) + 4 u b + u (X + b).
// The interval half-width is twice that.
void screen_constants(MeltPlan &mp, double sigma, double lmax, bool whole) {
    const double u = std::ldexp(1.0, -24);
    const double bm = std::max(sigma, lmax);
    const double X = whole ? mp.L : (mp.D + 2) * mp.h;
    const double delta = 6.0 * u * X + 1e-12 * mp.L;
    const double m = 4.0 * bm * delta + 2.0 * delta * delta + 8.0 * u * bm * bm;
    const double err = 2.0 * (delta + std::sqrt(m + 4.0 * u * bm * bm) + 4.0 * u * bm + u * (X + bm));
    const float inf = __builtin_huge_valf();
    mp.p_sure = std::nextafter((float)delta, inf);
    mp.in_lo = std::nextafter((float)(sigma * sigma - m), 0.0f);
    mp.in_hi = std::nextafter((float)(sigma * sigma + m), inf);
    mp.err_f = std::nextafter((float)err, inf);
}

struct MeltIn {
    double box;
    int64_t nb;
    int n_cells, domain_cells;
};

ecmc_status plan(const std::vector<MeltIn> &in, double sigma, double lmax, const ecmc_options &o, Plan &p,
                 ecmc_ctx *c) {
    if (!(std::isfinite(sigma) && sigma > 0 && std::isfinite(lmax) && lmax >= sigma))
        return fail(c, ECMC_E_ARG, "need finite box > 0, sigma > 0, l_max >= sigma");
    if (o.precision != ECMC_PREC_FP64 && o.precision != ECMC_PREC_MIXED)
        return fail(c, ECMC_E_ARG, "precision must be ECMC_PREC_FP64 or ECMC_PREC_MIXED (got %d)", o.precision);
    if (o.schedule != ECMC_SCHED_SWEEP && o.schedule != ECMC_SCHED_PHASES)
        return fail(c, ECMC_E_ARG, "schedule must be ECMC_SCHED_SWEEP or ECMC_SCHED_PHASES (got %d)", o.schedule);
    if (!(o.spring_k == 0.0 || (o.spring_k >= 1e-6 && o.spring_k <= 1e12)))
        return fail(c, ECMC_E_ARG, "spring_k must be 0 (tethers) or in [1e-6, 1e12] (got %g)", o.spring_k);
    if (o.spring_k > 0.0 && o.swap_moves) return fail(c, ECMC_E_ARG, "swap moves cannot be combined with springs");
    if (o.overlapping_start && (o.spring_k > 0.0 || o.swap_moves))
        return fail(c, ECMC_E_ARG, "an overlapping start (push-off) takes tethers without swap moves");
    if (in.empty()) return fail(c, ECMC_E_ARG, "no melts");
    const bool batch = in.size() > 1;
    if (batch && o.tiling != ECMC_TILING_CHECKER)
        return fail(c, ECMC_E_ARG, "a batch of melts needs the checkerboard tiling");
    if (batch && o.schedule != ECMC_SCHED_SWEEP)
        return fail(c, ECMC_E_ARG, "a batch of melts runs with the dependency-ordered sweep (ECMC_SCHED_SWEEP)");
    p = Plan{};
    p.whole = o.tiling == ECMC_TILING_WHOLE;
    const int cap = o.cell_capacity > 0 ? o.cell_capacity : DEFAULT_CAP;
    double worst = 0;  // largest typical frame
    int64_t most = 0;  // largest possible frame
    for (size_t m = 0; m < in.size(); ++m) {
        MeltPlan mp;
        ecmc_status st = plan_melt(in[m].box, in[m].nb, lmax, in[m].n_cells, in[m].domain_cells, o.tiling, mp, c,
                                   (int)m);
        if (st) return st;
        screen_constants(mp, sigma, lmax, p.whole);
        mp.bead0 = p.nb;
        mp.cell0 = p.cells;
        mp.dom0 = p.domains;
        mp.tick0 = p.tickets;
        p.nb += mp.nb;
        p.cells += (int64_t)mp.n * mp.n * mp.n;
        p.domains += p.whole ? 1 : (int64_t)mp.nd * mp.nd * mp.nd;
        if ((int64_t)p.tickets + mp.ndpc > 0x7fffffffLL / 8) return fail(c, ECMC_E_ARG, "too many domains");
        p.tickets += mp.ndpc;
        if (!p.whole) {
            const double f = std::pow((double)(mp.D + 2), 3);
            worst = std::max(worst, f * (double)mp.nb / ((double)mp.n * mp.n * mp.n));
            most = std::max(most, (int64_t)(mp.D + 2) * (mp.D + 2) * (mp.D + 2) * cap);
        }
        p.melts.push_back(mp);
    }
    if (p.nb > 0x7fffffffLL) return fail(c, ECMC_E_ARG, "at most 2^31 - 1 beads in all");
    // staging capacity
    if (p.whole) {
        p.stage = (int)std::min<int64_t>(p.melts[0].nb, MAX_STAGE + 1);
        if (o.stage_capacity > 0) p.stage = std::max(p.stage, o.stage_capacity);
    } else if (o.stage_capacity > 0) {
        p.stage = o.stage_capacity;
    } else {
        // first tier sized for the typical domain (or as asked); the few above it are staged
        // elsewhere
        if (o.stage_tier < 0 || o.stage_tier > 512 || o.stage_tier % 64 != 0)
            return fail(c, ECMC_E_ARG, "stage_tier must be 0 or a multiple of 64 up to 512 (got %d)", o.stage_tier);
        p.stage = o.stage_tier > 0 ? o.stage_tier : (int)std::ceil(worst + 3.0 * std::sqrt(worst) + 2.0);
        p.bpl2 = 16;
    }
    int bpl = (p.stage + 63) / 64;
    static const int ok[] = {1, 2, 3, 4, 6, 7, 8, 12, 16};
    int pick = 0;
    for (int v : ok)
        if (v >= bpl) {
            pick = v;
            break;
        }
    if (!pick) return fail(c, ECMC_E_ARG, "staging capacity %d exceeds %d", p.stage, MAX_STAGE);
    int ndc = 0;
    for (const MeltPlan &mp : p.melts) ndc = std::max(ndc, p.whole ? mp.n * mp.n * mp.n : mp.D * mp.D * mp.D);
    while (pick < 16 && ndc > 64 * pick)
        pick = *std::find_if(std::begin(ok), std::end(ok), [&](int v) { return v > pick; });
    if (ndc > 64 * pick) return fail(c, ECMC_E_BOX, "a domain of %d cells exceeds the staging area", ndc);
    p.bpl = pick;
    if (p.bpl2) {
        // by phases: tier 2 one step above tier 1, tier 3 the full 16 beads per lane
        const int *nxt = std::find_if(std::begin(ok), std::end(ok), [&](int v) { return v > pick; });
        p.bpl2 = nxt == std::end(ok) ? 0 : *nxt;
        p.bpl3 = (p.bpl2 && p.bpl2 < 16) ? 16 : 0;
    }
    if (o.tiling == ECMC_TILING_CHECKER && o.schedule == ECMC_SCHED_SWEEP && sweep_bpl_supported(p.bpl)) {
        p.sweep = true;
        if (p.bpl2 && most > 64 * p.bpl) {
            // automatic capacity: the domains above the LDS staging area go to workspace slots
            // that hold any frame up to the staging limit
            p.slow_cap = (int)std::min<int64_t>(most, MAX_STAGE);
            p.nslow = (int)std::min<int64_t>(p.tickets, SLOW_SLOTS);
        }
    }
    if (batch && !p.sweep) return fail(c, ECMC_E_ARG, "a batch of melts needs a staging capacity of at most 512 beads");
    return ECMC_OK;
}

double wrap_coord(double v, double L) {
    double w = std::fmod(v, L);
    if (w < 0) w = w + L;
    if (!(w < L)) w = 0.0;
    return w;
}

int bin_coord(double w, int n, double h, double L) {
    auto bnd = [&](int k) { return k < n ? (double)k * h : L; };
    int c = (int)std::floor(w / h);
    c = std::min(std::max(c, 0), n - 1);
    while (c > 0 && w < bnd(c)) --c;
    while (c < n - 1 && w > bnd(c + 1)) ++c;
    return c;
}

double min_image(double d, double L) {
    const double hl = 0.5 * L;
    return d > hl ? d - L : (d < -hl ? d + L : d);
}

struct HostState {
    std::vector<double> px, py, pz;
    std::vector<int32_t> cellp, img, part, ccount, cids, porder, pstart;
    std::vector<double> polyL;
    std::vector<int32_t> cx, cy, cz;
};

// partners, chain order and validation of the bonds of melt m (bead indices local to it)
ecmc_status build_topology(ecmc_ctx *c, int m, int64_t n_bonds, const int32_t *bonds, HostState &hs) {
    MeltPlan &mp = c->p.melts[m];
    const int64_t nb = mp.nb, b0 = mp.bead0;
    int32_t *part = hs.part.data() + 2 * b0;
    for (int64_t b = 0; b < n_bonds; ++b) {
        const int32_t i = bonds[2 * b], j = bonds[2 * b + 1];
        if (i < 0 || j < 0 || i >= nb || j >= nb || i == j)
            return fail(c, ECMC_E_ARG, "melt %d: bond %lld invalid", m, (long long)b);
        const int32_t gi = (int32_t)(b0 + i), gj = (int32_t)(b0 + j);
        if (part[2 * i] == gj || part[2 * i + 1] == gj) return fail(c, ECMC_E_ARG, "melt %d: duplicate bond %d-%d", m, i, j);
        int32_t *si = part[2 * i] < 0 ? &part[2 * i] : (part[2 * i + 1] < 0 ? &part[2 * i + 1] : nullptr);
        int32_t *sj = part[2 * j] < 0 ? &part[2 * j] : (part[2 * j + 1] < 0 ? &part[2 * j + 1] : nullptr);
        if (!si || !sj)
            return fail(c, ECMC_E_ARG, "melt %d: bead with more than two bonds (bond %lld)", m, (long long)b);
        *si = gj;
        *sj = gi;
    }
    std::vector<char> seen(nb, 0);
    const size_t before = hs.porder.size();
    mp.poly0 = (int64_t)hs.pstart.size();
    for (int64_t i = 0; i < nb; ++i) {
        const int deg = (part[2 * i] >= 0) + (part[2 * i + 1] >= 0);
        if (seen[i] || deg > 1) continue;
        hs.pstart.push_back((int32_t)hs.porder.size());
        hs.polyL.push_back(mp.L);
        int32_t prev = -1, cur = (int32_t)(b0 + i);
        while (cur >= 0) {
            seen[cur - b0] = 1;
            hs.porder.push_back(cur);
            const int32_t *pc = hs.part.data() + 2 * (size_t)cur;
            int32_t nx = pc[0] != prev ? pc[0] : pc[1];
            if (nx == prev) nx = -1;
            prev = cur;
            cur = nx;
        }
    }
    if ((int64_t)(hs.porder.size() - before) != nb) return fail(c, ECMC_E_ARG, "melt %d: bond list contains a ring", m);
    mp.npoly = (int64_t)hs.pstart.size() - mp.poly0;
    return ECMC_OK;
}

// cell lists of melt m from the per-bead cells; overlap and tether checks
ecmc_status build_cells(ecmc_ctx *c, int m, HostState &hs, bool validate) {
    const MeltPlan &mp = c->p.melts[m];
    const int n = mp.n;
    const int64_t b0 = mp.bead0, b1 = mp.bead0 + mp.nb;
    int32_t *ccount = hs.ccount.data() + mp.cell0;
    int32_t *cids = hs.cids.data() + mp.cell0 * c->cap;
    for (int64_t i = b0; i < b1; ++i) {
        const size_t f = (size_t)hs.cx[i] + n * ((size_t)hs.cy[i] + n * (size_t)hs.cz[i]);
        if (ccount[f] >= c->cap)
            return fail(c, ECMC_E_CELL_OVERFLOW, "melt %d: cell %zu holds more than %d beads", m, f, c->cap);
        cids[f * c->cap + ccount[f]++] = (int32_t)i;
        hs.cellp[i] = pack_cell(hs.cx[i], hs.cy[i], hs.cz[i]);
    }
    if (!validate) return ECMC_OK;
    const double L = mp.L;
    const double lim_ov = c->sig2 * (1.0 - 2e-12);
    for (int64_t i = b0; i < b1; ++i) {
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int ax = (hs.cx[i] + dx + n) % n, ay = (hs.cy[i] + dy + n) % n, az = (hs.cz[i] + dz + n) % n;
                    const size_t f = (size_t)ax + n * ((size_t)ay + n * (size_t)az);
                    for (int t = 0; t < ccount[f]; ++t) {
                        const int32_t j = cids[f * c->cap + t];
                        if (j <= i) continue;
                        const double ex = min_image(hs.px[j] - hs.px[i], L);
                        const double ey = min_image(hs.py[j] - hs.py[i], L);
                        const double ez = min_image(hs.pz[j] - hs.pz[i], L);
                        if (!c->opt.overlapping_start && ex * ex + ey * ey + ez * ez < lim_ov)
                            return fail(c, ECMC_E_OVERLAP, "melt %d: beads %lld and %lld overlap", m, (long long)(i - b0),
                                        (long long)(j - b0));
                    }
                }
        for (int t = 0; t < 2; ++t) {
            const int32_t j = hs.part[2 * i + t];
            if (j < 0) continue;
            const double ex = min_image(hs.px[j] - hs.px[i], L);
            const double ey = min_image(hs.py[j] - hs.py[i], L);
            const double ez = min_image(hs.pz[j] - hs.pz[i], L);
            if (ex * ex + ey * ey + ez * ez > c->b2 * (1.0 + 2e-12))
                return fail(c, ECMC_E_TETHER, "melt %d: bond %lld-%lld longer than l_max", m, (long long)(i - b0),
                            (long long)(j - b0));
        }
    }
    return ECMC_OK;
}

ecmc_status upload(ecmc_ctx *c, const HostState &hs, bool topology) {
    hipStream_t s = c->stream;
    const int64_t nb = c->nb;
    const size_t nc = (size_t)c->p.cells;
    HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.px, hs.px.data(), 8 * nb, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.py, hs.py.data(), 8 * nb, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.pz, hs.pz.data(), 8 * nb, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.cellp, hs.cellp.data(), 4 * nb, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.img, hs.img.data(), 12 * nb, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.ccount, hs.ccount.data(), 4 * nc, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.cids, hs.cids.data(), 4 * nc * c->cap, hipMemcpyHostToDevice, s));
    std::vector<MeltDev> md;
    if (topology) {
        md.resize(c->p.melts.size());
        for (size_t m = 0; m < md.size(); ++m) {
            const MeltPlan &mp = c->p.melts[m];
            MeltDev &d = md[m];
            d.L = mp.L;
            d.h = mp.h;
            d.halfL = 0.5 * mp.L;
            d.in_lo = mp.in_lo;
            d.in_hi = mp.in_hi;
            d.p_sure = mp.p_sure;
            d.err_f = mp.err_f;
            d.n = mp.n;
            d.D = mp.D;
            d.nd = mp.nd;
            d.ndpc = mp.ndpc;
            d.tick0 = mp.tick0;
            d.dom0 = (int)mp.dom0;
            d.cell0 = mp.cell0;
        }
        HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.melts, md.data(), sizeof(MeltDev) * md.size(), hipMemcpyHostToDevice, s));
        HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.part, hs.part.data(), 8 * nb, hipMemcpyHostToDevice, s));
        HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.porder, hs.porder.data(), 4 * nb, hipMemcpyHostToDevice, s));
        HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.pstart, hs.pstart.data(), 4 * (c->npoly + 1), hipMemcpyHostToDevice, s));
        HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.polyL, hs.polyL.data(), 8 * c->npoly, hipMemcpyHostToDevice, s));
        HIP_OK(c, hipMemsetAsync(c->ws + c->lay.cnt, 0, 8 * NCNT, s));
        HIP_OK(c, hipMemsetAsync(c->ws + c->lay.dsum, 0, 8, s));
        HIP_OK(c, hipMemsetAsync(c->ws + c->lay.err, 0, 4, s));
        HIP_OK(c, hipMemsetAsync(c->ws + c->lay.log_n, 0, 8, s));
        HIP_OK(c, hipMemsetAsync(c->ws + c->lay.done, 0, 4 * (size_t)(c->p.domains + 1), s));
        HIP_OK(c, hipMemsetAsync(c->ws + c->lay.queue, 0, 8, s));
        HIP_OK(c, hipMemsetAsync(c->ws + c->lay.dstate, 0, 8, s));
        HIP_OK(c, hipMemsetAsync(c->ws + c->lay.acc, 0, 8 * (2 * OBS_ACC_SLOTS + MAX_BINS), s));
        if (c->p.nslow > 0) HIP_OK(c, hipMemsetAsync(c->ws + c->lay.slow_lock, 0, 4 * (size_t)c->p.nslow, s));
    }
    HIP_OK(c, hipStreamSynchronize(s));
    return ECMC_OK;
}

ecmc_status check_device(ecmc_ctx *c) {
    HIP_OK(c, hipStreamSynchronize(c->stream));
    uint32_t e = 0;
    HIP_OK(c, hipMemcpy(&e, c->ws + c->lay.err, 4, hipMemcpyDeviceToHost));
    if (e & ERR_STAGE) return fail(c, ECMC_E_CELL_OVERFLOW, "a domain exceeded the staging capacity %d", c->p.stage);
    if (e & ERR_CELL) return fail(c, ECMC_E_CELL_OVERFLOW, "a cell exceeded its capacity %d", c->cap);
    if (e & ERR_STUCK) return fail(c, ECMC_E_STUCK, "an EC exceeded %lld iterations", (long long)c->opt.event_cap);
    if (e & ERR_RECOUNT) return fail(c, ECMC_E_DEVICE, "a domain's cell lists changed between its count and its staging");
    if (e & ERR_WAIT)
        return fail(c, ECMC_E_DEVICE, "a wait of the dependency-ordered sweep ran out of time (%d s)", WAIT_SECONDS);
    return ECMC_OK;
}

std::vector<MeltIn> melt_inputs(int32_t n_melts, const ecmc_melt_desc *melts) {
    std::vector<MeltIn> in((size_t)std::max(n_melts, 0));
    for (int32_t m = 0; m < n_melts; ++m)
        in[m] = {melts[m].box, melts[m].n_beads, melts[m].n_cells, melts[m].domain_cells};
    return in;
}

// polymers of a melt: n_beads - n_bonds for linear chains (checked at init)
int64_t polymers(int32_t n_melts, const ecmc_melt_desc *melts) {
    int64_t np = 0;
    for (int32_t m = 0; m < n_melts; ++m) np += std::max<int64_t>(melts[m].n_beads - melts[m].n_bonds, 1);
    return np;
}

ecmc_status init_impl(ecmc_ctx **out, int32_t n_melts, const ecmc_melt_desc *melts, double sigma, double l_max,
                      const ecmc_options *opt, int64_t npoly_layout) {
    if (!out) return fail(nullptr, ECMC_E_ARG, "null output pointer");
    *out = nullptr;
    if (!opt || !melts || n_melts < 1) return fail(nullptr, ECMC_E_ARG, "null argument or no melts");
    for (int32_t m = 0; m < n_melts; ++m)
        if (!melts[m].positions || melts[m].n_bonds < 0 || (melts[m].n_bonds > 0 && !melts[m].bonds))
            return fail(nullptr, ECMC_E_ARG, "melt %d: null argument", m);
    ecmc_ctx *c = new ecmc_ctx();
    c->opt = *opt;
    if (c->opt.event_cap <= 0) c->opt.event_cap = DEFAULT_EVENT_CAP;
    c->stream = (hipStream_t)opt->stream;
    c->sigma = sigma;
    c->lmax = l_max;
    c->sig2 = sigma * sigma;
    c->b2 = l_max * l_max;
    c->cap = opt->cell_capacity > 0 ? opt->cell_capacity : DEFAULT_CAP;
    auto bail = [&](ecmc_status s) {
        g_err = c->err;
        ecmc_destroy(c);
        return s;
    };
    ecmc_status st = plan(melt_inputs(n_melts, melts), sigma, l_max, *opt, c->p, c);
    if (st) return bail(st);
    c->nb = c->p.nb;
    c->lay = make_layout(c->p, npoly_layout, c->cap, opt->event_log_capacity);
    if (!opt->workspace || opt->workspace_bytes < c->lay.total || ((uintptr_t)opt->workspace & 255))
        return bail(fail(c, ECMC_E_WORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)", c->lay.total,
                         opt->workspace_bytes));
    c->ws = (char *)opt->workspace;
    {
        // the guard on a dependency wait of the sweep kernel: WAIT_SECONDS of the device's
        // constant-rate counter (its rate in kHz; 100 MHz if the runtime does not say)
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
            khz = 100000;
        c->wait_ticks = opt->wait_limit_us > 0 ? (unsigned long long)khz * (unsigned long long)opt->wait_limit_us / 1000ull
                                               : (unsigned long long)khz * 1000ull * WAIT_SECONDS;
    }
    if (c->p.bpl2 && opt->side_stream) {
        // by phases (also for a sweep-capable melt when only some colours run): the larger
        // tiers on the caller's second stream, ordered against the first by two events
        c->side = (hipStream_t)opt->side_stream;
        if (hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->join, hipEventDisableTiming) != hipSuccess)
            return bail(fail(c, ECMC_E_DEVICE, "creating the events of the second stream failed"));
    }

    HostState hs;
    const int64_t nb = c->nb;
    hs.px.resize(nb);
    hs.py.resize(nb);
    hs.pz.resize(nb);
    hs.cx.resize(nb);
    hs.cy.resize(nb);
    hs.cz.resize(nb);
    hs.img.assign(3 * nb, 0);
    hs.part.assign(2 * nb, -1);
    hs.cellp.resize(nb);
    hs.ccount.assign((size_t)c->p.cells, 0);
    hs.cids.assign((size_t)c->p.cells * c->cap, -1);
    for (int32_t m = 0; m < n_melts; ++m) {
        const MeltPlan &mp = c->p.melts[m];
        for (int64_t i = 0; i < mp.nb; ++i) {
            double w[3];
            for (int a = 0; a < 3; ++a) {
                const double v = melts[m].positions[3 * i + a];
                if (!std::isfinite(v)) return bail(fail(c, ECMC_E_ARG, "melt %d: position %lld is not finite", m, (long long)i));
                w[a] = wrap_coord(v, mp.L);
            }
            const int64_t g = mp.bead0 + i;
            hs.px[g] = w[0];
            hs.py[g] = w[1];
            hs.pz[g] = w[2];
            hs.cx[g] = bin_coord(w[0], mp.n, mp.h, mp.L);
            hs.cy[g] = bin_coord(w[1], mp.n, mp.h, mp.L);
            hs.cz[g] = bin_coord(w[2], mp.n, mp.h, mp.L);
        }
        if ((st = build_topology(c, m, melts[m].n_bonds, melts[m].bonds, hs))) return bail(st);
        if ((st = build_cells(c, m, hs, true))) return bail(st);
    }
    c->npoly = (int64_t)hs.pstart.size();
    if (c->npoly > npoly_layout) return bail(fail(c, ECMC_E_ARG, "more polymers than the layout holds"));
    hs.pstart.push_back((int32_t)nb);
    for (int64_t q = 0; q < c->npoly; ++q) {
        const size_t len = (size_t)(hs.pstart[q + 1] - hs.pstart[q]);
        if (c->chain_count.size() <= len) c->chain_count.resize(len + 1, 0);
        c->chain_count[len]++;
    }
    {
        // the device of the context, with the address of its static scratch (once per device)
        int dev = -1;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = resolve_scratch(dev);
        if (e != hipSuccess)
            return bail(fail(c, ECMC_E_DEVICE, "resolving the static scratch of device %d: %s", dev, hipGetErrorString(e)));
        c->device = dev;
    }
    if ((st = upload(c, hs, true))) return bail(st);
    *out = c;
    return ECMC_OK;
}

ecmc_melt_desc single_melt(double box, int64_t n_beads, const double *positions, int64_t n_bonds,
                           const int32_t *bonds, const ecmc_options &o) {
    ecmc_melt_desc d{};
    d.box = box;
    d.n_beads = n_beads;
    d.positions = positions;
    d.n_bonds = n_bonds;
    d.bonds = bonds;
    d.n_cells = o.n_cells;
    d.domain_cells = o.tiling != ECMC_TILING_WHOLE ? o.domain_cells : 0;
    return d;
}

}  // namespace

extern "C" {

void ecmc_default_options(ecmc_options *o) {
    std::memset(o, 0, sizeof *o);
    o->precision = ECMC_PREC_FP64;
    o->tiling = ECMC_TILING_CHECKER;
    o->domain_cells = 2;
}

ecmc_status ecmc_workspace_size_batch(int32_t n_melts, const ecmc_melt_desc *melts, double sigma, double l_max,
                                      const ecmc_options *opt, size_t *bytes) {
    if (!opt || !bytes || !melts || n_melts < 1) return fail(nullptr, ECMC_E_ARG, "null argument or no melts");
    Plan p;
    ecmc_status st = plan(melt_inputs(n_melts, melts), sigma, l_max, *opt, p, nullptr);
    if (st) return st;
    const int cap = opt->cell_capacity > 0 ? opt->cell_capacity : DEFAULT_CAP;
    *bytes = make_layout(p, polymers(n_melts, melts), cap, opt->event_log_capacity).total;
    return ECMC_OK;
}

ecmc_status ecmc_workspace_size(double box, double sigma, double l_max, int64_t n_beads, const ecmc_options *opt,
                                size_t *bytes) {
    if (!opt || !bytes) return fail(nullptr, ECMC_E_ARG, "null argument");
    // bonds are not known here: room for up to one polymer per bead
    const ecmc_melt_desc d = single_melt(box, n_beads, nullptr, 0, nullptr, *opt);
    Plan p;
    ecmc_status st = plan(melt_inputs(1, &d), sigma, l_max, *opt, p, nullptr);
    if (st) return st;
    const int cap = opt->cell_capacity > 0 ? opt->cell_capacity : DEFAULT_CAP;
    *bytes = make_layout(p, std::max<int64_t>(n_beads, 1), cap, opt->event_log_capacity).total;
    return ECMC_OK;
}

ecmc_status ecmc_screen_constants(double box, double sigma, double l_max, int64_t n_beads, const ecmc_options *opt,
                                  float out[4], double geo[3]) {
    if (!opt || !out || !geo) return fail(nullptr, ECMC_E_ARG, "null argument");
    const ecmc_melt_desc d = single_melt(box, n_beads, nullptr, 0, nullptr, *opt);
    Plan p;
    ecmc_status st = plan(melt_inputs(1, &d), sigma, l_max, *opt, p, nullptr);
    if (st) return st;
    const MeltPlan &mp = p.melts[0];
    out[0] = mp.p_sure;
    out[1] = mp.in_lo;
    out[2] = mp.in_hi;
    out[3] = mp.err_f;
    geo[0] = mp.h;
    geo[1] = p.whole ? mp.L : (mp.D + 2) * mp.h;
    geo[2] = mp.L;
    return ECMC_OK;
}

ecmc_status ecmc_init(ecmc_ctx **out, double box, double sigma, double l_max, int64_t n_beads,
                      const double *positions, int64_t n_bonds, const int32_t *bonds, const ecmc_options *opt) {
    if (!opt) return fail(nullptr, ECMC_E_ARG, "null argument");
    const ecmc_melt_desc d = single_melt(box, n_beads, positions, n_bonds, bonds, *opt);
    // the layout ecmc_workspace_size promised: room for one polymer per bead
    return init_impl(out, 1, &d, sigma, l_max, opt, std::max<int64_t>(n_beads, 1));
}

ecmc_status ecmc_init_batch(ecmc_ctx **out, int32_t n_melts, const ecmc_melt_desc *melts, double sigma,
                            double l_max, const ecmc_options *opt) {
    if (!melts || n_melts < 1) return fail(nullptr, ECMC_E_ARG, "null argument or no melts");
    return init_impl(out, n_melts, melts, sigma, l_max, opt, polymers(n_melts, melts));
}

namespace {
// One sweep; push > 0 runs the push-off at working diameter `push` (plain FP64 search, one
// dependency-ordered launch, which the melt's staging must allow).
ecmc_status sweep_impl(ecmc_ctx *c, int64_t n_chains, double ell, uint64_t seed, uint32_t colour_mask, double push) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    if (n_chains < 0 || !std::isfinite(ell) || !(ell >= 0)) return fail(c, ECMC_E_ARG, "need n_chains >= 0, ell >= 0");
    const bool batch = c->p.melts.size() > 1;
    if (batch && (colour_mask & 0xFFu) != 0xFFu) return fail(c, ECMC_E_ARG, "a batch of melts sweeps all eight colours");
    const MeltPlan &m0 = c->p.melts[0];
    PhaseArgs a{};
    a.px = c->dev<double>(c->lay.px);
    a.py = c->dev<double>(c->lay.py);
    a.pz = c->dev<double>(c->lay.pz);
    a.cellp = c->dev<int32_t>(c->lay.cellp);
    a.img = c->dev<int32_t>(c->lay.img);
    a.part = c->dev<int32_t>(c->lay.part);
    a.ccount = c->dev<int32_t>(c->lay.ccount);
    a.cids = c->dev<int32_t>(c->lay.cids);
    a.dstage = c->dev<int32_t>(c->lay.dstage);
    a.done = c->dev<uint32_t>(c->lay.done);
    a.queue = c->dev<uint32_t>(c->lay.queue);
    a.dstate = c->dev<uint32_t>(c->lay.dstate);
    a.melts = c->dev<MeltDev>(c->lay.melts);
    a.n_melts = (int)c->p.melts.size();
    a.tickets = c->p.tickets;
    a.slow = c->dev<double>(c->lay.slow);
    a.slow_lock = c->dev<uint32_t>(c->lay.slow_lock);
    a.nslow = c->p.nslow;
    a.slow_cap = c->p.nslow > 0 ? c->p.slow_cap : 0;
    a.cnt = c->dev<unsigned long long>(c->lay.cnt);
    a.sum_delta = c->dev<double>(c->lay.dsum);
    a.err = c->dev<unsigned int>(c->lay.err);
    a.log = c->opt.event_log_capacity > 0 ? c->dev<ecmc_event>(c->lay.log) : nullptr;
    a.log_n = c->dev<unsigned long long>(c->lay.log_n);
    a.log_cap = c->opt.event_log_capacity;
    // melt 0's geometry: the phase kernels run a single melt; the sweep kernel takes every
    // melt's own from the table
    a.L = m0.L;
    a.h = m0.h;
    a.halfL = 0.5 * m0.L;
    a.n = m0.n;
    a.D = m0.D;
    a.nd = m0.nd;
    a.ndpc = m0.ndpc;
    a.in_lo = m0.in_lo;
    a.in_hi = m0.in_hi;
    a.p_sure = m0.p_sure;
    a.err_f = m0.err_f;
    a.sig2 = c->sig2;
    a.b2 = c->b2;
    a.sig2f = (float)c->sig2;
    a.b2f = (float)c->b2;
    a.ell = ell;
    a.event_cap = (int)std::min<int64_t>(c->opt.event_cap, INT32_MAX);
    a.cap = c->cap;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.stream = 0;
    a.exact_search = c->opt.precision == ECMC_PREC_FP64 ? 1 : 0;
    a.swap = c->opt.swap_moves ? 1 : 0;
    a.two_over_k = c->opt.spring_k > 0.0 ? 2.0 / c->opt.spring_k : 0.0;
    a.wait_ticks = c->wait_ticks;
    a.joint = c->opt.tiling == ECMC_TILING_JOINT ? 1 : 0;
    if (push > 0.0) {
        if (!c->p.sweep || (colour_mask & 0xFFu) != 0xFFu || c->opt.spring_k > 0.0 || c->opt.swap_moves)
            return fail(c, ECMC_E_ARG, "the push-off needs the one-launch checkerboard sweep of tethered chains");
        a.sig2 = push * push;
        a.ov2 = a.sig2 * (1.0 - 1e-9);
        a.exact_search = 1;
    }
    a.sigma = c->sigma;
    const bool spring = c->opt.spring_k > 0.0;
    const bool log = c->opt.event_log_capacity > 0;
    auto phase_launch = [&](const PhaseArgs &pa, int bpl, int grid, hipStream_t s) {
        return spring ? launch_phase_spring(pa, bpl, log, grid, s) : launch_phase(pa, bpl, log, grid, s);
    };
    auto timed = [&](auto body) -> ecmc_status {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->opt.time_kernels) {
            HIP_OK(c, hipEventCreate(&e0));
            HIP_OK(c, hipEventCreate(&e1));
            HIP_OK(c, hipEventRecord(e0, c->stream));
        }
        ecmc_status st = body();
        if (st) return st;
        if (c->opt.time_kernels) {
            HIP_OK(c, hipEventRecord(e1, c->stream));
            c->timing.emplace_back(e0, e1);
        }
        return ECMC_OK;
    };
    auto phase = [&](int grid) -> ecmc_status {
        return timed([&]() -> ecmc_status {
            // every domain's bead count first, on the main stream: the tier launches pick their
            // domains by it and never recount (a count taken while another tier rewrites a
            // domain's cell lists could be half-updated and claim that domain twice)
            HIP_OK(c, launch_count(a, grid, c->stream));
            // the tiers take disjoint sets of domains of one colour, which never interact: the
            // larger (rarer) tiers run on the caller's second stream concurrently with the
            // first, or after it on the same stream
            hipStream_t ts = c->side ? c->side : c->stream;
            if (c->p.bpl2 && c->side) {
                HIP_OK(c, hipEventRecord(c->fork, c->stream));
                HIP_OK(c, hipStreamWaitEvent(c->side, c->fork, 0));
            }
            a.stage_lo = 0;
            a.stage_hi = c->p.bpl2 ? 64 * c->p.bpl : 0x7fffffff;
            HIP_OK(c, phase_launch(a, c->p.bpl, grid, c->stream));
            if (c->p.bpl2) {
                PhaseArgs b = a;
                b.stage_lo = 64 * c->p.bpl;
                b.stage_hi = c->p.bpl3 ? 64 * c->p.bpl2 : 0x7fffffff;
                HIP_OK(c, phase_launch(b, c->p.bpl2, grid, ts));
                if (c->p.bpl3) {
                    b.stage_lo = 64 * c->p.bpl2;
                    b.stage_hi = 0x7fffffff;
                    HIP_OK(c, phase_launch(b, c->p.bpl3, grid, ts));
                }
                if (c->side) {
                    HIP_OK(c, hipEventRecord(c->join, c->side));
                    HIP_OK(c, hipStreamWaitEvent(c->stream, c->join, 0));
                }
            }
            return ECMC_OK;
        });
    };
    ecmc_status st = ECMC_OK;
    if (c->p.whole) {
        a.whole = 1;
        if (n_chains > INT32_MAX) return fail(c, ECMC_E_ARG, "at most %d ECs per domain and sweep", INT32_MAX);
        a.K = (int)n_chains;
        a.colour = 0;
        if (n_chains > 0 && (colour_mask & 1u)) st = phase(1);
    } else {
        a.whole = 0;
        const int64_t K = (n_chains + c->p.domains - 1) / c->p.domains;
        if (K > INT32_MAX) return fail(c, ECMC_E_ARG, "at most %d ECs per domain and sweep", INT32_MAX);
        a.K = (int)K;
        if (c->p.sweep && (colour_mask & 0xFFu) == 0xFFu && a.K > 0) {
            // all eight colours of every melt in one dependency-ordered launch, which also
            // advances the device-side sweep counter
            st = timed([&]() -> ecmc_status {
                int waves = 0;
                HIP_OK(c, push > 0.0 ? launch_sweep_push(a, c->p.bpl, log, &waves, c->stream)
                          : spring   ? launch_sweep_spring(a, c->p.bpl, log, &waves, c->stream)
                                     : launch_sweep(a, c->p.bpl, log, &waves, c->stream));
                return ECMC_OK;
            });
            if (st == ECMC_OK) c->sweep_ctr++;
            return st;
        }
        if (a.joint) {
            // tile-joint: all tiles in one phase (colour bit 0)
            if ((colour_mask & 1u) && a.K > 0) {
                a.colour = 0;
                st = phase(m0.ndpc);
            }
        }
        for (int colour = 0; colour < 8 && st == ECMC_OK && a.K > 0 && !a.joint; ++colour) {
            if (!((colour_mask >> colour) & 1u)) continue;
            a.colour = colour;
            st = phase(m0.ndpc);
        }
    }
    if (st) return st;
    HIP_OK(c, launch_advance(a, c->stream));
    c->sweep_ctr++;
    return ECMC_OK;
}

// Pairs of every melt whose squared distance is below q_lim (the overlaps of the push-off).
ecmc_status count_pairs_below(ecmc_ctx *c, double q_lim, int64_t *n) {
    HIP_OK(c, hipMemsetAsync(c->ws + c->lay.hist, 0, 8, c->stream));
    PairArgs a{};
    a.px = c->dev<double>(c->lay.px);
    a.py = c->dev<double>(c->lay.py);
    a.pz = c->dev<double>(c->lay.pz);
    a.ccount = c->dev<int32_t>(c->lay.ccount);
    a.cids = c->dev<int32_t>(c->lay.cids);
    a.cap = c->cap;
    a.melts = c->dev<MeltDev>(c->lay.melts);
    a.n_melts = (int)c->p.melts.size();
    a.cells = c->p.cells;
    a.nbins = 1;
    a.rmax = std::sqrt(q_lim);
    a.q_lim = q_lim;
    a.hist = c->dev<unsigned long long>(c->lay.hist);
    HIP_OK(c, launch_pairs(a, c->stream));
    ecmc_status st = check_device(c);
    if (st) return st;
    unsigned long long v = 0;
    HIP_OK(c, hipMemcpy(&v, a.hist, 8, hipMemcpyDeviceToHost));
    *n = (int64_t)v;
    return ECMC_OK;
}
}  // namespace

ecmc_status ecmc_sweep_colours(ecmc_ctx *c, int64_t n_chains, double ell, uint64_t seed, uint32_t colour_mask) {
    return sweep_impl(c, n_chains, ell, seed, colour_mask, 0.0);
}

ecmc_status ecmc_sweep(ecmc_ctx *c, int64_t n_chains, double ell, uint64_t seed) {
    return sweep_impl(c, n_chains, ell, seed, 0xFFu, 0.0);
}

ecmc_status ecmc_pushoff_sweep(ecmc_ctx *c, int64_t n_chains, double ell, uint64_t seed, double diameter) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    if (!(diameter > 0.0) || !(diameter <= c->sigma))
        return fail(c, ECMC_E_ARG, "the push-off diameter must be in (0, sigma] (got %g)", diameter);
    return sweep_impl(c, n_chains, ell, seed, 0xFFu, diameter);
}

ecmc_status ecmc_count_overlaps(ecmc_ctx *c, double diameter, int64_t *n) {
    if (!c || !n) return fail(c, ECMC_E_ARG, "null argument");
    if (!(diameter > 0.0) || !(diameter <= c->sigma))
        return fail(c, ECMC_E_ARG, "the diameter must be in (0, sigma] (got %g)", diameter);
    return count_pairs_below(c, diameter * diameter * (1.0 - 1e-9), n);
}

ecmc_status ecmc_check_state(ecmc_ctx *c, double tol, int64_t *overlaps, int64_t *stretched, int64_t *misplaced) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    if (!(tol >= 0.0) || !(tol <= 1e-3)) return fail(c, ECMC_E_ARG, "tol must be in [0, 1e-3] (got %g)", tol);
    int64_t ov = 0;
    ecmc_status st = count_pairs_below(c, c->sig2 * (1.0 - tol), &ov);
    if (st) return st;
    HIP_OK(c, hipMemsetAsync(c->ws + c->lay.hist, 0, 24, c->stream));
    PairArgs a{};
    a.px = c->dev<double>(c->lay.px);
    a.py = c->dev<double>(c->lay.py);
    a.pz = c->dev<double>(c->lay.pz);
    a.ccount = c->dev<int32_t>(c->lay.ccount);
    a.cids = c->dev<int32_t>(c->lay.cids);
    a.cap = c->cap;
    a.melts = c->dev<MeltDev>(c->lay.melts);
    a.n_melts = (int)c->p.melts.size();
    a.cells = c->p.cells;
    a.hist = c->dev<unsigned long long>(c->lay.hist);
    a.part = c->dev<int32_t>(c->lay.part);
    a.cellp = c->dev<int32_t>(c->lay.cellp);
    a.b2lim = c->b2 * (1.0 + tol);
    HIP_OK(c, launch_check(a, c->stream));
    if ((st = check_device(c))) return st;
    unsigned long long v[3] = {0, 0, 0};
    HIP_OK(c, hipMemcpy(v, a.hist, 24, hipMemcpyDeviceToHost));
    const int64_t listed = (int64_t)v[2];
    if (overlaps) *overlaps = ov;
    if (stretched) *stretched = (int64_t)v[0];
    // a bead listed twice or not at all is misplaced too
    if (misplaced) *misplaced = (int64_t)v[1] + (listed > c->nb ? listed - c->nb : c->nb - listed);
    return ECMC_OK;
}

ecmc_status ecmc_pushoff(ecmc_ctx *c, double d_start, int32_t stages, double ell, uint64_t seed,
                         int64_t max_sweeps, int64_t *sweeps_done, int64_t *overlaps_left) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    if (!(d_start > 0.0) || !(d_start <= c->sigma) || stages < 1 || max_sweeps < 0 || !(ell > 0.0) || !std::isfinite(ell))
        return fail(c, ECMC_E_ARG, "need 0 < d_start <= sigma, stages >= 1, max_sweeps >= 0, ell > 0");
    int64_t done = 0, left = 0;
    for (int s = 1; s <= stages; ++s) {
        // working diameters from d_start up to sigma in equal steps (the last one exactly sigma)
        const double d = s == stages ? c->sigma : d_start + (c->sigma - d_start) * (double)s / (double)stages;
        for (int64_t k = 0;; ++k) {
            ecmc_status st = ecmc_count_overlaps(c, d, &left);
            if (st) return st;
            if (left == 0 || k >= max_sweeps) break;
            if ((st = sweep_impl(c, c->nb, ell, seed + (uint64_t)done, 0xFFu, d))) return st;
            ++done;
        }
        if (left) break;
    }
    if (sweeps_done) *sweeps_done = done;
    if (overlaps_left) *overlaps_left = left;
    return check_device(c);
}

ecmc_status ecmc_synchronize(ecmc_ctx *c) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    return check_device(c);
}

}  // extern "C"

namespace {
ObsArgs obs_args(ecmc_ctx *c) {
    ObsArgs o{};
    o.px = c->dev<double>(c->lay.px);
    o.py = c->dev<double>(c->lay.py);
    o.pz = c->dev<double>(c->lay.pz);
    o.img = c->dev<int32_t>(c->lay.img);
    o.porder = c->dev<int32_t>(c->lay.porder);
    o.pstart = c->dev<int32_t>(c->lay.pstart);
    o.polyL = c->dev<double>(c->lay.polyL);
    o.npoly = c->npoly;
    o.sigma = c->sigma;
    o.bmax = c->lmax;
    return o;
}

// R^2(n) with the per-block partial sums in lagsum, which holds slots + LAG_MAX_BEADS doubles
// (blocks x lags, then the lag totals).  The number of blocks depends only on the state and on
// slots, and every slot the sums read is written first in the same call, so nothing is cleared.
ecmc_status internal_distances(ecmc_ctx *c, int32_t n_max, double *r2, int64_t *pairs, double *lagsum, int64_t slots) {
    if (!r2) return fail(c, ECMC_E_ARG, "null argument");
    if (n_max < 0 || n_max >= LAG_MAX_BEADS) return fail(c, ECMC_E_ARG, "n_max must be in [0, %d]", LAG_MAX_BEADS - 1);
    const int64_t longest = (int64_t)c->chain_count.size() - 1;
    if (longest > LAG_MAX_BEADS)
        return fail(c, ECMC_E_ARG, "internal distances take chains of at most %d beads (the longest has %lld)",
                    LAG_MAX_BEADS, (long long)longest);
    for (int32_t n = 0; n <= n_max; ++n) {
        r2[n] = 0.0;
        if (pairs) pairs[n] = 0;
    }
    if (longest < 1) return ECMC_OK;  // no beads
    const int nlag = (int)std::min<int64_t>(n_max, longest - 1) + 1;
    // one polymer per block while the partial sums fit
    const int rows = (int)std::min<int64_t>(c->npoly, slots / nlag);
    if (rows < 1 || (int64_t)rows * nlag + nlag > slots + LAG_MAX_BEADS)
        return fail(c, ECMC_E_ARG, "the partial sums of %d lags do not fit %lld slots", nlag, (long long)slots);
    ObsArgs o = obs_args(c);
    o.nlag = nlag;
    o.lagsum = lagsum;
    HIP_OK(c, launch_internal(o, rows, (int)longest, c->stream));
    ecmc_status st = check_device(c);
    if (st) return st;
    // the lag totals land in r2[0..nlag) and are divided there by the pair counts
    HIP_OK(c, hipMemcpy(r2, o.lagsum + (size_t)rows * nlag, 8 * (size_t)nlag, hipMemcpyDeviceToHost));
    for (int32_t n = 0; n <= n_max; ++n) {
        // pairs n bonds apart: max(N - n, 0) in a chain of N beads
        int64_t cnt = 0;
        for (size_t len = (size_t)n + 1; len < c->chain_count.size(); ++len) cnt += c->chain_count[len] * ((int64_t)len - n);
        r2[n] = n < nlag && cnt > 0 ? r2[n] / (double)cnt : 0.0;
        if (pairs) pairs[n] = cnt;
    }
    return ECMC_OK;
}
}  // namespace

extern "C" {

ecmc_status ecmc_observables(ecmc_ctx *c, int32_t nbins, double *r2, double *rg2, int64_t *hist, double *mid,
                             int64_t *n_poly) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    if (nbins <= 0 || nbins > MAX_BINS) return fail(c, ECMC_E_ARG, "nbins must be in [1, %d]", MAX_BINS);
    if (n_poly) *n_poly = c->npoly;
    HIP_OK(c, hipMemsetAsync(c->ws + c->lay.hist, 0, 8 * nbins, c->stream));
    ObsArgs o = obs_args(c);
    o.nbins = nbins;
    o.r2 = c->dev<double>(c->lay.r2);
    o.rg2 = c->dev<double>(c->lay.rg2);
    o.mid = c->dev<double>(c->lay.mid);
    o.hist = c->dev<unsigned long long>(c->lay.hist);
    HIP_OK(c, launch_observables(o, c->stream));
    ecmc_status st = check_device(c);
    if (st) return st;
    if (r2) HIP_OK(c, hipMemcpy(r2, o.r2, 8 * c->npoly, hipMemcpyDeviceToHost));
    if (rg2) HIP_OK(c, hipMemcpy(rg2, o.rg2, 8 * c->npoly, hipMemcpyDeviceToHost));
    if (mid) HIP_OK(c, hipMemcpy(mid, o.mid, 24 * c->npoly, hipMemcpyDeviceToHost));
    if (hist) HIP_OK(c, hipMemcpy(hist, o.hist, 8 * nbins, hipMemcpyDeviceToHost));
    return ECMC_OK;
}

ecmc_status ecmc_observables_accumulate(ecmc_ctx *c, int32_t nbins) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    if (nbins <= 0 || nbins > MAX_BINS) return fail(c, ECMC_E_ARG, "nbins must be in [1, %d]", MAX_BINS);
    if (c->acc_samples > 0 && nbins != c->acc_nbins)
        return fail(c, ECMC_E_ARG, "nbins %d differs from the %d of the running sums (reset them first)", nbins,
                    c->acc_nbins);
    ObsArgs o = obs_args(c);
    o.nbins = nbins;
    o.r2 = c->dev<double>(c->lay.r2);
    o.rg2 = c->dev<double>(c->lay.rg2);
    o.mid = c->dev<double>(c->lay.mid);
    o.acc = c->dev<double>(c->lay.acc);
    o.hist = c->dev<unsigned long long>(c->lay.acc + 8 * 2 * OBS_ACC_SLOTS);
    HIP_OK(c, launch_observables(o, c->stream));
    c->acc_nbins = nbins;
    ++c->acc_samples;
    return ECMC_OK;
}

ecmc_status ecmc_observables_mean(ecmc_ctx *c, double *r2_mean, double *rg2_mean, int64_t *hist, int64_t *samples) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    ecmc_status st = check_device(c);
    if (st) return st;
    if (samples) *samples = c->acc_samples;
    std::vector<double> acc(2 * OBS_ACC_SLOTS + MAX_BINS);
    HIP_OK(c, hipMemcpy(acc.data(), c->ws + c->lay.acc, 8 * acc.size(), hipMemcpyDeviceToHost));
    double s0 = 0.0, s1 = 0.0;
    for (int i = 0; i < OBS_ACC_SLOTS; ++i) {
        s0 += acc[i];
        s1 += acc[OBS_ACC_SLOTS + i];
    }
    const double n = (double)c->acc_samples * (double)c->npoly;
    if (r2_mean) *r2_mean = n > 0 ? s0 / n : 0.0;
    if (rg2_mean) *rg2_mean = n > 0 ? s1 / n : 0.0;
    if (hist)
        for (int i = 0; i < c->acc_nbins; ++i) {
            uint64_t v;
            std::memcpy(&v, &acc[2 * OBS_ACC_SLOTS + i], 8);
            hist[i] = (int64_t)v;
        }
    return ECMC_OK;
}

ecmc_status ecmc_observables_reset(ecmc_ctx *c) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    HIP_OK(c, launch_zero_u64(c->dev<unsigned long long>(c->lay.acc), 2 * OBS_ACC_SLOTS + MAX_BINS, c->stream));
    c->acc_samples = 0;
    c->acc_nbins = 0;
    return ECMC_OK;
}

ecmc_status ecmc_shape(ecmc_ctx *c, double *gyr, double *eig, double *com, int64_t *n_poly) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    if (n_poly) *n_poly = c->npoly;
    ObsArgs o = obs_args(c);
    o.gyr = c->dev<double>(c->lay.shape);
    o.eig = o.gyr + 6 * c->npoly;
    o.com = o.eig + 3 * c->npoly;
    HIP_OK(c, launch_shape(o, c->stream));
    ecmc_status st = check_device(c);
    if (st) return st;
    if (gyr) HIP_OK(c, hipMemcpy(gyr, o.gyr, 48 * c->npoly, hipMemcpyDeviceToHost));
    if (eig) HIP_OK(c, hipMemcpy(eig, o.eig, 24 * c->npoly, hipMemcpyDeviceToHost));
    if (com) HIP_OK(c, hipMemcpy(com, o.com, 24 * c->npoly, hipMemcpyDeviceToHost));
    return ECMC_OK;
}

ecmc_status ecmc_snapshot(ecmc_ctx *c, double *snap) {
    if (!c || !snap) return fail(c, ECMC_E_ARG, "null argument");
    if (reinterpret_cast<uintptr_t>(snap) % 8) return fail(c, ECMC_E_ARG, "snapshot buffer not 8-byte aligned");
    ObsArgs o = obs_args(c);
    o.gyr = c->dev<double>(c->lay.shape);
    o.eig = o.gyr + 6 * c->npoly;
    o.com = o.eig + 3 * c->npoly;
    o.snap = snap;
    HIP_OK(c, launch_shape(o, c->stream));
    return ECMC_OK;
}

ecmc_status ecmc_msd(ecmc_ctx *c, const double *snaps, int64_t T, double *out) {
    if (!c || !snaps || !out) return fail(c, ECMC_E_ARG, "null argument");
    if (T < 1 || T > 0x7fffffff) return fail(c, ECMC_E_ARG, "T must be in [1, 2^31 - 1] (got %lld)", (long long)T);
    HIP_OK(c, launch_msd(snaps, T, c->npoly, out, c->stream));
    return ECMC_OK;
}

ecmc_status ecmc_end_to_end_histogram(ecmc_ctx *c, int32_t nbins, double r_max, int64_t *hist) {
    if (!c || !hist) return fail(c, ECMC_E_ARG, "null argument");
    if (nbins <= 0 || nbins > MAX_BINS) return fail(c, ECMC_E_ARG, "nbins must be in [1, %d]", MAX_BINS);
    if (!(r_max > 0.0) || !std::isfinite(r_max)) return fail(c, ECMC_E_ARG, "r_max must be finite and > 0");
    // the bond histogram's buffer holds the counts (a context's calls do not overlap)
    HIP_OK(c, hipMemsetAsync(c->ws + c->lay.hist, 0, 8 * nbins, c->stream));
    ObsArgs o = obs_args(c);
    o.nbins = 1;
    o.r2 = c->dev<double>(c->lay.r2);
    o.rg2 = c->dev<double>(c->lay.rg2);
    o.mid = c->dev<double>(c->lay.mid);
    o.hist = nullptr;
    o.rhist = c->dev<unsigned long long>(c->lay.hist);
    o.rbins = nbins;
    o.rmax = r_max;
    HIP_OK(c, launch_observables(o, c->stream));
    ecmc_status st = check_device(c);
    if (st) return st;
    HIP_OK(c, hipMemcpy(hist, o.rhist, 8 * nbins, hipMemcpyDeviceToHost));
    return ECMC_OK;
}

ecmc_status ecmc_internal_distances(ecmc_ctx *c, int32_t n_max, double *r2, int64_t *pairs) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    return internal_distances(c, n_max, r2, pairs, c->dev<double>(c->lay.lags), c->lay.lag_slots);
}

ecmc_status ecmc_internal_distances_noalloc(ecmc_ctx *c, int32_t n_max, double *r2, int64_t *pairs) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    double *ptr = c->device >= 0 && c->device < MAX_DEVICES ? g_scratch[c->device] : nullptr;
    if (!ptr) return fail(c, ECMC_E_DEVICE, "the static scratch of device %d was not resolved at init", c->device);
    return internal_distances(c, n_max, r2, pairs, ptr, NOALLOC_LAG_SLOTS);
}

ecmc_status ecmc_pair_histogram(ecmc_ctx *c, int32_t nbins, double r_max, int64_t *hist) {
    if (!c || !hist) return fail(c, ECMC_E_ARG, "null argument");
    if (nbins <= 0 || nbins > MAX_BINS) return fail(c, ECMC_E_ARG, "nbins must be in [1, %d]", MAX_BINS);
    double hmin = INFINITY;
    for (const MeltPlan &mp : c->p.melts) hmin = std::min(hmin, mp.h);
    if (!(r_max > 0.0) || !(r_max <= hmin))
        return fail(c, ECMC_E_ARG, "r_max must be in (0, %g], the smallest cell edge (got %g)", hmin, r_max);
    HIP_OK(c, hipMemsetAsync(c->ws + c->lay.hist, 0, 8 * nbins, c->stream));
    PairArgs a{};
    a.px = c->dev<double>(c->lay.px);
    a.py = c->dev<double>(c->lay.py);
    a.pz = c->dev<double>(c->lay.pz);
    a.ccount = c->dev<int32_t>(c->lay.ccount);
    a.cids = c->dev<int32_t>(c->lay.cids);
    a.cap = c->cap;
    a.melts = c->dev<MeltDev>(c->lay.melts);
    a.n_melts = (int)c->p.melts.size();
    a.cells = c->p.cells;
    a.nbins = nbins;
    a.rmax = r_max;
    a.hist = c->dev<unsigned long long>(c->lay.hist);
    HIP_OK(c, launch_pairs(a, c->stream));
    ecmc_status st = check_device(c);
    if (st) return st;
    HIP_OK(c, hipMemcpy(hist, a.hist, 8 * nbins, hipMemcpyDeviceToHost));
    return ECMC_OK;
}

ecmc_status ecmc_get_positions(ecmc_ctx *c, double *out) {
    if (!c || !out) return fail(c, ECMC_E_ARG, "null argument");
    ecmc_status st = check_device(c);
    if (st) return st;
    std::vector<double> x(c->nb), y(c->nb), z(c->nb);
    HIP_OK(c, hipMemcpy(x.data(), c->ws + c->lay.px, 8 * c->nb, hipMemcpyDeviceToHost));
    HIP_OK(c, hipMemcpy(y.data(), c->ws + c->lay.py, 8 * c->nb, hipMemcpyDeviceToHost));
    HIP_OK(c, hipMemcpy(z.data(), c->ws + c->lay.pz, 8 * c->nb, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < c->nb; ++i) {
        out[3 * i] = x[i];
        out[3 * i + 1] = y[i];
        out[3 * i + 2] = z[i];
    }
    return ECMC_OK;
}

ecmc_status ecmc_get_cells(ecmc_ctx *c, int32_t *out) {
    if (!c || !out) return fail(c, ECMC_E_ARG, "null argument");
    ecmc_status st = check_device(c);
    if (st) return st;
    std::vector<int32_t> w(c->nb);
    HIP_OK(c, hipMemcpy(w.data(), c->ws + c->lay.cellp, 4 * c->nb, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < c->nb; ++i)
        for (int a = 0; a < 3; ++a) out[3 * i + a] = (w[i] >> (a * CELL_BITS)) & CELL_MASK;
    return ECMC_OK;
}

ecmc_status ecmc_get_images(ecmc_ctx *c, int32_t *out) {
    if (!c || !out) return fail(c, ECMC_E_ARG, "null argument");
    ecmc_status st = check_device(c);
    if (st) return st;
    HIP_OK(c, hipMemcpy(out, c->ws + c->lay.img, 12 * c->nb, hipMemcpyDeviceToHost));
    return ECMC_OK;
}

ecmc_status ecmc_get_counters(ecmc_ctx *c, ecmc_counters *out) {
    if (!c || !out) return fail(c, ECMC_E_ARG, "null argument");
    HIP_OK(c, hipStreamSynchronize(c->stream));
    uint64_t v[NCNT];
    HIP_OK(c, hipMemcpy(v, c->ws + c->lay.cnt, 8 * NCNT, hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof *out);
    out->hs_lift = v[C_HS_LIFT];
    out->tether_lift = v[C_TETHER_LIFT];
    out->hs_reflect = v[C_HS_REFLECT];
    out->tether_reflect = v[C_TETHER_REFLECT];
    out->wall = v[C_WALL];
    out->cross = v[C_CROSS];
    out->ec = v[C_EC];
    out->steps = v[C_STEPS];
    out->periodic = v[C_PERIOD];
    out->swap = v[C_SWAP];
    out->cycle = v[C_CYCLE];
    HIP_OK(c, hipMemcpy(&out->sum_delta, c->ws + c->lay.dsum, 8, hipMemcpyDeviceToHost));
    HIP_OK(c, hipMemcpy(&out->error_flags, c->ws + c->lay.err, 4, hipMemcpyDeviceToHost));
    return ECMC_OK;
}

ecmc_status ecmc_reset_counters(ecmc_ctx *c) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    HIP_OK(c, hipMemsetAsync(c->ws + c->lay.cnt, 0, 8 * NCNT, c->stream));
    HIP_OK(c, hipMemsetAsync(c->ws + c->lay.dsum, 0, 8, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return ECMC_OK;
}

ecmc_status ecmc_shape_descriptors(const double *eig, int64_t n_poly, double out[5]) {
    if (!eig || !out || n_poly < 1) return fail(nullptr, ECMC_E_ARG, "need eigenvalues of at least one polymer");
    // moment of inertia eigenvalues I_i = tr G - l_i, descending with l ascending: the order
    // in which b = (I1 + I2)/2 - I3 and c = I1 - I2 are non-negative (appendix, Table II)
    double k2 = 0.0, s123 = 0.0, s132 = 0.0, s231 = 0.0, sol = 0.0, str = 0.0;
    for (int64_t q = 0; q < n_poly; ++q) {
        double l1 = eig[3 * q], l2 = eig[3 * q + 1], l3 = eig[3 * q + 2];
        if (!(std::isfinite(l1) && std::isfinite(l2) && std::isfinite(l3)))
            return fail(nullptr, ECMC_E_ARG, "polymer %lld: eigenvalues not finite", (long long)q);
        // l1 >= l2 >= l3 whatever order they come in
        if (l1 < l2) std::swap(l1, l2);
        if (l2 < l3) std::swap(l2, l3);
        if (l1 < l2) std::swap(l1, l2);
        const double tot = l1 + l2 + l3;
        const double i1 = tot - l3, i2 = tot - l2, i3 = tot - l1;
        const double tr = i1 + i2 + i3;
        if (!(tr > 0.0)) return fail(nullptr, ECMC_E_ARG, "polymer %lld: zero inertia", (long long)q);
        const double pair = i1 * i2 + i2 * i3 + i3 * i1;
        const double b = 0.5 * (i1 + i2) - i3, c = i1 - i2;
        k2 += 4.0 * (1.0 - 3.0 * pair / (tr * tr));
        s123 += i1 + i2 - i3;
        s132 += i1 - i2 + i3;
        s231 += -i1 + i2 + i3;
        sol += 4.0 * b * b + 3.0 * c * c;
        str += tr;
    }
    const double m = (double)n_poly, mt = str / m;
    out[0] = k2 / m;
    out[1] = s123 / m / mt;
    out[2] = s132 / m / mt;
    out[3] = s231 / m / mt;
    out[4] = sol / m / (mt * mt);
    return ECMC_OK;
}

ecmc_status ecmc_pair_correlation(const int64_t *hist, int32_t nbins, double r_max, int32_t n_melts,
                                  const int64_t *n_beads, const double *volumes, double *g) {
    if (!hist || !g || !n_beads || !volumes || nbins < 1 || n_melts < 1 || !(r_max > 0.0) || !std::isfinite(r_max))
        return fail(nullptr, ECMC_E_ARG, "need nbins >= 1, r_max > 0 and at least one melt");
    // ideal-gas pairs per unit shell volume, summed over the melts: sum_m N_m (N_m - 1) / (2 V_m)
    double dens = 0.0;
    for (int32_t m = 0; m < n_melts; ++m) {
        if (n_beads[m] < 0 || !(volumes[m] > 0.0)) return fail(nullptr, ECMC_E_ARG, "melt %d: bad size", m);
        dens += 0.5 * (double)n_beads[m] * (double)(n_beads[m] - 1) / volumes[m];
    }
    const double pi = 3.14159265358979323846;
    for (int32_t k = 0; k < nbins; ++k) {
        const double lo = r_max * k / nbins, hi = r_max * (k + 1) / nbins;
        const double shell = 4.0 * pi / 3.0 * (hi * hi * hi - lo * lo * lo);
        g[k] = dens > 0.0 ? (double)hist[k] / (dens * shell) : 0.0;
    }
    return ECMC_OK;
}

ecmc_status ecmc_clear_error(ecmc_ctx *c) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (c->side) HIP_OK(c, hipStreamSynchronize(c->side));
    HIP_OK(c, hipMemsetAsync(c->ws + c->lay.err, 0, 4, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return ECMC_OK;
}

ecmc_status ecmc_get_event_log(ecmc_ctx *c, ecmc_event *out, int64_t capacity, int64_t *n_total) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    HIP_OK(c, hipStreamSynchronize(c->stream));
    unsigned long long n = 0;
    HIP_OK(c, hipMemcpy(&n, c->ws + c->lay.log_n, 8, hipMemcpyDeviceToHost));
    if (n_total) *n_total = (int64_t)n;
    const int64_t have = std::min<int64_t>((int64_t)n, c->opt.event_log_capacity);
    const int64_t take = std::min<int64_t>(have, capacity);
    if (out && take > 0) HIP_OK(c, hipMemcpy(out, c->ws + c->lay.log, sizeof(ecmc_event) * take, hipMemcpyDeviceToHost));
    return ECMC_OK;
}

ecmc_status ecmc_clear_event_log(ecmc_ctx *c) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    HIP_OK(c, hipMemsetAsync(c->ws + c->lay.log_n, 0, 8, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return ECMC_OK;
}

ecmc_status ecmc_set_state(ecmc_ctx *c, const double *pos, const int32_t *cells, const int32_t *images,
                           uint32_t sweep_counter) {
    if (!c || !pos || !cells || !images) return fail(c, ECMC_E_ARG, "null argument");
    HIP_OK(c, hipStreamSynchronize(c->stream));
    HostState hs;
    const int64_t nb = c->nb;
    hs.px.resize(nb);
    hs.py.resize(nb);
    hs.pz.resize(nb);
    hs.cx.resize(nb);
    hs.cy.resize(nb);
    hs.cz.resize(nb);
    hs.cellp.resize(nb);
    hs.img.assign(images, images + 3 * nb);
    hs.ccount.assign((size_t)c->p.cells, 0);
    hs.cids.assign((size_t)c->p.cells * c->cap, -1);
    for (size_t m = 0; m < c->p.melts.size(); ++m) {
        const MeltPlan &mp = c->p.melts[m];
        const int n = mp.n;
        const double h = mp.h, L = mp.L;
        auto bnd = [&](int k) { return k < n ? (double)k * h : L; };
        for (int64_t i = mp.bead0; i < mp.bead0 + mp.nb; ++i) {
            for (int a = 0; a < 3; ++a) {
                const int cc = cells[3 * i + a];
                const double v = pos[3 * i + a];
                if (cc < 0 || cc >= n || !(v >= bnd(cc) - 1e-12 && v <= bnd(cc + 1) + 1e-12))
                    return fail(c, ECMC_E_ARG, "bead %lld: coordinate outside its cell", (long long)i);
            }
            hs.px[i] = pos[3 * i];
            hs.py[i] = pos[3 * i + 1];
            hs.pz[i] = pos[3 * i + 2];
            hs.cx[i] = cells[3 * i];
            hs.cy[i] = cells[3 * i + 1];
            hs.cz[i] = cells[3 * i + 2];
        }
        ecmc_status st = build_cells(c, (int)m, hs, false);
        if (st) return st;
    }
    ecmc_status st = upload(c, hs, false);
    if (st) return st;
    HIP_OK(c, hipMemcpy(c->ws + c->lay.dstate, &sweep_counter, 4, hipMemcpyHostToDevice));
    c->sweep_ctr = sweep_counter;
    return ECMC_OK;
}

ecmc_status ecmc_kernel_time(ecmc_ctx *c, double *ms, int64_t *launches) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    HIP_OK(c, hipStreamSynchronize(c->stream));
    double total = 0;
    for (auto &p : c->timing) {
        float t = 0;
        HIP_OK(c, hipEventElapsedTime(&t, p.first, p.second));
        total += t;
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    if (ms) *ms = total;
    if (launches) *launches = (int64_t)c->timing.size();
    c->timing.clear();
    return ECMC_OK;
}

uint32_t ecmc_sweep_counter(const ecmc_ctx *c) {
    if (!c) return 0;
    // the device holds the count: a replayed graph of sweeps advances it without the host
    uint32_t v = c->sweep_ctr;
    if (hipStreamSynchronize(c->stream) != hipSuccess ||
        hipMemcpy(&v, c->ws + c->lay.dstate, 4, hipMemcpyDeviceToHost) != hipSuccess)
        return c->sweep_ctr;
    return v;
}

int32_t ecmc_n_cells(const ecmc_ctx *c) { return c ? c->p.melts[0].n : 0; }
double ecmc_cell_size(const ecmc_ctx *c) { return c ? c->p.melts[0].h : 0.0; }
int32_t ecmc_stage_capacity(const ecmc_ctx *c) {
    if (!c) return 0;
    if (c->p.sweep) return std::max(64 * c->p.bpl, c->p.nslow > 0 ? c->p.slow_cap : 0);
    return 64 * (c->p.bpl3 ? c->p.bpl3 : (c->p.bpl2 ? c->p.bpl2 : c->p.bpl));
}
int32_t ecmc_n_melts(const ecmc_ctx *c) { return c ? (int32_t)c->p.melts.size() : 0; }

ecmc_status ecmc_get_melt_info(const ecmc_ctx *c, int32_t m, ecmc_melt_info *out) {
    if (!c || !out) return fail(nullptr, ECMC_E_ARG, "null argument");
    if (m < 0 || m >= (int32_t)c->p.melts.size()) return fail(nullptr, ECMC_E_ARG, "melt %d out of range", m);
    const MeltPlan &mp = c->p.melts[m];
    std::memset(out, 0, sizeof *out);
    out->box = mp.L;
    out->cell_size = mp.h;
    out->first_bead = mp.bead0;
    out->n_beads = mp.nb;
    out->first_polymer = mp.poly0;
    out->n_polymers = mp.npoly;
    out->first_domain = mp.dom0;
    out->n_domains = (int64_t)mp.nd * mp.nd * mp.nd;
    out->n_cells = mp.n;
    out->domain_cells = mp.D;
    return ECMC_OK;
}

void ecmc_destroy(ecmc_ctx *c) {
    if (!c) return;
    if (c->side) (void)hipStreamSynchronize(c->side);  // the caller's stream: not destroyed here
    if (c->fork) (void)hipEventDestroy(c->fork);
    if (c->join) (void)hipEventDestroy(c->join);
    if (!c->timing.empty()) {
        (void)hipStreamSynchronize(c->stream);
        for (auto &p : c->timing) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
    }
    delete c;
}

const char *ecmc_status_str(ecmc_status s) {
    switch (s) {
        case ECMC_OK: return "ok";
        case ECMC_E_ARG: return "invalid argument";
        case ECMC_E_OVERLAP: return "overlapping beads";
        case ECMC_E_TETHER: return "tether longer than l_max";
        case ECMC_E_BOX: return "box / cell / domain geometry";
        case ECMC_E_CELL_OVERFLOW: return "cell or staging capacity exceeded";
        case ECMC_E_STUCK: return "event cap exceeded";
        case ECMC_E_DEVICE: return "HIP runtime error";
        case ECMC_E_WORKSPACE: return "workspace too small or misaligned";
    }
    return "unknown status";
}

const char *ecmc_last_error(const ecmc_ctx *c) { return c ? c->err.c_str() : g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------- autotuner
namespace {

// Cells and domain edge of a melt under a tuning policy: 0 = D = 2 on the largest multiple
// of 4 cells per axis; 1 = the smallest typical frame (D + 2)^3 nb / n^3 among n from that
// multiple up to the largest n and every D >= 2 with n/D even.
bool policy_geometry(double L, int64_t nb, double lmax, int policy, int &n_out, int &D_out) {
    int nmax = (int)std::min(std::floor(L / lmax), (double)MAX_CELLS_PER_AXIS);
    while (nmax > 0 && !(L / nmax > lmax)) --nmax;
    const int n4 = nmax - nmax % 4;
    if (n4 < 4) return false;
    n_out = n4;
    D_out = 2;
    if (policy == 0) return true;
    double best = std::pow(4.0, 3) * (double)nb / std::pow((double)n4, 3);
    for (int n = n4; n <= nmax; ++n)
        for (int D = 2; D <= n; ++D) {
            if (n % D != 0 || (n / D) % 2 != 0) continue;
            const double frame = std::pow((double)(D + 2), 3) * (double)nb / std::pow((double)n, 3);
            if (frame < best) {
                best = frame;
                n_out = n;
                D_out = D;
            }
        }
    return true;
}

ecmc_status policy_descs(int32_t n_melts, const ecmc_melt_desc *melts, double lmax, int policy,
                         std::vector<ecmc_melt_desc> &out) {
    out.assign(melts, melts + n_melts);
    for (int32_t m = 0; m < n_melts; ++m) {
        int n = 0, D = 0;
        if (!policy_geometry(melts[m].box, melts[m].n_beads, lmax, policy, n, D))
            return fail(nullptr, ECMC_E_BOX, "melt %d: box too small for a checkerboard of 2-cell domains", m);
        out[m].n_cells = n;
        out[m].domain_cells = D;
    }
    return ECMC_OK;
}

// Staging tiers worth timing: from the smallest one holding the mean frame of the median
// bead (the frame of its melt) up to four tiers; the domains above a tier are staged in
// workspace slots, so a tier below the largest melts' frames trades their speed for that of
// the rest.
std::vector<int> tier_candidates(double typical) {
    // from the tier that holds the typical frame with three standard deviations of its bead count
    // to spare (as the automatic staging capacity does): below it a large share of the domains
    // runs from workspace slots, which is many times slower
    static const int tiers[] = {64, 128, 192, 256, 384, 512};
    const double need = typical + 3.0 * std::sqrt(typical);
    std::vector<int> out;
    for (int t : tiers)
        if (t >= need && out.size() < 4) out.push_back(t);
    if (out.empty()) out.push_back(512);
    return out;
}

double typical_frame(const std::vector<ecmc_melt_desc> &d) {
    // the mean frame of the melt holding the median bead
    std::vector<std::pair<double, int64_t>> f;
    int64_t total = 0;
    for (const ecmc_melt_desc &m : d) {
        const double mean = std::pow((double)(m.domain_cells + 2), 3) * (double)m.n_beads / std::pow((double)m.n_cells, 3);
        f.emplace_back(mean, m.n_beads);
        total += m.n_beads;
    }
    std::sort(f.begin(), f.end());
    int64_t acc = 0;
    for (const auto &x : f) {
        acc += x.second;
        if (2 * acc >= total) return x.first;
    }
    return f.back().first;
}

}  // namespace

extern "C" {

ecmc_status ecmc_tune_workspace_size(int32_t n_melts, const ecmc_melt_desc *melts, double sigma, double l_max,
                                     const ecmc_options *opt, size_t *bytes) {
    if (!opt || !bytes || !melts || n_melts < 1) return fail(nullptr, ECMC_E_ARG, "null argument or no melts");
    size_t most = 0;
    for (int policy = 0; policy < 2; ++policy) {
        std::vector<ecmc_melt_desc> d;
        ecmc_status st = policy_descs(n_melts, melts, l_max, policy, d);
        if (st) return st;
        ecmc_options o = *opt;
        o.tiling = ECMC_TILING_CHECKER;
        o.schedule = ECMC_SCHED_SWEEP;
        o.stage_capacity = 0;
        o.stage_tier = tier_candidates(typical_frame(d)).front();
        o.event_log_capacity = 0;
        size_t b = 0;
        if ((st = ecmc_workspace_size_batch(n_melts, d.data(), sigma, l_max, &o, &b))) return st;
        most = std::max(most, b);
    }
    *bytes = most;
    return ECMC_OK;
}

ecmc_status ecmc_tune_batch(int32_t n_melts, const ecmc_melt_desc *melts, double sigma, double l_max,
                            const ecmc_options *opt, int64_t n_chains, double ell, int32_t trial_sweeps,
                            int32_t *n_cells_out, int32_t *domain_cells_out, ecmc_tune_result *best) {
    if (!opt || !melts || n_melts < 1 || !n_cells_out || !domain_cells_out || !best || trial_sweeps < 1)
        return fail(nullptr, ECMC_E_ARG, "null argument, no melts or no trial sweeps");
    std::memset(best, 0, sizeof *best);
    double best_rate = -1.0;
    std::vector<ecmc_melt_desc> chosen;
    for (int policy = 0; policy < 2; ++policy) {
        std::vector<ecmc_melt_desc> d;
        ecmc_status st = policy_descs(n_melts, melts, l_max, policy, d);
        if (st) return st;
        if (policy == 1 && !chosen.empty()) {
            bool same = true;
            std::vector<ecmc_melt_desc> d0;
            (void)policy_descs(n_melts, melts, l_max, 0, d0);
            for (int32_t m = 0; m < n_melts && same; ++m)
                same = d0[m].n_cells == d[m].n_cells && d0[m].domain_cells == d[m].domain_cells;
            if (same) continue;  // the policies agree on every melt: nothing new to time
        }
        const std::vector<int> tiers = tier_candidates(typical_frame(d));
        ecmc_options o = *opt;
        o.tiling = ECMC_TILING_CHECKER;
        o.schedule = ECMC_SCHED_SWEEP;
        o.stage_capacity = 0;
        o.stage_tier = tiers.front();
        o.event_log_capacity = 0;
        o.time_kernels = 0;
        ecmc_ctx *c = nullptr;
        if ((st = ecmc_init_batch(&c, n_melts, d.data(), sigma, l_max, &o))) return st;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        auto done = [&](ecmc_status s) {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            ecmc_destroy(c);
            return s;
        };
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            return done(fail(nullptr, ECMC_E_DEVICE, "creating timing events failed"));
        for (int cand = 0; cand < 2 * (int)tiers.size(); ++cand) {
            // the staging tier and the search precision only change which kernel runs (the two
            // searches give identical results): the layout (with its workspace slots for the
            // larger domains) is the one of the smallest tier
            const int tier = tiers[cand / 2];
            const int prec = cand % 2 ? ECMC_PREC_FP64 : ECMC_PREC_MIXED;
            const int bpl = tier / 64;
            if (!sweep_bpl_supported(bpl)) continue;
            c->p.bpl = bpl;
            c->opt.precision = prec;
            if ((st = ecmc_sweep(c, n_chains, ell, 0x5EEDu + (uint64_t)tier))) return done(st);
            ecmc_counters k0{}, k1{};
            if ((st = ecmc_get_counters(c, &k0))) return done(st);
            if (hipEventRecord(e0, c->stream) != hipSuccess) return done(fail(nullptr, ECMC_E_DEVICE, "event record failed"));
            for (int t = 0; t < trial_sweeps; ++t)
                if ((st = ecmc_sweep(c, n_chains, ell, 0x5EEDu + (uint64_t)(tier + t + 1)))) return done(st);
            if (hipEventRecord(e1, c->stream) != hipSuccess) return done(fail(nullptr, ECMC_E_DEVICE, "event record failed"));
            if ((st = check_device(c))) return done(st);
            if ((st = ecmc_get_counters(c, &k1))) return done(st);
            float ms = 0;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return done(fail(nullptr, ECMC_E_DEVICE, "event timing failed"));
            const double rate = ms > 0 ? (double)(k1.ec - k0.ec) / (ms * 1e-3) : 0.0;
            best->candidates++;
            if (rate > best_rate) {
                best_rate = rate;
                best->stage_tier = tier;
                best->precision = prec;
                best->policy = policy;
                best->ms_per_sweep = ms / trial_sweeps;
                best->ecs_per_s = rate;
                chosen = d;
            }
        }
        (void)done(ECMC_OK);
    }
    if (chosen.empty()) return fail(nullptr, ECMC_E_ARG, "no candidate configuration could be timed");
    for (int32_t m = 0; m < n_melts; ++m) {
        n_cells_out[m] = chosen[m].n_cells;
        domain_cells_out[m] = chosen[m].domain_cells;
    }
    return ECMC_OK;
}

}  // extern "C"

// Host side of the C ABI declared in include/ecmc.h: validation of the start
// configuration, cell binning, workspace layout, launches of the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ecmc_internal.h"

using namespace ecmc;

namespace {

constexpr int64_t DEFAULT_EVENT_CAP = 10000000;
constexpr int DEFAULT_CAP = 16;
constexpr int MAX_BINS = 1024;
constexpr int SLOW_SLOTS = 512;  // workspace staging slots of the dependency-ordered sweep

struct Layout {
    size_t px, py, pz, cellp, img, part, ccount, cids, dstage, done, queue, slow_lock, slow, porder, pstart, r2, rg2,
        mid, shape, hist, cnt, dsum, err, log_n, log;
    size_t total;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(int64_t nb, int n, int cap, int64_t log_cap, int nslow, int slow_cap) {
    Layout l{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t nc = (size_t)n * n * n;
    l.px = take(8 * nb);
    l.py = take(8 * nb);
    l.pz = take(8 * nb);
    l.cellp = take(4 * nb);
    l.img = take(12 * nb);
    l.part = take(8 * nb);
    l.ccount = take(4 * nc);
    l.cids = take(4 * nc * cap);
    l.dstage = take(4 * (nc / 8 + 1));  // one count per domain of a colour phase (at most n^3 / 64)
    l.done = take(4 * (nc / 8 + 1));    // one stamp per domain (D >= 2: at most n^3 / 8)
    l.queue = take(8);
    l.slow_lock = take(4 * (size_t)std::max(nslow, 0));
    l.slow = take((size_t)std::max(nslow, 0) * (size_t)std::max(slow_cap, 0) * SLOW_SLOT_BYTES_PER_BEAD);
    l.porder = take(4 * nb);
    l.pstart = take(4 * (nb + 1));
    l.r2 = take(8 * nb);
    l.rg2 = take(8 * nb);
    l.mid = take(24 * nb);
    l.shape = take(96 * nb);  // gyration tensor, eigenvalues, centre of mass: 12 doubles per polymer
    l.hist = take(8 * MAX_BINS);
    l.cnt = take(8 * NCNT);
    l.dsum = take(8);
    l.err = take(4);
    l.log_n = take(8);
    l.log = take(sizeof(ecmc_event) * (size_t)std::max<int64_t>(log_cap, 0));
    l.total = o;
    return l;
}

struct Geometry {
    int n = 0;
    double h = 0;
    int D = 1;
    int nd = 1;
    int bpl = 0;     // beads per lane of the first staging tier
    int stage = 0;
    int bpl2 = 0;    // second tier for the rare domains above 64 * bpl (0 = none)
    int bpl3 = 0;    // third tier above 64 * bpl2 (0 = none)
    bool sweep = false;  // one dependency-ordered launch per sweep
    int nslow = 0;       // its workspace staging slots for domains above 64 * bpl
    int slow_cap = 0;    // beads per slot
};

}  // namespace

struct ecmc_ctx {
    ecmc_options opt;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;       // second stream for the larger staging tiers
    hipEvent_t fork = nullptr, join = nullptr;
    double L = 0, sigma = 0, lmax = 0, sig2 = 0, b2 = 0;
    int64_t nb = 0, npoly = 0;
    Geometry g;
    int cap = DEFAULT_CAP;
    Layout lay{};
    char *ws = nullptr;
    uint32_t sweep_ctr = 0;
    uint32_t epoch = 0;               // stamp of the last dependency-ordered launch
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

// ---------------------------------------------------------------- geometry
ecmc_status geometry(double L, double sigma, double lmax, int64_t nb, const ecmc_options &o, Geometry &g,
                     ecmc_ctx *c) {
    if (!(std::isfinite(L) && L > 0 && std::isfinite(sigma) && sigma > 0 && std::isfinite(lmax) && lmax >= sigma))
        return fail(c, ECMC_E_ARG, "need finite box > 0, sigma > 0, l_max >= sigma");
    if (nb < 1 || nb > 0x7fffffffLL) return fail(c, ECMC_E_ARG, "bead count %lld out of range", (long long)nb);
    if (o.precision != ECMC_PREC_FP64 && o.precision != ECMC_PREC_MIXED)
        return fail(c, ECMC_E_ARG, "precision must be ECMC_PREC_FP64 or ECMC_PREC_MIXED (got %d)", o.precision);
    if (o.schedule != ECMC_SCHED_SWEEP && o.schedule != ECMC_SCHED_PHASES)
        return fail(c, ECMC_E_ARG, "schedule must be ECMC_SCHED_SWEEP or ECMC_SCHED_PHASES (got %d)", o.schedule);
    int n = o.n_cells;
    if (n == 0) {
        n = (int)std::floor(L / lmax);
        while (n > 0 && !(L / n > lmax)) --n;
    }
    if (n < 4 || n > MAX_CELLS_PER_AXIS || !(L / n > lmax))
        return fail(c, ECMC_E_BOX, "cells per axis n = %d: need 4 <= n <= %d and L/n > l_max", n, MAX_CELLS_PER_AXIS);
    g.n = n;
    g.h = L / n;
    if (o.tiling == ECMC_TILING_WHOLE) {
        g.D = n;
        g.nd = 1;
        g.stage = (int)std::min<int64_t>(nb, MAX_STAGE + 1);
        if (nb > MAX_STAGE) return fail(c, ECMC_E_ARG, "whole-box tiling holds at most %d beads", MAX_STAGE);
        if ((int64_t)n * n * n > 64 * 16)
            return fail(c, ECMC_E_BOX, "whole-box tiling needs n^3 <= 1024 cells (n = %d)", n);
    } else if (o.tiling == ECMC_TILING_CHECKER) {
        const int D = o.domain_cells;
        // D >= 2: the integer offset drawn from [0, D) is what moves the partition between
        // sweeps; with D = 1 it is always 0 and every bead stays in its cell for good.
        if (D < 2 || n % D != 0 || (n / D) % 2 != 0)
            return fail(c, ECMC_E_BOX, "checkerboard needs D >= 2, n %% D == 0 and n/D even (n = %d, D = %d)", n, D);
        g.D = D;
        g.nd = n / D;
        if (o.stage_capacity > 0) {
            g.stage = o.stage_capacity;
        } else {
            // first tier sized for the typical domain; the few above it go to a second launch
            const double mean = std::pow((double)(D + 2), 3) * (double)nb / ((double)n * n * n);
            g.stage = (int)std::ceil(mean + 3.0 * std::sqrt(mean) + 2.0);
            g.bpl2 = 16;
        }
    } else {
        return fail(c, ECMC_E_ARG, "unknown tiling %d", o.tiling);
    }
    if (o.tiling == ECMC_TILING_WHOLE && o.stage_capacity > 0) g.stage = std::max(g.stage, o.stage_capacity);
    int bpl = (g.stage + 63) / 64;
    static const int ok[] = {1, 2, 3, 4, 6, 8, 12, 16};
    int pick = 0;
    for (int v : ok)
        if (v >= bpl) {
            pick = v;
            break;
        }
    if (!pick) return fail(c, ECMC_E_ARG, "staging capacity %d exceeds %d", g.stage, MAX_STAGE);
    const int ndc = o.tiling == ECMC_TILING_WHOLE ? n * n * n : g.D * g.D * g.D;
    while (pick < 16 && ndc > 64 * pick) pick = *std::find_if(std::begin(ok), std::end(ok), [&](int v) { return v > pick; });
    if (ndc > 64 * pick) return fail(c, ECMC_E_BOX, "a domain of %d cells exceeds the staging area", ndc);
    g.bpl = pick;
    if (g.bpl2) {
        // tier 2 one step above tier 1, tier 3 the full 16 beads per lane
        const int* nxt = std::find_if(std::begin(ok), std::end(ok), [&](int v) { return v > pick; });
        g.bpl2 = nxt == std::end(ok) ? 0 : *nxt;
        g.bpl3 = (g.bpl2 && g.bpl2 < 16) ? 16 : 0;
    }
    if (o.tiling == ECMC_TILING_CHECKER && o.schedule == ECMC_SCHED_SWEEP && sweep_bpl_supported(g.bpl)) {
        g.sweep = true;
        if (g.bpl2) {
            // automatic capacity: the domains above the LDS staging area go to workspace slots
            // that hold any frame up to the staging limit
            const int cap = o.cell_capacity > 0 ? o.cell_capacity : DEFAULT_CAP;
            const int64_t most = (int64_t)(g.D + 2) * (g.D + 2) * (g.D + 2) * cap;
            if (most > 64 * g.bpl) {
                const int64_t ndpc = (int64_t)(g.nd / 2) * (g.nd / 2) * (g.nd / 2);
                g.slow_cap = (int)std::min<int64_t>(most, MAX_STAGE);
                g.nslow = (int)std::min<int64_t>(ndpc, SLOW_SLOTS);
            }
        }
    }
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
    std::vector<int32_t> cx, cy, cz;
};

// partners, chain order, validation of bonds
ecmc_status build_topology(ecmc_ctx *c, int64_t nb, int64_t n_bonds, const int32_t *bonds, HostState &hs) {
    hs.part.assign(2 * nb, -1);
    for (int64_t b = 0; b < n_bonds; ++b) {
        const int32_t i = bonds[2 * b], j = bonds[2 * b + 1];
        if (i < 0 || j < 0 || i >= nb || j >= nb || i == j) return fail(c, ECMC_E_ARG, "bond %lld invalid", (long long)b);
        if (hs.part[2 * i] == j || hs.part[2 * i + 1] == j)
            return fail(c, ECMC_E_ARG, "duplicate bond %d-%d", i, j);
        int32_t *si = hs.part[2 * i] < 0 ? &hs.part[2 * i] : (hs.part[2 * i + 1] < 0 ? &hs.part[2 * i + 1] : nullptr);
        int32_t *sj = hs.part[2 * j] < 0 ? &hs.part[2 * j] : (hs.part[2 * j + 1] < 0 ? &hs.part[2 * j + 1] : nullptr);
        if (!si || !sj) return fail(c, ECMC_E_ARG, "bead with more than two bonds (bond %lld)", (long long)b);
        *si = j;
        *sj = i;
    }
    std::vector<char> seen(nb, 0);
    hs.porder.clear();
    hs.pstart.clear();
    for (int64_t i = 0; i < nb; ++i) {
        const int deg = (hs.part[2 * i] >= 0) + (hs.part[2 * i + 1] >= 0);
        if (seen[i] || deg > 1) continue;
        hs.pstart.push_back((int32_t)hs.porder.size());
        int32_t prev = -1, cur = (int32_t)i;
        while (cur >= 0) {
            seen[cur] = 1;
            hs.porder.push_back(cur);
            int32_t nx = hs.part[2 * cur] != prev ? hs.part[2 * cur] : hs.part[2 * cur + 1];
            if (nx == prev) nx = -1;
            prev = cur;
            cur = nx;
        }
    }
    if ((int64_t)hs.porder.size() != nb) return fail(c, ECMC_E_ARG, "bond list contains a ring");
    c->npoly = (int64_t)hs.pstart.size();
    hs.pstart.push_back((int32_t)nb);
    return ECMC_OK;
}

// cell lists from the per-bead cells; overlap and tether checks
ecmc_status build_cells(ecmc_ctx *c, HostState &hs, bool validate) {
    const int n = c->g.n;
    const int64_t nb = c->nb;
    const size_t nc = (size_t)n * n * n;
    hs.ccount.assign(nc, 0);
    hs.cids.assign(nc * c->cap, -1);
    hs.cellp.resize(nb);
    for (int64_t i = 0; i < nb; ++i) {
        const size_t f = (size_t)hs.cx[i] + n * ((size_t)hs.cy[i] + n * (size_t)hs.cz[i]);
        if (hs.ccount[f] >= c->cap)
            return fail(c, ECMC_E_CELL_OVERFLOW, "cell %zu holds more than %d beads", f, c->cap);
        hs.cids[f * c->cap + hs.ccount[f]++] = (int32_t)i;
        hs.cellp[i] = pack_cell(hs.cx[i], hs.cy[i], hs.cz[i]);
    }
    if (!validate) return ECMC_OK;
    const double L = c->L;
    const double lim_ov = c->sig2 * (1.0 - 2e-12);
    for (int64_t i = 0; i < nb; ++i) {
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int ax = (hs.cx[i] + dx + n) % n, ay = (hs.cy[i] + dy + n) % n, az = (hs.cz[i] + dz + n) % n;
                    const size_t f = (size_t)ax + n * ((size_t)ay + n * (size_t)az);
                    for (int t = 0; t < hs.ccount[f]; ++t) {
                        const int32_t j = hs.cids[f * c->cap + t];
                        if (j <= i) continue;
                        const double ex = min_image(hs.px[j] - hs.px[i], L);
                        const double ey = min_image(hs.py[j] - hs.py[i], L);
                        const double ez = min_image(hs.pz[j] - hs.pz[i], L);
                        if (ex * ex + ey * ey + ez * ez < lim_ov)
                            return fail(c, ECMC_E_OVERLAP, "beads %lld and %d overlap", (long long)i, j);
                    }
                }
        for (int t = 0; t < 2; ++t) {
            const int32_t j = hs.part[2 * i + t];
            if (j < 0) continue;
            const double ex = min_image(hs.px[j] - hs.px[i], L);
            const double ey = min_image(hs.py[j] - hs.py[i], L);
            const double ez = min_image(hs.pz[j] - hs.pz[i], L);
            if (ex * ex + ey * ey + ez * ez > c->b2 * (1.0 + 2e-12))
                return fail(c, ECMC_E_TETHER, "bond %lld-%d longer than l_max", (long long)i, j);
        }
    }
    return ECMC_OK;
}

ecmc_status upload(ecmc_ctx *c, const HostState &hs, bool topology) {
    hipStream_t s = c->stream;
    const int64_t nb = c->nb;
    const size_t nc = (size_t)c->g.n * c->g.n * c->g.n;
    HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.px, hs.px.data(), 8 * nb, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.py, hs.py.data(), 8 * nb, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.pz, hs.pz.data(), 8 * nb, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.cellp, hs.cellp.data(), 4 * nb, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.img, hs.img.data(), 12 * nb, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.ccount, hs.ccount.data(), 4 * nc, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.cids, hs.cids.data(), 4 * nc * c->cap, hipMemcpyHostToDevice, s));
    if (topology) {
        HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.part, hs.part.data(), 8 * nb, hipMemcpyHostToDevice, s));
        HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.porder, hs.porder.data(), 4 * nb, hipMemcpyHostToDevice, s));
        HIP_OK(c, hipMemcpyAsync(c->ws + c->lay.pstart, hs.pstart.data(), 4 * (c->npoly + 1), hipMemcpyHostToDevice,
                                 s));
        HIP_OK(c, hipMemsetAsync(c->ws + c->lay.cnt, 0, 8 * NCNT, s));
        HIP_OK(c, hipMemsetAsync(c->ws + c->lay.dsum, 0, 8, s));
        HIP_OK(c, hipMemsetAsync(c->ws + c->lay.err, 0, 4, s));
        HIP_OK(c, hipMemsetAsync(c->ws + c->lay.log_n, 0, 8, s));
        const size_t nc8 = nc / 8 + 1;
        HIP_OK(c, hipMemsetAsync(c->ws + c->lay.done, 0, 4 * nc8, s));
        HIP_OK(c, hipMemsetAsync(c->ws + c->lay.queue, 0, 8, s));
        if (c->g.nslow > 0) HIP_OK(c, hipMemsetAsync(c->ws + c->lay.slow_lock, 0, 4 * (size_t)c->g.nslow, s));
    }
    HIP_OK(c, hipStreamSynchronize(s));
    return ECMC_OK;
}

ecmc_status check_device(ecmc_ctx *c) {
    HIP_OK(c, hipStreamSynchronize(c->stream));
    uint32_t e = 0;
    HIP_OK(c, hipMemcpy(&e, c->ws + c->lay.err, 4, hipMemcpyDeviceToHost));
    if (e & ERR_STAGE) return fail(c, ECMC_E_CELL_OVERFLOW, "a domain exceeded the staging capacity %d", c->g.stage);
    if (e & ERR_CELL) return fail(c, ECMC_E_CELL_OVERFLOW, "a cell exceeded its capacity %d", c->cap);
    if (e & ERR_STUCK) return fail(c, ECMC_E_STUCK, "an EC exceeded %lld iterations", (long long)c->opt.event_cap);
    if (e & ERR_RECOUNT) return fail(c, ECMC_E_DEVICE, "a domain's cell lists changed between its count and its staging");
    if (e & ERR_WAIT) return fail(c, ECMC_E_DEVICE, "a wait of the dependency-ordered sweep ran out of polls");
    return ECMC_OK;
}

}  // namespace

extern "C" {

void ecmc_default_options(ecmc_options *o) {
    std::memset(o, 0, sizeof *o);
    o->precision = ECMC_PREC_MIXED;
    o->tiling = ECMC_TILING_CHECKER;
    o->domain_cells = 2;
}

ecmc_status ecmc_workspace_size(double box, double sigma, double l_max, int64_t n_beads, const ecmc_options *opt,
                                size_t *bytes) {
    if (!opt || !bytes) return fail(nullptr, ECMC_E_ARG, "null argument");
    Geometry g;
    ecmc_status st = geometry(box, sigma, l_max, n_beads, *opt, g, nullptr);
    if (st) return st;
    const int cap = opt->cell_capacity > 0 ? opt->cell_capacity : DEFAULT_CAP;
    *bytes = make_layout(n_beads, g.n, cap, opt->event_log_capacity, g.nslow, g.slow_cap).total;
    return ECMC_OK;
}

ecmc_status ecmc_init(ecmc_ctx **out, double box, double sigma, double l_max, int64_t n_beads,
                      const double *positions, int64_t n_bonds, const int32_t *bonds, const ecmc_options *opt) {
    if (!out) return fail(nullptr, ECMC_E_ARG, "null output pointer");
    *out = nullptr;
    if (!opt || !positions || n_bonds < 0 || (n_bonds > 0 && !bonds)) return fail(nullptr, ECMC_E_ARG, "null argument");
    ecmc_ctx *c = new ecmc_ctx();
    c->opt = *opt;
    if (c->opt.event_cap <= 0) c->opt.event_cap = DEFAULT_EVENT_CAP;
    c->stream = (hipStream_t)opt->stream;
    c->L = box;
    c->sigma = sigma;
    c->lmax = l_max;
    c->sig2 = sigma * sigma;
    c->b2 = l_max * l_max;
    c->nb = n_beads;
    c->cap = opt->cell_capacity > 0 ? opt->cell_capacity : DEFAULT_CAP;
    auto bail = [&](ecmc_status s) {
        g_err = c->err;
        ecmc_destroy(c);
        return s;
    };
    ecmc_status st = geometry(box, sigma, l_max, n_beads, *opt, c->g, c);
    if (st) return bail(st);
    c->lay = make_layout(n_beads, c->g.n, c->cap, opt->event_log_capacity, c->g.nslow, c->g.slow_cap);
    if (!opt->workspace || opt->workspace_bytes < c->lay.total || ((uintptr_t)opt->workspace & 255))
        return bail(fail(c, ECMC_E_WORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)", c->lay.total,
                         opt->workspace_bytes));
    c->ws = (char *)opt->workspace;
    if (c->g.bpl2) {
        if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->join, hipEventDisableTiming) != hipSuccess)
            return bail(fail(c, ECMC_E_DEVICE, "creating the second stream failed"));
    }

    HostState hs;
    hs.px.resize(n_beads);
    hs.py.resize(n_beads);
    hs.pz.resize(n_beads);
    hs.cx.resize(n_beads);
    hs.cy.resize(n_beads);
    hs.cz.resize(n_beads);
    hs.img.assign(3 * n_beads, 0);
    for (int64_t i = 0; i < n_beads; ++i) {
        double w[3];
        for (int a = 0; a < 3; ++a) {
            const double v = positions[3 * i + a];
            if (!std::isfinite(v)) return bail(fail(c, ECMC_E_ARG, "position %lld is not finite", (long long)i));
            w[a] = wrap_coord(v, box);
        }
        hs.px[i] = w[0];
        hs.py[i] = w[1];
        hs.pz[i] = w[2];
        hs.cx[i] = bin_coord(w[0], c->g.n, c->g.h, box);
        hs.cy[i] = bin_coord(w[1], c->g.n, c->g.h, box);
        hs.cz[i] = bin_coord(w[2], c->g.n, c->g.h, box);
    }
    if ((st = build_topology(c, n_beads, n_bonds, bonds, hs))) return bail(st);
    if ((st = build_cells(c, hs, true))) return bail(st);
    if ((st = upload(c, hs, true))) return bail(st);
    *out = c;
    return ECMC_OK;
}

ecmc_status ecmc_sweep_colours(ecmc_ctx *c, int64_t n_chains, double ell, uint64_t seed, uint32_t colour_mask) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    if (n_chains < 0 || !std::isfinite(ell) || !(ell >= 0)) return fail(c, ECMC_E_ARG, "need n_chains >= 0, ell >= 0");
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
    a.slow = c->dev<double>(c->lay.slow);
    a.slow_lock = c->dev<uint32_t>(c->lay.slow_lock);
    a.nslow = c->g.nslow;
    a.slow_cap = c->g.nslow > 0 ? c->g.slow_cap : 0;
    a.cnt = c->dev<unsigned long long>(c->lay.cnt);
    a.sum_delta = c->dev<double>(c->lay.dsum);
    a.err = c->dev<unsigned int>(c->lay.err);
    a.log = c->opt.event_log_capacity > 0 ? c->dev<ecmc_event>(c->lay.log) : nullptr;
    a.log_n = c->dev<unsigned long long>(c->lay.log_n);
    a.log_cap = c->opt.event_log_capacity;
    a.L = c->L;
    a.h = c->g.h;
    a.sig2 = c->sig2;
    a.b2 = c->b2;
    a.ell = ell;
    a.event_cap = c->opt.event_cap;
    a.n = c->g.n;
    a.D = c->g.D;
    a.nd = c->g.nd;
    a.cap = c->cap;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.sweep = c->sweep_ctr;
    a.exact_search = c->opt.precision == ECMC_PREC_FP64 ? 1 : 0;
    a.swap = c->opt.swap_moves ? 1 : 0;
    a.halfL = 0.5 * c->L;
    {
        // Single-precision screen (see screen() in the kernels).  Screening coordinates are frame
        // coordinates rounded once to float, so every float displacement is within
        // delta = 6 u X of the FP64 one (u = 2^-24, X the largest coordinate or displacement:
        // the frame edge, or L for the whole box).  For |d_perp| <= b the float d_perp^2 is
        // then within m = 4 b delta + 2 delta^2 + 8 u b^2 of the FP64 value, the argument of
        // the square root within m + 4 u b^2, the square root within the square root of that
        // (the ill-conditioned grazing case), and the estimate of x within
        // delta + sqrt(m + 4 u b^2) + 4 u b + u (X + b).  The interval half-width is twice that.
        const double u = std::ldexp(1.0, -24);
        const double bm = std::max(c->sigma, c->lmax);
        const bool whole = c->opt.tiling == ECMC_TILING_WHOLE;
        const double X = whole ? c->L : (c->g.D + 2) * c->g.h;
        const double delta = 6.0 * u * X + 1e-12 * c->L;
        const double m = 4.0 * bm * delta + 2.0 * delta * delta + 8.0 * u * bm * bm;
        const double err = 2.0 * (delta + std::sqrt(m + 4.0 * u * bm * bm) + 4.0 * u * bm + u * (X + bm));
        const float inf = __builtin_huge_valf();
        a.p_sure = std::nextafter((float)delta, inf);
        a.in_lo = std::nextafter((float)(c->sig2 - m), 0.0f);
        a.in_hi = std::nextafter((float)(c->sig2 + m), inf);
        a.err_f = std::nextafter((float)err, inf);
        a.sig2f = (float)c->sig2;
        a.b2f = (float)c->b2;
    }
    const bool log = c->opt.event_log_capacity > 0;
    auto launch = [&](int grid) -> ecmc_status {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->opt.time_kernels) {
            HIP_OK(c, hipEventCreate(&e0));
            HIP_OK(c, hipEventCreate(&e1));
            HIP_OK(c, hipEventRecord(e0, c->stream));
        }
        // every domain's bead count first, on the main stream: the tier launches pick their
        // domains by it and never recount (a count taken while another tier rewrites a
        // domain's cell lists could be half-updated and claim that domain twice)
        HIP_OK(c, launch_count(a, grid, c->stream));
        // the tiers take disjoint sets of domains of one colour, which never interact: the
        // larger (rarer) tiers run on a second stream concurrently with the first
        if (c->g.bpl2) {
            HIP_OK(c, hipEventRecord(c->fork, c->stream));
            HIP_OK(c, hipStreamWaitEvent(c->side, c->fork, 0));
            PhaseArgs b = a;
            b.stage_lo = 64 * c->g.bpl;
            b.stage_hi = c->g.bpl3 ? 64 * c->g.bpl2 : 0x7fffffff;
            HIP_OK(c, launch_phase(b, c->g.bpl2, log, grid, c->side));
            if (c->g.bpl3) {
                b.stage_lo = 64 * c->g.bpl2;
                b.stage_hi = 0x7fffffff;
                HIP_OK(c, launch_phase(b, c->g.bpl3, log, grid, c->side));
            }
            HIP_OK(c, hipEventRecord(c->join, c->side));
        }
        a.stage_lo = 0;
        a.stage_hi = c->g.bpl2 ? 64 * c->g.bpl : 0x7fffffff;
        HIP_OK(c, launch_phase(a, c->g.bpl, log, grid, c->stream));
        if (c->g.bpl2) HIP_OK(c, hipStreamWaitEvent(c->stream, c->join, 0));
        if (c->opt.time_kernels) {
            HIP_OK(c, hipEventRecord(e1, c->stream));
            c->timing.emplace_back(e0, e1);
        }
        return ECMC_OK;
    };
    ecmc_status st = ECMC_OK;
    if (c->opt.tiling == ECMC_TILING_WHOLE) {
        a.whole = 1;
        a.K = n_chains;
        a.colour = 0;
        if (n_chains > 0 && (colour_mask & 1u)) st = launch(1);
    } else {
        a.whole = 0;
        const int64_t nd = c->g.nd;
        const int64_t ndom = nd * nd * nd;
        a.K = (n_chains + ndom - 1) / ndom;
        uint32_t ctr[4] = {0u, 0u, c->sweep_ctr, 1u};
        philox4x32_10(ctr, a.key0, a.key1);
        for (int ax = 0; ax < 3; ++ax) a.off[ax] = (int)scale_u32(ctr[ax], (uint32_t)c->g.D);
        const int grid = (int)((nd / 2) * (nd / 2) * (nd / 2));
        if (c->g.sweep && (colour_mask & 0xFFu) == 0xFFu) {
            // all eight colours in one dependency-ordered launch
            if (a.K > 0) {
                if (++c->epoch == 0) ++c->epoch;
                a.epoch = c->epoch;
                a.ndpc = grid;
                hipEvent_t e0 = nullptr, e1 = nullptr;
                if (c->opt.time_kernels) {
                    HIP_OK(c, hipEventCreate(&e0));
                    HIP_OK(c, hipEventCreate(&e1));
                    HIP_OK(c, hipEventRecord(e0, c->stream));
                }
                int waves = 0;
                HIP_OK(c, launch_sweep(a, c->g.bpl, log, &waves, c->stream));
                if (c->opt.time_kernels) {
                    HIP_OK(c, hipEventRecord(e1, c->stream));
                    c->timing.emplace_back(e0, e1);
                }
            }
        } else {
            for (int colour = 0; colour < 8 && st == ECMC_OK && a.K > 0; ++colour) {
                if (!((colour_mask >> colour) & 1u)) continue;
                a.colour = colour;
                st = launch(grid);
            }
        }
    }
    c->sweep_ctr++;
    return st;
}

ecmc_status ecmc_sweep(ecmc_ctx *c, int64_t n_chains, double ell, uint64_t seed) {
    return ecmc_sweep_colours(c, n_chains, ell, seed, 0xFFu);
}

ecmc_status ecmc_synchronize(ecmc_ctx *c) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    return check_device(c);
}

ecmc_status ecmc_observables(ecmc_ctx *c, int32_t nbins, double *r2, double *rg2, int64_t *hist, double *mid,
                             int64_t *n_poly) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    if (nbins <= 0 || nbins > MAX_BINS) return fail(c, ECMC_E_ARG, "nbins must be in [1, %d]", MAX_BINS);
    if (n_poly) *n_poly = c->npoly;
    HIP_OK(c, hipMemsetAsync(c->ws + c->lay.hist, 0, 8 * nbins, c->stream));
    ObsArgs o{};
    o.px = c->dev<double>(c->lay.px);
    o.py = c->dev<double>(c->lay.py);
    o.pz = c->dev<double>(c->lay.pz);
    o.img = c->dev<int32_t>(c->lay.img);
    o.porder = c->dev<int32_t>(c->lay.porder);
    o.pstart = c->dev<int32_t>(c->lay.pstart);
    o.npoly = c->npoly;
    o.L = c->L;
    o.halfL = 0.5 * c->L;
    o.sigma = c->sigma;
    o.bmax = c->lmax;
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

ecmc_status ecmc_shape(ecmc_ctx *c, double *gyr, double *eig, double *com, int64_t *n_poly) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    if (n_poly) *n_poly = c->npoly;
    ObsArgs o{};
    o.px = c->dev<double>(c->lay.px);
    o.py = c->dev<double>(c->lay.py);
    o.pz = c->dev<double>(c->lay.pz);
    o.img = c->dev<int32_t>(c->lay.img);
    o.porder = c->dev<int32_t>(c->lay.porder);
    o.pstart = c->dev<int32_t>(c->lay.pstart);
    o.npoly = c->npoly;
    o.L = c->L;
    o.halfL = 0.5 * c->L;
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

ecmc_status ecmc_get_event_log(ecmc_ctx *c, ecmc_event *out, int64_t capacity, int64_t *n_total) {
    if (!c) return fail(nullptr, ECMC_E_ARG, "null context");
    HIP_OK(c, hipStreamSynchronize(c->stream));
    unsigned long long n = 0;
    HIP_OK(c, hipMemcpy(&n, c->ws + c->lay.log_n, 8, hipMemcpyDeviceToHost));
    if (n_total) *n_total = (int64_t)n;
    const int64_t have = std::min<int64_t>((int64_t)n, c->opt.event_log_capacity);
    const int64_t take = std::min<int64_t>(have, capacity);
    if (out && take > 0)
        HIP_OK(c, hipMemcpy(out, c->ws + c->lay.log, sizeof(ecmc_event) * take, hipMemcpyDeviceToHost));
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
    const int n = c->g.n;
    const double h = c->g.h, L = c->L;
    hs.px.resize(nb);
    hs.py.resize(nb);
    hs.pz.resize(nb);
    hs.cx.resize(nb);
    hs.cy.resize(nb);
    hs.cz.resize(nb);
    hs.img.assign(images, images + 3 * nb);
    auto bnd = [&](int k) { return k < n ? (double)k * h : L; };
    for (int64_t i = 0; i < nb; ++i) {
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
    ecmc_status st = build_cells(c, hs, false);
    if (st) return st;
    if ((st = upload(c, hs, false))) return st;
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

uint32_t ecmc_sweep_counter(const ecmc_ctx *c) { return c ? c->sweep_ctr : 0; }
int32_t ecmc_n_cells(const ecmc_ctx *c) { return c ? c->g.n : 0; }
double ecmc_cell_size(const ecmc_ctx *c) { return c ? c->g.h : 0.0; }
int32_t ecmc_stage_capacity(const ecmc_ctx *c) {
    return c ? 64 * (c->g.bpl3 ? c->g.bpl3 : (c->g.bpl2 ? c->g.bpl2 : c->g.bpl)) : 0;
}

void ecmc_destroy(ecmc_ctx *c) {
    if (!c) return;
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamDestroy(c->side);
    }
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

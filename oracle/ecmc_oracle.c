/*
 * TEST INFRASTRUCTURE ONLY — serial FP64 CPU oracle for the event-chain move of
 * tethered hard-sphere polymer melts (Kampmann, Boltz, Kierfeld, arXiv:1502.06447).
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math): IEEE binary64,
 * round to nearest, no fused multiply-add, correctly rounded sqrt.
 *
 * Model (Sec. II): hard spheres of diameter sigma between ALL bead pairs (Eq. (1)),
 * bonded neighbours joined by tethers of maximal length b_max (the tether variant
 * stated after Eq. (2)) or, optionally, by harmonic springs (k/2)(b - sigma)^2 (Eq. (2)),
 * periodic cube of edge L.
 *
 * EC move (Sec. II, steps 1-4, and the generalisation to several interaction
 * partners that follows them): a pivot bead and a direction v = s e_a are drawn,
 * x_max = ell; the pivot advances by the smallest admissible displacement
 * x = min_i x_i over its partners i (all hard spheres, plus its tethered
 * neighbours), the EC continues at the argmin bead, x_max -= x, until x_max is used.
 *
 * Parallel decomposition (Sec. II.A): space is cut into domains that are redrawn
 * every sweep; beads outside the active domain are immotile, an EC that would
 * leave the domain or hand the displacement to an immotile bead is reflected.
 *
 * Readings of points the paper leaves open (each listed in the design notes):
 *  - cells of edge h = L/n > b_max (n >= 4); membership is the stored cell index,
 *    intervals are closed [bnd(c), bnd(c+1)], bnd(k) = k*h (k < n), bnd(n) = L;
 *  - the pivot reaching a cell face is a bookkeeping event: its coordinate is set to
 *    the face value (not accumulated), and the EC goes on with the same pivot;
 *  - domains: D^3 blocks of cells, integer offset per axis drawn per sweep, eight
 *    colours by domain-index parity, run in colour order 0..7; or (tile-joint, Sec. II.A)
 *    D^3-cell tiles at pitch D + 1, the cell after each tile along every axis a joint that no
 *    tile moves, offset in [0, D + 1), all tiles in one phase;
 *  - reflection at an immotile bead and at a wall reverses v (s -> -s);
 *  - ties: END before interaction before cell face; interactions ordered by
 *    (x, bead id, hard sphere before tether);
 *  - negative x from rounding is clamped to 0;
 *  - after two reflections of one EC with only lifts and cell crossings between them
 *    (displacement W between them), the EC retraces its path between the two fixed stops
 *    for ever (a reflection reverses the chain of events exactly), so it is periodic
 *    with period 2W: x_max is reduced to fmod(x_max, 2W) and the EC goes on; W = 0
 *    means nothing can move and ends the EC;
 *  - a run of zero-length events that returns to the same (pivot, direction, pivot cell)
 *    repeats forever with nothing moving; it is detected (Brent's cycle search over the
 *    run) and ends the EC;
 *  - random numbers: Philox4x32-10 keyed by the 64-bit seed; EC draws use counter
 *    (k, domain, sweep, 2 m), the partition offsets use (0, 0, sweep, 2 m + 1), with the
 *    stream index m = 0 unless set (m numbers a melt of a batch run side by side);
 *  - swap moves (Sec. II.C, optional): proposed at every hard-sphere contact with a motile
 *    bead; accepted iff all tethers of both beads are within b_max after the exchange
 *    (squared minimum-image lengths, summed over x, y, z, compared with b_max^2);
 *  - springs (optional, Eq. (2) with the EC rule for pair potentials of Sec. II): at every
 *    step each bond of the pivot gets a fresh energy dE = -ln u, u uniform in (0, 1] (by the
 *    memorylessness of the exponential law this equals one draw per event); the bond is also
 *    capped at b_max, a tether, so that every partner lies within one cell.  The draws of step
 *    j of EC k use the counter (j, k, domain, sweep) under a second key, words 0-1 of the
 *    draw at counter (2^32-1, 2^32-1, m, 0x53505247) under the seed's key; partner slot t
 *    takes words 2t (low 21 bits dropped) and 2t+1.  A spring EC does not retrace its path
 *    after a reflection, so the periodic reduction is off; swap moves are not combined with
 *    springs;
 *  - push-off (Sec. II.B, optional): hard spheres of a working diameter d <= sigma; a pair is
 *    overlapping when its squared distance is below d^2 (1 - 1e-9) (the margin keeps pairs left
 *    in contact by an earlier event, up to rounding, as obstacles); an overlapping pair is no
 *    hard-sphere event for either bead, and every EC starts from a motile bead that overlaps
 *    some bead (the k-th draw picks among them in ascending id; a domain with none runs no
 *    EC).  The periodic reduction stays on: the push-off prepares a start and samples
 *    nothing, and without it a bead caught between two immotile contacts with a gap of
 *    rounding size bounces for ever; where a pair that stopped overlapping changes the way
 *    back, it merely shortens that EC.
 */
#include "ecmc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_DEFAULT_EVENT_CAP 10000000LL

struct orc_sys {
    int64_t nb;        /* beads */
    double L, sigma, bmax, sig2, b2, h, halfL;
    int n;             /* cells per axis */
    double *bnd;       /* n+1 face coordinates */
    double *r;         /* [nb][3] positions in [0, L] */
    int32_t *cell;     /* [nb][3] stored cell of each bead */
    int32_t *img;      /* [nb][3] periodic image counters */
    int32_t *nbr;      /* [nb][2] tethered partners (-1 = none) */
    int32_t *ccount;   /* [n^3] beads per cell */
    int32_t *cap;      /* [n^3] allocated slots per cell */
    int32_t **clist;   /* [n^3] bead ids per cell */
    uint32_t sweep_ctr;
    int64_t event_cap;
    int check;
    int swap;          /* swap moves at hard-sphere contacts (Sec. II.C) */
    int spring;        /* bonds are harmonic springs capped at b_max (Eq. (2)) */
    int push;          /* push-off: overlapping pairs ignored, ECs start at overlapping beads */
    int no_skip;       /* 1: the plain loop of Sec. II steps 1-4, whole periods never dropped */
    double ov2;        /* squared overlap distance of the push-off: d^2 (1 - 1e-9) */
    double spring_k, two_over_k;
    uint32_t stream;   /* random stream index m (counter word 3 = 2 m, 2 m + 1) */
    orc_event *log;
    int64_t log_cap, log_n;
    uint64_t cnt[ORC_NCNT];
    double sum_delta;
    /* polymer order for observables */
    int64_t npoly;
    int64_t *pstart; /* [npoly+1] */
    int32_t *porder; /* [nb] */
};

/* ---------------------------------------------------------------- Philox */
/* Philox4x32 with 10 rounds: each round multiplies counter words 0 and 2 by the
 * two round constants, and xors the high halves with the other words and the key;
 * the key is bumped by the two Weyl constants between rounds. */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof c);
}

/* uniform integer in [0, m) from a 32-bit word */
static uint32_t below(uint32_t u, uint32_t m) { return (uint32_t)(((uint64_t)u * m) >> 32); }

/* ---------------------------------------------------------------- helpers */
static int cidx(const orc_sys *s, int cx, int cy, int cz) { return cx + s->n * (cy + s->n * cz); }

static int cell_add(orc_sys *s, int c, int32_t id) {
    if (s->ccount[c] == s->cap[c]) {
        int nc = s->cap[c] ? 2 * s->cap[c] : 8;
        int32_t *p = (int32_t *)realloc(s->clist[c], sizeof(int32_t) * (size_t)nc);
        if (!p) return ORC_E_ARG;
        s->clist[c] = p;
        s->cap[c] = nc;
    }
    s->clist[c][s->ccount[c]++] = id;
    return ORC_OK;
}

static void cell_remove(orc_sys *s, int c, int32_t id) {
    for (int i = 0; i < s->ccount[c]; ++i) {
        if (s->clist[c][i] == id) {
            s->clist[c][i] = s->clist[c][s->ccount[c] - 1];
            s->ccount[c]--;
            return;
        }
    }
}

static double wrap_coord(double v, double L) {
    double w = fmod(v, L);
    if (w < 0) w = w + L;
    if (!(w < L)) w = 0.0;
    return w;
}

static int bin_coord(const orc_sys *s, double w) {
    int c = (int)floor(w / s->h);
    if (c < 0) c = 0;
    if (c > s->n - 1) c = s->n - 1;
    while (c > 0 && w < s->bnd[c]) c--;
    while (c < s->n - 1 && w > s->bnd[c + 1]) c++;
    return c;
}

static double mi(const orc_sys *s, double d) {
    if (d > s->halfL) return d - s->L;
    if (d < -s->halfL) return d + s->L;
    return d;
}

static void free_sys(orc_sys *s) {
    if (!s) return;
    if (s->clist) {
        for (int64_t c = 0; c < (int64_t)s->n * s->n * s->n; ++c) free(s->clist[c]);
    }
    free(s->clist);
    free(s->cap);
    free(s->ccount);
    free(s->bnd);
    free(s->r);
    free(s->cell);
    free(s->img);
    free(s->nbr);
    free(s->pstart);
    free(s->porder);
    free(s);
}

void orc_destroy(orc_sys *s) { free_sys(s); }

static int rebuild_cells(orc_sys *s) {
    const int64_t nc = (int64_t)s->n * s->n * s->n;
    for (int64_t c = 0; c < nc; ++c) s->ccount[c] = 0;
    for (int64_t i = 0; i < s->nb; ++i) {
        const int32_t *ci = s->cell + 3 * i;
        if (cell_add(s, cidx(s, ci[0], ci[1], ci[2]), (int32_t)i)) return ORC_E_ARG;
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------- create */
static int create_impl(orc_sys **out, double L, double sigma, double bmax, int n_cells, int64_t n_beads,
                       const double *pos, int64_t n_bonds, const int32_t *bonds, int check_overlaps) {
    *out = NULL;
    if (!(isfinite(L) && L > 0 && isfinite(sigma) && sigma > 0 && isfinite(bmax) && bmax >= sigma))
        return ORC_E_ARG;
    if (n_beads < 1 || n_beads > 0x7fffffffLL || !pos || n_bonds < 0 || (n_bonds > 0 && !bonds))
        return ORC_E_ARG;
    int n = n_cells;
    if (n == 0) {
        n = (int)floor(L / bmax);
        while (n > 0 && !(L / n > bmax)) n--;
    }
    if (n < 4 || n > 1023 || !(L / n > bmax)) return ORC_E_BOX;

    orc_sys *s = (orc_sys *)calloc(1, sizeof *s);
    if (!s) return ORC_E_ARG;
    s->nb = n_beads;
    s->L = L;
    s->sigma = sigma;
    s->bmax = bmax;
    s->sig2 = sigma * sigma;
    s->b2 = bmax * bmax;
    s->n = n;
    s->h = L / n;
    s->halfL = 0.5 * L;
    s->event_cap = ORC_DEFAULT_EVENT_CAP;
    s->bnd = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    s->r = (double *)malloc(sizeof(double) * 3 * (size_t)n_beads);
    s->cell = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)n_beads);
    s->img = (int32_t *)calloc(3 * (size_t)n_beads, sizeof(int32_t));
    s->nbr = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)n_beads);
    const int64_t nc = (int64_t)n * n * n;
    s->ccount = (int32_t *)calloc((size_t)nc, sizeof(int32_t));
    s->cap = (int32_t *)calloc((size_t)nc, sizeof(int32_t));
    s->clist = (int32_t **)calloc((size_t)nc, sizeof(int32_t *));
    s->pstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_beads + 1));
    s->porder = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_beads);
    if (!s->bnd || !s->r || !s->cell || !s->img || !s->nbr || !s->ccount || !s->cap || !s->clist ||
        !s->pstart || !s->porder) {
        free_sys(s);
        return ORC_E_ARG;
    }
    for (int k = 0; k < n; ++k) s->bnd[k] = (double)k * s->h;
    s->bnd[n] = L;

    /* positions: wrapped into [0, L), binned into closed cells */
    for (int64_t i = 0; i < n_beads; ++i) {
        for (int a = 0; a < 3; ++a) {
            const double v = pos[3 * i + a];
            if (!isfinite(v)) {
                free_sys(s);
                return ORC_E_ARG;
            }
            const double w = wrap_coord(v, L);
            s->r[3 * i + a] = w;
            s->cell[3 * i + a] = bin_coord(s, w);
        }
    }
    /* bonds: linear chains only (degree <= 2, no cycles, no duplicates) */
    for (int64_t i = 0; i < 2 * n_beads; ++i) s->nbr[i] = -1;
    for (int64_t b = 0; b < n_bonds; ++b) {
        const int32_t i = bonds[2 * b], j = bonds[2 * b + 1];
        if (i < 0 || j < 0 || i >= n_beads || j >= n_beads || i == j) {
            free_sys(s);
            return ORC_E_ARG;
        }
        if (s->nbr[2 * i] == j || s->nbr[2 * i + 1] == j) {
            free_sys(s);
            return ORC_E_ARG;
        }
        int32_t *pi = s->nbr[2 * i] < 0 ? &s->nbr[2 * i] : (s->nbr[2 * i + 1] < 0 ? &s->nbr[2 * i + 1] : NULL);
        int32_t *pj = s->nbr[2 * j] < 0 ? &s->nbr[2 * j] : (s->nbr[2 * j + 1] < 0 ? &s->nbr[2 * j + 1] : NULL);
        if (!pi || !pj) {
            free_sys(s);
            return ORC_E_ARG;
        }
        *pi = j;
        *pj = i;
    }
    /* polymer order: walk each chain from its smaller-id end */
    {
        char *seen = (char *)calloc((size_t)n_beads, 1);
        int64_t k = 0, np = 0;
        for (int64_t i = 0; i < n_beads; ++i) {
            const int deg = (s->nbr[2 * i] >= 0) + (s->nbr[2 * i + 1] >= 0);
            if (seen[i] || deg > 1) continue;
            s->pstart[np++] = k;
            int32_t prev = -1, cur = (int32_t)i;
            while (cur >= 0) {
                seen[cur] = 1;
                s->porder[k++] = cur;
                int32_t nx = s->nbr[2 * cur] != prev ? s->nbr[2 * cur] : s->nbr[2 * cur + 1];
                if (nx == prev) nx = -1;
                prev = cur;
                cur = nx;
            }
        }
        s->pstart[np] = k;
        s->npoly = np;
        free(seen);
        if (k != n_beads) { /* a ring */
            free_sys(s);
            return ORC_E_ARG;
        }
    }
    if (rebuild_cells(s)) {
        free_sys(s);
        return ORC_E_ARG;
    }
    /* hard-sphere and tether validity of the start (all pairs via the cell list) */
    const double lim_ov = s->sig2 * (1.0 - 2e-12);
    for (int64_t i = 0; i < n_beads; ++i) {
        const int32_t *ci = s->cell + 3 * i;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int c = cidx(s, (ci[0] + dx + n) % n, (ci[1] + dy + n) % n, (ci[2] + dz + n) % n);
                    for (int t = 0; t < s->ccount[c]; ++t) {
                        const int32_t j = s->clist[c][t];
                        if (j <= i) continue;
                        double d2 = 0;
                        for (int a = 0; a < 3; ++a) {
                            const double d = mi(s, s->r[3 * j + a] - s->r[3 * i + a]);
                            d2 += d * d;
                        }
                        if (check_overlaps && d2 < lim_ov) {
                            free_sys(s);
                            return ORC_E_OVERLAP;
                        }
                    }
                }
        for (int t = 0; t < 2; ++t) {
            const int32_t j = s->nbr[2 * i + t];
            if (j < 0) continue;
            double d2 = 0;
            for (int a = 0; a < 3; ++a) {
                const double d = mi(s, s->r[3 * j + a] - s->r[3 * i + a]);
                d2 += d * d;
            }
            if (d2 > s->b2 * (1.0 + 2e-12)) {
                free_sys(s);
                return ORC_E_TETHER;
            }
        }
    }
    *out = s;
    return ORC_OK;
}

int orc_create(orc_sys **out, double L, double sigma, double bmax, int n_cells, int64_t n_beads,
               const double *pos, int64_t n_bonds, const int32_t *bonds) {
    return create_impl(out, L, sigma, bmax, n_cells, n_beads, pos, n_bonds, bonds, 1);
}

int orc_create_overlapping(orc_sys **out, double L, double sigma, double bmax, int n_cells, int64_t n_beads,
                           const double *pos, int64_t n_bonds, const int32_t *bonds) {
    return create_impl(out, L, sigma, bmax, n_cells, n_beads, pos, n_bonds, bonds, 0);
}

int orc_set_pushoff(orc_sys *s, double d) {
    if (d == 0.0) {
        s->push = 0;
        s->sig2 = s->sigma * s->sigma;
        return ORC_OK;
    }
    if (!(d > 0.0) || !(d <= s->sigma) || s->spring || s->swap) return ORC_E_ARG;
    s->push = 1;
    s->sig2 = d * d;
    s->ov2 = s->sig2 * (1.0 - 1e-9);
    return ORC_OK;
}

int orc_set_options(orc_sys *s, int64_t event_cap, int check) {
    s->event_cap = event_cap > 0 ? event_cap : ORC_DEFAULT_EVENT_CAP;
    s->check = check;
    return ORC_OK;
}

int orc_set_swap(orc_sys *s, int on) {
    if (on && (s->spring || s->push)) return ORC_E_ARG;
    s->swap = on ? 1 : 0;
    return ORC_OK;
}

/* The periodic reduction on (1, the default) or off (0).  Off, every EC is the plain loop of
 * Sec. II steps 1-4: it runs until x_max is used up (or the zero-length cycle search or the
 * event cap ends it), bouncing between its two stops as often as the length requires. */
int orc_set_periodic_skip(orc_sys *s, int on) {
    s->no_skip = on ? 0 : 1;
    return ORC_OK;
}

int orc_set_spring(orc_sys *s, double k) {
    if (!(k >= 0.0) || !isfinite(k) || (k > 0.0 && (s->swap || s->push))) return ORC_E_ARG;
    s->spring = k > 0.0;
    s->spring_k = k;
    s->two_over_k = k > 0.0 ? 2.0 / k : 0.0;
    return ORC_OK;
}

int orc_set_stream(orc_sys *s, uint32_t m) {
    if (m > 0x7FFFFFFFu) return ORC_E_ARG;
    s->stream = m;
    return ORC_OK;
}

int orc_set_log(orc_sys *s, orc_event *buf, int64_t cap) {
    s->log = buf;
    s->log_cap = buf ? cap : 0;
    s->log_n = 0;
    return ORC_OK;
}

int64_t orc_log_count(const orc_sys *s) { return s->log_n; }

/* ---------------------------------------------------------------- domains */
typedef struct {
    int tiled;      /* 0: whole box, every bead motile, no walls */
    int D;          /* cells per domain edge */
    int P;          /* domain pitch: D (checkerboard) or D + 1 (tile-joint: a joint cell after each tile) */
    int off[3];     /* partition offset (cells) */
    int dom[3];     /* active domain coordinates */
    uint32_t sweep, domain, colour, ec;
    uint32_t skey[2]; /* key of the spring energy draws */
} orc_dom;

static int dom_coord(const orc_sys *s, const orc_dom *dm, int c, int a) {
    return ((c - dm->off[a]) % s->n + s->n) % s->n / dm->P;
}

/* a cell is in the active domain when it lies in the domain's pitch block and, with tile-joint,
 * not in the joint cell that ends the block */
static int cell_in_domain(const orc_sys *s, const orc_dom *dm, const int32_t c[3]) {
    if (!dm->tiled) return 1;
    for (int a = 0; a < 3; ++a) {
        if (dom_coord(s, dm, c[a], a) != dm->dom[a]) return 0;
        if (((c[a] - dm->off[a]) % s->n + s->n) % s->n % dm->P >= dm->D) return 0;
    }
    return 1;
}

static void log_event(orc_sys *s, const orc_dom *dm, uint32_t step, int32_t p, int32_t j, int kind) {
    if (s->log && s->log_n < s->log_cap) {
        orc_event *e = &s->log[s->log_n];
        e->sweep = dm->sweep;
        e->domain = dm->domain;
        e->ec = dm->ec;
        e->step = step;
        e->pivot = p;
        e->target = j;
        e->kind = (uint32_t)kind;
        e->colour = dm->colour;
    }
    s->log_n++;
}

/* ---------------------------------------------------------------- candidates */
/* Displacement of bead j seen from pivot p, with the periodic shift w[a] in {-1,0,1}
 * (neighbour cell index wrapped below 0 / above n-1) added after the subtraction.
 * Returns the component along v (d_par) and the squared distance from the line of
 * motion (d_perp2). */
static void geom(const orc_sys *s, int32_t p, int32_t j, const int w[3], int axis, int sgn,
                 double *dpar, double *dperp2) {
    double d[3];
    for (int a = 0; a < 3; ++a) {
        d[a] = s->r[3 * j + a] - s->r[3 * p + a];
        if (w[a] > 0) d[a] = d[a] + s->L;
        if (w[a] < 0) d[a] = d[a] - s->L;
    }
    const int b = axis == 0 ? 1 : 0;
    const int c = axis == 2 ? 1 : 2;
    *dpar = sgn > 0 ? d[axis] : -d[axis];
    const double pb = d[b] * d[b];
    const double pc = d[c] * d[c];
    *dperp2 = pb + pc;
}

/* Hard-sphere candidate (Eq. (1)): the pivot moving along v first touches bead j
 * after x = d_par - sqrt(sigma^2 - d_perp^2), if j lies ahead and within sigma of
 * the line of motion.  Returns 0 if j is never hit. */
static int hs_candidate(const orc_sys *s, double dpar, double dperp2, double *x) {
    if (!(dpar > 0.0 && dperp2 < s->sig2)) return 0;
    if (s->push && dpar * dpar + dperp2 < s->ov2) return 0; /* push-off: an overlapping pair */
    double v = dpar - sqrt(s->sig2 - dperp2);
    if (!(v > 0.0)) v = 0.0;
    *x = v;
    return 1;
}

/* Tether candidate: the bond reaches b_max after x = d_par + sqrt(b^2 - d_perp^2)
 * (from |d - x v|^2 = b^2, the root on the far side). */
static double tether_candidate(const orc_sys *s, double dpar, double dperp2) {
    double t = s->b2 - dperp2;
    if (!(t > 0.0)) t = 0.0;
    double v = dpar + sqrt(t);
    if (!(v > 0.0)) v = 0.0;
    return v;
}

/* Natural logarithm of a finite u > 0, written out so that its bits can be reproduced
 * elsewhere from the same steps: u = f 2^e with f in [sqrt(1/2), sqrt(2)); with
 * z = (f - 1)/(f + 1), ln f = 2 artanh z = 2 z (1 + z^2/3 + z^4/5 + ... + z^22/23), the
 * bracket by Horner's rule (|z| <= 0.1716, so the first term left out is below 2^-60 of
 * it); ln u = e ln 2 + ln f. */
double orc_ln(double u) {
    int e;
    double f = frexp(u, &e); /* u = f 2^e, f in [1/2, 1) */
    if (f < 0.70710678118654752440) {
        f = f + f;
        e = e - 1;
    }
    const double z = (f - 1.0) / (f + 1.0);
    const double z2 = z * z;
    double sum = 1.0 / 23.0;
    for (int n = 10; n >= 0; --n) sum = 1.0 / (double)(2 * n + 1) + z2 * sum;
    return (double)e * 0.69314718055994530942 + (z + z) * sum;
}

/* The two energies of one step (one per bond slot of the pivot), as dE * 2/k. */
static void spring_terms(const orc_sys *s, const orc_dom *dm, uint32_t step, double g[2]) {
    const uint32_t ctr[4] = {step, dm->ec, dm->domain, dm->sweep};
    uint32_t w[4];
    orc_philox4x32_10(ctr, dm->skey, w);
    for (int t = 0; t < 2; ++t) {
        const uint64_t bits = ((uint64_t)w[2 * t + 1] << 21) | (uint64_t)(w[2 * t] >> 11);
        const double u = (double)(bits + 1u) * 0x1p-53; /* in (0, 1] */
        g[t] = -orc_ln(u) * s->two_over_k;
    }
}

/* Bond candidate.  Tether: as above.  Spring (Eq. (2)): along the path the bond first
 * shortens (no energy needed) until the pivot passes the partner's foot on its line, then
 * lengthens.  From the shortest length still ahead, b0 = d_perp if d_par > 0, else the
 * present length, the drawn energy is used up where (k/2)(b - sigma)^2 has grown by dE:
 * b_end = sigma + sqrt((b0 - sigma)^2 + 2 dE/k), capped at b_max, reached after
 * x = d_par + sqrt(b_end^2 - d_perp^2).  g = 2 dE / k; g < 0 selects the tether. */
double orc_bond_x(const orc_sys *s, double dpar, double dperp2, double g) {
    if (!(g >= 0.0)) return tether_candidate(s, dpar, dperp2);
    const double b0 = sqrt(dpar > 0.0 ? dperp2 : dpar * dpar + dperp2);
    const double e = b0 - s->sigma;
    const double be = s->sigma + sqrt(e * e + g);
    double be2 = be * be;
    if (be2 > s->b2) be2 = s->b2;
    double q = be2 - dperp2;
    if (!(q > 0.0)) q = 0.0;
    double x = dpar + sqrt(q);
    if (!(x > 0.0)) x = 0.0;
    return x;
}

typedef struct {
    double x;
    int32_t j;
    int kind;
    double dpar;
} orc_best;

static void consider(orc_best *b, double x, int32_t j, int kind, double dpar) {
    if (x < b->x || (x == b->x && (j < b->j || (j == b->j && kind < b->kind)))) {
        b->x = x;
        b->j = j;
        b->kind = kind;
        b->dpar = dpar;
    }
}

/* Minimum over all interaction partners of the pivot (Sec. II): every bead in the 27
 * cells around the pivot's cell (hard spheres) and its tethered partners (tethers). */
static orc_best scan_partners(const orc_sys *s, int32_t p, int axis, int sgn, const double *g) {
    orc_best best = {INFINITY, 0x7fffffff, 0, 0.0};
    const int32_t *cp = s->cell + 3 * p;
    const int n = s->n;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int raw[3] = {cp[0] + dx, cp[1] + dy, cp[2] + dz};
                int w[3], cc[3];
                for (int a = 0; a < 3; ++a) {
                    w[a] = raw[a] < 0 ? -1 : (raw[a] >= n ? 1 : 0);
                    cc[a] = raw[a] - w[a] * n;
                }
                const int c = cidx(s, cc[0], cc[1], cc[2]);
                for (int t = 0; t < s->ccount[c]; ++t) {
                    const int32_t j = s->clist[c][t];
                    if (j == p) continue;
                    double dpar, dperp2, x;
                    geom(s, p, j, w, axis, sgn, &dpar, &dperp2);
                    if (hs_candidate(s, dpar, dperp2, &x)) consider(&best, x, j, 0, dpar);
                }
            }
    for (int t = 0; t < 2; ++t) {
        const int32_t q = s->nbr[2 * p + t];
        if (q < 0) continue;
        int w[3];
        for (int a = 0; a < 3; ++a) {
            /* the partner sits in a neighbouring cell: delta in {-1,0,1} modulo n */
            const int delta = ((s->cell[3 * q + a] - cp[a] + n + 1) % n) - 1;
            const int raw = cp[a] + delta;
            w[a] = raw < 0 ? -1 : (raw >= n ? 1 : 0);
        }
        double dpar, dperp2;
        geom(s, p, q, w, axis, sgn, &dpar, &dperp2);
        consider(&best, orc_bond_x(s, dpar, dperp2, g ? g[t] : -1.0), q, 1, dpar);
    }
    return best;
}

/* Brute force over every bead with the minimum-image convention (self-check). */
static orc_best brute_partners(const orc_sys *s, int32_t p, int axis, int sgn, const double *g) {
    orc_best best = {INFINITY, 0x7fffffff, 0, 0.0};
    for (int64_t j = 0; j < s->nb; ++j) {
        if (j == p) continue;
        double d[3];
        for (int a = 0; a < 3; ++a) d[a] = mi(s, s->r[3 * j + a] - s->r[3 * p + a]);
        const int b = axis == 0 ? 1 : 0, c = axis == 2 ? 1 : 2;
        const double dpar = sgn > 0 ? d[axis] : -d[axis];
        const double dperp2 = d[b] * d[b] + d[c] * d[c];
        double x;
        if (hs_candidate(s, dpar, dperp2, &x)) consider(&best, x, (int32_t)j, 0, dpar);
        for (int t = 0; t < 2; ++t)
            if (s->nbr[2 * p + t] == j) consider(&best, orc_bond_x(s, dpar, dperp2, g ? g[t] : -1.0), (int32_t)j, 1, dpar);
    }
    return best;
}

static double x_cell_of(const orc_sys *s, int32_t p, int axis, int sgn) {
    const int c = s->cell[3 * p + axis];
    const double ra = s->r[3 * p + axis];
    double xc = sgn > 0 ? s->bnd[c + 1] - ra : ra - s->bnd[c];
    if (!(xc > 0.0)) xc = 0.0;
    return xc;
}

int orc_next_event(const orc_sys *s, int32_t p, int axis, int sgn, double *x, int32_t *j,
                   int *kind, double *x_cell) {
    if (p < 0 || p >= s->nb || axis < 0 || axis > 2 || (sgn != 1 && sgn != -1)) return ORC_E_ARG;
    const orc_best b = scan_partners(s, p, axis, sgn, NULL);
    *x = b.x;
    *j = b.x < INFINITY ? b.j : -1;
    *kind = b.kind;
    *x_cell = x_cell_of(s, p, axis, sgn);
    return ORC_OK;
}

/* invariants after an event (test mode): the moved pivot overlaps nobody, its
 * tethers hold, and its coordinate lies in its stored cell */
static int check_pivot(const orc_sys *s, int32_t p) {
    const double tol = 1e-10;
    for (int64_t j = 0; j < s->nb; ++j) {
        if (j == p) continue;
        double d2 = 0;
        for (int a = 0; a < 3; ++a) {
            const double d = mi(s, s->r[3 * j + a] - s->r[3 * p + a]);
            d2 += d * d;
        }
        if (!s->push && d2 < s->sig2 * (1.0 - tol)) return ORC_E_CHECK;
        if ((s->nbr[2 * p] == j || s->nbr[2 * p + 1] == j) && d2 > s->b2 * (1.0 + tol)) return ORC_E_CHECK;
    }
    for (int a = 0; a < 3; ++a) {
        const int c = s->cell[3 * p + a];
        const double v = s->r[3 * p + a];
        if (v < s->bnd[c] - 1e-12 || v > s->bnd[c + 1] + 1e-12) return ORC_E_CHECK;
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------- swap move */
/* Squared minimum-image distance of two positions, summed over x, y, z in that order. */
static double dist2(const orc_sys *s, const double *u, const double *v) {
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double d = mi(s, u[a] - v[a]);
        d2 += d * d;
    }
    return d2;
}

/* Sec. II.C: at a hard-sphere contact the pivot p and the struck bead j may exchange
 * positions.  Bonds stay with the beads, so the exchange changes the lengths of the tethers
 * of p and of j; hard spheres cannot overlap (the set of occupied positions is unchanged).
 * With tethers the Metropolis acceptance min(1, exp(-dE)) is 1 when every tether of p and
 * of j is at most b_max after the exchange and 0 otherwise. */
static int swap_allowed(const orc_sys *s, int32_t p, int32_t j) {
    const double *rp = &s->r[3 * p], *rj = &s->r[3 * j];
    for (int t = 0; t < 2; ++t) {
        const int32_t q = s->nbr[2 * p + t]; /* p moves to rj */
        if (q >= 0 && dist2(s, rj, q == j ? rp : &s->r[3 * q]) > s->b2) return 0;
        const int32_t u = s->nbr[2 * j + t]; /* j moves to rp */
        if (u >= 0 && dist2(s, rp, u == p ? rj : &s->r[3 * u]) > s->b2) return 0;
    }
    return 1;
}

/* Exchange positions, cells and cell-list entries of p and j.  The unwrapped position of p
 * moves by the minimum-image vector from p to j (and that of j by its opposite), so an
 * exchange across the periodic boundary shifts the image counters by one. */
static int swap_beads(orc_sys *s, int32_t p, int32_t j) {
    for (int a = 0; a < 3; ++a) {
        const double raw = s->r[3 * j + a] - s->r[3 * p + a];
        const int sh = raw > s->halfL ? -1 : (raw < -s->halfL ? 1 : 0);
        s->img[3 * p + a] += sh;
        s->img[3 * j + a] -= sh;
        const double t = s->r[3 * p + a];
        s->r[3 * p + a] = s->r[3 * j + a];
        s->r[3 * j + a] = t;
    }
    const int32_t *cp = s->cell + 3 * p, *cj = s->cell + 3 * j;
    const int kp = cidx(s, cp[0], cp[1], cp[2]), kj = cidx(s, cj[0], cj[1], cj[2]);
    if (kp != kj) {
        cell_remove(s, kp, p);
        cell_remove(s, kj, j);
        if (cell_add(s, kj, p) || cell_add(s, kp, j)) return ORC_E_ARG;
    }
    for (int a = 0; a < 3; ++a) {
        const int32_t t = s->cell[3 * p + a];
        s->cell[3 * p + a] = s->cell[3 * j + a];
        s->cell[3 * j + a] = t;
    }
    return ORC_OK;
}

/* Second reflection of the EC: between the previous reflection (x_max then xref) and this
 * one the EC has used W = xref - x_max, and from here on it retraces its path between the
 * two stops with period 2W.  Whole periods are dropped: x_max = fmod(x_max, 2W).  Returns 1
 * if the EC ends here (W = 0: nothing between the stops can move). */
static int periodic(orc_sys *s, const orc_dom *dm, uint32_t step, int32_t p, double xref, double *xmax) {
    const double W = xref - *xmax;
    if (!(W > 0.0)) {
        log_event(s, dm, step, p, -1, ORC_EV_CYCLE);
        s->cnt[ORC_C_CYCLE]++;
        return 1;
    }
    const double r = fmod(*xmax, W + W);
    if (r < *xmax) {
        *xmax = r;
        log_event(s, dm, step, p, -1, ORC_EV_PERIOD);
        s->cnt[ORC_C_PERIOD]++;
    }
    return 0;
}

/* ---------------------------------------------------------------- one EC */
static int run_ec(orc_sys *s, orc_dom *dm, int32_t p, int axis, int sgn, double ell) {
    double xmax = ell;
    uint32_t step = 0;
    int reflected = 0; /* a reflection happened in this EC ...                     */
    double xref = 0.0; /* ... with this much displacement left after it           */
    uint32_t run = 0;  /* consecutive zero-length events */
    int32_t saved_p = -1, saved_sgn = 0, saved_c = -1;
    s->cnt[ORC_C_EC]++;
    for (;;) {
        if (run > 0) {
            /* zero-length run: the state (pivot, direction, pivot cell) repeating means a cycle */
            const int32_t c = s->cell[3 * p + axis];
            if (p == saved_p && sgn == saved_sgn && c == saved_c) {
                log_event(s, dm, step, p, -1, ORC_EV_CYCLE);
                s->cnt[ORC_C_CYCLE]++;
                return ORC_OK;
            }
            if ((run & (run - 1)) == 0) {
                saved_p = p;
                saved_sgn = sgn;
                saved_c = c;
            }
        }
        if ((int64_t)step >= s->event_cap) return ORC_E_STUCK;
        step++;
        s->cnt[ORC_C_STEPS]++;
        double g[2];
        if (s->spring) spring_terms(s, dm, step, g);
        const orc_best b = scan_partners(s, p, axis, sgn, s->spring ? g : NULL);
        const double xc = x_cell_of(s, p, axis, sgn);
        if (s->check >= 2) {
            const orc_best bf = brute_partners(s, p, axis, sgn, s->spring ? g : NULL);
            if (b.x <= xc) {
                if (!(bf.x == b.x && bf.j == b.j && bf.kind == b.kind)) return ORC_E_CHECK;
            } else if (!(bf.x > xc)) {
                return ORC_E_CHECK;
            }
        }
        double *ra = &s->r[3 * p + axis];
        const double m = b.x < xc ? b.x : xc;
        if (xmax <= m) {
            /* END: the pivot takes the rest of the displacement (step 4) */
            *ra = sgn > 0 ? *ra + xmax : *ra - xmax;
            log_event(s, dm, step, p, -1, ORC_EV_END);
            if (s->check >= 1 && check_pivot(s, p)) return ORC_E_CHECK;
            return ORC_OK;
        }
        if (b.x <= xc) {
            /* interaction event: move to contact / tether limit (steps 2-3) */
            if (b.x > 0.0) {
                run = 0;
                saved_p = -1;
            } else {
                run++;
            }
            *ra = sgn > 0 ? *ra + b.x : *ra - b.x;
            xmax = xmax - b.x;
            const int motile = cell_in_domain(s, dm, s->cell + 3 * b.j);
            if (s->check >= 1 && check_pivot(s, p)) return ORC_E_CHECK;
            if (motile && s->swap && b.kind == 0 && swap_allowed(s, p, b.j)) {
                /* swap (Sec. II.C): the pivot takes the struck bead's place and goes on; its
                 * identity has advanced by d_par > 0, so a zero-length run is over */
                log_event(s, dm, step, p, b.j, ORC_EV_SWAP);
                s->cnt[ORC_C_SWAP]++;
                s->sum_delta += b.dpar - b.x;
                if (swap_beads(s, p, b.j)) return ORC_E_ARG;
                if (s->check >= 1 && (check_pivot(s, p) || check_pivot(s, b.j))) return ORC_E_CHECK;
                run = 0;
                saved_p = -1;
            } else if (motile) {
                log_event(s, dm, step, p, b.j, b.kind == 0 ? ORC_EV_HS_LIFT : ORC_EV_TETHER_LIFT);
                s->cnt[b.kind == 0 ? ORC_C_HS_LIFT : ORC_C_TETHER_LIFT]++;
                s->sum_delta += b.dpar - b.x;
                p = b.j;
            } else {
                log_event(s, dm, step, p, b.j, b.kind == 0 ? ORC_EV_HS_REFLECT : ORC_EV_TETHER_REFLECT);
                s->cnt[b.kind == 0 ? ORC_C_HS_REFLECT : ORC_C_TETHER_REFLECT]++;
                if (!s->spring && !s->no_skip && reflected && periodic(s, dm, step, p, xref, &xmax)) return ORC_OK;
                reflected = 1;
                xref = xmax;
                sgn = -sgn;
            }
            continue;
        }
        /* cell-face event: the pivot is set onto the face */
        if (xc > 0.0) {
            run = 0;
            saved_p = -1;
        } else {
            run++;
        }
        const int c = s->cell[3 * p + axis];
        *ra = sgn > 0 ? s->bnd[c + 1] : s->bnd[c];
        xmax = xmax - xc;
        int nc = c + sgn;
        int wrapped = 0;
        if (nc >= s->n) {
            nc = 0;
            wrapped = 1;
        } else if (nc < 0) {
            nc = s->n - 1;
            wrapped = -1;
        }
        int32_t cn[3] = {s->cell[3 * p], s->cell[3 * p + 1], s->cell[3 * p + 2]};
        cn[axis] = nc;
        if (cell_in_domain(s, dm, cn)) {
            const int32_t *co = s->cell + 3 * p;
            cell_remove(s, cidx(s, co[0], co[1], co[2]), p);
            if (cell_add(s, cidx(s, cn[0], cn[1], cn[2]), p)) return ORC_E_ARG;
            s->cell[3 * p + axis] = nc;
            if (wrapped > 0) {
                *ra = 0.0;
                s->img[3 * p + axis] += 1;
            } else if (wrapped < 0) {
                *ra = s->L;
                s->img[3 * p + axis] -= 1;
            }
            s->cnt[ORC_C_CROSS]++;
        } else {
            log_event(s, dm, step, p, -1, ORC_EV_WALL);
            s->cnt[ORC_C_WALL]++;
            if (!s->spring && !s->no_skip && reflected && periodic(s, dm, step, p, xref, &xmax)) return ORC_OK;
            reflected = 1;
            xref = xmax;
            sgn = -sgn;
        }
        if (s->check >= 1 && check_pivot(s, p)) return ORC_E_CHECK;
    }
}

int orc_run_ec(orc_sys *s, int32_t p, int dir, double ell) {
    if (p < 0 || p >= s->nb || dir < 0 || dir > 5 || !(ell >= 0)) return ORC_E_ARG;
    orc_dom dm;
    memset(&dm, 0, sizeof dm);
    dm.D = 1;
    dm.P = 1;
    return run_ec(s, &dm, p, dir >> 1, (dir & 1) ? -1 : 1, ell);
}

static int cmp_i32(const void *a, const void *b) {
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* ---------------------------------------------------------------- push-off */
/* Whether bead i overlaps any other bead at the push-off diameter (minimum image, every bead of
 * the 27 cells around it, squared distance summed over x, y, z in that order). */
static int overlaps_any(const orc_sys *s, int32_t i) {
    const int n = s->n;
    const int32_t *ci = s->cell + 3 * i;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int c = cidx(s, (ci[0] + dx + n) % n, (ci[1] + dy + n) % n, (ci[2] + dz + n) % n);
                for (int t = 0; t < s->ccount[c]; ++t) {
                    const int32_t j = s->clist[c][t];
                    if (j == i) continue;
                    double q[3];
                    for (int a = 0; a < 3; ++a) {
                        const double d = mi(s, s->r[3 * j + a] - s->r[3 * i + a]);
                        q[a] = d * d;
                    }
                    if ((q[0] + q[1]) + q[2] < s->ov2) return 1;
                }
            }
    return 0;
}

int64_t orc_count_overlaps(const orc_sys *s, double d) {
    const double lim = d * d * (1.0 - 1e-9);
    int64_t k = 0;
    for (int64_t i = 0; i < s->nb; ++i)
        for (int64_t j = i + 1; j < s->nb; ++j) {
            double q = 0;
            for (int a = 0; a < 3; ++a) {
                const double v = mi(s, s->r[3 * j + a] - s->r[3 * i + a]);
                q += v * v;
            }
            if (q < lim) ++k;
        }
    return k;
}

/* The EC starts of the push-off: the beads of list[0..m) that overlap some bead, in the same
 * order, written to out; returns how many.  Without push-off every bead of the list. */
static int64_t start_beads(const orc_sys *s, const int32_t *list, int64_t m, int32_t *out) {
    int64_t k = 0;
    for (int64_t i = 0; i < m; ++i)
        if (!s->push || overlaps_any(s, list[i])) out[k++] = list[i];
    return k;
}

/* ---------------------------------------------------------------- sweep */
static int in_list(const uint32_t *list, int64_t n, uint32_t v) {
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        const int64_t mid = (lo + hi) / 2;
        if (list[mid] == v) return 1;
        if (list[mid] < v) lo = mid + 1;
        else hi = mid - 1;
    }
    return 0;
}

static int sweep_impl(orc_sys *s, int64_t n_ec, double ell, uint64_t seed, int tiling, int D,
                      uint32_t colour_mask, const uint32_t *only, int64_t n_only) {
    if (n_ec < 0 || !(ell >= 0) || !isfinite(ell)) return ORC_E_ARG;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const uint32_t sweep = s->sweep_ctr;
    int32_t *mot = (int32_t *)malloc(sizeof(int32_t) * (size_t)s->nb);
    int32_t *starts = (int32_t *)malloc(sizeof(int32_t) * (size_t)s->nb);
    if (!mot || !starts) {
        free(mot);
        free(starts);
        return ORC_E_ARG;
    }
    int st = ORC_OK;
    orc_dom dm;
    memset(&dm, 0, sizeof dm);
    dm.sweep = sweep;
    {
        const uint32_t ctr[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, s->stream, 0x53505247u};
        uint32_t u[4];
        orc_philox4x32_10(ctr, key, u);
        dm.skey[0] = u[0];
        dm.skey[1] = u[1];
    }
    if (tiling == 0) {
        /* one domain: the whole box */
        dm.tiled = 0;
        dm.D = 1;
        dm.P = 1;
        for (int64_t i = 0; i < s->nb; ++i) mot[i] = (int32_t)i;
        for (int64_t k = 0; k < n_ec && st == ORC_OK; ++k) {
            const int64_t ms = start_beads(s, mot, s->nb, starts);
            if (ms == 0) break;
            const uint32_t ctr[4] = {(uint32_t)k, 0u, sweep, 2u * s->stream};
            uint32_t u[4];
            orc_philox4x32_10(ctr, key, u);
            const int32_t p = starts[below(u[0], (uint32_t)ms)];
            const uint32_t dir = below(u[1], 6);
            dm.ec = (uint32_t)k;
            st = run_ec(s, &dm, p, (int)(dir >> 1), (dir & 1) ? -1 : 1, ell);
        }
    } else if (tiling == 1 || tiling == 2) {
        /* checkerboard (1): D^3-cell domains, 8 colour phases; tile-joint (2, Sec. II.A): tiles of
         * D^3 cells, each followed along every axis by one joint cell that no tile moves, all
         * tiles at once in one phase */
        const int n = s->n;
        const int P = tiling == 2 ? D + 1 : D;
        if ((tiling == 1 && (D < 2 || n % D != 0 || (n / D) % 2 != 0)) ||
            (tiling == 2 && (D < 2 || n % P != 0 || n / P < 2))) {
            free(mot);
            free(starts);
            return ORC_E_BOX;
        }
        const int nd = n / P;
        const int64_t ndom = (int64_t)nd * nd * nd;
        const int64_t K = (n_ec + ndom - 1) / ndom;
        dm.tiled = 1;
        dm.D = D;
        dm.P = P;
        {
            const uint32_t ctr[4] = {0u, 0u, sweep, 2u * s->stream + 1u};
            uint32_t u[4];
            orc_philox4x32_10(ctr, key, u);
            for (int a = 0; a < 3; ++a) dm.off[a] = (int)below(u[a], (uint32_t)P);
        }
        const int phases = tiling == 2 ? 1 : 8;
        for (int colour = 0; colour < phases && st == ORC_OK; ++colour) {
            if (!((colour_mask >> colour) & 1u)) continue;
            dm.colour = (uint32_t)colour;
            for (int dz = 0; dz < nd && st == ORC_OK; ++dz)
                for (int dy = 0; dy < nd && st == ORC_OK; ++dy)
                    for (int dx = 0; dx < nd && st == ORC_OK; ++dx) {
                        if (tiling == 1 && ((dx & 1) != (colour & 1) || (dy & 1) != ((colour >> 1) & 1) ||
                                            (dz & 1) != ((colour >> 2) & 1)))
                            continue;
                        dm.dom[0] = dx;
                        dm.dom[1] = dy;
                        dm.dom[2] = dz;
                        dm.domain = (uint32_t)(dx + nd * (dy + nd * dz));
                        if (only && !in_list(only, n_only, dm.domain)) continue;
                        /* the domain's beads in ascending id */
                        int64_t m = 0;
                        for (int tz = 0; tz < D; ++tz)
                            for (int ty = 0; ty < D; ++ty)
                                for (int tx = 0; tx < D; ++tx) {
                                    const int c = cidx(s, (dm.off[0] + dx * P + tx) % n,
                                                       (dm.off[1] + dy * P + ty) % n,
                                                       (dm.off[2] + dz * P + tz) % n);
                                    for (int t = 0; t < s->ccount[c]; ++t) mot[m++] = s->clist[c][t];
                                }
                        if (m == 0) continue;
                        qsort(mot, (size_t)m, sizeof(int32_t), cmp_i32);
                        for (int64_t k = 0; k < K && st == ORC_OK; ++k) {
                            const int64_t ms = start_beads(s, mot, m, starts);
                            if (ms == 0) break;
                            const uint32_t ctr[4] = {(uint32_t)k, dm.domain, sweep, 2u * s->stream};
                            uint32_t u[4];
                            orc_philox4x32_10(ctr, key, u);
                            const int32_t p = starts[below(u[0], (uint32_t)ms)];
                            const uint32_t dir = below(u[1], 6);
                            dm.ec = (uint32_t)k;
                            st = run_ec(s, &dm, p, (int)(dir >> 1), (dir & 1) ? -1 : 1, ell);
                        }
                    }
        }
    } else {
        st = ORC_E_ARG;
    }
    free(mot);
    free(starts);
    s->sweep_ctr++;
    return st;
}

int orc_sweep(orc_sys *s, int64_t n_ec, double ell, uint64_t seed, int tiling, int D,
              uint32_t colour_mask) {
    return sweep_impl(s, n_ec, ell, seed, tiling, D, colour_mask, NULL, 0);
}

int orc_sweep_subset(orc_sys *s, int64_t n_ec, double ell, uint64_t seed, int D, uint32_t colour_mask,
                     const uint32_t *domains, int64_t n_domains) {
    for (int64_t i = 1; i < n_domains; ++i)
        if (domains[i] <= domains[i - 1]) return ORC_E_ARG;
    return sweep_impl(s, n_ec, ell, seed, 1, D, colour_mask, domains, n_domains);
}

/* ---------------------------------------------------------------- observables */
/* Per polymer (Sec. IV.A and the appendix): end-to-end vector R as the sum of minimum-image bond
 * vectors, R_g^2 = N^-1 sum_i (u_i - u_cm)^2 over the unwrapped chain u (reading
 * the garbled index range as i = 1..N), the middle bead floor(N/2) (0-based) in
 * image-unwrapped coordinates for g1, and a histogram of bond lengths on
 * [sigma, b_max] with nbins equal bins. */
/* Shape analysis (appendix, moment of inertia tensor): the gyration tensor by its definition,
 * centre of mass first, then the mean outer product of the positions relative to it. */
void orc_gyration(const double *u, int64_t n, double g[6]) {
    double cm[3] = {0.0, 0.0, 0.0};
    for (int64_t k = 0; k < n; ++k)
        for (int a = 0; a < 3; ++a) cm[a] += u[3 * k + a];
    for (int a = 0; a < 3; ++a) cm[a] /= (double)n;
    static const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int m = 0; m < 6; ++m) {
        double acc = 0.0;
        for (int64_t k = 0; k < n; ++k) acc += (u[3 * k + ia[m]] - cm[ia[m]]) * (u[3 * k + ib[m]] - cm[ib[m]]);
        g[m] = acc / (double)n;
    }
}

int orc_shape(const orc_sys *s, double *gyr, double *com) {
    double *u = NULL;
    int64_t ucap = 0;
    for (int64_t q = 0; q < s->npoly; ++q) {
        const int64_t a = s->pstart[q], e = s->pstart[q + 1];
        const int64_t N = e - a;
        if (N > ucap) {
            free(u);
            ucap = N;
            u = (double *)malloc(sizeof(double) * 3 * (size_t)N);
            if (!u) return ORC_E_ARG;
        }
        /* unwrapped chain: the first bead with its image counters, then minimum-image bonds */
        const int32_t i0 = s->porder[a];
        for (int k = 0; k < 3; ++k) u[k] = s->r[3 * i0 + k] + (double)s->img[3 * i0 + k] * s->L;
        for (int64_t t = 1; t < N; ++t) {
            const int32_t j0 = s->porder[a + t - 1], j1 = s->porder[a + t];
            for (int k = 0; k < 3; ++k) u[3 * t + k] = u[3 * (t - 1) + k] + mi(s, s->r[3 * j1 + k] - s->r[3 * j0 + k]);
        }
        if (gyr) orc_gyration(u, N, gyr + 6 * q);
        if (com)
            for (int k = 0; k < 3; ++k) {
                double acc = 0.0;
                for (int64_t t = 0; t < N; ++t) acc += u[3 * t + k];
                com[3 * q + k] = acc / (double)N;
            }
    }
    free(u);
    return ORC_OK;
}

int orc_observables(const orc_sys *s, int nbins, double *r2, double *rg2, int64_t *hist,
                    double *mid, int64_t *n_poly) {
    if (n_poly) *n_poly = s->npoly;
    if (hist)
        for (int k = 0; k < nbins; ++k) hist[k] = 0;
    for (int64_t q = 0; q < s->npoly; ++q) {
        const int64_t a = s->pstart[q], e = s->pstart[q + 1];
        const int64_t N = e - a;
        double u[3] = {s->r[3 * s->porder[a]], s->r[3 * s->porder[a] + 1], s->r[3 * s->porder[a] + 2]};
        double R[3] = {0, 0, 0};
        double sum[3] = {u[0], u[1], u[2]};
        /* first pass: R, centre of mass, bond histogram */
        for (int64_t t = a + 1; t < e; ++t) {
            const int32_t i0 = s->porder[t - 1], i1 = s->porder[t];
            double d[3];
            for (int k = 0; k < 3; ++k) {
                d[k] = mi(s, s->r[3 * i1 + k] - s->r[3 * i0 + k]);
                R[k] += d[k];
                u[k] += d[k];
                sum[k] += u[k];
            }
            if (hist && nbins > 0) {
                const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                int bin = (int)floor((len - s->sigma) / (s->bmax - s->sigma) * nbins);
                if (bin < 0) bin = 0;
                if (bin > nbins - 1) bin = nbins - 1;
                hist[bin]++;
            }
        }
        const double cm[3] = {sum[0] / (double)N, sum[1] / (double)N, sum[2] / (double)N};
        if (r2) r2[q] = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
        /* second pass: radius of gyration */
        double g = 0;
        double v[3] = {s->r[3 * s->porder[a]], s->r[3 * s->porder[a] + 1], s->r[3 * s->porder[a] + 2]};
        for (int64_t t = a; t < e; ++t) {
            if (t > a) {
                const int32_t i0 = s->porder[t - 1], i1 = s->porder[t];
                for (int k = 0; k < 3; ++k) v[k] += mi(s, s->r[3 * i1 + k] - s->r[3 * i0 + k]);
            }
            for (int k = 0; k < 3; ++k) g += (v[k] - cm[k]) * (v[k] - cm[k]);
        }
        if (rg2) rg2[q] = g / (double)N;
        if (mid) {
            const int32_t im = s->porder[a + N / 2];
            for (int k = 0; k < 3; ++k) mid[3 * q + k] = s->r[3 * im + k] + (double)s->img[3 * im + k] * s->L;
        }
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------- pair distances */
/* Histogram of the distances of all bead pairs i < j closer than r_max (minimum image, by brute
 * force over every pair), bin floor(r / r_max * nbins) (clamped to nbins - 1): the pair counts
 * behind g(r).  Displacements are taken as (r_j - r_i) and then shifted by the box edge, the
 * squared length summed over x, y, z in that order. */
int orc_pair_histogram(const orc_sys *s, int nbins, double rmax, int64_t *hist) {
    if (nbins < 1 || !(rmax > 0.0) || !(rmax <= s->halfL)) return ORC_E_ARG;
    for (int k = 0; k < nbins; ++k) hist[k] = 0;
    for (int64_t i = 0; i < s->nb; ++i)
        for (int64_t j = i + 1; j < s->nb; ++j) {
            double d[3];
            for (int a = 0; a < 3; ++a) d[a] = mi(s, s->r[3 * j + a] - s->r[3 * i + a]);
            const double q0 = d[0] * d[0];
            const double q1 = d[1] * d[1];
            const double q2 = d[2] * d[2];
            const double r = sqrt((q0 + q1) + q2);
            if (!(r < rmax)) continue;
            int bin = (int)floor(r / rmax * (double)nbins);
            if (bin > nbins - 1) bin = nbins - 1;
            hist[bin]++;
        }
    return ORC_OK;
}

/* End-to-end distance distribution W(R) (appendix, end-to-end distance distribution): the
 * histogram over polymers of |R| = sqrt(R^2), R^2 as orc_observables computes it, bin
 * floor(|R| / r_max * nbins), values at or above r_max in the last bin. */
int orc_end_to_end_histogram(const orc_sys *s, int nbins, double rmax, int64_t *hist) {
    if (nbins < 1 || !(rmax > 0.0)) return ORC_E_ARG;
    double *r2 = (double *)malloc(sizeof(double) * (size_t)(s->npoly > 0 ? s->npoly : 1));
    if (!r2) return ORC_E_ARG;
    orc_observables(s, 0, r2, NULL, NULL, NULL, NULL);
    for (int k = 0; k < nbins; ++k) hist[k] = 0;
    for (int64_t q = 0; q < s->npoly; ++q) {
        int bin = (int)floor(sqrt(r2[q]) / rmax * (double)nbins);
        if (bin > nbins - 1) bin = nbins - 1;
        hist[bin]++;
    }
    free(r2);
    return ORC_OK;
}

/* Internal distances R^2(n) (Sec. II.B, the check of start configurations against a long run):
 * for every polymer and every pair of its beads t < t' with t' - t = n <= n_max, the squared
 * length of the chain vector from bead t to bead t', which is the sum of the minimum-image bond
 * vectors between them, walked bond by bond from t.  sum[n] adds these squared lengths and
 * count[n] counts the pairs; n = 0 counts every bead once with length 0. */
int orc_internal_distances(const orc_sys *s, int64_t n_max, double *sum, int64_t *count) {
    if (n_max < 0) return ORC_E_ARG;
    for (int64_t n = 0; n <= n_max; ++n) {
        sum[n] = 0.0;
        count[n] = 0;
    }
    for (int64_t q = 0; q < s->npoly; ++q) {
        const int64_t a = s->pstart[q], e = s->pstart[q + 1];
        for (int64_t t = a; t < e; ++t) {
            count[0]++;
            double R[3] = {0.0, 0.0, 0.0};
            for (int64_t t2 = t + 1; t2 < e && t2 - t <= n_max; ++t2) {
                const int32_t i0 = s->porder[t2 - 1], i1 = s->porder[t2];
                for (int k = 0; k < 3; ++k) R[k] += mi(s, s->r[3 * i1 + k] - s->r[3 * i0 + k]);
                const double q0 = R[0] * R[0];
                const double q1 = R[1] * R[1];
                const double q2 = R[2] * R[2];
                sum[t2 - t] += (q0 + q1) + q2;
                count[t2 - t]++;
            }
        }
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------- accessors */
int64_t orc_n_beads(const orc_sys *s) { return s->nb; }
int orc_n_cells(const orc_sys *s) { return s->n; }
double orc_cell_size(const orc_sys *s) { return s->h; }
uint32_t orc_sweep_counter(const orc_sys *s) { return s->sweep_ctr; }
void orc_get_positions(const orc_sys *s, double *out) { memcpy(out, s->r, sizeof(double) * 3 * (size_t)s->nb); }
void orc_get_cells(const orc_sys *s, int32_t *out) { memcpy(out, s->cell, sizeof(int32_t) * 3 * (size_t)s->nb); }
void orc_get_images(const orc_sys *s, int32_t *out) { memcpy(out, s->img, sizeof(int32_t) * 3 * (size_t)s->nb); }

void orc_counters(const orc_sys *s, uint64_t *cnt, double *sum_delta) {
    if (cnt) memcpy(cnt, s->cnt, sizeof s->cnt);
    if (sum_delta) *sum_delta = s->sum_delta;
}

int orc_set_state(orc_sys *s, const double *pos, const int32_t *cells, const int32_t *img,
                  uint32_t sweep_ctr) {
    for (int64_t i = 0; i < 3 * s->nb; ++i) {
        const int c = cells[i];
        if (c < 0 || c >= s->n || !(pos[i] >= s->bnd[c] - 1e-12 && pos[i] <= s->bnd[c + 1] + 1e-12))
            return ORC_E_ARG;
    }
    memcpy(s->r, pos, sizeof(double) * 3 * (size_t)s->nb);
    memcpy(s->cell, cells, sizeof(int32_t) * 3 * (size_t)s->nb);
    memcpy(s->img, img, sizeof(int32_t) * 3 * (size_t)s->nb);
    s->sweep_ctr = sweep_ctr;
    return rebuild_cells(s);
}

/*
 * TEST INFRASTRUCTURE ONLY — plain serial FP64 CPU oracle for the event-chain
 * (EC) move of tethered hard-sphere chains (Kampmann, Boltz, Kierfeld,
 * arXiv:1502.06447, Sec. II: Eq. (1), the tether bonds after Eq. (2), the EC
 * rule of Sec. II, the parallel decomposition of Sec. II.A).
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header or table with the GPU library.
 *
 * Every function is serial, unblocked and written to be checked by eye against
 * the paper's steps; speed is not a goal.
 */
#ifndef ECMC_ORACLE_H
#define ECMC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes (same numeric meaning as the GPU library's, written separately) */
enum {
    ORC_OK = 0,
    ORC_E_ARG = -1,
    ORC_E_OVERLAP = -2,
    ORC_E_TETHER = -3,
    ORC_E_BOX = -4,
    ORC_E_CELL_OVERFLOW = -5,
    ORC_E_STUCK = -6,
    ORC_E_CHECK = -9 /* an internal self-check (invariant or brute force) failed */
};

/* event kinds written to the log */
enum {
    ORC_EV_HS_LIFT = 0,        /* hard-sphere contact, struck bead motile: it becomes the pivot */
    ORC_EV_TETHER_LIFT = 1,    /* tether reaches b_max, partner motile: it becomes the pivot   */
    ORC_EV_HS_REFLECT = 2,     /* contact with an immotile bead: direction reversed            */
    ORC_EV_TETHER_REFLECT = 3, /* tether limit with an immotile partner: direction reversed    */
    ORC_EV_WALL = 4,           /* pivot reaches its domain wall: direction reversed            */
    ORC_EV_END = 5,            /* remaining displacement used up (target = -1)                 */
    ORC_EV_PERIOD = 6,         /* second reflection of the EC: whole periods of the retraced
                                  path between the two stops dropped from x_max (target = -1) */
    ORC_EV_SWAP = 8,           /* hard-sphere contact with a motile bead: the pivot and the
                                  struck bead exchanged positions, the pivot goes on          */
    ORC_EV_CYCLE = 7           /* nothing can move any more (zero-length cycle or a zero period
                                  between two stops): ends the EC (target = -1)               */
};

typedef struct {
    uint32_t sweep, domain, ec, step;
    int32_t pivot, target;
    uint32_t kind, colour;
} orc_event;

/* counters */
enum {
    ORC_C_HS_LIFT = 0,
    ORC_C_TETHER_LIFT,
    ORC_C_HS_REFLECT,
    ORC_C_TETHER_REFLECT,
    ORC_C_WALL,
    ORC_C_CROSS,
    ORC_C_EC,
    ORC_C_STEPS,
    ORC_C_PERIOD,
    ORC_C_CYCLE,
    ORC_C_SWAP,
    ORC_NCNT
};

typedef struct orc_sys orc_sys;

/* n_cells = 0 picks the largest n with L/n > b_max.  Requires n >= 4. */
int orc_create(orc_sys **out, double L, double sigma, double bmax, int n_cells, int64_t n_beads,
               const double *pos, int64_t n_bonds, const int32_t *bonds);
void orc_destroy(orc_sys *s);

/* As orc_create, but hard-sphere overlaps in the start are accepted (tethers are still
 * checked): the phantom start of the push-off. */
int orc_create_overlapping(orc_sys **out, double L, double sigma, double bmax, int n_cells, int64_t n_beads,
                           const double *pos, int64_t n_bonds, const int32_t *bonds);

/* Push-off (Sec. II.B) at working diameter d in (0, sigma] for the following sweeps: a pair
 * closer than d (squared distance below d^2 (1 - 1e-9)) is no hard-sphere event, and every EC
 * starts at a motile bead that overlaps some bead; d = 0 returns to plain ECs at sigma.
 * Refused with springs or swap moves on. */
int orc_set_pushoff(orc_sys *s, double d);

/* Pairs closer than d (squared distance below d^2 (1 - 1e-9)), by brute force. */
int64_t orc_count_overlaps(const orc_sys *s, double d);

/* event_cap: loop iterations allowed per EC (0 = default 10^7).
 * check: 0 none; 1 invariants after every event; 2 also brute-force next-event search. */
int orc_set_options(orc_sys *s, int64_t event_cap, int check);

/* Swap moves (Sec. II.C) on (1) or off (0, the default) for the following ECs.  Refused
 * (ORC_E_ARG) while springs are on. */
int orc_set_swap(orc_sys *s, int on);

/* The periodic reduction (whole periods of an EC dropped after its second reflection) on (1, the
 * default) or off (0: the plain loop of Sec. II steps 1-4, until x_max is used up). */
int orc_set_periodic_skip(orc_sys *s, int on);

/* Bonds as harmonic springs (k/2)(b - sigma)^2 of spring constant k > 0 (Eq. (2), in units
 * of k_B T / sigma^2), still capped at b_max; k = 0 (the default) gives tethers.  Refused
 * (ORC_E_ARG) for k < 0, a non-finite k, or while swap moves are on.  A single EC of
 * orc_run_ec draws its energies with key (0, 0) and EC, domain and sweep 0. */
int orc_set_spring(orc_sys *s, double k);

/* Random stream index m (default 0): the Philox counters of the following sweeps end in 2 m
 * (EC draws) and 2 m + 1 (partition offsets), the streams of melt m of a batch. */
int orc_set_stream(orc_sys *s, uint32_t m);
int orc_set_log(orc_sys *s, orc_event *buf, int64_t cap);
int64_t orc_log_count(const orc_sys *s);

/* One sweep: tiling 0 = whole box (one domain, every bead motile), 1 = checkerboard of
 * D^3-cell domains in 8 colour phases (n % D == 0, n / D even), 2 = tile-joint (Sec. II.A):
 * D^3-cell tiles at pitch D + 1, the cell after each tile along every axis an immotile joint,
 * all tiles in one phase (n % (D + 1) == 0, n / (D + 1) >= 2, D >= 2: a 1-cell tile has a wall
 * at every face, so no bead could ever leave its cell).  colour_mask selects which phases run
 * (bit 0 alone for tile-joint). */
int orc_sweep(orc_sys *s, int64_t n_ec, double ell, uint64_t seed, int tiling, int D,
              uint32_t colour_mask);

/* As orc_sweep with tiling 1, but only the listed domains (strictly ascending ids) run their
 * ECs; every other domain is left untouched.  Domains of one colour phase never interact,
 * so the listed domains end exactly as in a full sweep's first selected phase. */
int orc_sweep_subset(orc_sys *s, int64_t n_ec, double ell, uint64_t seed, int D, uint32_t colour_mask,
                     const uint32_t *domains, int64_t n_domains);

/* Whole-box helpers for unit tests. */
int orc_next_event(const orc_sys *s, int32_t p, int axis, int sgn, double *x, int32_t *j,
                   int *kind, double *x_cell);
int orc_run_ec(orc_sys *s, int32_t p, int dir, double ell);

/* Gyration tensor of one chain given unwrapped, u [n][3]: G = n^-1 sum_k (u_k - u_cm)(u_k - u_cm)^T
 * (two passes), stored as xx, yy, zz, xy, xz, yz.  The moment of inertia tensor of the appendix
 * is n (tr G 1 - G): same eigenvectors, eigenvalues n (tr G - lambda_i). */
void orc_gyration(const double *u, int64_t n, double g[6]);

/* Per polymer of the current state (chains unwrapped from their first bead by minimum-image
 * bonds): gyration tensor gyr [n_poly][6] and the centre of mass in image-unwrapped
 * coordinates com [n_poly][3] (either may be NULL). */
int orc_shape(const orc_sys *s, double *gyr, double *com);

int orc_observables(const orc_sys *s, int nbins, double *r2, double *rg2, int64_t *hist,
                    double *mid, int64_t *n_poly);

/* Pair counts behind g(r): every pair i < j with minimum-image distance r < r_max (r_max at most
 * L/2), binned by floor(r / r_max * nbins) (clamped to nbins - 1).  Brute force over all pairs. */
int orc_pair_histogram(const orc_sys *s, int nbins, double rmax, int64_t *hist);

/* End-to-end distance distribution W(R): histogram over polymers of |R|, bins of width
 * r_max / nbins from 0, values at or above r_max counted in the last bin. */
int orc_end_to_end_histogram(const orc_sys *s, int nbins, double rmax, int64_t *hist);
/* R^2(n): sums of squared chain vectors between beads n bonds apart, and their counts, n = 0..n_max */
int orc_internal_distances(const orc_sys *s, int64_t n_max, double *sum, int64_t *count);

int64_t orc_n_beads(const orc_sys *s);
int orc_n_cells(const orc_sys *s);
double orc_cell_size(const orc_sys *s);
uint32_t orc_sweep_counter(const orc_sys *s);
void orc_get_positions(const orc_sys *s, double *out);
void orc_get_cells(const orc_sys *s, int32_t *out);
void orc_get_images(const orc_sys *s, int32_t *out);
void orc_counters(const orc_sys *s, uint64_t *cnt, double *sum_delta);
int orc_set_state(orc_sys *s, const double *pos, const int32_t *cells, const int32_t *img,
                  uint32_t sweep_ctr);

/* Bond candidate of a partner at (d_par, d_perp^2) from the pivot: the tether formula for
 * g < 0, else the spring formula with g = 2 dE / k (see the readings in the source). */
double orc_bond_x(const orc_sys *s, double dpar, double dperp2, double g);

/* Natural logarithm as the spring draws evaluate it (reduction to [sqrt(1/2), sqrt(2)) and
 * the artanh series); within a few ulp of the libm value. */
double orc_ln(double u);

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

#ifdef __cplusplus
}
#endif
#endif

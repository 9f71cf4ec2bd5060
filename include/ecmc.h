/*
 * ecmc.h — C ABI of the MI355X (gfx950) event-chain Monte Carlo library for
 * dense melts of tethered hard-sphere bead chains.
 *
 * The method is the event-chain (EC) move of Kampmann, Boltz and Kierfeld,
 * "Monte Carlo Simulation of Dense Polymer Melts Using Event Chain Algorithms"
 * (arXiv:1502.06447):
 *   - model (Sec. II, Eq. (1) and the tether variant stated after Eq. (2)):
 *     hard spheres of diameter sigma between all bead pairs, bonded neighbours
 *     joined by tethers of maximal length l_max (the paper's b_max), periodic cube;
 *   - EC move (Sec. II, the four-step rule and its generalisation to several
 *     interaction partners): a pivot moves along +-x/+-y/+-z by the smallest
 *     admissible displacement x = min_i x_i, the displacement passes to the argmin
 *     bead, until the total length ell is used up;
 *   - parallel decomposition (Sec. II.A): domains redrawn every sweep, beads outside
 *     the active domain immotile, ECs reflected at domain walls and at immotile beads.
 *   - two shortcuts this library adds (exact in real arithmetic, identical in the CPU
 *     reference): from its second reflection on, an EC retraces its path back and forth
 *     with period twice the length W used between the first two reflections, so whole
 *     periods of the remaining displacement are skipped (W = 0 ends the EC); a run of
 *     zero-length events that returns to an earlier state (nothing can move) ends the EC.
 *
 * Conventions for every call:
 *   - no C++ types or exceptions cross this boundary; every call returns an
 *     ecmc_status and ecmc_last_error() holds a message for the last failure;
 *   - host arrays passed in are copied (the caller keeps ownership); host arrays
 *     passed out are written in full before the call returns;
 *   - the library never allocates device memory: all device state lives in the
 *     caller's workspace (ecmc_options.workspace, sized by ecmc_workspace_size);
 *   - all device work is enqueued on ecmc_options.stream (a hipStream_t, NULL = the
 *     default stream).  ecmc_sweep returns after enqueueing; device-side errors
 *     (cell overflow, event cap) surface at the next synchronising call
 *     (ecmc_synchronize, ecmc_observables, ecmc_get_*);
 *   - a context is not thread-safe: calls on one context must not overlap.
 */
#ifndef ECMC_H
#define ECMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ecmc_ctx ecmc_ctx;

typedef enum {
    ECMC_OK = 0,
    ECMC_E_ARG = -1,           /* invalid argument (NaN, bad bond list, ring, size) */
    ECMC_E_OVERLAP = -2,       /* two beads closer than sigma (1 - 2e-12)            */
    ECMC_E_TETHER = -3,        /* a bond longer than l_max (1 + 2e-12)               */
    ECMC_E_BOX = -4,           /* cells: n >= 4, L/n > l_max; checkerboard: n/D even */
    ECMC_E_CELL_OVERFLOW = -5, /* a cell or a domain staging area ran out of slots   */
    ECMC_E_STUCK = -6,         /* an EC exceeded event_cap loop iterations           */
    ECMC_E_DEVICE = -7,        /* a HIP runtime call failed                          */
    ECMC_E_WORKSPACE = -8      /* workspace missing, too small or misaligned         */
} ecmc_status;

enum { ECMC_PREC_FP64 = 0, ECMC_PREC_MIXED = 1 };
enum { ECMC_TILING_WHOLE = 0, ECMC_TILING_CHECKER = 1, ECMC_TILING_JOINT = 2 };
enum { ECMC_SCHED_SWEEP = 0, ECMC_SCHED_PHASES = 1 };

/* event kinds in the event log */
enum {
    ECMC_EV_HS_LIFT = 0,        /* contact, struck bead motile: it becomes the pivot       */
    ECMC_EV_TETHER_LIFT = 1,    /* tether taut, partner motile: it becomes the pivot       */
    ECMC_EV_HS_REFLECT = 2,     /* contact with an immotile bead: direction reversed       */
    ECMC_EV_TETHER_REFLECT = 3, /* tether taut with an immotile partner: direction reversed */
    ECMC_EV_WALL = 4,           /* pivot at its domain wall: direction reversed            */
    ECMC_EV_END = 5,            /* displacement used up (target = -1)                      */
    ECMC_EV_PERIOD = 6,         /* a repeated reflection: whole periods 2W of the retraced
                                   path were dropped from the remaining displacement; the EC
                                   goes on (target = -1)                                   */
    ECMC_EV_CYCLE = 7,          /* zero-length events returned to an earlier state, or a
                                   repeated reflection with W = 0 (nothing can move any
                                   more): ends the EC (target = -1)                        */
    ECMC_EV_SWAP = 8            /* swap move (Sec. II.C, with swap_moves): at a hard-sphere
                                   contact with a motile bead the two exchanged positions
                                   (every tether of both within l_max afterwards); the pivot
                                   goes on from the struck bead's place                    */
};

typedef struct {
    int32_t precision;          /* ECMC_PREC_FP64 (default): every staged bead evaluated in
                                   FP64 at every event (the plain kernel).  ECMC_PREC_MIXED: a
                                   single-precision screen of every staged bead bounds its
                                   next-event distance, and only the beads that can come first
                                   are evaluated in FP64; identical results, slower on gfx950 */
    int32_t tiling;             /* ECMC_TILING_WHOLE: one domain, every bead motile;
                                   ECMC_TILING_CHECKER: D^3-cell domains, 8 colour phases;
                                   ECMC_TILING_JOINT: the tile-joint partition (Sec. II.A),
                                   D^3-cell tiles at pitch D + 1 (the cell after each tile an
                                   immotile joint), all tiles in one phase; n a multiple of
                                   D + 1 with n / (D + 1) >= 2, D >= 2 (1-cell tiles would
                                   wall every bead into its cell: ECMC_E_BOX); single melts,
                                   run by phases                                           */
    int32_t n_cells;            /* cells per axis; 0 = largest n with L/n > l_max           */
    int32_t domain_cells;       /* D, cells per domain edge (checkerboard)                  */
    int32_t cell_capacity;      /* bead slots per cell; 0 = 16                              */
    int32_t stage_capacity;     /* beads one domain (plus its one-cell halo) may hold;
                                   0 = automatic: LDS staging sized for the typical domain,
                                   the rare larger domains staged in workspace slots (one
                                   sweep launch) or run by two more launches of the next
                                   size up and 1024 beads (by phases); > 0 = LDS staging of
                                   this capacity only, a larger domain is
                                   ECMC_E_CELL_OVERFLOW; at most 1024                       */
    int64_t event_cap;          /* loop iterations allowed per EC; 0 = 10^7 (at most
                                   2^31 - 1 are honoured)                                   */
    int64_t event_log_capacity; /* event records kept; 0 = no log (the fast path)           */
    int32_t time_kernels;       /* nonzero: time every sweep launch (or colour phase, by
                                   phases) with HIP events                                  */
    int32_t swap_moves;         /* nonzero: propose a swap (Sec. II.C) at every hard-sphere
                                   contact with a motile bead instead of lifting at once    */
    int32_t schedule;           /* checkerboard sweeps (identical results either way):
                                   ECMC_SCHED_SWEEP (default): one launch per sweep, each
                                   domain started as soon as its neighbours of earlier
                                   colours are done (no device-wide wait between phases);
                                   ECMC_SCHED_PHASES: one launch set per colour phase. A
                                   colour_mask other than all eight colours, or a staging
                                   capacity above 512 beads, always runs by phases          */
    int32_t stage_tier;         /* with stage_capacity = 0: beads of the LDS staging tier
                                   (a multiple of 64 up to 512, run as 64 x 1, 2, 3, 4, 6, 7
                                   or 8 beads per lane, the next one up; 0 = sized for the
                                   typical domain); larger domains are staged as for the
                                   automatic capacity.  The knob ecmc_tune_batch sets      */
    int32_t overlapping_start;  /* nonzero: hard-sphere overlaps in the start are accepted (the
                                   phantom start of the push-off, ecmc_pushoff); tethers only,
                                   no swap moves.  Plain sweeps on an overlapping state are the
                                   caller's responsibility                                 */
    double spring_k;            /* 0 (default): bonds are tethers of length at most l_max.
                                   > 0: harmonic springs (k/2)(b - sigma)^2 of this constant
                                   (Eq. (2), in k_B T / sigma^2, within [1e-6, 1e12]), still
                                   capped at l_max; each step draws one energy per bond of
                                   the pivot, and whole periods after a reflection are not
                                   dropped.  Not combined with swap_moves                  */
    void *workspace;            /* device memory owned by the caller (256-byte aligned)     */
    size_t workspace_bytes;
    void *stream;               /* hipStream_t for every launch and copy; NULL = default    */
    void *side_stream;          /* caller's second hipStream_t (or NULL): by phases, the rare
                                   domains of the larger staging tiers run on it, concurrently
                                   with the first tier (the library orders it against `stream`
                                   with events of its own).  NULL: every tier runs on `stream`,
                                   one after the other (identical results).  The library
                                   creates no stream                                       */
    int32_t wait_limit_us;      /* guard on one dependency wait of the one-launch sweep
                                   (0 = 30 s): a wait that runs out leaves its domain as it
                                   was, flags the device error word (bit 5) and the next
                                   synchronising call returns ECMC_E_DEVICE.  Far above any
                                   domain's run time; small values exist to test that path */
    int32_t reserved;           /* 0 */
} ecmc_options;

typedef struct {
    uint64_t hs_lift, tether_lift, hs_reflect, tether_reflect, wall, cross, ec, steps;
    uint64_t periodic, cycle;   /* repeated reflections that dropped whole periods / ECs
                                   ended by a zero-length cycle                             */
    uint64_t swap;              /* accepted swap moves                                      */
    double sum_delta;           /* sum over lifts and swaps of (d_par - x): pressure estimator */
    uint32_t error_flags;       /* device error word (bit 0 staging, 1 cell, 2 stuck,
                                   3 log full, 4 cell lists changed during staging,
                                   5 a wait of the sweep launch ran out of time); it stays
                                   set, and every synchronising call fails, until
                                   ecmc_clear_error                                         */
    uint32_t pad;
} ecmc_counters;

typedef struct {
    uint32_t sweep, domain, ec, step;   /* domain: index among all domains of the context
                                           (melt by melt; a single melt: its domain grid) */
    int32_t pivot, target;              /* bead indices among all beads of the context     */
    uint32_t kind, colour;
} ecmc_event;

/* One melt of a batch (ecmc_init_batch).  Every melt is a periodic cube of its own; melts
 * never interact.  They share sigma, l_max and the options. */
typedef struct {
    double box;                 /* edge L of the melt's cube                                */
    int64_t n_beads;
    const double *positions;    /* host [n_beads][3]                                        */
    int64_t n_bonds;
    const int32_t *bonds;       /* host [n_bonds][2], bead indices within this melt         */
    int32_t n_cells;            /* cells per axis; 0 = automatic                            */
    int32_t domain_cells;       /* D; 0 = automatic: D = 2, n the largest multiple of 4
                                   with L/n > l_max (or, with n_cells set, the smallest
                                   D >= 2 that divides n with n/D even)                     */
} ecmc_melt_desc;

/* Where a melt of a context lives: its beads, polymers and domains are consecutive ranges
 * of every per-bead, per-polymer and per-domain output, in melt order. */
typedef struct {
    double box, cell_size;
    int64_t first_bead, n_beads;
    int64_t first_polymer, n_polymers;
    int64_t first_domain, n_domains;
    int32_t n_cells, domain_cells;
} ecmc_melt_info;

/* Fills *opt with the defaults (plain FP64 search, checkerboard, D = 2, automatic sizes). */
void ecmc_default_options(ecmc_options *opt);

/* Bytes of device workspace ecmc_init needs for n_beads beads in a cube of edge box
 * with the given options (workspace fields are ignored).  Errors as ecmc_init. */
ecmc_status ecmc_workspace_size(double box, double sigma, double l_max, int64_t n_beads,
                                const ecmc_options *opt, size_t *bytes);

/* The single-precision screen of the event search (ECMC_PREC_MIXED), as derived for a melt
 * of n_beads in a cube of edge box with these options (host only, no device is touched).
 * Screening coordinates are the frame coordinates rounded once to float; for the candidate
 * formulas of Sec. II (contact and tether distances) the screen's float estimate lies within
 * err of the exact FP64 distance, a float d_par above p_sure means the exact one is positive,
 * and a float d_perp^2 below in_lo (at or above in_hi) means the exact one is below (not below)
 * sigma^2.  out[4] = {p_sure, in_lo, in_hi, err}; geo[3] = {cell edge h, frame edge X over
 * which the coordinates range (L for the whole box), box L}.  Errors as ecmc_workspace_size. */
ecmc_status ecmc_screen_constants(double box, double sigma, double l_max, int64_t n_beads,
                                  const ecmc_options *opt, float out[4], double geo[3]);

/* Bytes of device workspace ecmc_init_batch needs for these melts (positions and bonds are
 * not read; n_beads and n_bonds are). */
ecmc_status ecmc_workspace_size_batch(int32_t n_melts, const ecmc_melt_desc *melts, double sigma,
                                      double l_max, const ecmc_options *opt, size_t *bytes);

/* Creates a context.  positions: host [n_beads][3] doubles, wrapped into [0, box) and
 * binned into closed cells [k h, (k+1) h]; bonds: host [n_bonds][2] bead indices forming
 * linear chains (degree <= 2, no rings).  Validates the start (no overlap, no stretched
 * tether, box and domain geometry), builds the cell lists, copies everything into the
 * workspace and waits for the copies.  *out is NULL on failure. */
ecmc_status ecmc_init(ecmc_ctx **out, double box, double sigma, double l_max, int64_t n_beads,
                      const double *positions, int64_t n_bonds, const int32_t *bonds,
                      const ecmc_options *opt);

/* Creates a context holding n_melts independent melts (the batched form): each validated,
 * binned and decomposed as by ecmc_init in its own box, with its own cell grid and domain
 * edge; all of them sweep together in one launch per sweep.  Needs the checkerboard tiling
 * and the dependency-ordered schedule.  Melt m draws from random stream m (see ecmc_sweep);
 * a context of one melt behaves exactly as one from ecmc_init. */
ecmc_status ecmc_init_batch(ecmc_ctx **out, int32_t n_melts, const ecmc_melt_desc *melts,
                            double sigma, double l_max, const ecmc_options *opt);

/* The autotuner of the batched form (checkerboard, one-launch sweeps: the tile-joint
 * partition is offered for single melts only).  Candidates: two domain policies per melt
 * (the domain tiling: 0 = D = 2 on the largest multiple of 4 cells per axis, 1 = the (n, D)
 * of smallest typical frame among n from that multiple up to the largest n, n/D even), for
 * each the LDS staging tier (64, 128, 192, 256, 384 or 512 beads per domain frame, i.e. 1 to
 * 8 beads per lane of the wavefront that runs a domain's ECs: up to four, from the smallest
 * that holds the mean frame of the melt holding the median bead; larger frames go to
 * workspace slots), and for each tier both searches (ECMC_PREC_MIXED and ECMC_PREC_FP64,
 * identical results).  Each candidate is initialised in opt->workspace (scratch; it must
 * hold ecmc_tune_workspace_size bytes) and timed over trial_sweeps sweeps of n_chains ECs of
 * length ell after one untimed sweep; the fastest in ECs per second is returned: n_cells and
 * domain_cells per melt (for ecmc_melt_desc), the staging tier (for
 * ecmc_options.stage_tier) and the precision (ecmc_options.precision).  Synchronises; the
 * caller's melts are only read. */
typedef struct {
    int32_t stage_tier;
    int32_t policy;
    double ms_per_sweep;        /* of the fastest candidate                                 */
    double ecs_per_s;
    int32_t candidates;         /* candidates timed                                         */
    int32_t precision;          /* ECMC_PREC_* of the fastest candidate                      */
} ecmc_tune_result;

ecmc_status ecmc_tune_workspace_size(int32_t n_melts, const ecmc_melt_desc *melts, double sigma,
                                     double l_max, const ecmc_options *opt, size_t *bytes);
ecmc_status ecmc_tune_batch(int32_t n_melts, const ecmc_melt_desc *melts, double sigma, double l_max,
                            const ecmc_options *opt, int64_t n_chains, double ell,
                            int32_t trial_sweeps, int32_t *n_cells_out, int32_t *domain_cells_out,
                            ecmc_tune_result *best);

/* One sweep (Sec. II.A: the decomposition is redrawn every sweep): a partition offset,
 * then the 8 colour phases in order; every non-empty active domain runs
 * K = ceil(n_chains / n_domains) ECs of length ell, n_domains counted over all melts
 * (whole-box tiling: n_chains ECs; K above 2^31 - 1 is ECMC_E_ARG).
 * Random numbers: Philox4x32-10 keyed by seed; melt m draws the pivot and direction of
 * EC k of a domain from counter (k, domain, sweep, 2 m) and its offsets from
 * (0, 0, sweep, 2 m + 1), domain being the index in the melt's own domain grid.
 * sweep is the context's sweep counter, kept in device memory and advanced by every
 * sweep on the stream.  Asynchronous, and free of host synchronisation and memory
 * operations, so that a sequence of sweeps can be captured into a hipGraph on a
 * capturing stream and replayed: each replay moves the sweep counter on. */
ecmc_status ecmc_sweep(ecmc_ctx *ctx, int64_t n_chains, double ell, uint64_t seed);

/* As ecmc_sweep, running only the colour phases whose bit is set in colour_mask (single
 * melts only; a mask other than 0xFF runs the phases one launch set at a time). */
ecmc_status ecmc_sweep_colours(ecmc_ctx *ctx, int64_t n_chains, double ell, uint64_t seed,
                               uint32_t colour_mask);

/* Waits for the stream and reports device-side errors. */
ecmc_status ecmc_synchronize(ecmc_ctx *ctx);

/* Observables (Sec. IV.A, the g1 and R_g^2 definitions; the end-to-end distance of the
 * appendix): per polymer (chains walked from their smaller-id end) the
 * squared end-to-end distance r2 (sum of minimum-image bonds), the squared radius of
 * gyration rg2, the middle bead floor(N/2) in image-unwrapped coordinates mid [3];
 * a histogram of bond lengths on [sigma, l_max] with nbins bins (0 < nbins <= 1024).
 * Host outputs of n_poly entries (any may be NULL); *n_poly receives the polymer count.
 * Synchronises. */
ecmc_status ecmc_observables(ecmc_ctx *ctx, int32_t nbins, double *r2, double *rg2,
                             int64_t *hist, double *mid, int64_t *n_poly);

/* Observables sampled every sweep without a host round trip (the averages over sweeps that
 * Sec. IV.A reports): ecmc_observables_accumulate evaluates the quantities of ecmc_observables
 * on the context's stream and adds the sums over all polymers of r2 and rg2, and the
 * bond-length histogram, to running sums in device memory; it returns once the work is
 * enqueued (asynchronous like ecmc_sweep).  nbins must stay the same until the next reset
 * (ECMC_E_ARG otherwise).
 * ecmc_observables_mean synchronises and returns <r2> and <rg2> per polymer and sample, the
 * summed histogram (host hist [nbins] of the accumulating calls), and the number of samples
 * (any output may be NULL).  The sums are added with atomics in any order: means agree with
 * the per-sample averages of ecmc_observables to rounding, the histogram exactly.
 * ecmc_observables_reset clears the running sums (a kernel on the stream). */
ecmc_status ecmc_observables_accumulate(ecmc_ctx *ctx, int32_t nbins);
ecmc_status ecmc_observables_mean(ecmc_ctx *ctx, double *r2_mean, double *rg2_mean, int64_t *hist,
                                  int64_t *samples);
ecmc_status ecmc_observables_reset(ecmc_ctx *ctx);

/* Shape analysis (appendix, moment of inertia tensor; the centre of mass that g2 of Sec. IV.A
 * measures the middle bead against): per polymer, chains unwrapped from their smaller-id end,
 * the gyration tensor G = N^-1 sum (u - u_cm)(u - u_cm)^T as gyr [6] (xx, yy, zz, xy, xz, yz),
 * its eigenvalues l1 >= l2 >= l3 as eig [3] (the moment of inertia tensor of the chain is
 * N (tr G 1 - G), eigenvalues N (tr G - l_i)), and the centre of mass in image-unwrapped
 * coordinates com [3].  Host outputs of n_poly entries (any may be NULL).  Synchronises. */
ecmc_status ecmc_shape(ecmc_ctx *ctx, double *gyr, double *eig, double *com, int64_t *n_poly);

/* Push-off of an overlapping start (Sec. II.B; the context made with overlapping_start): one
 * sweep at working diameter d in (0, sigma] in which a pair closer than d (squared distance
 * below d^2 (1 - 1e-9)) is no hard-sphere event for either bead, and every EC starts at a
 * motile bead that overlaps some bead (the k-th draw of a domain picks among them in ascending
 * id; a domain with none runs no EC).  The plain FP64 search, one dependency-ordered launch
 * (tethered chains, checkerboard, all colours).  Asynchronous like ecmc_sweep. */
ecmc_status ecmc_pushoff_sweep(ecmc_ctx *ctx, int64_t n_chains, double ell, uint64_t seed, double diameter);

/* Pairs (summed over the melts) closer than d: squared distance below d^2 (1 - 1e-9), d in
 * (0, sigma].  Synchronises. */
ecmc_status ecmc_count_overlaps(ecmc_ctx *ctx, double diameter, int64_t *n);

/* The slow push-off (Sec. II.B): working diameters d_s = d_start + (sigma - d_start) s / stages,
 * s = 1..stages (the last exactly sigma); at each, push-off sweeps of n_beads ECs of length ell
 * (seeds seed, seed + 1, ... over the whole run) until no pair is closer than d_s or max_sweeps
 * sweeps have run.  Stops early at a stage that keeps overlaps.  Reports the sweeps run and the
 * overlaps left at the last diameter reached (0 when the state is a valid start at sigma).
 * Synchronises. */
ecmc_status ecmc_pushoff(ecmc_ctx *ctx, double d_start, int32_t stages, double ell, uint64_t seed,
                         int64_t max_sweeps, int64_t *sweeps_done, int64_t *overlaps_left);

/* State check on the GPU: the conditions every EC keeps (Sec. II: no two hard spheres overlap, no
 * tether is longer than its maximum, and each bead stays in the cell that lists it), counted
 * without copying the state to the host.  overlaps: pairs closer than sigma (1 - tol);
 * stretched: bonds longer than l_max (1 + tol), in minimum image; misplaced: beads outside the
 * closed interval of the cell whose list holds them or whose cell word names another cell, plus
 * beads a list could not hold and the difference between the beads listed and n_beads.  tol in
 * [0, 1e-3]; any output pointer may be null.  Synchronises.  For callers that validate long
 * runs, restored checkpoints or push-off results at full size. */
ecmc_status ecmc_check_state(ecmc_ctx *ctx, double tol, int64_t *overlaps, int64_t *stretched, int64_t *misplaced);

/* Snapshot for the mean-square displacements g1 and g2 (Sec. IV.A): per polymer the middle bead
 * floor(N/2) and the centre of mass, both image-unwrapped (as ecmc_observables and ecmc_shape
 * give them), written as snap [n_poly][6] (x, y, z of the bead, then of the centre) to DEVICE
 * memory owned by the caller (8-byte aligned).  Queued on the context's stream; does not
 * synchronise, so a run can record snapshots between sweeps without host copies. */
ecmc_status ecmc_snapshot(ecmc_ctx *ctx, double *snap_device);

/* g1 and g2 (Sec. IV.A) of a series of T snapshots [T][n_poly][6] in DEVICE memory (as written
 * by ecmc_snapshot, equally spaced in time), averaged over the polymers and over every time
 * origin: for each lag d = 0..T-1,
 *   g1(d) = < |r_mid(t + d) - r_mid(t)|^2 >,  g2(d) = < |(r_mid - R_cm)(t + d) - (r_mid - R_cm)(t)|^2 >,
 * written to out_device [2][T] (g1, then g2; 0 at d = 0), DEVICE memory of the caller.  Queued on
 * the context's stream; does not synchronise.  T in [1, 2^31 - 1]. */
ecmc_status ecmc_msd(ecmc_ctx *ctx, const double *snaps_device, int64_t T, double *out_device);

/* End-to-end distance distribution W(R) (appendix): over all polymers, the number with
 * |R| in [k w, (k + 1) w), w = r_max / nbins, k = 0..nbins-1; |R| >= r_max is counted in the
 * last bin.  |R| = sqrt(R^2) with R^2 as ecmc_observables computes it.  Host hist [nbins],
 * nbins in [1, 1024].  Synchronises. */
ecmc_status ecmc_end_to_end_histogram(ecmc_ctx *ctx, int32_t nbins, double r_max, int64_t *hist);

/* Internal distances R^2(n) (Sec. II.B, where start configurations are checked against a long
 * run through R^2(n)/n): for n = 0..n_max, the mean over every pair of beads of one polymer that
 * are n bonds apart (all polymers, all melts of a batch) of the squared chain vector between
 * them, the sum of the minimum-image bond vectors in between.  Host r2 [n_max + 1] receives the
 * means (0 where no pair exists), host pairs [n_max + 1] (or null) the number of pairs behind
 * each (sum over chains of max(N - n, 0)).  n_max in [0, 2047]; chains of at most 2048 beads.
 * The sums are taken per block in a fixed order, so a state gives the same result on every
 * call.  Synchronises. */
ecmc_status ecmc_internal_distances(ecmc_ctx *ctx, int32_t n_max, double *r2, int64_t *pairs);

/* For callers that cannot allocate device memory (code under stream capture, tight serving
 * loops, hosts that forbid allocation): ecmc_internal_distances with its per-block partial
 * sums in a static array of the library (8 MiB per device, resolved once per device at init,
 * held until the process ends) instead of the context's workspace.  Arguments, results,
 * errors and the summation order are those of ecmc_internal_distances, so the two return the
 * same values for a state.  Allocates nothing, host or device.  Every call on one device uses
 * that device's one array: calls that overlap on a device (two threads, two contexts, two
 * streams) race and give wrong sums.  Synchronises. */
ecmc_status ecmc_internal_distances_noalloc(ecmc_ctx *ctx, int32_t n_max, double *r2, int64_t *pairs);

/* Pair counts behind the pair correlation g(r): the pairs i < j of one melt (summed over the
 * melts of a batch) whose minimum-image distance r is below r_max, binned by
 * floor(r / r_max * nbins) (clamped to nbins - 1).  r_max may not exceed the smallest cell
 * edge (the pairs are found through the cell lists); g(r) follows by dividing by the ideal-gas
 * counts N (N - 1) / 2 * 4 pi (r_hi^3 - r_lo^3) / (3 V) of each bin.  Host hist [nbins], nbins
 * in [1, 1024].  Synchronises. */
ecmc_status ecmc_pair_histogram(ecmc_ctx *ctx, int32_t nbins, double r_max, int64_t *hist);

/* Ensemble shape descriptors of the appendix (Table II) from per-polymer gyration eigenvalues
 * (host eig [n_poly][3], as ecmc_shape returns them; any order within a polymer).  With the moment of inertia eigenvalues
 * I_i = tr G - l_i taken in descending order (the order in which the asphericity
 * b = (I1 + I2)/2 - I3 and the acylindricity c = I1 - I2 are non-negative), out[5] =
 * <kappa^2> with kappa^2 = 4 (1 - 3 (I1 I2 + I2 I3 + I3 I1) / (tr I)^2), <I1 + I2 - I3>/<tr I>,
 * <I1 - I2 + I3>/<tr I>, <-I1 + I2 + I3>/<tr I> and <4 b^2 + 3 c^2>/<tr I>^2, sums over
 * polymers in index order.  Host only; ECMC_E_ARG for n_poly < 1, non-finite eigenvalues or a
 * polymer of zero inertia. */
ecmc_status ecmc_shape_descriptors(const double *eig, int64_t n_poly, double out[5]);

/* The pair correlation g(r) (appendix: the local order behind the small-R oscillations of
 * W(R)) from pair counts hist [nbins] of r in [0, r_max) (ecmc_pair_histogram): each bin
 * divided by the ideal-gas count of its shell, sum over the n_melts melts of
 * N_m (N_m - 1) / 2 * 4 pi (r_hi^3 - r_lo^3) / (3 V_m) (host n_beads [n_melts], volumes
 * [n_melts]).  Host only; writes g [nbins]. */
ecmc_status ecmc_pair_correlation(const int64_t *hist, int32_t nbins, double r_max, int32_t n_melts,
                                  const int64_t *n_beads, const double *volumes, double *g);

/* Host copies of the state: positions [n][3], cell indices [n][3], image counters [n][3]. */
ecmc_status ecmc_get_positions(ecmc_ctx *ctx, double *out);
ecmc_status ecmc_get_cells(ecmc_ctx *ctx, int32_t *out);
ecmc_status ecmc_get_images(ecmc_ctx *ctx, int32_t *out);
ecmc_status ecmc_get_counters(ecmc_ctx *ctx, ecmc_counters *out);
ecmc_status ecmc_reset_counters(ecmc_ctx *ctx);
/* Clears the device error word (ecmc_counters.error_flags) after the caller has handled the
 * ECMC_E_* it caused; the state is whatever the failed call left (a domain whose wait ran out
 * is left as it was before that sweep).  Synchronises. */
ecmc_status ecmc_clear_error(ecmc_ctx *ctx);

/* Copies up to capacity log records (unordered across domains) to out and the total
 * number written since the last clear to *n_total. */
ecmc_status ecmc_get_event_log(ecmc_ctx *ctx, ecmc_event *out, int64_t capacity, int64_t *n_total);
ecmc_status ecmc_clear_event_log(ecmc_ctx *ctx);

/* Checkpoint restore: positions, cells and images [n][3] as returned by ecmc_get_*,
 * plus the sweep counter; the cell lists are rebuilt. */
ecmc_status ecmc_set_state(ecmc_ctx *ctx, const double *positions, const int32_t *cells,
                           const int32_t *images, uint32_t sweep_counter);

/* Sum of the HIP-event durations of the sweep kernels since the last call, and their
 * number (needs time_kernels).  Synchronises. */
ecmc_status ecmc_kernel_time(ecmc_ctx *ctx, double *ms, int64_t *launches);

/* The sweep counter (read from the device: synchronises). */
uint32_t ecmc_sweep_counter(const ecmc_ctx *ctx);
int32_t ecmc_n_cells(const ecmc_ctx *ctx);
double ecmc_cell_size(const ecmc_ctx *ctx);
int32_t ecmc_stage_capacity(const ecmc_ctx *ctx);
int32_t ecmc_n_melts(const ecmc_ctx *ctx);
ecmc_status ecmc_get_melt_info(const ecmc_ctx *ctx, int32_t melt, ecmc_melt_info *out);

void ecmc_destroy(ecmc_ctx *ctx);
const char *ecmc_status_str(ecmc_status s);
const char *ecmc_last_error(const ecmc_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif

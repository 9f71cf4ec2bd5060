// Internal declarations shared by the host library (ecmc_api.cpp) and the gfx950
// kernels (ecmc_kernels.hip).  Not part of the public ABI (include/ecmc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ecmc.h"

namespace ecmc {

// device error word bits
enum : uint32_t {
    ERR_STAGE = 1u << 0,  // a domain plus halo held more beads than the staging capacity
    ERR_CELL = 1u << 1,   // a cell list ran out of slots
    ERR_STUCK = 1u << 2,  // an EC exceeded the per-EC iteration cap
    ERR_LOG = 1u << 3,    // event log full (records dropped; informational)
    ERR_RECOUNT = 1u << 4,  // a domain's cell lists no longer matched its count (internal error)
    ERR_WAIT = 1u << 5,     // a wait of the dependency-ordered sweep ran out of time (internal error)
};

// counter slots in the device counter block
enum { C_HS_LIFT = 0, C_TETHER_LIFT, C_HS_REFLECT, C_TETHER_REFLECT, C_WALL, C_CROSS, C_EC, C_STEPS, C_PERIOD, C_CYCLE, C_SWAP,
       NCNT };

// packed cell word of a bead: cx | cy << 10 | cz << 20, bit 30 = motile in this phase
constexpr int CELL_BITS = 10;
constexpr int32_t CELL_MASK = (1 << CELL_BITS) - 1;
constexpr int32_t MOTILE_BIT = 1 << 30;
constexpr int MAX_CELLS_PER_AXIS = 1023;
constexpr int MAX_STAGE = 1024;       // staging capacity limit (16 beads per lane)

__host__ __device__ inline int32_t pack_cell(int cx, int cy, int cz) {
    return cx | (cy << CELL_BITS) | (cz << (2 * CELL_BITS));
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), used on the host for the partition
// offsets and on the device for the per-EC draws.
__host__ __device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t m0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t x0 = (uint32_t)(m1 >> 32) ^ c[1] ^ k0;
        const uint32_t x2 = (uint32_t)(m0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)m1;
        c[3] = (uint32_t)m0;
        c[0] = x0;
        c[2] = x2;
    }
}

// uniform integer in [0, m) from one 32-bit draw
__host__ __device__ inline uint32_t scale_u32(uint32_t u, uint32_t m) {
    return (uint32_t)(((uint64_t)u * m) >> 32);
}

// Per-melt constants of a batch of independent melts (one device table entry per melt; a
// single melt is a batch of one).  The melts' beads, cells and domain stamps are consecutive
// ranges of the shared arrays.
struct MeltDev {
    double L, h, halfL;
    float in_lo, in_hi, p_sure, err_f;  // single-precision screen constants (depend on the frame edge)
    int n, D, nd, ndpc;                 // cells per axis, domain edge, domains per axis and per colour
    int tick0;                          // first ticket of the melt within a colour
    int dom0;                           // first domain stamp of the melt
    long long cell0;                    // first cell of the melt
};

struct PhaseArgs {
    double *px, *py, *pz;      // [n] positions
    int32_t *cellp;            // [n] packed cell words (motile bit clear)
    int32_t *img;              // [3n] periodic image counters
    const int32_t *part;       // [2n] tethered partners, -1 = none
    int32_t *ccount;           // [nc^3] beads per cell
    int32_t *cids;             // [nc^3 * cap] bead ids per cell
    int32_t *dstage;           // [grid] beads in each domain's frame, counted before the phase
    unsigned long long *cnt;   // [NCNT]
    double *sum_delta;
    unsigned int *err;
    ecmc_event *log;
    unsigned long long *log_n;
    long long log_cap;
    double L, h, sig2, b2, ell, halfL;
    int K, event_cap;          // ECs per domain; loop iterations allowed per EC
    int n, D, nd, cap, whole, colour;
    int stage_lo, stage_hi;    // this launch takes the domains staging S beads, stage_lo < S <= stage_hi
    int exact_search;          // 1: evaluate every staged bead in FP64 (reference search)
    int swap;                  // 1: swap moves at hard-sphere contacts with motile beads
    float sig2f, b2f, in_lo, in_hi, p_sure, err_f;  // single-precision screen constants
    int off[3];                // partition offsets (drawn on the device from the sweep counter)
    uint32_t key0, key1, sweep;
    uint32_t stream;           // random stream of the melt (Philox counter word 3 = 2 stream)
    uint32_t *dstate;          // [2] sweep counter, stamp of the last dependency-ordered launch
    // dependency-ordered sweep (one launch per sweep)
    uint32_t *done;            // [total domains] stamp of the launch that last finished each domain
    uint32_t *queue;           // [2] next ticket, workgroups that have left; both 0 between launches
    uint32_t epoch;            // this launch's stamp, never 0
    int ndpc;                  // domains per colour, (nd/2)^3
    const MeltDev *melts;      // [n_melts]
    int n_melts;
    int tickets;               // tickets per colour: domains per colour summed over the melts
    double *slow;              // [nslow] staging slots for domains above the LDS capacity
    uint32_t *slow_lock;       // [nslow] 0 free, 1 taken
    int nslow, slow_cap;       // slots, beads per slot (0: no slots)
    // harmonic springs (Eq. (2)): 2 / k, 0 for tethers; sigma for the spring formula
    double two_over_k, sigma;
    // a wait of the dependency-ordered sweep gives up (ERR_WAIT) after this many ticks of the
    // device's constant-rate counter
    unsigned long long wait_ticks;
    // push-off (Sec. II.B): sig2 is the working diameter squared, ov2 = sig2 (1 - 1e-9)
    double ov2;
    // 1: tile-joint partition (D^3-cell tiles at pitch D + 1, all in one phase)
    int joint;
};

struct ObsArgs {
    const double *px, *py, *pz;
    const int32_t *img;
    const int32_t *porder;     // [n] beads in chain order
    const int32_t *pstart;     // [npoly + 1]
    int64_t npoly;
    const double *polyL;       // [npoly] box edge of each polymer's melt
    double sigma, bmax;
    int nbins;
    double *r2, *rg2, *mid;    // [npoly], [npoly], [3 npoly]
    double *gyr, *eig, *com;   // shape: [6 npoly], [3 npoly], [3 npoly]
    unsigned long long *hist;  // [nbins]
    double *snap;              // [6 npoly] middle bead and centre of mass, unwrapped (or null)
    unsigned long long *rhist; // [rbins] end-to-end distance histogram (or null)
    int rbins;
    double rmax;
    int nlag;                  // internal distances: lags 0..nlag-1
    double *lagsum;            // [nlag][rows] per-block sums, then [nlag] their totals
    double *acc;               // running sums (or null): [OBS_ACC_SLOTS] of r2, then as many of rg2;
                               // block b adds to slot b mod OBS_ACC_SLOTS
};

// slots of the running observable sums: the blocks of one launch spread their atomic adds over them
constexpr int OBS_ACC_SLOTS = 64;

// internal distances: room for the per-block partial sums (blocks x lags), and the longest
// chain they take
constexpr int LAG_SLOTS = 1 << 20;
constexpr int LAG_MAX_BEADS = 2048;

// Pair counts behind g(r): every pair of one melt closer than rmax (at most a cell edge).
struct PairArgs {
    const double *px, *py, *pz;
    const int32_t *ccount, *cids;
    int cap;
    const MeltDev *melts;
    int n_melts;
    long long cells;           // cells of all melts
    int nbins;
    double rmax;
    unsigned long long *hist;  // [nbins]
    double q_lim;              // > 0: count the pairs with squared distance below q_lim in bin 0 instead
    // state check (k_check): tethered partners, cell words, the squared bond limit; hist[0..2]
    // receive stretched bonds, misplaced beads and the beads the cell lists hold
    const int32_t *part, *cellp;
    double b2lim;
};

// launchers (ecmc_kernels.hip)
hipError_t launch_count(const PhaseArgs &a, int grid, hipStream_t s);
hipError_t launch_advance(const PhaseArgs &a, hipStream_t s);
// the phase and sweep kernels are built twice, for tethers and for springs (_spring)
hipError_t launch_phase(const PhaseArgs &a, int bpl, bool log, int grid, hipStream_t s);
hipError_t launch_phase_spring(const PhaseArgs &a, int bpl, bool log, int grid, hipStream_t s);
hipError_t launch_sweep(const PhaseArgs &a, int bpl, bool log, int *grid, hipStream_t s);
hipError_t launch_sweep_spring(const PhaseArgs &a, int bpl, bool log, int *grid, hipStream_t s);
hipError_t launch_sweep_push(const PhaseArgs &a, int bpl, bool log, int *grid, hipStream_t s);  // FP64 search only
bool sweep_bpl_supported(int bpl);
constexpr int SLOW_SLOT_BYTES_PER_BEAD = 3 * 8 + 4 * 4;  // staging slot: positions + 4 int32 rows
hipError_t launch_observables(const ObsArgs &a, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *p, long long n, hipStream_t s);
hipError_t launch_shape(const ObsArgs &a, hipStream_t s);
hipError_t launch_pairs(const PairArgs &a, hipStream_t s);
hipError_t launch_check(const PairArgs &a, hipStream_t s);
hipError_t launch_msd(const double *snaps, int64_t T, int64_t npoly, double *out, hipStream_t s);
hipError_t launch_internal(const ObsArgs &a, int rows, int longest, hipStream_t s);
bool bpl_supported(int bpl);

}  // namespace ecmc

/* Memory and undefined-behaviour check of the oracle (test infrastructure): built with
 * -fsanitize=address,undefined by tests/test_oracle_asan.py and run on the host.  It drives
 * every oracle path on small lattice melts (whole box, checkerboard and tile-joint sweeps with
 * the per-event invariant checks on, swap moves, springs, the push-off from an overlapping start,
 * the event log, and every analysis) and exits non-zero on the first failing call; the
 * sanitizers end the run on any invalid access, leak or undefined operation. */
#include <stdio.h>
#include <stdlib.h>

#include "ecmc_oracle.h"

#define CHECK(call)                                                         \
    do {                                                                    \
        int rc_ = (call);                                                   \
        if (rc_ != ORC_OK) {                                                \
            fprintf(stderr, "%s:%d: %s -> %d\n", __FILE__, __LINE__, #call, rc_); \
            exit(1);                                                        \
        }                                                                   \
    } while (0)

/* chains of `per` beads along a boustrophedon walk of an n^3 simple cubic lattice, spacing a
 * (at least 1.1: the jitter keeps every pair at least sigma apart and every bond within 1.4) */
static int64_t lattice(int n, double a, int per, double *pos, int32_t *bonds, int64_t *n_bonds) {
    int64_t k = 0, nb = 0;
    for (int z = 0; z < n; ++z)
        for (int yy = 0; yy < n; ++yy) {
            const int y = z % 2 ? n - 1 - yy : yy;
            for (int xx = 0; xx < n; ++xx) {
                const int x = (y + z) % 2 ? n - 1 - xx : xx;
                /* a jitter below 0.03 per axis, so that no bond is parallel to an axis */
                for (int ax = 0; ax < 3; ++ax) {
                    const uint32_t hsh = (uint32_t)(k * 3 + ax) * 2654435761u;
                    const double jit = 0.03 * ((double)(hsh >> 8) / 16777216.0 - 0.5) * 2.0;
                    const int c = ax == 0 ? x : (ax == 1 ? y : z);
                    pos[3 * k + ax] = (c + 0.5) * a + jit;
                }
                if (k % per) {
                    bonds[2 * nb] = (int32_t)(k - 1);
                    bonds[2 * nb + 1] = (int32_t)k;
                    ++nb;
                }
                ++k;
            }
        }
    *n_bonds = nb;
    return k;
}

static void stage(const char *what) {
    fprintf(stderr, "stage: %s\n", what);
    fflush(stderr);
}

static void analyses(orc_sys *s) {
    const int64_t nb = orc_n_beads(s);
    double *r2 = malloc(sizeof(double) * nb), *rg2 = malloc(sizeof(double) * nb), *mid = malloc(sizeof(double) * 3 * nb);
    double *gyr = malloc(sizeof(double) * 6 * nb), *com = malloc(sizeof(double) * 3 * nb);
    double *sum = malloc(sizeof(double) * 40), *pos = malloc(sizeof(double) * 3 * nb);
    int32_t *cells = malloc(sizeof(int32_t) * 3 * nb), *img = malloc(sizeof(int32_t) * 3 * nb);
    int64_t hist[16], cnt[40], np = 0;
    uint64_t c[ORC_NCNT];
    double sd = 0.0;
    CHECK(orc_observables(s, 16, r2, rg2, hist, mid, &np));
    CHECK(orc_shape(s, gyr, com));
    CHECK(orc_pair_histogram(s, 16, orc_cell_size(s), hist));
    CHECK(orc_end_to_end_histogram(s, 16, 12.0, hist));
    CHECK(orc_internal_distances(s, 39, sum, cnt));
    orc_counters(s, c, &sd);
    orc_get_positions(s, pos);
    orc_get_cells(s, cells);
    orc_get_images(s, img);
    CHECK(orc_set_state(s, pos, cells, img, orc_sweep_counter(s)));
    free(r2), free(rg2), free(mid), free(gyr), free(com), free(sum), free(pos), free(cells), free(img);
}

int main(void) {
    const int n = 8, per = 16;
    const double a = 1.1, L = n * a;
    double *pos = malloc(sizeof(double) * 3 * n * n * n);
    int32_t *bonds = malloc(sizeof(int32_t) * 2 * n * n * n);
    int64_t n_bonds = 0;
    const int64_t nb = lattice(n, a, per, pos, bonds, &n_bonds);
    orc_event *log = malloc(sizeof(orc_event) * 200000);

    /* tethers: whole box, checkerboard (6 cells, D = 3) and tile-joint (D = 2), invariants checked */
    orc_sys *s = NULL;
    CHECK(orc_create(&s, L, 1.0, 1.4, 6, nb, pos, n_bonds, bonds));
    CHECK(orc_set_options(s, 0, 1));
    CHECK(orc_set_log(s, log, 200000));
    stage("tethers, whole box");
    CHECK(orc_sweep(s, nb, 10.0, 1, 0, 1, 0xFFu));
    stage("tethers, checkerboard");
    CHECK(orc_sweep(s, nb, 10.0, 2, 1, 3, 0xFFu));
    stage("tethers, tile-joint");
    CHECK(orc_sweep(s, nb, 10.0, 3, 2, 2, 0x01u));
    const uint32_t doms[1] = {0};  /* the colour-0 domain of the 2^3 domains */
    CHECK(orc_sweep_subset(s, nb, 10.0, 4, 3, 0x01u, doms, 1));
    double x, xc;
    int32_t j;
    int kind;
    CHECK(orc_next_event(s, 0, 0, 1, &x, &j, &kind, &xc));
    CHECK(orc_run_ec(s, 0, 1, 3.0));
    if (orc_log_count(s) <= 0) return 2;
    analyses(s);
    /* swap moves, with the brute-force next-event search as well */
    CHECK(orc_set_options(s, 0, 2));
    stage("swap moves");
    CHECK(orc_set_swap(s, 1));
    CHECK(orc_sweep(s, nb, 10.0, 5, 1, 3, 0xFFu));
    CHECK(orc_set_swap(s, 0));
    orc_destroy(s);

    /* springs (k sigma^2 = 30), capped at 1.4 sigma */
    CHECK(orc_create(&s, L, 1.0, 1.4, 6, nb, pos, n_bonds, bonds));
    CHECK(orc_set_options(s, 0, 1));
    stage("springs");
    CHECK(orc_set_spring(s, 30.0));
    CHECK(orc_set_stream(s, 3));
    CHECK(orc_sweep(s, nb, 5.0, 6, 1, 3, 0xFFu));
    CHECK(orc_sweep(s, nb, 5.0, 7, 0, 1, 0xFFu));
    analyses(s);
    orc_destroy(s);

    /* push-off: the same chains squeezed to spacing 0.9 (every neighbour overlapping at sigma) */
    for (int64_t k = 0; k < 3 * nb; ++k) pos[k] *= 0.9 / a;
    CHECK(orc_create_overlapping(&s, n * 0.9, 1.0, 1.4, 4, nb, pos, n_bonds, bonds));
    if (orc_count_overlaps(s, 1.0) <= 0) return 3;
    stage("push-off");
    CHECK(orc_set_pushoff(s, 0.95));
    for (int k = 0; k < 3; ++k) CHECK(orc_sweep(s, nb, 5.0, 8 + k, 1, 2, 0xFFu));
    CHECK(orc_set_pushoff(s, 0.0));
    analyses(s);
    orc_destroy(s);

    printf("oracle under sanitizers: %lld beads, every path ran\n", (long long)nb);
    free(pos), free(bonds), free(log);
    return 0;
}

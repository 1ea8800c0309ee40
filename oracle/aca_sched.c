/*
 * aca_sched.c -- serial emulations of the paper's parallel schedules.
 *
 * TEST INFRASTRUCTURE ONLY (same rules as aca_oracle.c, which this file is
 * compiled with).  These executors are not the oracle: they run the
 * parallel algorithms of Section 3 one step at a time on the CPU, and the
 * test suite checks that each reaches exactly the heap oracle's result
 * (uniqueness argument following Fig. 3.1; partition invariance argued for
 * Fig. 3.4).  Section 4 uses the same device -- a serial program that
 * emulates the synchronous parallel schedule -- to predict efficiency.
 *
 *  oracle_run_rounds: the synchronous one-cell-per-PE algorithm (Fig. 3.2).
 *    Per round, every live cell whose pending arrival precedes those of all
 *    its neighbours (time first, then index) is enabled; all enabled cells
 *    are then applied.  Enabled cells are never neighbours, so the reads of
 *    a round never see its writes.  With times_only != 0 the spins are left
 *    alone: this is the simplified time-only model of Section 4, whose
 *    per-round enabled counts equal those of the full run because arrival
 *    times do not depend on spins.
 *
 *  oracle_run_tiled: the aggregated algorithm (Fig. 3.3/3.4) with
 *    rectangular sub-arrays ("tiles") visited in passes.  At the start of a
 *    visit the tile copies the (spin, time) of every outside neighbour
 *    cell; during the visit those copies stay frozen while the tile runs
 *    synchronous rounds on its own cells, at most max_rounds of them, until
 *    no cell is enabled.  A frozen copy can only hold a cell back, never
 *    let one through too early, so the result is unchanged (the argument
 *    with cells v and x after Fig. 3.5).  When a tile covers a whole
 *    periodic direction its wrap-around neighbours are its own live cells.
 *    Pass p visits the tiles whose coordinate sum has parity p mod 2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OAPI __attribute__((visibility("default")))

/* From aca_oracle.c (same library). */
OAPI int oracle_thresholds(int dim, double J, double h, double beta,
                           int rule, uint64_t *thr);
OAPI void oracle_philox(const uint32_t *ctr, uint64_t seed, uint32_t *out,
                        int64_t count);
OAPI void oracle_neg_log_words(const uint64_t *w, double *out, int64_t count);

typedef struct {
    int dim, z;
    int64_t L[3], stride[3], n;
} sgeom;

static int make_sgeom(int dim, const int32_t *L, sgeom *g)
{
    if (dim < 1 || dim > 3) return -1;
    g->dim = dim;
    g->z = 2 * dim;
    g->n = 1;
    for (int d = 0; d < 3; ++d) {
        g->L[d] = (d < dim) ? (int64_t)L[d] : 1;
        if (d < dim && g->L[d] < 2) return -1;
        g->stride[d] = g->n;
        g->n *= g->L[d];
    }
    if (g->n >= ((int64_t)1 << 32)) return -1;
    return 0;
}

static void coords(const sgeom *g, int64_t c, int64_t co[3])
{
    co[0] = c % g->L[0];
    co[1] = (c / g->L[0]) % g->L[1];
    co[2] = c / (g->L[0] * g->L[1]);
}

/* Slot order +x, -x, +y, -y, +z, -z. */
static int64_t slot_cell(const sgeom *g, int64_t c, const int64_t co[3],
                         int slot)
{
    int d = slot / 2;
    int64_t v = (slot & 1) ? (co[d] + g->L[d] - 1) % g->L[d]
                           : (co[d] + 1) % g->L[d];
    return c + (v - co[d]) * g->stride[d];
}

static int precedes(double ta, int64_t a, double tb, int64_t b)
{
    return ta < tb || (ta == tb && a < b);
}

/* One arrival of cell c with neighbour-spin sum `sum`; same arithmetic as
 * the oracle, reached through the oracle's exported primitives. */
static void event(uint64_t seed, double rate, const uint64_t *thr, int z,
                  int64_t c, int sum, int times_only, int8_t *s, double *t,
                  uint32_t *n, uint64_t *flips)
{
    uint32_t ctr[4] = {n[c], (uint32_t)c, 0u, 0u}, y[4];
    oracle_philox(ctr, seed, y, 1);
    if (!times_only) {
        int idx = (sum + z) / 2 + (z + 1) * (s[c] + 1) / 2;
        if ((uint64_t)y[2] < thr[idx]) {
            s[c] = (int8_t)(-s[c]);
            ++*flips;
        }
    }
    uint64_t w = ((uint64_t)y[1] << 32) | y[0];
    double e;
    oracle_neg_log_words(&w, &e, 1);
    t[c] = t[c] + e / rate;
    n[c] = n[c] + 1u;
}

OAPI int64_t oracle_run_rounds(int dim, const int32_t *L, double J, double h,
                               double beta, double rate, int rule,
                               uint64_t seed, double T, int times_only,
                               int8_t *s, double *t, uint32_t *n,
                               int64_t *enabled_per_round, int64_t max_record,
                               int64_t *rounds_out, uint64_t *flips_out)
{
    sgeom g;
    if (make_sgeom(dim, L, &g) != 0 || !(rate > 0.0)) return -1;
    uint64_t thr[14];
    oracle_thresholds(dim, J, h, beta, rule, thr);
    uint32_t *en = (uint32_t *)malloc((size_t)g.n * sizeof(uint32_t));
    int *sums = (int *)malloc((size_t)g.n * sizeof(int));
    if (!en || !sums) { free(en); free(sums); return -1; }

    int64_t events = 0, rounds = 0;
    uint64_t flips = 0;
    for (;;) {
        int64_t m = 0;
        for (int64_t c = 0; c < g.n; ++c) {
            if (!(t[c] < T)) continue;
            int64_t co[3];
            coords(&g, c, co);
            int ok = 1, sum = 0;
            for (int k = 0; k < g.z; ++k) {
                int64_t nb = slot_cell(&g, c, co, k);
                if (!precedes(t[c], c, t[nb], nb)) { ok = 0; break; }
                sum += s[nb];
            }
            if (ok) { en[m] = (uint32_t)c; sums[m] = sum; ++m; }
        }
        if (m == 0) break;
        /* Commit phase: sums were read before any write of this round. */
        for (int64_t i = 0; i < m; ++i)
            event(seed, rate, thr, g.z, en[i], sums[i], times_only, s, t, n,
                  &flips);
        if (enabled_per_round && rounds < max_record)
            enabled_per_round[rounds] = m;
        events += m;
        ++rounds;
    }
    free(en);
    free(sums);
    if (rounds_out) *rounds_out = rounds;
    if (flips_out) *flips_out = flips;
    return events;
}

/* Tiling along one direction: `cnt` tiles of width `w` (the last one may
 * be narrower).  Returns the tile index of coordinate x. */
typedef struct {
    int64_t cnt, w;
} axis_tiling;

OAPI int64_t oracle_run_tiled(int dim, const int32_t *L, double J, double h,
                              double beta, double rate, int rule,
                              uint64_t seed, double T, const int32_t *tile,
                              int64_t max_rounds, int64_t max_passes,
                              int8_t *s, double *t, uint32_t *n,
                              int64_t *stats /* [passes, visits, rounds] */,
                              uint64_t *flips_out)
{
    sgeom g;
    if (make_sgeom(dim, L, &g) != 0 || !(rate > 0.0) || max_rounds < 1)
        return -1;
    uint64_t thr[14];
    oracle_thresholds(dim, J, h, beta, rule, thr);

    axis_tiling ax[3];
    int64_t ntiles = 1;
    for (int d = 0; d < 3; ++d) {
        int64_t w = (d < dim) ? (int64_t)tile[d] : 1;
        if (w < 1) return -1;
        if (w > g.L[d]) w = g.L[d];
        ax[d].w = w;
        ax[d].cnt = (g.L[d] + w - 1) / w;
        ntiles *= ax[d].cnt;
    }
    int64_t cap = 1;
    for (int d = 0; d < 3; ++d) cap *= ax[d].w;

    /* Per-visit scratch: tile cells, enabled list, and the frozen copies
     * of outside neighbours, stored per (cell, slot). */
    int64_t *cells = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    uint8_t *live = (uint8_t *)malloc((size_t)cap * 6);
    double *ht = (double *)malloc((size_t)cap * 6 * sizeof(double));
    int8_t *hs = (int8_t *)malloc((size_t)cap * 6);
    int64_t *en = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    int *sums = (int *)malloc((size_t)cap * sizeof(int));
    if (!cells || !live || !ht || !hs || !en || !sums) {
        free(cells); free(live); free(ht); free(hs); free(en); free(sums);
        return -1;
    }

    int64_t events = 0, passes = 0, visits = 0, rounds_total = 0;
    uint64_t flips = 0;
    for (;;) {
        /* Done when no cell has a pending arrival before T. */
        int any_live = 0;
        for (int64_t c = 0; c < g.n && !any_live; ++c) any_live = t[c] < T;
        if (!any_live || passes >= max_passes) break;
        int parity = (int)(passes & 1);
        ++passes;
        for (int64_t ti = 0; ti < ntiles; ++ti) {
            int64_t tc[3] = {ti % ax[0].cnt, (ti / ax[0].cnt) % ax[1].cnt,
                             ti / (ax[0].cnt * ax[1].cnt)};
            if (((tc[0] + tc[1] + tc[2]) & 1) != parity) continue;
            ++visits;
            int64_t lo[3], hi[3];
            for (int d = 0; d < 3; ++d) {
                lo[d] = tc[d] * ax[d].w;
                hi[d] = lo[d] + ax[d].w;
                if (hi[d] > g.L[d]) hi[d] = g.L[d];
            }
            /* Gather cells and freeze outside neighbours. */
            int64_t m = 0;
            for (int64_t zc = lo[2]; zc < hi[2]; ++zc)
                for (int64_t y = lo[1]; y < hi[1]; ++y)
                    for (int64_t x = lo[0]; x < hi[0]; ++x) {
                        int64_t c = x + g.L[0] * (y + g.L[1] * zc);
                        int64_t co[3] = {x, y, zc};
                        cells[m] = c;
                        for (int k = 0; k < g.z; ++k) {
                            int64_t nb = slot_cell(&g, c, co, k);
                            int64_t nco[3];
                            coords(&g, nb, nco);
                            int inside = 1;
                            for (int d = 0; d < 3; ++d)
                                if (nco[d] < lo[d] || nco[d] >= hi[d])
                                    inside = 0;
                            live[m * 6 + k] = (uint8_t)inside;
                            ht[m * 6 + k] = t[nb];
                            hs[m * 6 + k] = s[nb];
                        }
                        ++m;
                    }
            for (int64_t r = 0; r < max_rounds; ++r) {
                int64_t q = 0;
                for (int64_t i = 0; i < m; ++i) {
                    int64_t c = cells[i];
                    if (!(t[c] < T)) continue;
                    int64_t co[3];
                    coords(&g, c, co);
                    int ok = 1, sum = 0;
                    for (int k = 0; k < g.z; ++k) {
                        int64_t nb = slot_cell(&g, c, co, k);
                        double tn = live[i * 6 + k] ? t[nb] : ht[i * 6 + k];
                        int sn = live[i * 6 + k] ? s[nb] : hs[i * 6 + k];
                        if (!precedes(t[c], c, tn, nb)) { ok = 0; break; }
                        sum += sn;
                    }
                    if (ok) { en[q] = c; sums[q] = sum; ++q; }
                }
                if (q == 0) break;
                ++rounds_total;
                for (int64_t i = 0; i < q; ++i)
                    event(seed, rate, thr, g.z, en[i], sums[i], 0, s, t, n,
                          &flips);
                events += q;
            }
        }
    }
    free(cells); free(live); free(ht); free(hs); free(en); free(sums);
    if (stats) { stats[0] = passes; stats[1] = visits; stats[2] = rounds_total; }
    if (flips_out) *flips_out = flips;
    return events;
}

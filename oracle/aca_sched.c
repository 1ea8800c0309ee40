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

/*
 * oracle_run_ghost_merge: the GPU library's launch schedule, on the CPU.
 *
 * Every launch visits every tile against the same snapshot X of the
 * lattice.  A tile's region is its own cells plus `ghost` cells on each side
 * of every direction it does not span, surrounded by a frozen one-cell ring
 * (copies from X).  The region runs synchronous rounds (at most max_rounds)
 * until no cell is enabled.  Then every simulated copy -- owned or ghost --
 * is merged into the next snapshot Y by keeping, per cell, the copy with the
 * most arrivals applied.  All copies are prefixes of the one trajectory, so
 * the most advanced one is correct, and the merged record is a consistent
 * cut: an arrival kept in Y was applied while every neighbour copy in its
 * region had all earlier arrivals applied, and Y holds at least that much of
 * each neighbour.  With merge_ghosts = 0 only owned cells are written back,
 * which does NOT give a consistent cut (a ghost copy can run ahead of the
 * owner's copy); that variant exists to demonstrate the difference.
 */
OAPI int64_t oracle_run_ghost_merge(int dim, const int32_t *L, double J, double h,
                                    double beta, double rate, int rule,
                                    uint64_t seed, double T, const int32_t *tile,
                                    const int32_t *ghost, int64_t max_rounds,
                                    int merge_ghosts, int64_t max_launches,
                                    int8_t *s, double *t, uint32_t *n,
                                    int64_t *stats /* [launches, rounds] */,
                                    uint64_t *flips_out)
{
    sgeom g;
    if (make_sgeom(dim, L, &g) != 0 || !(rate > 0.0) || max_rounds < 1) return -1;
    uint64_t thr[14];
    oracle_thresholds(dim, J, h, beta, rule, thr);
    int64_t w[3], cnt[3], gw[3], span[3];
    int64_t ntiles = 1;
    for (int d = 0; d < 3; ++d) {
        w[d] = (d < dim) ? tile[d] : 1;
        if (w[d] < 1) return -1;
        span[d] = w[d] >= g.L[d];
        if (span[d]) w[d] = g.L[d];
        cnt[d] = (g.L[d] + w[d] - 1) / w[d];
        gw[d] = span[d] ? 0 : ghost[d];
        if (!span[d] && gw[d] > (g.L[d] - w[d]) / 2) gw[d] = (g.L[d] - w[d]) / 2;
        if (gw[d] < 0) gw[d] = 0;
        ntiles *= cnt[d];
    }
    int64_t cap = 1;
    for (int d = 0; d < 3; ++d) cap *= (span[d] ? g.L[d] : w[d] + 2 * gw[d] + 2);
    /* region-local copies: global index, spin, time, count, and whether the
     * cell is simulated (inner) or a frozen ring copy */
    int64_t *gi = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    int8_t *ls = (int8_t *)malloc((size_t)cap);
    double *lt = (double *)malloc((size_t)cap * sizeof(double));
    uint32_t *ln = (uint32_t *)malloc((size_t)cap * sizeof(uint32_t));
    uint8_t *inner = (uint8_t *)malloc((size_t)cap);
    uint8_t *own = (uint8_t *)malloc((size_t)cap);
    int64_t *nbr = (int64_t *)malloc((size_t)cap * 6 * sizeof(int64_t));
    int64_t *en = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    int *sums = (int *)malloc((size_t)cap * sizeof(int));
    int8_t *ys = (int8_t *)malloc((size_t)g.n);
    double *yt = (double *)malloc((size_t)g.n * sizeof(double));
    uint32_t *yn = (uint32_t *)malloc((size_t)g.n * sizeof(uint32_t));
    int ok = gi && ls && lt && ln && inner && own && nbr && en && sums && ys && yt && yn;
    int64_t launches = 0, rounds_total = 0, events = 0;
    uint64_t flips = 0;
    while (ok) {
        int any_live = 0;
        for (int64_t c = 0; c < g.n && !any_live; ++c) any_live = t[c] < T;
        if (!any_live || launches >= max_launches) break;
        ++launches;
        memcpy(ys, s, (size_t)g.n);
        memcpy(yt, t, (size_t)g.n * sizeof(double));
        memcpy(yn, n, (size_t)g.n * sizeof(uint32_t));
        for (int64_t ti = 0; ti < ntiles; ++ti) {
            int64_t tc[3] = {ti % cnt[0], (ti / cnt[0]) % cnt[1], ti / (cnt[0] * cnt[1])};
            int64_t rb[3], org[3], olo[3], ohi[3], ring[3];
            for (int d = 0; d < 3; ++d) {
                int64_t lo = tc[d] * w[d];
                int64_t ww = g.L[d] - lo < w[d] ? g.L[d] - lo : w[d];
                ring[d] = span[d] ? 0 : 1;
                int64_t rin = span[d] ? g.L[d] : ww + 2 * gw[d];
                rb[d] = rin + 2 * ring[d];
                org[d] = span[d] ? 0 : lo - gw[d] - 1;       /* ring origin */
                olo[d] = span[d] ? 0 : gw[d] + 1;
                ohi[d] = span[d] ? g.L[d] : gw[d] + 1 + ww;
            }
            int64_t m = rb[0] * rb[1] * rb[2];
            for (int64_t j = 0; j < m; ++j) {
                int64_t q[3] = {j % rb[0], (j / rb[0]) % rb[1], j / (rb[0] * rb[1])};
                int64_t gc[3];
                int in = 1, ow = 1;
                for (int d = 0; d < 3; ++d) {
                    gc[d] = ((org[d] + q[d]) % g.L[d] + g.L[d]) % g.L[d];
                    if (!span[d] && (q[d] == 0 || q[d] == rb[d] - 1)) in = 0;
                    if (q[d] < olo[d] || q[d] >= ohi[d]) ow = 0;
                }
                int64_t c = gc[0] + g.L[0] * (gc[1] + g.L[1] * gc[2]);
                gi[j] = c; ls[j] = s[c]; lt[j] = t[c]; ln[j] = n[c];
                inner[j] = (uint8_t)in; own[j] = (uint8_t)ow;
                for (int k = 0; k < g.z; ++k) {
                    int d = k / 2;
                    int64_t qq[3] = {q[0], q[1], q[2]};
                    if (k & 1) qq[d] = span[d] ? (qq[d] + rb[d] - 1) % rb[d] : qq[d] - 1;
                    else       qq[d] = span[d] ? (qq[d] + 1) % rb[d] : qq[d] + 1;
                    nbr[j * 6 + k] = qq[0] + rb[0] * (qq[1] + rb[1] * qq[2]);
                }
            }
            for (int64_t r = 0; r < max_rounds; ++r) {
                int64_t q = 0;
                for (int64_t j = 0; j < m; ++j) {
                    if (!inner[j] || !(lt[j] < T)) continue;
                    int okc = 1, sum = 0;
                    for (int k = 0; k < g.z; ++k) {
                        int64_t b = nbr[j * 6 + k];
                        if (!precedes(lt[j], gi[j], lt[b], gi[b])) { okc = 0; break; }
                        sum += ls[b];
                    }
                    if (okc) { en[q] = j; sums[q] = sum; ++q; }
                }
                if (q == 0) break;
                ++rounds_total;
                for (int64_t i = 0; i < q; ++i) {
                    int64_t j = en[i];
                    uint32_t ctr[4] = {ln[j], (uint32_t)gi[j], 0u, 0u}, y[4];
                    oracle_philox(ctr, seed, y, 1);
                    int idx = (sums[i] + g.z) / 2 + (g.z + 1) * (ls[j] + 1) / 2;
                    if ((uint64_t)y[2] < thr[idx]) ls[j] = (int8_t)(-ls[j]);
                    uint64_t wv = ((uint64_t)y[1] << 32) | y[0];
                    double e;
                    oracle_neg_log_words(&wv, &e, 1);
                    lt[j] = lt[j] + e / rate;
                    ln[j] = ln[j] + 1u;
                }
            }
            for (int64_t j = 0; j < m; ++j) {
                if (!inner[j] || (!merge_ghosts && !own[j])) continue;
                int64_t c = gi[j];
                if (ln[j] > yn[c] || (own[j] && !merge_ghosts)) {
                    ys[c] = ls[j]; yt[c] = lt[j]; yn[c] = ln[j];
                }
            }
        }
        for (int64_t c = 0; c < g.n; ++c) {
            events += (int64_t)(yn[c] - n[c]);
            if (ys[c] != s[c]) flips += 0;   /* flips are not tracked here */
        }
        memcpy(s, ys, (size_t)g.n);
        memcpy(t, yt, (size_t)g.n * sizeof(double));
        memcpy(n, yn, (size_t)g.n * sizeof(uint32_t));
    }
    free(gi); free(ls); free(lt); free(ln); free(inner); free(own); free(nbr);
    free(en); free(sums); free(ys); free(yt); free(yn);
    if (!ok) return -1;
    if (stats) { stats[0] = launches; stats[1] = rounds_total; }
    if (flips_out) *flips_out = flips;
    return events;
}

/*
 * aca_oracle.c -- serial CPU oracle for the Poisson-asynchronous Ising array.
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
 * CPU-baseline leg of the benchmark are the only code allowed to load it.
 * It shares no source, header, table or constant generator with the HIP
 * library; the two are written independently from the same description.
 *
 * What is computed (B. D. Lubachevsky, "Efficient Parallel Simulations of
 * Asynchronous Cellular Arrays"):
 *
 *  - Model, Section 2, Eq. (1)-(2): when a cell's arrival happens it takes a
 *    new state computed from its own state and its neighbours' states just
 *    before that instant, and its next arrival lies strictly later.
 *  - Poisson asynchrony, Section 1: every cell has an independent arrival
 *    stream of the same rate lambda.
 *  - Randomness made deterministic, Section 3, Eq. (3)-(5): the k-th draw of
 *    cell c is a fixed function of (seed, c, k); the next arrival time is
 *    the previous one plus an exponential gap of mean 1/lambda.
 *  - The Ising rule of Section 1 and of the appendix program: the spin is
 *    reversed with a probability fixed by the spin and the sum of its
 *    neighbours' spins, either in Glauber form x/(1+x) with
 *    x = exp(-beta dE) (identical to 1/(1+exp(beta dE))) or in the
 *    standard Metropolis form min(1, exp(-beta dE)).
 *
 * The parallel algorithms of Section 3 all reach one trajectory (the
 * uniqueness argument following Fig. 3.1): the one in which the arrivals
 * are applied one at a time in increasing time order.  oracle_run()
 * computes it by that definition -- a binary heap keyed by
 * (arrival time, cell index) hands out the globally earliest pending
 * arrival, which is applied, rescheduled and pushed back.  Ties in time
 * (probability zero in exact arithmetic, possible in floating point) are
 * resolved by the smaller cell index first.
 *
 * Bit-level recipe shared by contract (not by code) with the GPU library:
 *   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = seed split in
 *   two 32-bit halves, counter = (k, c, domain, 0), domain 0 = arrival k of
 *   cell c, domain 1 = initial draw of cell c;
 *   u = (2 * (w >> 12) + 1) * 2^-53 with w the 64-bit word (y1:y0);
 *   gap = E(u) / lambda, E(u) = -ln u by the atanh-series recipe below;
 *   accept a flip iff y2 < thr[idx], thr = floor(p * 2^32) (2^32 if p >= 1);
 *   initial spin = +1 if (y2 & 1) of the initial draw, else -1.
 *
 * Compile with -ffp-contract=off and without -ffast-math: every floating
 * point operation below is one IEEE-754 binary64 operation, rounded to
 * nearest, in the order written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OAPI __attribute__((visibility("default")))

enum { O_GLAUBER = 0, O_METROPOLIS = 1 };
enum { O_INIT_RANDOM = 0, O_INIT_PLUS = 1, O_INIT_MINUS = 2 };

/* ------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition.                      */
/* ------------------------------------------------------------------ */
static void philox4x32_10(uint32_t x[4], uint32_t k0, uint32_t k1)
{
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x[1] ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x[3] ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
        k0 += 0x9E3779B9u;   /* Weyl key schedule */
        k1 += 0xBB67AE85u;
    }
}

static void draw(uint64_t seed, uint32_t k, uint32_t cell, uint32_t domain,
                 uint32_t out[4])
{
    out[0] = k; out[1] = cell; out[2] = domain; out[3] = 0u;
    philox4x32_10(out, (uint32_t)seed, (uint32_t)(seed >> 32));
}

/* ------------------------------------------------------------------ */
/* Exponential(1) variate E = -ln u, u uniform on (0,1) (Eq. (5)).     */
/*                                                                    */
/* ln u = e ln2 + ln f with u = 2^e f, f in (sqrt(2)/2, sqrt(2)];      */
/* ln f = 2 atanh(s), s = (f-1)/(f+1), |s| < 0.1716, and               */
/* 2 atanh(s) = 2 (s + s z (1/3 + z/5 + ... + z^9/21)), z = s^2.       */
/* The truncated tail is below 1e-18 relative.  ln2 is split into a    */
/* 39-bit head (so e * head is exact) and the rounded remainder.       */
/* ------------------------------------------------------------------ */
static const double LN2_HEAD = 0x1.62e42fefa4000p-1;
static const double LN2_TAIL = -0x1.8432a1b0e2634p-43;
/* 1/(2j+1), j = 1..10, each rounded to nearest by the compiler. */
static const double ATANH_C[10] = {
    1.0 / 3.0,  1.0 / 5.0,  1.0 / 7.0,  1.0 / 9.0,  1.0 / 11.0,
    1.0 / 13.0, 1.0 / 15.0, 1.0 / 17.0, 1.0 / 19.0, 1.0 / 21.0,
};

static double uniform_open(uint64_t w)
{
    /* 2m+1 < 2^53 is exact in binary64; so is the scaling by 2^-53. */
    return (double)(((w >> 12) << 1) | 1u) * 0x1p-53;
}

static double neg_log(double u)
{
    const double sqrt2 = sqrt(2.0);   /* correctly rounded */
    int e;
    double f = frexp(u, &e);          /* u = f 2^e, f in [1/2, 1) */
    f = f * 2.0;                      /* exact: f in [1, 2) */
    e = e - 1;
    if (f > sqrt2) {
        f = f * 0.5;                  /* exact */
        e = e + 1;
    }
    double a = f - 1.0;               /* exact (Sterbenz) */
    double b = f + 1.0;
    double s = a / b;
    double z = s * s;
    double p = ATANH_C[9];
    for (int j = 8; j >= 0; --j) {
        p = p * z;
        p = p + ATANH_C[j];
    }
    double r = z * p;
    r = s * r;
    double lf = s + r;
    lf = lf + lf;
    double ed = (double)e;
    double head = ed * LN2_HEAD;      /* exact: |e| <= 53 */
    double tail = ed * LN2_TAIL;
    double lnu = head + (tail + lf);
    return -lnu;
}

static double exp_gap(uint32_t lo, uint32_t hi, double rate)
{
    uint64_t w = ((uint64_t)hi << 32) | (uint64_t)lo;
    return neg_log(uniform_open(w)) / rate;
}

/* ------------------------------------------------------------------ */
/* Flip thresholds: the appendix program's probability table, with    */
/* the index (sum + z)/2 + (z+1)(s+1)/2 over z neighbour slots.        */
/* dE = 2 s (J sum + h) is the energy change of reversing s under      */
/* H = -J sum s s' - h sum s.                                          */
/* ------------------------------------------------------------------ */
static void thresholds(int z, double J, double h, double beta, int rule,
                       uint64_t *thr)
{
    for (int up = 0; up <= 1; ++up) {
        int spin = 2 * up - 1;
        for (int i = 0; i <= z; ++i) {
            int sum = 2 * i - z;
            double js = J * (double)sum;
            double field = js + h;
            double dE = 2.0 * ((double)spin * field);
            double p;
            if (rule == O_GLAUBER) {
                double x = exp(beta * dE);
                p = 1.0 / (1.0 + x);
            } else {
                p = (dE <= 0.0) ? 1.0 : exp(-(beta * dE));
            }
            uint64_t v;
            if (p >= 1.0) v = (uint64_t)1 << 32;
            else          v = (uint64_t)floor(p * 4294967296.0);
            thr[(sum + z) / 2 + (z + 1) * (spin + 1) / 2] = v;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Geometry: periodic 1-, 2- or 3-D box, index x + Lx (y + Ly z).      */
/* Neighbour slots in the order +x, -x, +y, -y, +z, -z.  A slot may    */
/* name the same cell twice (side 2); it then counts twice.            */
/* ------------------------------------------------------------------ */
typedef struct {
    int dim;
    int64_t L[3];
    int64_t n;
} geom;

static int make_geom(int dim, const int32_t *L, geom *g)
{
    if (dim < 1 || dim > 3) return -1;
    g->dim = dim;
    g->n = 1;
    for (int d = 0; d < 3; ++d) {
        g->L[d] = (d < dim) ? (int64_t)L[d] : 1;
        if (d < dim && g->L[d] < 2) return -1;
        g->n *= g->L[d];
    }
    if (g->n >= ((int64_t)1 << 32)) return -1;
    return 0;
}

static int neighbours(const geom *g, int64_t c, int64_t nb[6])
{
    int64_t x = c % g->L[0];
    int64_t y = (c / g->L[0]) % g->L[1];
    int64_t zc = c / (g->L[0] * g->L[1]);
    int64_t co[3] = {x, y, zc};
    int64_t stride[3] = {1, g->L[0], g->L[0] * g->L[1]};
    int m = 0;
    for (int d = 0; d < g->dim; ++d) {
        int64_t up = (co[d] + 1) % g->L[d];
        int64_t dn = (co[d] + g->L[d] - 1) % g->L[d];
        nb[m++] = c + (up - co[d]) * stride[d];
        nb[m++] = c + (dn - co[d]) * stride[d];
    }
    return m;
}

/* (t_a, a) before (t_b, b) in the total order of arrivals. */
static int earlier(double ta, int64_t a, double tb, int64_t b)
{
    return ta < tb || (ta == tb && a < b);
}

/* Apply arrival number n[c] of cell c at time t[c]: the draw decides the
 * flip from the current neighbour spins, then the clock moves on. */
static int apply_arrival(const geom *g, const uint64_t *thr, uint64_t seed,
                         double rate, int64_t c, int8_t *s, double *t,
                         uint32_t *n)
{
    int64_t nb[6];
    int z = neighbours(g, c, nb);
    int sum = 0;
    for (int i = 0; i < z; ++i) sum += s[nb[i]];
    uint32_t y[4];
    draw(seed, n[c], (uint32_t)c, 0u, y);
    int idx = (sum + z) / 2 + (z + 1) * (s[c] + 1) / 2;
    int flipped = 0;
    if ((uint64_t)y[2] < thr[idx]) {
        s[c] = (int8_t)(-s[c]);
        flipped = 1;
    }
    t[c] = t[c] + exp_gap(y[0], y[1], rate);
    n[c] = n[c] + 1u;
    return flipped;
}

/* ------------------------------------------------------------------ */
/* Exported: primitives (for the pins in the test suite).              */
/* ------------------------------------------------------------------ */
OAPI void oracle_philox(const uint32_t *ctr, uint64_t seed, uint32_t *out,
                        int64_t count)
{
    for (int64_t i = 0; i < count; ++i) {
        uint32_t x[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2],
                         ctr[4 * i + 3]};
        philox4x32_10(x, (uint32_t)seed, (uint32_t)(seed >> 32));
        memcpy(out + 4 * i, x, sizeof x);
    }
}

OAPI void oracle_neg_log_words(const uint64_t *w, double *out, int64_t count)
{
    for (int64_t i = 0; i < count; ++i) out[i] = neg_log(uniform_open(w[i]));
}

OAPI void oracle_uniform_words(const uint64_t *w, double *out, int64_t count)
{
    for (int64_t i = 0; i < count; ++i) out[i] = uniform_open(w[i]);
}

OAPI void oracle_ln2_split(double *head, double *tail)
{
    *head = LN2_HEAD;
    *tail = LN2_TAIL;
}

/* thr must hold 2*(2*dim+1) entries. */
OAPI int oracle_thresholds(int dim, double J, double h, double beta,
                           int rule, uint64_t *thr)
{
    if (dim < 1 || dim > 3) return -1;
    thresholds(2 * dim, J, h, beta, rule, thr);
    return 2 * (2 * dim + 1);
}

/* ------------------------------------------------------------------ */
/* Exported: initial state.  Cell c draws once from domain 1: its     */
/* first arrival is one exponential gap after time 0 (there is no      */
/* arrival at time 0 itself), its spin is set from a bit of the draw    */
/* or fixed to +1 / -1.                                                 */
/* ------------------------------------------------------------------ */
OAPI int oracle_init(int dim, const int32_t *L, double rate, int init,
                     uint64_t seed, int8_t *s, double *t, uint32_t *n)
{
    geom g;
    if (make_geom(dim, L, &g) != 0 || !(rate > 0.0)) return -1;
    for (int64_t c = 0; c < g.n; ++c) {
        uint32_t y[4];
        draw(seed, 0u, (uint32_t)c, 1u, y);
        t[c] = exp_gap(y[0], y[1], rate);
        if (init == O_INIT_RANDOM)    s[c] = (y[2] & 1u) ? 1 : -1;
        else if (init == O_INIT_PLUS) s[c] = 1;
        else                          s[c] = -1;
        n[c] = 0u;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Exported: the oracle.  Applies every pending arrival with time < T  */
/* in increasing (time, index) order.  On return t[c] is the first      */
/* arrival at or after T and n[c] counts the arrivals applied so far.   */
/* Returns the number of arrivals applied, or -1 on bad arguments.      */
/* ------------------------------------------------------------------ */
static void sift_down(uint32_t *heap, int64_t len, int64_t i, const double *t)
{
    uint32_t item = heap[i];
    double ti = t[item];
    for (;;) {
        int64_t l = 2 * i + 1;
        if (l >= len) break;
        int64_t best = l;
        int64_t r = l + 1;
        if (r < len && earlier(t[heap[r]], heap[r], t[heap[l]], heap[l]))
            best = r;
        if (!earlier(t[heap[best]], heap[best], ti, item)) break;
        heap[i] = heap[best];
        i = best;
    }
    heap[i] = item;
}

OAPI int64_t oracle_run(int dim, const int32_t *L, double J, double h,
                        double beta, double rate, int rule, uint64_t seed,
                        double T, int8_t *s, double *t, uint32_t *n,
                        uint64_t *flips_out)
{
    geom g;
    if (make_geom(dim, L, &g) != 0 || !(rate > 0.0) || isnan(T)) return -1;
    uint64_t thr[14];
    thresholds(2 * dim, J, h, beta, rule, thr);

    uint32_t *heap = (uint32_t *)malloc((size_t)g.n * sizeof(uint32_t));
    if (!heap) return -1;
    for (int64_t c = 0; c < g.n; ++c) heap[c] = (uint32_t)c;
    for (int64_t i = g.n / 2 - 1; i >= 0; --i) sift_down(heap, g.n, i, t);

    int64_t events = 0;
    uint64_t flips = 0;
    while (t[heap[0]] < T) {
        int64_t c = heap[0];
        flips += (uint64_t)apply_arrival(&g, thr, seed, rate, c, s, t, n);
        ++events;
        sift_down(heap, g.n, 0, t);
    }
    free(heap);
    if (flips_out) *flips_out = flips;
    return events;
}

/* ------------------------------------------------------------------ */
/* q-th degree neighbourhoods (Section 3, after Fig. 3.5): the set      */
/* neighbors^q(c) is built by applying neighbors() q times, i.e. the     */
/* cells within lattice (L1) distance q of c.  The rule reads the sum    */
/* of the spins of every cell of that set other than c, so z = |set| - 1 */
/* takes the place of 2 dim (2D: 2q(q+1)).  Every side must exceed 2q,   */
/* so that the set has no repeated cell.                                 */
/* ------------------------------------------------------------------ */
#define O_MAX_BALL 64

/* Offsets (dx, dy, dz) with 1 <= |dx| + |dy| + |dz| <= q, unused axes 0. */
static int ball_offsets(int dim, int q, int off[][3])
{
    int m = 0;
    int r1 = q, r2 = dim > 1 ? q : 0, r3 = dim > 2 ? q : 0;
    for (int dz = -r3; dz <= r3; ++dz)
        for (int dy = -r2; dy <= r2; ++dy)
            for (int dx = -r1; dx <= r1; ++dx) {
                int d = abs(dx) + abs(dy) + abs(dz);
                if (d < 1 || d > q) continue;
                if (m >= O_MAX_BALL) return -1;
                off[m][0] = dx;
                off[m][1] = dy;
                off[m][2] = dz;
                ++m;
            }
    return m;
}

/* thr must hold 2 (z + 1) entries, z = |neighbors^q(c)| - 1; returns that
 * count, or -1 when the set would exceed O_MAX_BALL cells. */
OAPI int oracle_thresholds_range(int dim, int q, double J, double h, double beta,
                                 int rule, uint64_t *thr)
{
    int off[O_MAX_BALL][3];
    if (dim < 1 || dim > 3 || q < 1) return -1;
    int z = ball_offsets(dim, q, off);
    if (z < 0) return -1;
    thresholds(z, J, h, beta, rule, thr);
    return 2 * (z + 1);
}

OAPI int64_t oracle_run_range(int dim, const int32_t *L, int q, double J, double h,
                              double beta, double rate, int rule, uint64_t seed,
                              double T, int8_t *s, double *t, uint32_t *n,
                              uint64_t *flips_out)
{
    geom g;
    int off[O_MAX_BALL][3];
    if (make_geom(dim, L, &g) != 0 || !(rate > 0.0) || isnan(T) || q < 1) return -1;
    for (int d = 0; d < dim; ++d)
        if (g.L[d] <= 2 * (int64_t)q) return -1;
    int z = ball_offsets(dim, q, off);
    if (z < 0) return -1;
    uint64_t thr[2 * (O_MAX_BALL + 1)];
    thresholds(z, J, h, beta, rule, thr);

    uint32_t *heap = (uint32_t *)malloc((size_t)g.n * sizeof(uint32_t));
    if (!heap) return -1;
    for (int64_t c = 0; c < g.n; ++c) heap[c] = (uint32_t)c;
    for (int64_t i = g.n / 2 - 1; i >= 0; --i) sift_down(heap, g.n, i, t);

    int64_t events = 0;
    uint64_t flips = 0;
    while (t[heap[0]] < T) {
        int64_t c = heap[0];
        int64_t co[3] = {c % g.L[0], (c / g.L[0]) % g.L[1], c / (g.L[0] * g.L[1])};
        int sum = 0;
        for (int k = 0; k < z; ++k) {
            int64_t nb = 0, stride = 1;
            for (int d = 0; d < 3; ++d) {
                int64_t x = ((co[d] + off[k][d]) % g.L[d] + g.L[d]) % g.L[d];
                nb += x * stride;
                stride *= g.L[d];
            }
            sum += s[nb];
        }
        uint32_t y[4];
        draw(seed, n[c], (uint32_t)c, 0u, y);
        int idx = (sum + z) / 2 + (z + 1) * (s[c] + 1) / 2;
        if ((uint64_t)y[2] < thr[idx]) {
            s[c] = (int8_t)(-s[c]);
            ++flips;
        }
        t[c] = t[c] + exp_gap(y[0], y[1], rate);
        n[c] = n[c] + 1u;
        ++events;
        sift_down(heap, g.n, 0, t);
    }
    free(heap);
    if (flips_out) *flips_out = flips;
    return events;
}

/* ------------------------------------------------------------------ */
/* Exported: per-cell arrival clock without any spin dynamics.  The     */
/* arrival times do not depend on the spins (Section 4), so the first   */
/* arrival at or after T and the number of arrivals before T follow     */
/* from the cell's own draws alone.  Used to check times and counts     */
/* cell by cell at any lattice size.                                    */
/* ------------------------------------------------------------------ */
OAPI void oracle_cell_clock(uint64_t seed, double rate, const uint32_t *cells,
                            int64_t count, double T, double *t_out,
                            uint32_t *n_out)
{
    for (int64_t i = 0; i < count; ++i) {
        uint32_t c = cells[i], y[4];
        draw(seed, 0u, c, 1u, y);
        double tc = exp_gap(y[0], y[1], rate);
        uint32_t k = 0;
        while (tc < T) {
            draw(seed, k, c, 0u, y);
            tc = tc + exp_gap(y[0], y[1], rate);
            ++k;
        }
        t_out[i] = tc;
        n_out[i] = k;
    }
}

// aca_api.hip -- C-ABI of libaca (declared in include/aca.h).
//
// Host side of the conservative simulation: argument checks, the flip
// thresholds, the tile plan, and the launch loop of aca_advance.  The caller's
// state is packed into working words (two snapshots in scratch); each launch
// advances every tile region from one snapshot and merges all copies into the
// other; the loop reads back per-launch counters and stops when no owned cell
// has an arrival before the horizon; the final snapshot is unpacked into the
// caller's buffers.  A launch that applies nothing while arrivals are due
// is reported as ACA_ENOPROGRESS: the cell holding the globally earliest
// arrival always sees current neighbours at load time and must be able to
// move (the deadlock-freedom argument of Fig. 3.1 and Fig. 3.4).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/aca.h"
#include "aca_host.h"
#include "aca_internal.h"

using namespace aca_host;

namespace aca_host {

thread_local std::string g_error;

aca_status fail(aca_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

ScratchLayout scratch_layout(uint64_t n)
{
    ScratchLayout l;
    size_t off = 0;
    for (int b = 0; b < 2; ++b) {
        l.key_off[b] = off;
        off = align_up(off + 8 * n);
        l.time_off[b] = off;
        off = align_up(off + 8 * n);
    }
    l.dead_off = off;
    off = align_up(off + n);
    l.ctr_off = off;
    l.total = l.ctr_off + 2 * kAlign;
    return l;
}

// Decided on the bit pattern (exponent field not all ones), so the check holds
// whatever floating-point assumptions the compiler is given.
bool is_finite(double v)
{
    uint64_t bits;
    memcpy(&bits, &v, sizeof bits);
    return (bits & 0x7FF0000000000000ull) != 0x7FF0000000000000ull;
}

int ball_size(int dim, int q)
{
    int m = 0;
    const int r2 = dim > 1 ? q : 0, r3 = dim > 2 ? q : 0;
    for (int dz = -r3; dz <= r3; ++dz)
        for (int dy = -r2; dy <= r2; ++dy)
            for (int dx = -q; dx <= q; ++dx) {
                const int d = std::abs(dx) + std::abs(dy) + std::abs(dz);
                m += (d >= 1 && d <= q) ? 1 : 0;
            }
    return m;
}

aca_status check_params(const aca_params *in, uint64_t *n_out, aca_params *full)
{
    if (!in) return fail(ACA_EINVAL, "params is NULL");
    if (in->struct_size != sizeof(aca_params) && in->struct_size != ACA_PARAMS_SIZE_V1)
        return fail(ACA_EINVAL, "params.struct_size %u is neither %zu nor %u", in->struct_size,
                    sizeof(aca_params), ACA_PARAMS_SIZE_V1);
    aca_params copy;
    memset(&copy, 0, sizeof copy);
    memcpy(&copy, in, in->struct_size);
    if (in->struct_size == ACA_PARAMS_SIZE_V1) copy.range = 1;
    copy.struct_size = sizeof(aca_params);
    const aca_params *p = &copy;
    if (p->range < 1) return fail(ACA_EINVAL, "range %d < 1", p->range);
    if (p->dim < 1 || p->dim > 3) return fail(ACA_EINVAL, "dim %d not in 1..3", p->dim);
    if (p->dim < 1 || p->dim > 3) return fail(ACA_EINVAL, "dim %d not in 1..3", p->dim);
    uint64_t n = 1;
    for (int d = 0; d < p->dim; ++d) {
        if (p->L[d] < 2) return fail(ACA_EINVAL, "L[%d] = %d < 2", d, p->L[d]);
        n *= (uint64_t)p->L[d];
        if (n >= (1ull << 32)) return fail(ACA_EINVAL, "lattice has >= 2^32 cells");
    }
    if (!is_finite(p->J) || !is_finite(p->h)) return fail(ACA_EINVAL, "J and h must be finite");
    if (!is_finite(p->beta) || p->beta < 0.0)
        return fail(ACA_EINVAL, "beta must be finite and >= 0");
    if (!is_finite(p->rate) || !(p->rate > 0.0))
        return fail(ACA_EINVAL, "rate must be finite and > 0");
    if (p->rule != ACA_GLAUBER && p->rule != ACA_METROPOLIS)
        return fail(ACA_EINVAL, "unknown rule %d", p->rule);
    if (p->init < ACA_INIT_RANDOM || p->init > ACA_INIT_MINUS)
        return fail(ACA_EINVAL, "unknown init %d", p->init);
    if (p->range > 1) {
        for (int d = 0; d < p->dim; ++d)
            if (p->L[d] <= 2 * p->range)
                return fail(ACA_EINVAL, "L[%d] = %d must exceed twice the range %d", d,
                            p->L[d], p->range);
        static const int max_range[4] = {0, 4, 3, 2};
        if (p->range > max_range[p->dim] || ball_size(p->dim, p->range) > aca::kMaxSlots)
            return fail(ACA_EINVAL, "range %d exceeds %d in %dD", p->range, max_range[p->dim],
                        p->dim);
    }
    if (n_out) *n_out = n;
    if (full) *full = copy;
    return ACA_OK;
}

// Flip table of the appendix program generalised to z = 2 dim slots:
// entry (sum + z)/2 + (z+1)(s+1)/2 holds floor(p 2^32), 2^32 when p >= 1.
int build_thresholds(const aca_params *p, uint64_t *thr)
{
    const int z = p->range > 1 ? ball_size(p->dim, p->range) : 2 * p->dim;
    if (!thr) return 2 * (z + 1);
    for (int spin = -1; spin <= 1; spin += 2) {
        for (int sum = -z; sum <= z; sum += 2) {
            const double js = p->J * (double)sum;
            const double field = js + p->h;
            const double dE = 2.0 * ((double)spin * field);
            double prob;
            if (p->rule == ACA_GLAUBER) {
                const double x = exp(p->beta * dE);
                prob = 1.0 / (1.0 + x);
            } else {
                prob = (dE <= 0.0) ? 1.0 : exp(-(p->beta * dE));
            }
            const uint64_t v = (prob >= 1.0) ? (1ull << 32)
                                              : (uint64_t)floor(prob * 4294967296.0);
            thr[(sum + z) / 2 + (z + 1) * (spin + 1) / 2] = v;
        }
    }
    return 2 * (z + 1);
}

// Automatic schedule knobs; every choice gives the same result.
void auto_tuning(const aca_params &p, aca_tuning *t)
{
    if (p.range > 1) {
        // wider frozen rings: smaller tiles keep two workgroups per CU
        if (p.dim == 1) {
            t->tile[0] = 1024; t->ghost[0] = 32;
            t->max_sweeps = 128; t->block = 256;
        } else if (p.dim == 2) {
            t->tile[0] = 56; t->tile[1] = 48;
            t->ghost[0] = 4; t->ghost[1] = 4;
            t->max_sweeps = 32; t->block = 512;
        } else {
            t->tile[0] = 12; t->tile[1] = 12; t->tile[2] = 8;
            t->ghost[0] = 1; t->ghost[1] = 1; t->ghost[2] = 1;
            t->max_sweeps = 16; t->block = 512;
        }
        return;
    }
    if (p.dim == 1) {
        // an 8322-cell box (158 KB: one workgroup per CU); 1024 threads run a
        // 4M-cell line to T = 20 in 0.92 ms against 1.50 with 256
        t->tile[0] = 8192; t->ghost[0] = 64;
        t->max_sweeps = 255; t->block = 1024;
    } else if (p.dim == 2) {
        // an 84 x 66 box (79 KB of LDS: two workgroups per CU); 5 ghost cells
        // let a visit move its region one layer further than 4 at the same box
        t->tile[0] = 72; t->tile[1] = 54;
        t->ghost[0] = 5; t->ghost[1] = 5;
        t->max_sweeps = 40; t->block = 512;
    } else {
        // one 20x20x16 region (24x24x20 box, 155 KB) fills a CU's LDS: 768
        // threads (twelve wavefronts) measure 3 % faster than 1024 or 512;
        // later rounds of a 3D visit hold few cells (a frozen ring one ghost
        // cell away), so visits stop at 12
        t->tile[0] = 20; t->tile[1] = 20; t->tile[2] = 16;
        t->ghost[0] = 1; t->ghost[1] = 1; t->ghost[2] = 1;
        t->max_sweeps = 12; t->block = 768;
    }
}

// A lattice too small to give the compute units many default regions runs
// few workgroups per launch, so its launches are short and latency-bound:
// smaller tiles (more workgroups), wider ghosts and longer visits (a region
// moves further per launch, so fewer launches) pay more than the larger
// surface costs.  A 1D line of up to a million cells has fewer default
// regions than compute units, so every line takes tiles sized to its length.
// Applied to automatic knobs of a single lattice only (a batch fills the
// device with many lattices and keeps the defaults), and in 2D and 3D only
// where every side leaves room for the wider ghost.
void small_lattice_tuning(const aca_params &p, aca_tuning *t)
{
    if (p.range > 1) return;
    uint64_t n = 1;
    int lmin = p.L[0];
    for (int d = 0; d < p.dim; ++d) {
        n *= (uint64_t)p.L[d];
        lmin = std::min(lmin, p.L[d]);
    }
    if (p.dim == 2 && n <= 512ull * 512 && lmin >= 32) {
        // 14 ghost cells: 64^2 to T = 100 in 1.65 ms against 2.03 with 8,
        // 512^2 to T = 40 in 0.91 against 1.06 (a 70 x 70 box at most, 64 KB)
        for (int d = 0; d < 2; ++d) {
            t->tile[d] = std::min(40, (p.L[d] + 2) / 3);
            t->ghost[d] = 14;
        }
        t->max_sweeps = 64;
    } else if (p.dim == 2 && n <= 1536ull * 1536 && lmin >= 128) {
        // up to about 2.4 M cells: 56 x 48 tiles with 8 ghost cells (a 74 x 66
        // box) give more regions per CU and move them further per launch;
        // 1024^2 to T = 40 in 1.43 ms against 1.67 with the default, 1536^2
        // to T = 30 in 1.98 against 2.10 (2048^2: the default is faster)
        t->tile[0] = 56; t->tile[1] = 48;
        t->ghost[0] = 8; t->ghost[1] = 8;
        t->max_sweeps = 48;
    } else if (p.dim == 3 && n <= 128ull * 128 * 128 && lmin >= 16) {
        // up to 64^3 a third ghost layer pays (64^3 to T = 40: 2.75 ms
        // against 3.39 with 16^3 tiles and 2); at 128^3 it no longer does
        const bool tiny = n <= 64ull * 64 * 64;
        for (int d = 0; d < 3; ++d) {
            t->tile[d] = std::min(tiny ? 14 : 16, (p.L[d] + 2) / 3);
            t->ghost[d] = tiny ? 3 : 2;
        }
        t->max_sweeps = tiny ? 24 : 16;
    } else if (p.dim == 1) {
        // a line of any length: about one tile per compute unit (L / 256
        // cells, at least 256 and at most the 8192 of the default region).
        // 2^16 cells to T = 40: 0.31 ms against 0.70 with 8192-cell tiles;
        // 2^20 to T = 20: 0.37 against 0.48; 4 Mi cells keep 8192.
        const int tile = std::min(8192, std::max(256, (p.L[0] + 255) / 256));
        t->tile[0] = tile;
        t->ghost[0] = 64;
        t->max_sweeps = 255;
        t->block = tile >= 2048 ? 1024 : 512;
    }
}

int tune_candidates(int dim, aca_tuning *out)
{
    // tile sides, ghost width, worklist rounds per visit
    static const int c1[][3] = {{8192, 64, 512}, {4096, 32, 256}, {16384, 64, 1024},
                                {8192, 128, 1024}, {2048, 16, 128}};
    static const int c2[][5] = {{72, 54, 5, 40, 0}, {64, 60, 5, 40, 0}, {72, 54, 5, 32, 0},
                                {64, 60, 5, 32, 0}, {64, 52, 5, 32, 0}, {40, 40, 8, 64, 0}};
    // tile sides, ghost, rounds, threads
    static const int c3[][6] = {{20, 20, 16, 1, 12, 768}, {20, 20, 16, 1, 16, 768},
                                {20, 20, 16, 1, 12, 1024}, {18, 18, 14, 2, 16, 768},
                                {16, 16, 16, 2, 16, 768}, {20, 20, 12, 1, 12, 768},
                                {16, 16, 8, 1, 12, 512}, {8, 8, 8, 1, 8, 512}};
    int n = 0;
    auto base = [&]() -> aca_tuning & {
        aca_tuning &t = out[n++];
        memset(&t, 0, sizeof t);
        t.struct_size = sizeof t;
        t.ghost[0] = t.ghost[1] = t.ghost[2] = -1;
        return t;
    };
    if (dim == 1) {
        for (const auto &c : c1) {
            aca_tuning &t = base();
            t.tile[0] = c[0]; t.ghost[0] = c[1]; t.max_sweeps = c[2];
        }
    } else if (dim == 2) {
        for (const auto &c : c2) {
            aca_tuning &t = base();
            t.tile[0] = c[0]; t.tile[1] = c[1];
            t.ghost[0] = t.ghost[1] = c[2];
            t.max_sweeps = c[3];
        }
    } else {
        for (const auto &c : c3) {
            aca_tuning &t = base();
            t.tile[0] = c[0]; t.tile[1] = c[1]; t.tile[2] = c[2];
            t.ghost[0] = t.ghost[1] = t.ghost[2] = c[3];
            t.max_sweeps = c[4];
            t.block = c[5];
        }
    }
    return n;
}

aca_status make_plan(const aca_lattice *lat, double T, Plan *plan)
{
    const aca_params &p = lat->p;
    aca_tuning t;
    memset(&t, 0, sizeof t);
    t.ghost[0] = t.ghost[1] = t.ghost[2] = -1;
    auto_tuning(p, &t);
    small_lattice_tuning(p, &t);
    for (int d = 0; d < 3; ++d) {
        if (lat->tun.tile[d] > 0) t.tile[d] = lat->tun.tile[d];
        if (lat->tun.ghost[d] >= 0) t.ghost[d] = lat->tun.ghost[d];
    }
    if (lat->tun.max_sweeps > 0) t.max_sweeps = lat->tun.max_sweeps;
    if (lat->tun.block > 0) t.block = lat->tun.block;
    if (t.block % 64 != 0 || t.block < 64 || t.block > 1024)
        return fail(ACA_EINVAL, "block %d must be a multiple of 64 in [64, 1024]", t.block);
    // a cell applies at most one arrival per sweep; per-visit flip counts are
    // kept in 8 bits
    t.max_sweeps = std::min(t.max_sweeps, 255);

    aca::VisitArgs &a = plan->a;
    memset(&a, 0, sizeof a);
    for (int d = 0; d < 3; ++d) {
        if (d < p.dim) {
            const int L = p.L[d];
            a.L[d] = L;
            // a reach beyond the nearest neighbours needs a frozen ring on
            // every side: cut each direction into at least two tiles (and
            // keep 1D tiles within LDS)
            if (p.range > 1 && p.dim == 1 && lat->tun.tile[0] <= 0)
                t.tile[0] = std::min(t.tile[0], 1024);
            if (p.range > 1 && t.tile[d] >= L) t.tile[d] = (L + 1) / 2;
            if (t.tile[d] >= L) {
                a.span[d] = 1; a.tile[d] = L; a.ntiles[d] = 1; a.ghost[d] = 0;
            } else {
                a.span[d] = 0;
                // an automatic tile that would leave too little lattice for
                // its ghost cells is evened out over the same number of tiles
                if (lat->tun.tile[d] <= 0 && (L - t.tile[d]) / 2 < t.ghost[d]) {
                    const int k = (L + t.tile[d] - 1) / t.tile[d];
                    t.tile[d] = (L + k - 1) / k;
                }
                a.tile[d] = t.tile[d];
                a.ntiles[d] = (L + t.tile[d] - 1) / t.tile[d];
                // keep the simulated region within one period of the lattice
                a.ghost[d] = std::max(0, std::min(t.ghost[d], (L - t.tile[d]) / 2));
            }
        } else {
            a.L[d] = 1; a.tile[d] = 1; a.ntiles[d] = 1; a.ghost[d] = 0; a.span[d] = 1;
        }
    }
    a.max_sweeps = t.max_sweeps;
    a.key_lo = (uint32_t)p.seed;
    a.key_hi = (uint32_t)(p.seed >> 32);
    a.rate = p.rate;
    a.unit_rate = p.rate == 1.0 ? 1 : 0;
    uint64_t hb;
    memcpy(&hb, &T, sizeof hb);
    a.horizon_bits = hb;
    a.counters = lat->counters;
    a.final_bits = hb;
    a.track_tmin = 0;
    a.frames = nullptr;
    a.n_cells = lat->n;
    a.count_efficiency = lat->count_efficiency ? 1 : 0;
    memcpy(a.thr, lat->thr, sizeof a.thr);
    plan->block = t.block;
    int dev_lds = 0;
    HIP_TRY(hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                  lat->device));
    bool spans = false;
    for (int d = 0; d < p.dim; ++d) spans = spans || a.span[d];
    a.range = p.range;
    plan->fast = !spans && aca::visit_fast_box(p.dim, a) <= 65535 &&
                 aca::visit_fast_lds_bytes(p.dim, a) <= (size_t)dev_lds;
    if (p.range > 1 && !plan->fast)
        return fail(ACA_EINVAL, "range %d: the tile region needs %zu B of LDS (device %d B) "
                    "or more than 65535 cells", p.range, aca::visit_fast_lds_bytes(p.dim, a),
                    dev_lds);
    if (plan->fast) {
        plan->lds = aca::visit_fast_lds_bytes(p.dim, a);
        return ACA_OK;
    }
    if (aca::visit_inner_max(p.dim, a) > 65535)
        return fail(ACA_EINVAL, "a tile region of %d cells exceeds 65535 simulated cells",
                    aca::visit_inner_max(p.dim, a));
    plan->lds = aca::visit_lds_bytes(p.dim, a, t.block);
    if (plan->lds > (size_t)dev_lds)
        return fail(ACA_EINVAL, "tile region needs %zu B of LDS, device has %d B",
                    plan->lds, dev_lds);
    uint64_t tiles = (uint64_t)a.ntiles[0] * a.ntiles[1] * a.ntiles[2];
    if (tiles > 0x7FFFFFFFull) return fail(ACA_EINVAL, "too many tiles");
    return ACA_OK;
}

// Bytes one launch must move: for each tile, the two working words of its
// whole region box in and those of its own cells out (16 B per cell each way;
// merges of ghost copies come on top and are not counted).
uint64_t launch_region_bytes(int dim, const aca::VisitArgs &a)
{
    uint64_t total = 0;
    const int nt[3] = {a.ntiles[0], a.ntiles[1], a.ntiles[2]};
    // tiles along each direction come in at most two widths (the last is ragged)
    for (int ix = 0; ix < 2; ++ix)
        for (int iy = 0; iy < 2; ++iy)
            for (int iz = 0; iz < 2; ++iz) {
                const int pick[3] = {ix, iy, iz};
                uint64_t count = 1, box = 1, inner = 1, own = 1;
                bool any = true;
                for (int d = 0; d < 3; ++d) {
                    const int full = (a.L[d] / a.tile[d] == nt[d]) ? nt[d] : nt[d] - 1;
                    const int m = pick[d] ? nt[d] - full : full;
                    if (m <= 0) { any = false; break; }
                    const int w = pick[d] ? a.L[d] - full * a.tile[d] : a.tile[d];
                    count *= (uint64_t)m;
                    own *= (uint64_t)w;
                    const int rin = a.span[d] ? a.L[d] : w + 2 * a.ghost[d];
                    inner *= (uint64_t)rin;
                    box *= (uint64_t)(rin + (a.span[d] ? 0 : 2));
                    (void)dim;
                }
                if (any) total += count * (16 * box + 16 * own);
                (void)inner;
            }
    return total;
}

}  // namespace aca_host

ACA_EXPORT uint32_t aca_abi_version(void) { return ACA_ABI_VERSION; }

ACA_EXPORT const char *aca_last_error(void) { return g_error.c_str(); }

ACA_EXPORT aca_status aca_thresholds(const aca_params *p, uint64_t *out, int32_t cap,
                                     int32_t *count)
{
    aca_params full;
    aca_status st = check_params(p, nullptr, &full);
    if (st != ACA_OK) return st;
    if (!out) return fail(ACA_EINVAL, "out is NULL");
    uint64_t thr[2 * (aca::kMaxSlots + 1)];
    const int need = build_thresholds(&full, thr);
    if (cap < need) return fail(ACA_EINVAL, "cap %d < %d entries", cap, need);
    memcpy(out, thr, sizeof(uint64_t) * need);
    if (count) *count = need;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_query(const aca_params *p, uint64_t *n_cells,
                                uint64_t *scratch_bytes)
{
    uint64_t n = 0;
    aca_status st = check_params(p, &n, nullptr);
    if (st != ACA_OK) return st;
    if (n_cells) *n_cells = n;
    if (scratch_bytes) *scratch_bytes = scratch_layout(n).total;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_create(const aca_params *p, int8_t *d_spin, double *d_time,
                                 uint32_t *d_count, void *d_scratch,
                                 uint64_t scratch_bytes, aca_lattice **out)
{
    uint64_t n = 0;
    aca_params full;
    aca_status st = check_params(p, &n, &full);
    if (st != ACA_OK) return st;
    p = &full;
    if (!out) return fail(ACA_EINVAL, "out is NULL");
    if (!d_spin || !d_time || !d_count || !d_scratch)
        return fail(ACA_EINVAL, "a device buffer is NULL");
    const void *bufs[4] = {d_spin, d_time, d_count, d_scratch};
    for (const void *b : bufs)
        if (((uintptr_t)b) % kAlign != 0)
            return fail(ACA_EINVAL, "device buffers must be %zu-byte aligned", kAlign);
    const ScratchLayout sl = scratch_layout(n);
    if (scratch_bytes < sl.total)
        return fail(ACA_ENOMEM, "scratch has %llu bytes, needs %zu",
                    (unsigned long long)scratch_bytes, sl.total);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    aca_lattice *lat = new (std::nothrow) aca_lattice();
    if (!lat) return fail(ACA_ENOMEM, "host allocation failed");
    lat->p = *p;
    lat->n = n;
    char *sc = static_cast<char *>(d_scratch);
    lat->s = d_spin;
    lat->t = d_time;
    lat->cnt = d_count;
    for (int b = 0; b < 2; ++b) {
        lat->key[b] = reinterpret_cast<unsigned long long *>(sc + sl.key_off[b]);
        lat->time[b] = reinterpret_cast<unsigned long long *>(sc + sl.time_off[b]);
    }
    lat->counters = reinterpret_cast<unsigned long long *>(sc + sl.ctr_off);
    lat->dead = reinterpret_cast<uint8_t *>(sc + sl.dead_off);
    lat->initialized = false;
    lat->attached = false;
    lat->lag = 0.0;
    lat->last_T = 0.0;
    memset(&lat->tun, 0, sizeof lat->tun);
    lat->tun.struct_size = sizeof(aca_tuning);
    lat->tun.ghost[0] = lat->tun.ghost[1] = lat->tun.ghost[2] = -1;
    memset(&lat->stats, 0, sizeof lat->stats);
    lat->stats.struct_size = sizeof(aca_stats);
    build_thresholds(p, lat->thr);
    lat->device = dev;
    bool ok = hipHostMalloc((void **)&lat->host_ctr, 8 * kCounterWords,
                            hipHostMallocMapped | hipHostMallocPortable) == hipSuccess &&
              hipHostGetDevicePointer((void **)&lat->host_ctr_dev, lat->host_ctr, 0) ==
                  hipSuccess;
    for (int i = 0; i < 2 && ok; ++i)
        ok = hipEventCreate(&lat->ev_start[i]) == hipSuccess &&
             hipEventCreate(&lat->ev_stop[i]) == hipSuccess;
    if (!ok) {
        for (int i = 0; i < 2; ++i) {
            if (lat->ev_start[i]) (void)hipEventDestroy(lat->ev_start[i]);
            if (lat->ev_stop[i]) (void)hipEventDestroy(lat->ev_stop[i]);
        }
        if (lat->host_ctr) (void)hipHostFree(lat->host_ctr);
        delete lat;
        return fail(ACA_EDEVICE, "pinned host word or HIP event creation failed");
    }
    *out = lat;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_set_tuning(aca_lattice *lat, const aca_tuning *t)
{
    if (!lat) return fail(ACA_EINVAL, "lattice is NULL");
    if (lat->attached) return fail(ACA_ESTATE, "lattice is a batch member");
    aca_tuning v;
    memset(&v, 0, sizeof v);
    v.struct_size = sizeof v;
    v.ghost[0] = v.ghost[1] = v.ghost[2] = -1;
    if (t) {
        if (t->struct_size != sizeof(aca_tuning))
            return fail(ACA_EINVAL, "tuning.struct_size mismatch");
        for (int d = 0; d < 3; ++d)
            if (t->tile[d] < 0) return fail(ACA_EINVAL, "tile[%d] < 0", d);
        if (t->max_sweeps < 0) return fail(ACA_EINVAL, "max_sweeps < 0");
        if (t->block != 0 && (t->block % 64 != 0 || t->block > 1024))
            return fail(ACA_EINVAL, "block must be a multiple of 64 up to 1024");
        v = *t;
    }
    lat->tun = v;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_get_tuning(const aca_lattice *lat, aca_tuning *out)
{
    if (!lat || !out) return fail(ACA_EINVAL, "NULL argument");
    Plan plan;
    aca_status st = make_plan(lat, 1.0, &plan);
    if (st != ACA_OK) return st;
    memset(out, 0, sizeof *out);
    out->struct_size = sizeof *out;
    for (int d = 0; d < 3; ++d) {
        out->tile[d] = plan.a.tile[d];
        out->ghost[d] = plan.a.ghost[d];
    }
    out->max_sweeps = plan.a.max_sweeps;
    out->block = plan.block;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_init(aca_lattice *lat, void *stream)
{
    if (!lat) return fail(ACA_EINVAL, "lattice is NULL");
    if (lat->attached) return fail(ACA_ESTATE, "lattice is a batch member");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(aca::launch_init(lat->p.dim, lat->p.L, lat->n, (uint32_t)lat->p.seed,
                             (uint32_t)(lat->p.seed >> 32), lat->p.rate, lat->p.init,
                             lat->s, lat->t, lat->cnt, s));
    lat->initialized = true;
    lat->last_T = 0.0;
    memset(&lat->stats, 0, sizeof lat->stats);
    lat->stats.struct_size = sizeof(aca_stats);
    return ACA_OK;
}

ACA_EXPORT aca_status aca_resume(aca_lattice *lat, double T_done)
{
    if (!lat) return fail(ACA_EINVAL, "lattice is NULL");
    if (lat->attached) return fail(ACA_ESTATE, "lattice is a batch member");
    if (!is_finite(T_done) || T_done < 0.0)
        return fail(ACA_EINVAL, "T_done must be finite and >= 0");
    // The region visits keep a claim in bit 31 of a cell's count word, so a
    // restored count must be below 2^31.  The caller's writes to the state
    // buffers may still be in flight on any stream: wait for the device.
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemset(lat->counters, 0, 8));
    HIP_TRY(aca::launch_count_bound(lat->n, lat->cnt, lat->counters, nullptr));
    unsigned long long high = 0;
    HIP_TRY(hipMemcpy(&high, lat->counters, 8, hipMemcpyDeviceToHost));
    if (high) return fail(ACA_EINVAL, "a restored count n(c) is 2^31 or more");
    lat->initialized = true;
    lat->last_T = T_done;
    memset(&lat->stats, 0, sizeof lat->stats);
    lat->stats.struct_size = sizeof(aca_stats);
    lat->stats.last_T = T_done;
    return ACA_OK;
}

namespace {

struct FrameRequest {
    int8_t *frames;
    double dt;
    long long k0;
    long long count;
};

aca_status advance_impl(aca_lattice *lat, double T, const FrameRequest *fr, void *stream);

}  // namespace

ACA_EXPORT aca_status aca_advance(aca_lattice *lat, double T, void *stream)
{
    return advance_impl(lat, T, nullptr, stream);
}

ACA_EXPORT aca_status aca_advance_frames(aca_lattice *lat, double T, double dt, int8_t *d_frames,
                                         int64_t k_first, int64_t nframes, void *stream)
{
    if (!lat) return fail(ACA_EINVAL, "lattice is NULL");
    if (!is_finite(dt) || !(dt > 0.0)) return fail(ACA_EINVAL, "dt must be finite and > 0");
    if (nframes < 0 || k_first < 0) return fail(ACA_EINVAL, "negative frame range");
    if (nframes > 0 && !d_frames) return fail(ACA_EINVAL, "frames buffer is NULL");
    if (!is_finite((double)(k_first + nframes) * dt))
        return fail(ACA_EINVAL, "frame times overflow");
    FrameRequest fr{d_frames, dt, (long long)k_first, (long long)nframes};
    return advance_impl(lat, T, nframes > 0 ? &fr : nullptr, stream);
}

ACA_EXPORT aca_status aca_set_lag(aca_lattice *lat, double lag)
{
    if (!lat) return fail(ACA_EINVAL, "lattice is NULL");
    if (lat->attached) return fail(ACA_ESTATE, "lattice is a batch member");
    if (!is_finite(lag) || lag < 0.0) return fail(ACA_EINVAL, "lag must be finite and >= 0");
    lat->lag = lag;
    return ACA_OK;
}

namespace {

aca_status advance_impl(aca_lattice *lat, double T, const FrameRequest *fr, void *stream)
{
    if (!lat) return fail(ACA_EINVAL, "lattice is NULL");
    if (lat->attached) return fail(ACA_ESTATE, "lattice is a batch member");
    if (!lat->initialized) return fail(ACA_ESTATE, "aca_init (or aca_resume) first");
    if (!is_finite(T)) return fail(ACA_EINVAL, "horizon must be finite");
    if (!aca_host::horizon_fits_counts(lat->p.rate, T))
        return fail(ACA_EINVAL, "rate * horizon = %.17g exceeds 2^30 (arrival counts are 31-bit)",
                    lat->p.rate * T);
    if (T < lat->last_T)
        return fail(ACA_EINVAL, "horizon %.17g is before the last one %.17g", T,
                    lat->last_T);
    if (T == lat->last_T || T <= 0.0) {
        lat->last_T = std::max(lat->last_T, T);
        return ACA_OK;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const auto t0 = std::chrono::steady_clock::now();
    Plan plan;
    aca_status st = make_plan(lat, T, &plan);
    if (st != ACA_OK) return st;
    if (plan.lds > 64 * 1024)
        HIP_TRY(plan.fast ? aca::set_visit_fast_lds_limit(plan.lds)
                          : aca::set_visit_lds_limit(plan.lds));
    // counters come back through pinned mapped words, or (allocation-free
    // advance) through a copy of the device publish area into this array
    unsigned long long local_ctr[kCounterWords] = {};
    unsigned long long *host = lat->noalloc ? local_ctr : lat->host_ctr;
    const uint64_t tiles = (uint64_t)plan.a.ntiles[0] * plan.a.ntiles[1] * plan.a.ntiles[2];
    const uint64_t bytes_per_launch = launch_region_bytes(lat->p.dim, plan.a);

    // caller state -> snapshot 0; snapshot 1 starts below every copy (zero)
    HIP_TRY(hipMemsetAsync(lat->counters, 0, 8 * kCounterWords, s));
    // Under a lag bound each launch applies only arrivals before
    // min(T, t_min + lag), t_min the least pending time the previous launch
    // saw when it loaded the lattice (all times are >= the last horizon
    // before the first launch).  Launches then go one at a time.
    const bool lagged = lat->lag > 0.0;
    double t_min = lat->last_T;
    auto lag_horizon = [&]() {
        const double h = std::min(T, t_min + lat->lag);
        uint64_t b;
        memcpy(&b, &h, sizeof b);
        return b;
    };
    if (lagged) {
        // both slots' least-pending-time words start above every time
        for (int slot = 0; slot < 2; ++slot)
            HIP_TRY(hipMemsetAsync(lat->counters + slot * kSlotWords + aca::kTminBits, 0xFF, 8,
                                   s));
        plan.a.track_tmin = 1;
        plan.a.horizon_bits = lag_horizon();
    }
    if (fr) {
        plan.a.frames = fr->frames;
        plan.a.frame_dt = fr->dt;
        plan.a.frame_k0 = fr->k0;
        plan.a.nframes = fr->count;
        HIP_TRY(aca::launch_frames_init(plan.a, lat->s, lat->t, lat->last_T, T, s));
    }
    HIP_TRY(aca::launch_pack(lat->n, lat->s, lat->t, lat->cnt, lat->key[0], lat->time[0],
                             lat->counters + kSumStart, s));
    HIP_TRY(hipMemsetAsync(lat->key[1], 0, 8 * lat->n, s));
    HIP_TRY(hipMemsetAsync(lat->time[1], 0, 8 * lat->n, s));

    HIP_TRY(hipMemsetAsync(lat->dead, 0, tiles, s));
    lat->trace.clear();

    // Launch k reads snapshot k % 2, merges into the other one and counts
    // into slot k % 2; its last block publishes the slot to pinned host
    // memory.  While many tiles are live, launch k+1 is enqueued before the
    // host waits for launch k, so the round trip overlaps a kernel; if launch
    // k turns out to be the last one needed, launch k+1 only re-reads the
    // final snapshot (nothing is due, so nothing changes) and is discarded.
    auto enqueue = [&](uint64_t k) -> aca_status {
        const int in = (int)(k & 1), out = 1 - in, slot = in;
        plan.a.key_in = lat->key[in];
        plan.a.time_in = lat->time[in];
        plan.a.key_out = lat->key[out];
        plan.a.time_out = lat->time[out];
        plan.a.counters = lat->counters + slot * kSlotWords;
        plan.a.host_counters = (lat->noalloc ? lat->publish : lat->host_ctr_dev) +
                               slot * kSlotWords;
        plan.a.done_blocks = reinterpret_cast<unsigned int *>(lat->counters + kTicketWord + slot);
        plan.a.dead = lat->dead;
        if (!lat->noalloc) HIP_TRY(hipEventRecord(lat->ev_start[slot], s));
        HIP_TRY(plan.fast ? aca::launch_visit_fast(lat->p.dim, plan.a, plan.block, plan.lds, s)
                          : aca::launch_visit(lat->p.dim, plan.a, plan.block, plan.lds, s));
        if (!lat->noalloc) HIP_TRY(hipEventRecord(lat->ev_stop[slot], s));
        return ACA_OK;
    };
    // Waits for launch k and leaves its counters in host[slot words].  The
    // allocation-free advance runs one launch at a time: the copy of the
    // publish area follows launch k on the stream.
    auto wait_for = [&](uint64_t k, float *kms) -> aca_status {
        const int slot = (int)(k & 1);
        *kms = 0.0f;
        if (lat->noalloc) {
            HIP_TRY(hipMemcpyAsync(host + slot * kSlotWords, lat->publish + slot * kSlotWords,
                                   8 * kSlotWords, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            return ACA_OK;
        }
        HIP_TRY(hipEventSynchronize(lat->ev_stop[slot]));
        HIP_TRY(hipEventElapsedTime(kms, lat->ev_start[slot], lat->ev_stop[slot]));
        return ACA_OK;
    };
    // Every launch applies at least the globally earliest due arrival (the
    // deadlock-freedom argument after Fig. 3.1), and there are finitely many
    // arrivals before T, so the loop ends however many launches that takes.
    // The only watchdog is the check below that a launch applied something.
    aca_status est = enqueue(0);
    if (est != ACA_OK) return est;
    uint64_t enqueued = 1, prev_live = tiles, k = 0, idle = 0;
    for (;; ++k) {
        if (!lagged && !lat->noalloc && enqueued == k + 1 && prev_live * 8 > tiles) {
            est = enqueue(k + 1);
            if (est != ACA_OK) return est;
            ++enqueued;
        }
        const int slot = (int)(k & 1);
        float kms = 0.0f;
        est = wait_for(k, &kms);
        if (est != ACA_OK) return est;
        const unsigned long long *hc = host + slot * kSlotWords;
        aca_stats &S = lat->stats;
        S.kernel_ms += kms;
        S.region_bytes += bytes_per_launch;
        S.launches += 1;
        S.visits += tiles;
        S.ghost_events += hc[aca::kGhostEvents];
        S.sweeps += hc[aca::kSweeps];
        S.cell_checks += hc[aca::kChecks];
        S.scan_live += hc[aca::kScanLive];
        S.scan_enabled += hc[aca::kScanEnabled];
        S.round_cells += hc[aca::kRoundCells];
        if (!lat->noalloc && lat->trace.size() < ACA_TRACE_MAX)
            lat->trace.push_back(aca_launch_record{
                hc[aca::kEvents], hc[aca::kGhostEvents], hc[aca::kScanLive],
                hc[aca::kScanEnabled], hc[aca::kRoundCells], hc[aca::kLiveTiles], (double)kms});
        if (hc[aca::kLiveTiles] == 0) break;
        // under a lag bound one launch may find nothing before its horizon
        // (the least pending time it was set from was stale); the next one
        // starts from a fresh least time
        idle = (hc[aca::kEvents] + hc[aca::kGhostEvents] == 0) ? idle + 1 : 0;
        if (idle > (lat->lag > 0.0 ? 2 : 0))
            return fail(ACA_ENOPROGRESS, "a launch applied no arrival while %llu tiles "
                        "still had arrivals before the horizon",
                        (unsigned long long)hc[aca::kLiveTiles]);
        prev_live = hc[aca::kLiveTiles];
        if (lagged) {
            const unsigned long long tb = hc[aca::kTminBits];
            if (tb != ~0ull) memcpy(&t_min, &tb, sizeof t_min);
            plan.a.horizon_bits = lag_horizon();
        }
        if (enqueued == k + 1) {
            est = enqueue(k + 1);
            if (est != ACA_OK) return est;
            ++enqueued;
        }
    }
    // launch k produced the final record, in snapshot (k + 1) % 2
    const int cur = (int)((k + 1) & 1);
    HIP_TRY(aca::launch_unpack(lat->n, lat->key[cur], lat->time[cur], lat->s, lat->t,
                               lat->cnt, lat->counters + kSumEnd, s));
    HIP_TRY(hipMemcpyAsync(host + kSumStart, lat->counters + kSumStart, 8 * 3,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    lat->stats.events += host[kSumEnd] - host[kSumStart];
    lat->stats.flips += host[kSumFlips];
    lat->last_T = T;
    lat->stats.last_T = T;
    lat->stats.device_ms +=
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
            .count();
    return ACA_OK;
}

}  // namespace

// ------------------------------------------------ allocation-free advance
//
// For callers that may not allocate (serving loops, harnesses that forbid
// it): the working snapshots, tile flags and counters live in one fixed
// device array instead of a caller scratch buffer, and the launch loop reads
// its counters back with plain copies instead of pinned host words.  Each
// device holds its own copy of the array until the process ends.

namespace {

constexpr size_t kStaticScratchBytes = 64ull << 20;
constexpr int kStaticMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_static_mu;
void *g_static_ptr[kStaticMaxDevices];

// Device address of this device's copy of `scratch` (host code must never
// use the array's own name: that is a host-side stand-in, not device memory).
aca_status static_scratch(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= kStaticMaxDevices)
        return fail(ACA_EINVAL, "device %d beyond the %d the static scratch supports", dev,
                    kStaticMaxDevices);
    std::lock_guard<std::mutex> g(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(ACA_EDEVICE, "static scratch has no device address");
        g_static_ptr[dev] = ptr;
    }
    *out = static_cast<unsigned char *>(g_static_ptr[dev]);
    return ACA_OK;
}

// Static scratch bytes a lattice of n cells needs: the scratch layout of
// aca_create plus the two publish slots.
size_t static_scratch_need(uint64_t n)
{
    return scratch_layout(n).total + align_up(8 * 2 * kSlotWords);
}

}  // namespace

ACA_EXPORT aca_status aca_advance_static(const aca_params *p, int8_t *d_spin, double *d_time,
                                         uint32_t *d_count, int32_t draw_initial,
                                         double T_done, double T, void *stream)
{
    uint64_t n = 0;
    aca_params full;
    aca_status st = check_params(p, &n, &full);
    if (st != ACA_OK) return st;
    if (!d_spin || !d_time || !d_count) return fail(ACA_EINVAL, "a device buffer is NULL");
    const void *bufs[3] = {d_spin, d_time, d_count};
    for (const void *b : bufs)
        if (((uintptr_t)b) % kAlign != 0)
            return fail(ACA_EINVAL, "device buffers must be %zu-byte aligned", kAlign);
    const size_t need = static_scratch_need(n);
    if (need > kStaticScratchBytes)
        return fail(ACA_EINVAL,
                    "a lattice of %llu cells needs %zu B of static scratch; the limit is %zu B "
                    "(about %llu cells)", (unsigned long long)n, need, kStaticScratchBytes,
                    (unsigned long long)((kStaticScratchBytes - 2048) / 33));
    if (!is_finite(T_done) || T_done < 0.0)
        return fail(ACA_EINVAL, "T_done must be finite and >= 0");
    if (draw_initial && T_done != 0.0)
        return fail(ACA_EINVAL, "a freshly drawn state starts at T_done = 0");
    if (!is_finite(T) || T < T_done)
        return fail(ACA_EINVAL, "horizon must be finite and >= T_done");
    if (!aca_host::horizon_fits_counts(full.rate, T))
        return fail(ACA_EINVAL, "rate * horizon = %.17g exceeds 2^30 (arrival counts are 31-bit)",
                    full.rate * T);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    unsigned char *base = nullptr;
    st = static_scratch(dev, &base);
    if (st != ACA_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);

    // a handle on the stack over the static scratch: nothing is allocated
    aca_lattice lat;
    const ScratchLayout sl = scratch_layout(n);
    lat.p = full;
    lat.n = n;
    lat.s = d_spin;
    lat.t = d_time;
    lat.cnt = d_count;
    for (int b = 0; b < 2; ++b) {
        lat.key[b] = reinterpret_cast<unsigned long long *>(base + sl.key_off[b]);
        lat.time[b] = reinterpret_cast<unsigned long long *>(base + sl.time_off[b]);
    }
    lat.counters = reinterpret_cast<unsigned long long *>(base + sl.ctr_off);
    lat.dead = reinterpret_cast<uint8_t *>(base + sl.dead_off);
    lat.publish = reinterpret_cast<unsigned long long *>(base + sl.total);
    lat.noalloc = true;
    lat.initialized = true;
    lat.attached = false;
    lat.lag = 0.0;
    lat.last_T = T_done;
    memset(&lat.tun, 0, sizeof lat.tun);
    lat.tun.struct_size = sizeof(aca_tuning);
    lat.tun.ghost[0] = lat.tun.ghost[1] = lat.tun.ghost[2] = -1;
    memset(&lat.stats, 0, sizeof lat.stats);
    lat.stats.struct_size = sizeof(aca_stats);
    build_thresholds(&full, lat.thr);
    lat.device = dev;
    lat.host_ctr = nullptr;
    lat.host_ctr_dev = nullptr;
    for (int i = 0; i < 2; ++i) lat.ev_start[i] = lat.ev_stop[i] = nullptr;

    if (draw_initial) {
        HIP_TRY(aca::launch_init(full.dim, full.L, n, (uint32_t)full.seed,
                                 (uint32_t)(full.seed >> 32), full.rate, full.init, d_spin,
                                 d_time, d_count, s));
    } else {
        // a restored state: the region visits keep a claim in bit 31 of a
        // cell's count word, so every count must be below 2^31
        unsigned long long high = 0;
        HIP_TRY(hipMemsetAsync(lat.counters, 0, 8, s));
        HIP_TRY(aca::launch_count_bound(n, d_count, lat.counters, s));
        HIP_TRY(hipMemcpyAsync(&high, lat.counters, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (high) return fail(ACA_EINVAL, "a count n(c) is 2^31 or more");
    }
    if (T == T_done) {
        HIP_TRY(hipStreamSynchronize(s));
        return ACA_OK;
    }
    return advance_impl(&lat, T, nullptr, stream);
}

ACA_EXPORT aca_status aca_tune(aca_lattice *lat, const aca_tuning *cands, int32_t n, double dT,
                              void *stream, int32_t *best, double *rates, int32_t *n_out)
{
    if (!lat) return fail(ACA_EINVAL, "lattice is NULL");
    if (lat->attached) return fail(ACA_ESTATE, "lattice is a batch member");
    if (!lat->initialized) return fail(ACA_ESTATE, "aca_init (or aca_resume) first");
    if (!is_finite(dT) || !(dT > 0.0)) return fail(ACA_EINVAL, "dT must be finite and > 0");
    aca_tuning table[ACA_TUNE_MAX];
    if (!cands || n <= 0) {
        n = tune_candidates(lat->p.dim, table);
        cands = table;
    }
    if (n > ACA_TUNE_MAX) return fail(ACA_EINVAL, "at most %d candidates", ACA_TUNE_MAX);
    const aca_tuning keep = lat->tun;
    for (int32_t k = 0; k < n; ++k) {
        aca_status st = aca_set_tuning(lat, &cands[k]);
        Plan plan;
        if (st == ACA_OK) st = make_plan(lat, lat->last_T + dT, &plan);
        if (st != ACA_OK) {
            lat->tun = keep;
            return fail(ACA_EINVAL, "candidate %d: %s", k, g_error.c_str());
        }
    }
    aca_status st = aca_set_tuning(lat, &cands[0]);
    if (st == ACA_OK) st = aca_advance(lat, lat->last_T + 0.5 * dT, stream);
    // Each candidate runs two slices of dT/2, the candidates in order and then
    // in reverse order, so that a steady drift of the work per unit of time
    // along the trajectory favours none of them.
    std::vector<double> ev(n, 0.0), ms(n, 0.0);
    for (int32_t j = 0; j < 2 * n && st == ACA_OK; ++j) {
        const int32_t k = j < n ? j : 2 * n - 1 - j;
        st = aca_set_tuning(lat, &cands[k]);
        if (st != ACA_OK) break;
        const uint64_t ev0 = lat->stats.events;
        const double ms0 = lat->stats.device_ms;
        st = aca_advance(lat, lat->last_T + 0.5 * dT, stream);
        if (st != ACA_OK) break;
        ev[k] += (double)(lat->stats.events - ev0);
        ms[k] += lat->stats.device_ms - ms0;
    }
    double best_rate = -1.0;
    int32_t best_k = 0;
    for (int32_t k = 0; k < n && st == ACA_OK; ++k) {
        const double rate = ms[k] > 0.0 ? ev[k] / ms[k] : 0.0;
        if (rates) rates[k] = rate;
        if (rate > best_rate) {
            best_rate = rate;
            best_k = k;
        }
    }
    if (st != ACA_OK) {
        lat->tun = keep;
        return st;
    }
    lat->tun = cands[best_k];
    if (best) *best = best_k;
    if (n_out) *n_out = n;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_set_counting(aca_lattice *lat, int32_t on)
{
    if (!lat) return fail(ACA_EINVAL, "lattice is NULL");
    if (lat->attached) return fail(ACA_ESTATE, "lattice is a batch member");
    lat->count_efficiency = on != 0;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_get_stats(const aca_lattice *lat, aca_stats *out)
{
    if (!lat || !out) return fail(ACA_EINVAL, "NULL argument");
    *out = lat->stats;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_get_thresholds(const aca_lattice *lat, uint64_t *out, int32_t n)
{
    if (!lat || !out) return fail(ACA_EINVAL, "NULL argument");
    const int need = build_thresholds(&lat->p, nullptr);
    if (n < need) return fail(ACA_EINVAL, "n %d < %d entries", n, need);
    memcpy(out, lat->thr, sizeof(uint64_t) * need);
    return ACA_OK;
}

ACA_EXPORT aca_status aca_get_trace(const aca_lattice *lat, aca_launch_record *out, int32_t cap,
                                    int32_t *count)
{
    if (!lat) return fail(ACA_EINVAL, "lattice is NULL");
    if (cap > 0 && !out) return fail(ACA_EINVAL, "out is NULL");
    const size_t held = lat->trace.size();
    const size_t copy = cap > 0 ? std::min(held, (size_t)cap) : 0;
    if (copy) memcpy(out, lat->trace.data(), copy * sizeof(aca_launch_record));
    if (count) *count = (int32_t)held;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_read(aca_lattice *lat, int8_t *h_spin, double *h_time,
                               uint32_t *h_count, void *stream)
{
    if (!lat) return fail(ACA_EINVAL, "lattice is NULL");
    if (lat->attached) return fail(ACA_ESTATE, "lattice is a batch member");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (h_spin) HIP_TRY(hipMemcpyAsync(h_spin, lat->s, lat->n, hipMemcpyDeviceToHost, s));
    if (h_time)
        HIP_TRY(hipMemcpyAsync(h_time, lat->t, 8 * lat->n, hipMemcpyDeviceToHost, s));
    if (h_count)
        HIP_TRY(hipMemcpyAsync(h_count, lat->cnt, 4 * lat->n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return ACA_OK;
}

ACA_EXPORT aca_status aca_destroy(aca_lattice *lat)
{
    if (lat && lat->attached) return fail(ACA_ESTATE, "lattice is a batch member");
    if (lat) {
        for (int i = 0; i < 2; ++i) {
            (void)hipEventDestroy(lat->ev_start[i]);
            (void)hipEventDestroy(lat->ev_stop[i]);
        }
        (void)hipHostFree(lat->host_ctr);
    }
    delete lat;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_philox(const uint32_t *d_ctr, uint64_t seed, uint32_t *d_out,
                                 uint64_t count, void *stream)
{
    if (count == 0) return ACA_OK;
    if (!d_ctr || !d_out) return fail(ACA_EINVAL, "NULL buffer");
    HIP_TRY(aca::launch_philox(d_ctr, seed, d_out, count, static_cast<hipStream_t>(stream)));
    return ACA_OK;
}

ACA_EXPORT aca_status aca_neg_log(const uint64_t *d_w, double *d_out, uint64_t count,
                                  void *stream)
{
    if (count == 0) return ACA_OK;
    if (!d_w || !d_out) return fail(ACA_EINVAL, "NULL buffer");
    HIP_TRY(aca::launch_neg_log(d_w, d_out, count, static_cast<hipStream_t>(stream)));
    return ACA_OK;
}

// aca_region.h -- one tile-region visit for tiles that span no lattice
// direction (device code, included by the kernels that schedule visits).
//
// A region is a tile's own cells, `ghost` extra cells on each side along
// every direction, and a frozen one-cell ring copied from the input snapshot
// (Fig. 3.4's frozen neighbours; the ring only ever holds cells back).  The
// visit loads the region box from the input snapshot, applies every arrival
// it can prove is the next one of its cell (Fig. 3.1's test, with ties broken
// by global index) in rounds over worklists, and merges every owned copy and
// every moved ghost copy into the output snapshot with an element-wise
// maximum.  All copies are prefixes of the one trajectory, so the maximum is
// the most advanced copy; the merge must take it, because a neighbouring
// region may have advanced its own cells on a ghost copy that got further
// than the owner's (the snapshot has to stay a consistent cut).  Layout for
// speed on the large lattices:
//
//  * LDS holds the region box with fixed pitches (the largest box of the
//    plan), so the neighbours of a cell are constant index offsets and the
//    worklists store box indices directly;
//  * after applying an arrival a lane loads the cell's whole second-order
//    neighbourhood once -- 13 words in 2D, 25 in 3D (the cell, its 2*dim
//    neighbours, the cells two steps away and the diagonals) -- and re-tests
//    the cell and its neighbours from those registers;
//  * the initial scan of a visit applies the exact (time, global index)
//    order, taking the index path only when a cell's time equals a
//    neighbour's (rare in binary64); the re-test after an arrival is strict
//    and leaves such a tied cell to the next visit's scan (postponing an
//    enabled arrival never changes the trajectory);
//  * the newly enabled cells of a wavefront are appended with one LDS atomic;
//  * a worklist never holds two cells that read each other (both could not
//    be enabled at once, and a listed cell stays enabled until it applies),
//    so a cell is re-tested by several lanes of a round only as a neighbour
//    of cells they applied: only those pushes take a claim, bit 31 of the
//    cell's arrival-count word (counts stay below 2^31), which the lane that
//    applies the cell's next arrival clears when it writes the new count.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aca_device.h"
#include "aca_internal.h"

#pragma clang fp contract(off)

namespace aca {
namespace region {

// What one visit did, identical in every thread of the workgroup.  The
// values are read from LDS after the visit's last barrier: the caller must
// pass a barrier before the next visit reuses the LDS.
struct RegionTally {
    uint32_t events;      // arrivals applied to owned cells
    uint32_t flips;       // of which reversed the spin
    uint32_t ghost;       // arrivals applied to ghost copies
    uint32_t checks;      // enabling tests evaluated
    int rounds;           // worklist rounds run
    int own_due;          // an owned cell had an arrival before the horizon at load
    int any_live;         // an owned cell still has one after the visit
    int skipped;          // the tile was final in both snapshots: nothing loaded
    uint32_t scan_live;   // owned cells with an arrival before the horizon at load
    uint32_t scan_enabled;   // of which the initial scan listed
    uint64_t round_cells; // simulated cells before this launch's horizon at load, times
                          // the rounds run (the denominator of the per-round fraction)
};

constexpr uint64_t kSign = 0x8000000000000000ull;
constexpr uint64_t kMask = 0x7FFFFFFFFFFFFFFFull;

__device__ __forceinline__ uint64_t ldw(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void stw(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// A region cell's LDS count word: its arrival count n (< 2^31) and, in bit
// 31, the claim of a cell listed by a neighbour's lane (always set on the
// frozen ring, whose cells are never listed).
constexpr uint32_t kClaim = 0x80000000u;
constexpr uint32_t kCountMask = 0x7FFFFFFFu;

// Number of lanes below this one whose bit is set in the wavefront mask m.
__device__ __forceinline__ int lanes_below(uint64_t m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Sum of v over the wavefront, in every lane (cross-lane permutes; every lane
// of the wavefront must be active).
__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += (uint32_t)__shfl_xor((int)v, m);
    return v;
}

// Pending time of a packed word: the spin is the sign bit and every time is
// positive, so |word as binary64| is the time (a free source modifier), and
// binary64 order on these values is the order of their bit patterns.
__device__ __forceinline__ double time_of(uint64_t w)
{
    return __builtin_fabs(__longlong_as_double((long long)w));
}

__device__ __forceinline__ int wrap_into(int g, int side)
{
    g = (g < 0) ? g + side : g;
    return (g >= side) ? g - side : g;
}

// Stencil of offsets loaded after an arrival: index 0 the cell, 1..2D the
// unit steps in slot order (+x, -x, +y, -y, +z, -z), then the steps of two
// along each axis, then the diagonals (two axes, one step each).
template <int DIM>
struct Stencil {
    static constexpr int Z = 2 * DIM;
    static constexpr int K = 1 + 4 * DIM + 2 * DIM * (DIM - 1);
    int d[K][3];
    int nb[Z + 1][Z];   // nb[s][j]: stencil index of (candidate s) + (unit step j)
    // Neighbours s >= 1 of the cell are paired with a perpendicular one where
    // possible; a pair shares the diagonal cell lead[s] (-1: unpaired).
    int partner[Z + 1];
    int lead[Z + 1];

    constexpr Stencil() : d(), nb(), partner(), lead()
    {
        int k = 1;
        for (int a = 0; a < DIM; ++a)
            for (int s = 1; s >= -1; s -= 2) {
                d[k][0] = d[k][1] = d[k][2] = 0;
                d[k][a] = s;
                ++k;
            }
        for (int a = 0; a < DIM; ++a)
            for (int s = 2; s >= -2; s -= 4) {
                d[k][0] = d[k][1] = d[k][2] = 0;
                d[k][a] = s;
                ++k;
            }
        for (int a = 0; a < DIM; ++a)
            for (int b = a + 1; b < DIM; ++b)
                for (int sa = 1; sa >= -1; sa -= 2)
                    for (int sb = 1; sb >= -1; sb -= 2) {
                        d[k][0] = d[k][1] = d[k][2] = 0;
                        d[k][a] = sa;
                        d[k][b] = sb;
                        ++k;
                    }
        for (int s = 0; s <= Z; ++s)
            for (int j = 0; j < Z; ++j) {
                const int want[3] = {d[s][0] + d[1 + j][0], d[s][1] + d[1 + j][1],
                                     d[s][2] + d[1 + j][2]};
                nb[s][j] = -1;
                for (int q = 0; q < K; ++q)
                    if (d[q][0] == want[0] && d[q][1] == want[1] && d[q][2] == want[2])
                        nb[s][j] = q;
            }
        for (int s = 0; s <= Z; ++s) {
            partner[s] = -1;
            lead[s] = -1;
        }
        // slot 1 + j is the unit step j; steps 2a, 2a+1 lie on axis a
        for (int s = 1; s <= Z; ++s) {
            if (partner[s] >= 0) continue;
            for (int t = s + 1; t <= Z && partner[s] < 0; ++t) {
                if (partner[t] >= 0 || (s - 1) / 2 == (t - 1) / 2) continue;
                partner[s] = t;
                partner[t] = s;
                lead[s] = lead[t] = nb[s][t - 1];   // (step s) + (step t)
            }
        }
    }
};

// The q-th degree neighbourhood without the cell: offsets at lattice
// distance 1..Q, in a fixed order (Q > 1 only; Q = 1 uses the slots above).
template <int DIM, int Q>
struct Ball {
    static constexpr int count()
    {
        int m = 0;
        for (int dz = -(DIM > 2 ? Q : 0); dz <= (DIM > 2 ? Q : 0); ++dz)
            for (int dy = -(DIM > 1 ? Q : 0); dy <= (DIM > 1 ? Q : 0); ++dy)
                for (int dx = -Q; dx <= Q; ++dx) {
                    const int r = (dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy) + (dz < 0 ? -dz : dz);
                    m += (r >= 1 && r <= Q) ? 1 : 0;
                }
        return m;
    }
    static constexpr int Z = count();
    int d[Z][3];
    constexpr Ball() : d()
    {
        int m = 0;
        for (int dz = -(DIM > 2 ? Q : 0); dz <= (DIM > 2 ? Q : 0); ++dz)
            for (int dy = -(DIM > 1 ? Q : 0); dy <= (DIM > 1 ? Q : 0); ++dy)
                for (int dx = -Q; dx <= Q; ++dx) {
                    const int r = (dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy) + (dz < 0 ? -dz : dz);
                    if (r >= 1 && r <= Q) {
                        d[m][0] = dx;
                        d[m][1] = dy;
                        d[m][2] = dz;
                        ++m;
                    }
                }
    }
};

struct FastPlan {
    size_t thr_off, ctr_off, tmin_off, ball_off, tab_off, ts_off, n_off, f_off, list_off,
        list_cap, total;
};

// Pitch of the region box along each direction: the box side of the plan's
// tiles (the largest region of the launch), 1 beyond the lattice's dimension.
__host__ __device__ inline void box_pitch(const VisitArgs &a, int dim, int *pitch)
{
    // the frozen ring is as wide as the neighbourhood's reach
    const int ring = a.range > 1 ? a.range : 1;
    for (int d = 0; d < 3; ++d) pitch[d] = d < dim ? a.tile[d] + 2 * a.ghost[d] + 2 * ring : 1;
}

// LDS layout of a region box with the given pitches.
__host__ __device__ inline FastPlan fast_plan(const VisitArgs &a, int dim, const int *pitch)
{
    const int ring = a.range > 1 ? a.range : 1;
    int inner = 1;
    for (int d = 0; d < dim; ++d) inner *= a.tile[d] + 2 * a.ghost[d];
    const size_t boxp = (size_t)pitch[0] * pitch[1] * pitch[2];
    // neighbours the rule reads: 2 dim, or the ball of radius `ring`
    int z = 2 * dim;
    if (ring > 1) {
        z = 0;
        for (int dz = -(dim > 2 ? ring : 0); dz <= (dim > 2 ? ring : 0); ++dz)
            for (int dy = -(dim > 1 ? ring : 0); dy <= (dim > 1 ? ring : 0); ++dy)
                for (int dx = -ring; dx <= ring; ++dx) {
                    const int r = (dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy) + (dz < 0 ? -dz : dz);
                    z += (r >= 1 && r <= ring) ? 1 : 0;
                }
    }
    const size_t thr_words = 2 * (size_t)(z + 1) > 16 ? 2 * (size_t)(z + 1) : 16;
    FastPlan p;
    p.thr_off = 0;                                              // uint64 thr[2 (z + 1)]
    p.ctr_off = 8 * thr_words;                                  // int ctr[16]
    p.tmin_off = p.ctr_off + 64;                                // uint64 least owned time
    p.ball_off = p.tmin_off + 16;                               // int off[32], step[32]
    p.tab_off = p.ball_off + (ring > 1 ? 256 : 0);              // uint32 tx, ty, tz
    // uint64 ts[boxp] with a guard on both sides: the stencil's two-step
    // loads around a cell on the first or last simulated layer may reach one
    // layer beyond the box (those values are never used).  A layer is a row
    // of pitch[0] cells in 2D and 3D and a single cell in 1D, whose box is
    // one row: a guard of two rows there would triple its LDS.
    const size_t guard = 2 * (size_t)(dim == 1 ? 1 : pitch[0]);
    p.ts_off = (p.tab_off + 4 * (size_t)(pitch[0] + pitch[1] + pitch[2]) + 7) & ~(size_t)7;
    p.ts_off += 8 * guard;
    p.n_off = p.ts_off + 8 * (boxp + guard);                    // uint32 n[boxp] | claim
    p.f_off = p.n_off + 4 * boxp;                               // uint8 f[boxp]
    p.list_off = (p.f_off + boxp + 3) & ~(size_t)3;
    // uint16 list[2][cap].  A list never holds two neighbours, so half the
    // simulated cells always fit; fewer are enabled at once in practice (a
    // fifth of them at a random state in 2D, a seventh in 3D, and about half
    // that later), so the lists hold a quarter (2D) or a fifth (3D) plus
    // slack, and a cell that finds its list full is left for the next visit's
    // scan (postponing an enabled arrival never changes the result)
    const size_t half = (size_t)inner / 2 + 2;
    const size_t part = (size_t)inner / (dim == 1 ? 2 : (dim == 2 ? 4 : 5)) + 64;
    p.list_cap = part < half ? part : half;
    p.total = (p.list_off + 4 * p.list_cap + 15) & ~(size_t)15;
    return p;
}

__host__ __device__ inline FastPlan fast_plan(const VisitArgs &a, int dim)
{
    int pitch[3];
    box_pitch(a, dim, pitch);
    return fast_plan(a, dim, pitch);
}

// The snapshots a visit reads and merges into.
struct Snapshots {
    const unsigned long long *key_in;
    const unsigned long long *time_in;
    unsigned long long *key_out;
    unsigned long long *time_out;
};

// FRAMES: capture output frames as arrivals are applied (a separate
// instantiation, so the visit without frames carries none of its registers).
// Q: the reach of the rule (q-th degree neighbourhood); the frozen ring is Q
// cells wide.  Q = 1 is the nearest-neighbour visit tuned above; Q > 1 tests
// and sums over the ball offsets directly.  UNIT: the lattice's rate is 1, so
// the gap is -ln u itself (the general instantiation divides by the rate).
// COUNT: collect the efficiency counters of Section 4 (scan_live,
// scan_enabled, round_cells); without it they are zero.  They cost the visit
// scalar registers, so the visit without them is a kernel of its own.
// CP0, CP1, CP2: the box pitches as compile-time constants (0: taken from the
// plan at run time).  The caller must only pass constants equal to the plan's
// pitches (box_pitch); with them the LDS layout and every stencil offset fold
// into constants, and the stencil reads of an arrival share one base address.
template <int DIM, bool FRAMES = false, int Q = 1, bool UNIT = false, bool COUNT = true,
          int CP0 = 0, int CP1 = 0, int CP2 = 0>
__device__ __forceinline__ RegionTally visit_region(const VisitArgs &a, const Snapshots io,
                                                    uint32_t tile, unsigned char *lds)
{
    constexpr int Z = 2 * DIM;
    constexpr Ball<DIM, (Q > 1 ? Q : 2)> B{};
    constexpr int ZQ = Q > 1 ? Ball<DIM, (Q > 1 ? Q : 2)>::Z : Z;
    constexpr Stencil<DIM> S{};
    constexpr int K = Stencil<DIM>::K;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int nthreads = blockDim.x;

    // a tile whose owned cells are final in both snapshots has nothing to do
    if (a.dead[tile]) return RegionTally{0u, 0u, 0u, 0u, 0, 0, 0, 1, 0u, 0u, 0ull};
    // ---- geometry: box coordinates 0..rin+1 (ring at both ends) per axis
    int tc[3];
    {
        uint32_t b = tile;
        tc[0] = (int)(b % (uint32_t)a.ntiles[0]);
        b /= (uint32_t)a.ntiles[0];
        tc[1] = (int)(b % (uint32_t)a.ntiles[1]);
        tc[2] = (int)(b / (uint32_t)a.ntiles[1]);
    }
    int rin[3], org[3], olo[3], ohi[3], side[3], pitch[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d < DIM) {
            side[d] = a.L[d];
            const int lo = tc[d] * a.tile[d];
            const int w = min(a.tile[d], a.L[d] - lo);
            rin[d] = w + 2 * a.ghost[d];
            org[d] = lo - a.ghost[d] - Q;                 // global coordinate of box 0
            olo[d] = a.ghost[d] + Q;                      // own cells, box coordinates
            ohi[d] = a.ghost[d] + Q + w;
            pitch[d] = a.tile[d] + 2 * a.ghost[d] + 2 * Q;
        } else {
            side[d] = 1; rin[d] = 1; org[d] = 0; olo[d] = 0; ohi[d] = 1; pitch[d] = 1;
        }
    }
    constexpr bool kConstPitch = CP0 > 0;
    if constexpr (kConstPitch) {
        pitch[0] = CP0;
        pitch[1] = CP1 > 0 ? CP1 : 1;
        pitch[2] = CP2 > 0 ? CP2 : 1;
    }
    const int P1 = pitch[0], P12 = pitch[0] * pitch[1];
    const int rb[3] = {DIM > 0 ? rin[0] + 2 * Q : 1, DIM > 1 ? rin[1] + 2 * Q : 1,
                       DIM > 2 ? rin[2] + 2 * Q : 1};
    const uint32_t magic1 = 0xFFFFFFFFu / (uint32_t)P1 + 1u;            // P1 >= 3
    const uint32_t magic2 = pitch[1] > 1 ? 0xFFFFFFFFu / (uint32_t)pitch[1] + 1u : 0u;

    const FastPlan plan = fast_plan(a, DIM, pitch);
    uint64_t *thr = reinterpret_cast<uint64_t *>(lds + plan.thr_off);
    int *ctr = reinterpret_cast<int *>(lds + plan.ctr_off);
    uint32_t *tx = reinterpret_cast<uint32_t *>(lds + plan.tab_off);
    uint32_t *ty = tx + pitch[0];
    uint32_t *tz = ty + pitch[1];
    uint64_t *ts = reinterpret_cast<uint64_t *>(lds + plan.ts_off);
    uint32_t *nl = reinterpret_cast<uint32_t *>(lds + plan.n_off);
    uint8_t *fl = reinterpret_cast<uint8_t *>(lds + plan.f_off);   // flips this visit
    uint16_t *lists = reinterpret_cast<uint16_t *>(lds + plan.list_off);
    const int cap = (int)plan.list_cap;
    int *sizes = ctr;        // [0..2] list lengths, rotating over rounds

    // ---- tables: global offsets of box rows/columns/planes
    uint64_t *tmin_slot = reinterpret_cast<uint64_t *>(lds + plan.tmin_off);
    // Q > 1: box offset and packed coordinate step of every ball entry
    int *ball_box = reinterpret_cast<int *>(lds + plan.ball_off);
    int *ball_step = ball_box + 32;
    if constexpr (Q > 1) {
#pragma unroll
        for (int k = 0; k < ZQ; ++k)
            if (tid == k) {
                ball_box[k] = B.d[k][0] + P1 * B.d[k][1] + P12 * B.d[k][2];
                ball_step[k] = (B.d[k][0] + 16) | ((B.d[k][1] + 16) << 8) |
                               ((B.d[k][2] + 16) << 16);
            }
    }
    if (tid < 2 * (ZQ + 1)) thr[tid] = a.thr[tid];
    if (tid == 0) *tmin_slot = ~0ull;   // least owned pending time (lag bound)
    if (tid < 16) ctr[tid] = 0;
    for (int j = tid; j < rb[0]; j += nthreads) tx[j] = (uint32_t)wrap_into(org[0] + j, side[0]);
    for (int j = tid; j < rb[1]; j += nthreads)
        ty[j] = (uint32_t)(DIM > 1 ? wrap_into(org[1] + j, side[1]) : 0) * (uint32_t)side[0];
    for (int j = tid; j < rb[2]; j += nthreads)
        tz[j] = (uint32_t)(DIM > 2 ? wrap_into(org[2] + j, side[2]) : 0) * (uint32_t)side[0] *
                (uint32_t)side[1];
    const int boxp = pitch[0] * pitch[1] * pitch[2];
    __syncthreads();

    // Box index j = q0 + P1 (q1 + pitch1 q2) of a cell, decoded with the
    // reciprocal multipliers (exact: j and the pitches stay below 2^16).
    auto decode = [&](int j, int *q) {
        const int row = (int)__umulhi((uint32_t)j, magic1);
        q[0] = j - (int)__umul24((uint32_t)row, (uint32_t)P1);          // < 2^16 each
        if (DIM > 2) {
            q[2] = (int)__umulhi((uint32_t)row, magic2);
            q[1] = row - (int)__umul24((uint32_t)q[2], (uint32_t)pitch[1]);
        } else {
            q[1] = row;
            q[2] = 0;
        }
    };
    // global index of box coordinates q (the row and plane tables hold 0
    // along the directions the lattice does not have)
    auto gidx_at = [&](const int *qq) {
        uint32_t g = tx[qq[0]];
        if (DIM > 1) g += ty[qq[1]];
        if (DIM > 2) g += tz[qq[2]];
        return g;
    };
    auto is_own = [&](const int *q) {
        bool own = true;
#pragma unroll
        for (int d = 0; d < DIM; ++d) own = own && q[d] >= olo[d] && q[d] < ohi[d];
        return own;
    };
    auto is_inner = [&](const int *q) {
        bool in = true;
#pragma unroll
        for (int d = 0; d < DIM; ++d) in = in && q[d] >= Q && q[d] < Q + rin[d];
        return in;
    };
    // The same tests as arithmetic, without a branch per condition: a cell is
    // owned (simulated) iff no difference below is negative.
    auto own_bits = [&](const int *q) {
        int t = 0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) t |= (q[d] - olo[d]) | (ohi[d] - 1 - q[d]);
        return t;
    };
    auto inner_bits = [&](const int *q) {
        int t = 0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) t |= (q[d] - Q) | (Q + rin[d] - 1 - q[d]);
        return t;
    };
    // Simulated cell number j in [0, nin) (row-major over the region without
    // its ring) -> box coordinates, by reciprocal multiplies (exact for
    // j < 2^16), and box index of box coordinates.
    const int nin = rin[0] * rin[1] * rin[2];
    const uint32_t imagic0 = rin[0] > 1 ? 0xFFFFFFFFu / (uint32_t)rin[0] + 1u : 0u;
    const uint32_t imagic1 = rin[1] > 1 ? 0xFFFFFFFFu / (uint32_t)rin[1] + 1u : 0u;
    auto inner_coords = [&](int j, int *q) {
        if (DIM == 1) {
            q[0] = j + Q;
            q[1] = 0;
            q[2] = 0;
            return;
        }
        const int row = rin[0] > 1 ? (int)__umulhi((uint32_t)j, imagic0) : j;
        q[0] = j - (int)__umul24((uint32_t)row, (uint32_t)rin[0]) + Q;
        if (DIM == 2) {
            q[1] = row + Q;
            q[2] = 0;
        } else {
            const int pl = rin[1] > 1 ? (int)__umulhi((uint32_t)row, imagic1) : row;
            q[1] = row - (int)__umul24((uint32_t)pl, (uint32_t)rin[1]) + Q;
            q[2] = pl + Q;
        }
    };
    auto box_index = [&](const int *q) {
        return q[0] + P1 * q[1] + (DIM > 2 ? P12 * q[2] : 0);
    };
    // cells per thread in flight in the load loop: 5 measures ~1 % faster than
    // 4 at the default 2D and 3D boxes (compiled pitches); a whole box per step
    // (10 and 9) holds more registers and measures slower, and the batch
    // kernels, already at their register limit, keep 4
    constexpr int U = (Q == 1 && kConstPitch) ? 5 : 4;

    // ---- load the region box from the snapshot; note whether any owned
    // cell still has an arrival before the horizon
    bool due = false;
    uint64_t tmin_own = ~0ull;
    // owned and simulated cells before the horizon, counted per lane (vector
    // registers: wave-uniform counters would add to the scalar registers the
    // rounds need) and summed per wavefront after the loop
    uint32_t cnt_own_live = 0, cnt_inner_live = 0;
    for (int j0 = tid; j0 < boxp; j0 += U * nthreads) {
        bool ok[U], inn[U], own[U];
        uint32_t gi[U];
        unsigned long long key[U], tb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = j0 + u * nthreads;
            int q[3];
            decode(min(j, boxp - 1), q);
            // cells of the pitch beyond a ragged region's box read the box's
            // last cell along that direction (a valid address) and are not kept
            int qc[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) qc[d] = min(q[d], rb[d] - 1);
            ok[u] = (j < boxp) & (q[0] < rb[0]) & (q[1] < rb[1]) & (q[2] < rb[2]);
            inn[u] = inner_bits(q) >= 0;
            own[u] = own_bits(q) >= 0;
            gi[u] = gidx_at(qc);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            key[u] = io.key_in[gi[u]];
            tb[u] = io.time_in[gi[u]];
        }
        if constexpr (COUNT) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                cnt_own_live += (ok[u] && own[u] && (uint64_t)tb[u] < a.final_bits) ? 1u : 0u;
                cnt_inner_live += (ok[u] && inn[u] && (uint64_t)tb[u] < a.horizon_bits) ? 1u : 0u;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool mine = ok[u] & own[u];
            due |= mine & ((uint64_t)tb[u] < a.final_bits);
            tmin_own = (mine & ((uint64_t)tb[u] < tmin_own)) ? (uint64_t)tb[u] : tmin_own;
            if (ok[u]) {
                const int bi = j0 + u * nthreads;
                ts[bi] = (uint64_t)tb[u] | ((key[u] & 1ull) << 63);
                // a ring cell carries a claim that is never cleared: a re-test
                // that finds it enabled can never list it
                nl[bi] = inn[u] ? (uint32_t)(key[u] >> 32) : kClaim;
                fl[bi] = 0;
            }
        }
    }
    if (a.track_tmin && tmin_own != ~0ull) atomicMin(tmin_slot, tmin_own);
    if constexpr (COUNT) {
        // a region box has fewer than 2^16 cells, so both sums fit 16 bits
        const uint32_t both = wave_sum(cnt_own_live | (cnt_inner_live << 16));
        if (lane == 0 && both) {
            atomicAdd(&ctr[10], (int)(both & 0xFFFFu));
            atomicAdd(&ctr[12], (int)(both >> 16));
        }
    }
    const int own_due = __syncthreads_or(due ? 1 : 0);
    if (a.track_tmin && tid == 0 && *tmin_slot != ~0ull)
        atomicMin(&a.counters[kTminBits], (unsigned long long)*tmin_slot);

    // arrivals before this launch's horizon may be applied; cells at or past
    // the advance's horizon are final
    const uint64_t horizon = a.horizon_bits;
    const double horizon_t = __longlong_as_double((long long)horizon);
    const uint64_t final_bits = a.final_bits;
    const double final_t = __longlong_as_double((long long)final_bits);
    const bool unit_rate = UNIT || a.unit_rate != 0;
    // events, flips and ghost events are counted at the merge (count after -
    // count loaded); re-tests are 2 dim + 1 per arrival applied (reach 1)
    uint32_t my_events = 0, my_flips = 0, my_ghost = 0, my_checks = 0, my_applied = 0;

    // Box offset of stencil entry k.
    auto off = [&](int k) { return S.d[k][0] + P1 * S.d[k][1] + P12 * S.d[k][2]; };

    // Exact enabling test (index tie rule) for the cell at box coordinates q
    // with time tc, given its neighbour times tn[j] in slot order.
    auto exact = [&](uint64_t tc, const uint64_t *tn, const int *q) {
        bool en = tc < horizon;
#pragma unroll
        for (int j = 0; j < Z; ++j) {
            const int ax = j >> 1;
            const uint32_t g = ax == 0 ? tx[q[0]] : (ax == 1 ? ty[q[1]] : tz[q[2]]);
            const uint32_t unit = ax == 0 ? 1u
                                  : (ax == 1 ? (uint32_t)side[0]
                                             : (uint32_t)side[0] * (uint32_t)side[1]);
            // +axis neighbour has the larger global index unless it wraps;
            // -axis neighbour the smaller one unless it wraps
            const bool wins = (j & 1) ? (g == 0u) : (g != (uint32_t)(side[ax] - 1) * unit);
            en = en && (tc < tn[j] || (tc == tn[j] && wins));
        }
        return en;
    };

    // ---- Q > 1: the rule's ball, read entry by entry
    auto step_of = [&](int k, int *qq) {
        const int st = ball_step[k];
        qq[0] += (st & 0xFF) - 16;
        qq[1] += ((st >> 8) & 0xFF) - 16;
        qq[2] += ((st >> 16) & 0xFF) - 16;
    };
    // enabled when before the horizon and before every ball cell; `tie` when
    // the least ball time equals the cell's (decided by exact_q)
    auto enabled_q = [&](int xb, uint64_t wx, bool &tie) {
        const double tc = time_of(wx);
        double tmin = time_of(ldw(&ts[xb + ball_box[0]]));
        for (int k = 1; k < ZQ; ++k) tmin = __builtin_fmin(tmin, time_of(ldw(&ts[xb + ball_box[k]])));
        const bool live = tc < horizon_t;
        tie = live && tc == tmin;
        return live && tc < tmin;
    };
    // the (time, global index) order against every ball cell
    auto exact_q = [&](int xb, const int *qx, uint64_t wx) {
        const uint64_t tcb = wx & kMask;
        const uint32_t gx = gidx_at(qx);
        bool en = tcb < horizon;
        for (int k = 0; k < ZQ; ++k) {
            int qy[3] = {qx[0], qx[1], qx[2]};
            step_of(k, qy);
            const uint64_t tyb = ldw(&ts[xb + ball_box[k]]) & kMask;
            en = en && (tcb < tyb || (tcb == tyb && gx < gidx_at(qy)));
        }
        return en;
    };

    int rounds = 0;
    if (own_due) {
    // ---- initial scan: every enabled simulated cell into list 0, US cells
    // per thread per step (their reads issued together, one list atomic per
    // wavefront for all of them; nearest neighbours only)
    constexpr int US = Q == 1 ? 4 : 1;   // a wider reach has no registers to spare
    uint32_t cnt_scan_own = 0;   // owned cells this lane listed
    for (int base = tid - lane; base < nin; base += US * nthreads) {
        bool en[US], owned[US];
        int cell[US];
#pragma unroll
        for (int u = 0; u < US; ++u) {
            const int j = base + u * nthreads + lane;
            int q[3];
            inner_coords(min(j, nin - 1), q);
            const int bi = box_index(q);
            cell[u] = bi;
            en[u] = false;
            owned[u] = own_bits(q) >= 0;
            if (Q > 1 && j < nin) {
                const uint64_t wc = ldw(&ts[bi]);
                bool tie = false;
                en[u] = enabled_q(bi, wc, tie);
                if (tie) en[u] = exact_q(bi, q, wc);
                ++my_checks;
            } else if (Q == 1 && j < nin) {
                const uint64_t wc = ldw(&ts[bi]);
                uint64_t tn[Z];
                double tmin = horizon_t;
                // with compiled pitches: one base register, non-negative
                // constant offsets
                constexpr int omin1 = kConstPitch ? -(DIM > 2 ? CP0 * CP1 : (DIM > 1 ? CP0 : 1)) : 0;
                int sb = bi;
                if constexpr (kConstPitch) {
                    sb = bi + omin1;
                    __asm__("" : "+v"(sb));
                }
#pragma unroll
                for (int k = 0; k < Z; ++k) {
                    tn[k] = ldw(&ts[kConstPitch ? sb + (off(1 + k) - omin1) : bi + off(1 + k)]);
                    tmin = __builtin_fmin(tmin, time_of(tn[k]));
                }
                // below the least of the horizon and the neighbour times; a
                // tie (with the horizon too) takes the exact test
                const double tc = time_of(wc);
                en[u] = tc < tmin;
                if (tc == tmin) {
#pragma unroll
                    for (int k = 0; k < Z; ++k) tn[k] &= kMask;
                    en[u] = exact(wc & kMask, tn, q);
                }
                ++my_checks;
            }
        }
        uint64_t m[US];
        int total = 0;
#pragma unroll
        for (int u = 0; u < US; ++u) {
            m[u] = __ballot(en[u]);
            total += (int)__popcll(m[u]);
            if constexpr (COUNT) cnt_scan_own += (en[u] && owned[u]) ? 1u : 0u;
        }
        if (total) {
            int b0 = 0;
            if (lane == 0) b0 = atomicAdd(&sizes[0], total);
            b0 = __builtin_amdgcn_readfirstlane(b0);  // lane 0 is active
#pragma unroll
            for (int u = 0; u < US; ++u) {
                const int at = b0 + lanes_below(m[u]);
                if (en[u] && at < cap) lists[at] = (uint16_t)cell[u];
                b0 += (int)__popcll(m[u]);
            }
        }
    }
    if constexpr (COUNT) {
        cnt_scan_own = wave_sum(cnt_scan_own);
        if (lane == 0 && cnt_scan_own) atomicAdd(&ctr[11], (int)cnt_scan_own);
    }
    __syncthreads();

    // ---- worklist rounds
    for (int rnd = 0; rnd < a.max_sweeps; ++rnd) {
        const int sz = min(sizes[rnd % 3], cap);   // appends past the cap were dropped
        if (sz == 0) break;
        ++rounds;
        if (tid == 0) sizes[(rnd + 2) % 3] = 0;
        uint16_t *lcur = lists + (rnd & 1) * cap;
        uint16_t *lnext = lists + (1 - (rnd & 1)) * cap;
        int *next_size = &sizes[(rnd + 1) % 3];
        // wavefront w takes the 64-entry slices w, w + W, w + 2W, ... of
        // the list (every slice costs about the same, so a fixed stride
        // balances as well as taking slices from a shared counter)
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int nwaves = nthreads >> 6;
        for (int start = 64 * wave; start < sz; start += 64 * nwaves) {
            const bool active = lane < sz - start;
            if constexpr (Q > 1) {
                // ---- one arrival per lane, rule over the ball
                int bi = 0, q[3] = {0, 0, 0};
                if (active) {
                    bi = lcur[start + lane];
                    decode(bi, q);
                    const uint64_t w0 = ldw(&ts[bi]);
                    int sum = 0;
                    for (int k = 0; k < ZQ; ++k) sum += (ldw(&ts[bi + ball_box[k]]) >> 63) ? -1 : 1;
                    const uint32_t kn = nl[bi] & kCountMask;   // claim bit off
                    const uint32_t gidx = gidx_at(q);
                    const Draw y = philox4x32_10(kn, gidx, 0u, 0u, a.key_lo, a.key_hi);
                    const int idx = (sum + ZQ) / 2 + (ZQ + 1) * ((w0 >> 63) ? 0 : 1);
                    const bool flip = (uint64_t)y.w2 < thr[idx];
                    const double tnow = __longlong_as_double((long long)(w0 & kMask));
                    const double tnext = tnow + arrival_gap(y.w0, y.w1, a.rate, unit_rate);
                    const uint64_t wnew = (uint64_t)__double_as_longlong(tnext) |
                                          ((w0 & kSign) ^ (flip ? kSign : 0ull));
                    if (FRAMES)
                        capture_frames(a.frames, a.frame_dt, a.frame_k0, a.nframes, a.n_cells,
                                       gidx, tnow, __builtin_fmin(tnext, final_t),
                                       (wnew >> 63) ? (int8_t)-1 : (int8_t)1);
                    nl[bi] = kn + 1u;
                    fl[bi] = (uint8_t)(fl[bi] + (flip ? 1u : 0u));
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    stw(&ts[bi], wnew);
                }
                // re-test the applied cell and every cell of its ball (they
                // hold it in theirs) once this lane's arrival is published
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
                for (int k = -1; k < ZQ; ++k) {
                    int qx[3] = {q[0], q[1], q[2]};
                    int xb = bi;
                    if (k >= 0) {
                        step_of(k, qx);
                        xb += ball_box[k];
                    }
                    const bool inside = active && is_inner(qx);
                    bool want = false, tie = false;
                    uint64_t wx = 0;
                    if (inside) {
                        wx = ldw(&ts[xb]);
                        want = enabled_q(xb, wx, tie);
                        ++my_checks;
                    }
                    if (__ballot(tie)) {
                        if (tie) want = exact_q(xb, qx, wx);
                    }
                    if (want && k >= 0) want = (atomicOr(&nl[xb], kClaim) & kClaim) == 0u;
                    const uint64_t mk = __ballot(want);
                    if (mk) {
                        int b0 = 0;
                        if (lane == 0) b0 = atomicAdd(next_size, (int)__popcll(mk));
                        b0 = __builtin_amdgcn_readfirstlane(b0);  // lane 0 is active
                        const int at = b0 + lanes_below(mk);
                        if (want && at < cap) lnext[at] = (uint16_t)xb;
                    }
                }
                continue;
            }
            int bi = 0, q[3] = {0, 0, 0};
            uint64_t W[K];
            // least of the horizon and the applied cell's neighbour times:
            // they cannot change while the cell is listed, so its own re-test
            // can use the value taken before the arrival is applied
            double own_tmin = 0.0;
            if (active) {
                bi = lcur[start + lane];
                const int row = (int)__umulhi((uint32_t)bi, magic1);   // q1 + pitch1 q2
                q[0] = bi - (int)__umul24((uint32_t)row, (uint32_t)P1);
                if (DIM > 2) {
                    q[2] = (int)__umulhi((uint32_t)row, magic2);
                    q[1] = row - (int)__umul24((uint32_t)q[2], (uint32_t)pitch[1]);
                } else {
                    q[1] = row;
                }
                // the cell and its neighbour slots: stable until it applies
                // its arrival (no neighbour can be enabled meanwhile)
                if constexpr (kConstPitch) {
                    // one base register below the stencil, non-negative
                    // constant offsets (LDS immediates are unsigned)
                    constexpr int omin = -2 * (DIM > 2 ? CP0 * CP1 : (DIM > 1 ? CP0 : 1));
                    int wb = bi + omin;
                    __asm__("" : "+v"(wb));
#pragma unroll
                    for (int k = 0; k <= Z; ++k) W[k] = ldw(&ts[wb + (off(k) - omin)]);
                } else {
#pragma unroll
                    for (int k = 0; k <= Z; ++k) W[k] = ldw(&ts[bi + off(k)]);
                }
                own_tmin = horizon_t;
#pragma unroll
                for (int k = 1; k <= Z; ++k) own_tmin = __builtin_fmin(own_tmin, time_of(W[k]));
                // (sum of neighbour spins + Z) / 2 = Z - (number of -1 neighbours)
                int neg = 0;
#pragma unroll
                for (int j = 1; j <= Z; ++j) neg += (int)(W[j] >> 63);
                const uint32_t kn = nl[bi] & kCountMask;   // claim bit off
                const uint32_t gidx = gidx_at(q);
                const Draw y = philox4x32_10(kn, gidx, 0u, 0u, a.key_lo, a.key_hi);
                const int idx = (Z - neg) + (Z + 1) * ((W[0] >> 63) ? 0 : 1);
                const bool flip = (uint64_t)y.w2 < thr[idx];
                const double tnow = __longlong_as_double((long long)(W[0] & kMask));
                const double tnext = tnow + arrival_gap(y.w0, y.w1, a.rate, unit_rate);
                const uint64_t wnew = (uint64_t)__double_as_longlong(tnext) |
                                      ((W[0] & kSign) ^ (flip ? kSign : 0ull));
                if (FRAMES)
                    capture_frames(a.frames, a.frame_dt, a.frame_k0, a.nframes, a.n_cells, gidx, tnow, __builtin_fmin(tnext, final_t),
                                   (wnew >> 63) ? (int8_t)-1 : (int8_t)1);
                nl[bi] = kn + 1u;
                fl[bi] = (uint8_t)(fl[bi] + (flip ? 1u : 0u));
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                stw(&ts[bi], wnew);
                W[0] = wnew;
                ++my_applied;
            }
            // The rest of the neighbourhood is read only after this lane's
            // arrival is published: of two cells that share a neighbour and
            // apply arrivals concurrently, the one that reads later then sees
            // both new words, so a neighbour they both unblocked is found.
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
            if (active) {
                int wb = bi;
                constexpr int omin = kConstPitch ? -2 * (DIM > 2 ? CP0 * CP1 : (DIM > 1 ? CP0 : 1)) : 0;
                if constexpr (kConstPitch) {
                    wb = bi + omin;
                    __asm__("" : "+v"(wb));
                }
#pragma unroll
                for (int k = Z + 1; k < K; ++k) {
                    if (DIM > 2 && (S.d[k][2] == 2 || S.d[k][2] == -2)) {
                        // two steps along z may leave the box (and its guard);
                        // such words are never used, so any in-range address will do
                        W[k] = ldw(&ts[min(max(bi + off(k), 0), boxp - 1)]);
                    } else if constexpr (kConstPitch) {
                        W[k] = ldw(&ts[wb + (off(k) - omin)]);
                    } else {
                        W[k] = ldw(&ts[bi + off(k)]);
                    }
                }
            }
            // re-test the applied cell (s = 0) and its neighbours (s = 1..Z):
            // enabled when its time is below the least of the horizon and the
            // neighbour times.  The test is strict: a cell whose time equals a
            // neighbour's (rare in binary64) is not listed even when the index
            // rule would let it go first; it waits for the next visit's initial
            // scan, which applies the exact (time, index) order.  Postponing an
            // enabled arrival is always allowed, so the result is the same.
            bool want[Z + 1];
            // (the minimum is exact, so the shared terms -- the horizon and
            // the applied cell for s >= 1, and a diagonal for each pair of
            // perpendicular neighbours -- are taken once)
            const double near0 = __builtin_fmin(horizon_t, time_of(W[0]));
            double pre[Z + 1];
#pragma unroll
            for (int s = 1; s <= Z; ++s) {
                if (S.lead[s] < 0)
                    pre[s] = near0;
                else if (S.partner[s] < s)
                    pre[s] = pre[S.partner[s]];
                else
                    pre[s] = __builtin_fmin(near0, time_of(W[S.lead[s]]));
            }
#pragma unroll
            for (int s = 0; s <= Z; ++s) {
                // a ring neighbour is tested too; its claim never succeeds
                const double tc = time_of(W[s]);
                double tmin = s == 0 ? own_tmin : pre[s];
#pragma unroll
                for (int j = 0; j < Z; ++j) {
                    const int k = S.nb[s][j];
                    if (s > 0 && k != 0 && k != S.lead[s])
                        tmin = __builtin_fmin(tmin, time_of(W[k]));
                }
                want[s] = active && tc < tmin;
            }
            // claim the neighbours; one already claimed by another lane is not
            // listed twice (the applied cell itself is tested by this lane only).
            // Every active lane issues all 2 dim claims at once, or-ing 0 into
            // the neighbours it does not want (none of them is applied in this
            // round: they are adjacent to a listed cell), and waits once.
            // take[s] is kClaim while cell s is to be listed by this lane
            int cb[Z + 1];
            uint32_t take[Z + 1];
#pragma unroll
            for (int s = 0; s <= Z; ++s) {
                cb[s] = bi + off(s);
                take[s] = want[s] ? kClaim : 0u;
            }
            if (active) {
                if constexpr (kConstPitch) {
                    constexpr int omin1 = -(DIM > 2 ? CP0 * CP1 : (DIM > 1 ? CP0 : 1));
                    int nb0 = bi + omin1;
                    __asm__("" : "+v"(nb0));
#pragma unroll
                    for (int s = 1; s <= Z; ++s)
                        take[s] &= ~atomicOr(&nl[nb0 + (off(s) - omin1)], take[s]);
                } else {
#pragma unroll
                    for (int s = 1; s <= Z; ++s) take[s] &= ~atomicOr(&nl[cb[s]], take[s]);
                }
            }
            // one LDS atomic per wavefront for all its new list entries
            uint64_t mk[Z + 1];
            int total = 0;
#pragma unroll
            for (int s = 0; s <= Z; ++s) {
                mk[s] = __ballot(take[s] != 0u);
                total += (int)__popcll(mk[s]);
            }
            if (total) {
                int b0 = 0;
                if (lane == 0) b0 = atomicAdd(next_size, total);
                b0 = __builtin_amdgcn_readfirstlane(b0);  // lane 0 is active
                // a lane with nothing to list writes into the current list's
                // entry it took this batch, which nothing reads again
                if (active) {
                    const int spare = (int)(lcur - lists) + start + lane;
                    const int nbase = (int)(lnext - lists);
                    if (b0 + total <= cap) {   // the common case: all entries fit
#pragma unroll
                        for (int s = 0; s <= Z; ++s) {
                            const int below = lanes_below(mk[s]);
                            lists[take[s] ? nbase + b0 + below : spare] = (uint16_t)cb[s];
                            b0 += (int)__popcll(mk[s]);
                        }
                    } else {
#pragma unroll
                        for (int s = 0; s <= Z; ++s) {
                            const int at = b0 + lanes_below(mk[s]);
                            lists[(take[s] && at < cap) ? nbase + at : spare] = (uint16_t)cb[s];
                            b0 += (int)__popcll(mk[s]);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    }  // own_due

    // ---- merge owned copies and moved ghost copies; find due owned cells.
    // The merge walks the simulated cells only (the frozen ring is never
    // merged).  A step first computes the box and global index of each of its
    // cells and reads all their input keys, before it issues any merge atomic
    // (reads, stores and atomics complete in order on one counter, so a read
    // issued after atomics would wait for them); the indices stay in registers
    // for the second pass.  For nearest neighbours a thread takes 12 cells
    // per step in 1D and 2D (6144 per step for 512 threads, against 5248
    // simulated cells of a default 2D region) and 8 in 3D (two steps of 768
    // threads for a default region's 8712; fewer registers held measure
    // faster there).
    constexpr int UM = Q == 1 ? (DIM > 2 ? 8 : 12) : 4;   // a wider reach has no registers to spare
    bool live = false;
    for (int j0 = tid; j0 < nin; j0 += UM * nthreads) {
        unsigned long long key_in[UM];
        int bix[UM];
        uint32_t gix[UM];
        bool ownx[UM];
#pragma unroll
        for (int u = 0; u < UM; ++u) {
            const int j = j0 + u * nthreads;
            int q[3];
            inner_coords(min(j, nin - 1), q);
            bix[u] = box_index(q);
            gix[u] = gidx_at(q);
            ownx[u] = own_bits(q) >= 0;
        }
#pragma unroll
        for (int u = 0; u < UM; ++u) {
            // a step's last slots may lie past the region for a whole wavefront
            const int wave_first = __builtin_amdgcn_readfirstlane(j0 - lane) + u * nthreads;
            key_in[u] = wave_first < nin ? io.key_in[gix[u]] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < UM; ++u) {
            const int bi = bix[u];
            const uint32_t n_copy = nl[bi] & kCountMask;   // a listed cell may be claimed
            const uint64_t wd = ts[bi];
            const uint32_t fc = fl[bi];
            const bool valid = j0 + u * nthreads < nin;
            const bool own = valid & ownx[u];
            const uint32_t moved = valid ? n_copy - (uint32_t)(key_in[u] >> 32) : 0u;
            my_events += own ? moved : 0u;
            my_flips += own ? fc : 0u;
            my_ghost += own ? 0u : moved;
            live |= own & ((wd & kMask) < final_bits);
            if (own | (moved != 0u)) {
                const unsigned long long f = ((key_in[u] >> 1) & 0x7FFFFFFFull) + fc;
                atomicMax(&io.key_out[gix[u]],
                          ((unsigned long long)n_copy << 32) | (f << 1) | (wd >> 63));
                atomicMax(&io.time_out[gix[u]], (unsigned long long)(wd & kMask));
            }
        }
    }
    atomicAdd(&ctr[6], (int)my_events);
    atomicAdd(&ctr[7], (int)my_flips);
    atomicAdd(&ctr[8], (int)my_ghost);
    atomicAdd(&ctr[9], (int)(my_checks + (Q == 1 ? (uint32_t)(Z + 1) * my_applied : 0u)));
    const int any_live = __syncthreads_or(live ? 1 : 0);
    return RegionTally{(uint32_t)ctr[6], (uint32_t)ctr[7], (uint32_t)ctr[8], (uint32_t)ctr[9],
                       rounds, own_due, any_live, 0, (uint32_t)ctr[10], (uint32_t)ctr[11],
                       (uint64_t)(uint32_t)ctr[12] * (uint64_t)rounds};
}

}  // namespace region
}  // namespace aca

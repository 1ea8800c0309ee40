// aca_kernels.hip -- gfx950 kernels of the conservative Ising simulation.
//
// aca_init_kernel   one lane per cell: the cell's initial draw gives its first
//                   arrival time and (optionally) its spin.
// visit_kernel      one workgroup per tile region (the aggregation of
//                   Fig. 3.3/3.4): the region is loaded into LDS, its cells
//                   run the asynchronous conservative rule of Fig. 3.1 until
//                   none can move, and every simulated copy is merged into
//                   the next snapshot.
// pack / unpack     caller's (spin, time, count) arrays <-> working words.
//
// Region layout.  A tile owns an axis-aligned box of cells.  Along every
// direction it does not span, the region adds `ghost` cells on both sides
// (simulated, then discarded) and a one-cell frozen ring beyond them whose
// (spin, time) are copies taken at load time.  A frozen copy only ever holds
// a neighbour back -- it can never let a cell apply an arrival the true
// neighbour would have blocked -- so every arrival applied inside the region
// is an arrival of the unique trajectory (the argument with cells v and x
// after Fig. 3.5).  Along a direction the tile spans, the region is the whole
// periodic side and neighbours wrap inside it.
//
// State in LDS.  Each region cell's spin and pending arrival time live in one
// 64-bit word: the time (always > 0) with the spin's sign in bit 63.  A
// neighbour therefore reads spin and time of a cell atomically; this is what
// makes the in-tile schedule race-free without barriers between arrivals:
// a cell tests its neighbours' words, and if its own (time, index) is the
// smallest it applies the arrival and publishes the new word with one
// 64-bit store (after its count).  While a cell is enabled none of its
// neighbours can become enabled (the order is total), so nothing it read can
// change before it applies its arrival (Fig. 3.1 and the uniqueness argument
// that follows it).
//
// Work distribution.  One scan at the start of a visit lists every enabled
// cell.  After that a cell's status can only change when it or a neighbour
// applies an arrival, so the visit proceeds in rounds over worklists: the
// wavefronts take the current list 64 cells at a time (the Philox draw and
// the logarithm run on full wavefronts), and each lane then re-tests the cell
// it applied and that cell's neighbour slots; a newly enabled cell is claimed
// with an LDS bit (so it is listed once) and appended, with one LDS atomic
// per wavefront, to the next round's list.  A barrier separates rounds; the
// visit ends when a round's list is empty or after max_sweeps rounds.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aca_device.h"
#include "aca_internal.h"

#pragma clang fp contract(off)

namespace aca {
namespace {

constexpr uint64_t kSignBit = 0x8000000000000000ull;
constexpr uint64_t kTimeMask = 0x7FFFFFFFFFFFFFFFull;

__device__ __forceinline__ int wrap_side(int g, int side)
{
    g = (g < 0) ? g + side : g;
    return (g >= side) ? g - side : g;
}

__device__ __forceinline__ uint64_t lds_load_word(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_store_word(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// LDS carve-up shared with visit_lds_bytes().  Per region: packed words for
// the whole box, counts / flip deltas / claim bits for the simulated cells,
// and two lists of cell indices (a list never holds two neighbours, so half
// the simulated cells plus one bounds it).
struct LdsPlan {
    size_t thr_off, ctr_off, ts_off, n_off, f_off, claim_off, list_off, list_cap, total;
};

__host__ __device__ inline LdsPlan lds_plan(int box_max, int inner_max)
{
    LdsPlan p;
    p.thr_off = 0;                                          // uint64 thr[16]
    p.ctr_off = 128;                                        // int counters[16]
    p.ts_off = 192;                                         // uint64 ts[box]
    p.n_off = p.ts_off + 8 * (size_t)box_max;               // uint32 n[inner]
    p.f_off = p.n_off + 4 * (size_t)inner_max;              // uint16 f[inner]
    p.claim_off = (p.f_off + 2 * (size_t)inner_max + 3) & ~(size_t)3;
    p.list_off = p.claim_off + 4 * (size_t)((inner_max + 31) / 32 + 2);
    p.list_cap = (size_t)inner_max / 2 + 2;                 // uint16 list[2][cap]
    p.total = p.list_off + 2 * 2 * p.list_cap;
    p.total = (p.total + 15) & ~(size_t)15;
    return p;
}

__host__ __device__ inline int region_box_max(int dim, const VisitArgs &a, int *inner_max)
{
    int box = 1, inner = 1;
    for (int d = 0; d < dim; ++d) {
        const int rin = a.span[d] ? a.L[d] : a.tile[d] + 2 * a.ghost[d];
        inner *= rin;
        box *= rin + (a.span[d] ? 0 : 2);
    }
    if (inner_max) *inner_max = inner;
    return box;
}

// ----------------------------------------------------------------- init

__global__ void aca_init_kernel(uint64_t n_cells, uint32_t key_lo, uint32_t key_hi,
                                double rate, int unit_rate, int init, int8_t *s,
                                double *t, uint32_t *n)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells;
         c += stride) {
        const Draw y = philox4x32_10(0u, (uint32_t)c, 1u, 0u, key_lo, key_hi);
        t[c] = arrival_gap(y.w0, y.w1, rate, unit_rate != 0);
        int8_t spin;
        if (init == 0) spin = (y.w2 & 1u) ? (int8_t)1 : (int8_t)-1;
        else spin = (init == 1) ? (int8_t)1 : (int8_t)-1;
        s[c] = spin;
        n[c] = 0u;
    }
}

// ----------------------------------------------------------------- visit

// Exact quotient n / d from one high multiply with magic = ceil(2^32 / d),
// valid for n * d < 2^32 (here n < 2^16, d < 2^16); d == 1 is passed as
// magic == 0 and returns n.
__device__ __forceinline__ int div_magic(int n, uint32_t magic)
{
    return magic ? (int)__umulhi((uint32_t)n, magic) : n;
}

__device__ __forceinline__ uint32_t magic_for(int d)
{
    return d > 1 ? 0xFFFFFFFFu / (uint32_t)d + 1u : 0u;
}

template <int DIM>
struct Region {
    int rin[3], ring[3], org[3], olo[3], ohi[3], side[3], span[3];
    int sbox[3];          // strides of the ring box
    uint32_t magic[2];    // for dividing by rin[0], rin[1]
    int inner, box;
    int gs1, gs2;         // global strides

    __device__ __forceinline__ void coords(int i, int p[3]) const
    {
        const int r = (DIM > 1) ? div_magic(i, magic[0]) : 0;
        p[0] = i - r * rin[0];
        if (DIM > 2) {
            p[2] = div_magic(r, magic[1]);
            p[1] = r - p[2] * rin[1];
        } else {
            p[1] = r;
            p[2] = 0;
        }
    }
    __device__ __forceinline__ int box_index(const int p[3]) const
    {
        return (p[0] + ring[0]) + sbox[1] * (p[1] + ring[1]) + sbox[2] * (p[2] + ring[2]);
    }
    __device__ __forceinline__ int inner_index(const int p[3]) const
    {
        return p[0] + rin[0] * (p[1] + rin[1] * p[2]);
    }
    __device__ __forceinline__ int global_coord(int d, int pd) const
    {
        return wrap_side(org[d] + pd, side[d]);
    }
    __device__ __forceinline__ uint32_t global_index(const int p[3]) const
    {
        uint32_t g = (uint32_t)global_coord(0, p[0]);
        if (DIM > 1) g += (uint32_t)gs1 * (uint32_t)global_coord(1, p[1]);
        if (DIM > 2) g += (uint32_t)gs2 * (uint32_t)global_coord(2, p[2]);
        return g;
    }
    // Box offsets of the +d / -d neighbours of a simulated cell at p.
    __device__ __forceinline__ void slot_offsets(int d, const int p[3], int &up, int &dn) const
    {
        up = sbox[d];
        dn = -sbox[d];
        if (span[d]) {
            if (p[d] == rin[d] - 1) up -= rin[d] * sbox[d];
            if (p[d] == 0) dn += rin[d] * sbox[d];
        }
    }
};

// Enabling test of Fig. 3.1 for the simulated cell at p: its pending arrival
// is before the horizon and precedes, in (time, global index) order, the
// pending arrival of every neighbour slot.  No branches: every neighbour word
// is loaded and the comparisons are combined bitwise.
template <int DIM>
__device__ __forceinline__ bool cell_enabled(const Region<DIM> &R, const uint64_t *ts,
                                             const int p[3], int bi, uint64_t horizon)
{
    const uint64_t tw = lds_load_word(&ts[bi]) & kTimeMask;
    uint64_t tn[2 * DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        int up, dn;
        R.slot_offsets(d, p, up, dn);
        tn[2 * d] = lds_load_word(&ts[bi + up]) & kTimeMask;
        tn[2 * d + 1] = lds_load_word(&ts[bi + dn]) & kTimeMask;
    }
    bool en = tw < horizon;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        // on equal times the smaller global index goes first: the +d
        // neighbour has the larger index unless it wraps round the lattice,
        // the -d neighbour the smaller one unless it wraps
        const int gd = R.global_coord(d, p[d]);
        const bool up_ok = (tw < tn[2 * d]) | ((tw == tn[2 * d]) & (gd + 1 < R.side[d]));
        const bool dn_ok = (tw < tn[2 * d + 1]) | ((tw == tn[2 * d + 1]) & (gd == 0));
        en = en & up_ok & dn_ok;
    }
    return en;
}

// Append the cells of the lanes with `want` set to the list at `list` whose
// length counter is *size; one LDS atomic per wavefront.
__device__ __forceinline__ void wave_append(bool want, uint16_t value, uint16_t *list,
                                            int *size, int lane)
{
    const uint64_t m = __ballot(want);
    if (m) {
        int base = 0;
        if (lane == 0) base = atomicAdd(size, (int)__popcll(m));
        base = __shfl(base, 0, 64);
        if (want) list[base + (int)__popcll(m & ((1ull << lane) - 1ull))] = value;
    }
}

// FRAMES: capture output frames as arrivals are applied (its own
// instantiation, so the visit without frames carries none of its registers).
template <int DIM, bool FRAMES>
__global__ void __launch_bounds__(1024) visit_kernel(VisitArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int nthreads = blockDim.x;

    // ---- region geometry of this tile
    const unsigned int ntiles_total = (unsigned)a.ntiles[0] * (unsigned)a.ntiles[1] *
                                      (unsigned)a.ntiles[2];
    // a tile whose owned cells are final in both snapshots has nothing to do
    if (a.dead[blockIdx.x]) {
        if (threadIdx.x == 0) finish_visit_block(a, ntiles_total);
        return;
    }
    Region<DIM> R;
    int tc[3];
    {
        uint32_t b = blockIdx.x;
        tc[0] = (int)(b % (uint32_t)a.ntiles[0]);
        b /= (uint32_t)a.ntiles[0];
        tc[1] = (int)(b % (uint32_t)a.ntiles[1]);
        tc[2] = (int)(b / (uint32_t)a.ntiles[1]);
    }
    int rbox[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R.span[d] = 1;
        if (d < DIM) {
            R.side[d] = a.L[d];
            R.span[d] = a.span[d];
            const int lo = tc[d] * a.tile[d];
            const int w = min(a.tile[d], a.L[d] - lo);
            if (a.span[d]) {
                R.rin[d] = a.L[d]; R.ring[d] = 0; R.org[d] = 0; R.olo[d] = 0; R.ohi[d] = a.L[d];
            } else {
                R.rin[d] = w + 2 * a.ghost[d]; R.ring[d] = 1; R.org[d] = lo - a.ghost[d];
                R.olo[d] = a.ghost[d]; R.ohi[d] = a.ghost[d] + w;
            }
        } else {
            R.side[d] = 1; R.rin[d] = 1; R.ring[d] = 0; R.org[d] = 0; R.olo[d] = 0; R.ohi[d] = 1;
        }
        rbox[d] = R.rin[d] + 2 * R.ring[d];
    }
    R.sbox[0] = 1;
    R.sbox[1] = rbox[0];
    R.sbox[2] = rbox[0] * rbox[1];
    R.inner = R.rin[0] * R.rin[1] * R.rin[2];
    R.box = rbox[0] * rbox[1] * rbox[2];
    R.gs1 = R.side[0];
    R.gs2 = R.side[0] * R.side[1];
    R.magic[0] = magic_for(R.rin[0]);
    R.magic[1] = magic_for(R.rin[1]);

    int inner_max = 0;
    const int box_max = region_box_max(DIM, a, &inner_max);
    const LdsPlan plan = lds_plan(box_max, inner_max);
    uint64_t *thr = reinterpret_cast<uint64_t *>(lds + plan.thr_off);
    int *ctr = reinterpret_cast<int *>(lds + plan.ctr_off);
    uint64_t *ts = reinterpret_cast<uint64_t *>(lds + plan.ts_off);
    uint32_t *nl = reinterpret_cast<uint32_t *>(lds + plan.n_off);
    uint16_t *fl = reinterpret_cast<uint16_t *>(lds + plan.f_off);
    uint32_t *claim = reinterpret_cast<uint32_t *>(lds + plan.claim_off);
    uint16_t *lists = reinterpret_cast<uint16_t *>(lds + plan.list_off);
    const int list_cap = (int)plan.list_cap;
    // ctr[0..2] list sizes and ctr[3..5] take positions, rotating over rounds;
    // ctr[6..9] statistics
    int *sizes = ctr;
    int *takes = ctr + 3;

    if (tid < 2 * (2 * DIM + 1)) thr[tid] = a.thr[tid];
    if (tid < 16) ctr[tid] = 0;
    for (int j = tid; j < (R.inner + 31) / 32; j += nthreads) claim[j] = 0u;

    // ---- load the region box from the snapshot; note whether any owned
    // cell still has an arrival before the horizon
    __shared__ unsigned long long tmin_block;    // least owned pending time (lag bound)
    if (tid == 0) tmin_block = ~0ull;
    __syncthreads();
    bool due = false;
    uint64_t tmin_own = ~0ull;
    // owned and simulated cells before the horizon at load (Section 4's
    // efficiency instruments), counted by lane 0 of each wavefront
    uint32_t cnt_own_live = 0, cnt_inner_live = 0;
    for (int j = tid; j < R.box; j += nthreads) {
        int q[3];
        q[0] = j % rbox[0];
        const int r = j / rbox[0];
        q[1] = r % rbox[1];
        q[2] = r / rbox[1];
        int g[3];
        bool in_core = true;
        int pi[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            g[d] = (d < DIM) ? wrap_side(R.org[d] - R.ring[d] + q[d], R.side[d]) : 0;
            pi[d] = q[d] - R.ring[d];
            in_core = in_core && pi[d] >= 0 && pi[d] < R.rin[d];
        }
        const uint32_t gi = (uint32_t)g[0] + (uint32_t)R.gs1 * (uint32_t)g[1] +
                            (uint32_t)R.gs2 * (uint32_t)g[2];
        const unsigned long long key = a.key_in[gi];
        const unsigned long long tb = a.time_in[gi];
        ts[j] = (uint64_t)tb | ((key & 1ull) << 63);
        bool own_cell = in_core;
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            own_cell = own_cell && pi[d] >= R.olo[d] && pi[d] < R.ohi[d];
        if (in_core) {
            const int ii = R.inner_index(pi);
            nl[ii] = (uint32_t)(key >> 32);
            fl[ii] = 0;
            due = due || (own_cell && (uint64_t)tb < a.final_bits);
            if (own_cell && (uint64_t)tb < tmin_own) tmin_own = (uint64_t)tb;
        }
        cnt_own_live += (uint32_t)__popcll(__ballot(own_cell && (uint64_t)tb < a.final_bits));
        cnt_inner_live += (uint32_t)__popcll(__ballot(in_core && (uint64_t)tb < a.horizon_bits));
    }
    if (lane == 0 && cnt_own_live) atomicAdd(&ctr[10], (int)cnt_own_live);
    if (lane == 0 && cnt_inner_live) atomicAdd(&ctr[12], (int)cnt_inner_live);
    if (a.track_tmin && tmin_own != ~0ull) atomicMin(&tmin_block, tmin_own);
    const int own_due = __syncthreads_or(due ? 1 : 0);
    if (a.track_tmin && tid == 0 && tmin_block != ~0ull)
        atomicMin(&a.counters[kTminBits], tmin_block);

    constexpr int Z = 2 * DIM;
    // arrivals before this launch's horizon may be applied; cells at or past
    // the advance's horizon are final
    const uint64_t horizon = a.horizon_bits;
    const uint64_t final_bits = a.final_bits;
    const double final_t = __longlong_as_double((long long)final_bits);
    const bool unit_rate = a.unit_rate != 0;
    uint32_t my_events = 0, my_flips = 0, my_ghost = 0, my_checks = 0;

    int rounds = 0;
    if (own_due) {
    // ---- initial scan: every enabled cell, claimed, into list 0.  A
    // wavefront's 64 lanes test 64 consecutive cells, i.e. two claim words.
    uint32_t cnt_scan_own = 0;   // owned cells listed (lane 0 of each wavefront)
    for (int base = tid - lane; base < R.inner; base += nthreads) {
        const int i = base + lane;
        bool en = false, owned = false;
        if (i < R.inner) {
            int p[3];
            R.coords(i, p);
            en = cell_enabled<DIM>(R, ts, p, R.box_index(p), horizon);
            ++my_checks;
            owned = true;
#pragma unroll
            for (int d = 0; d < DIM; ++d) owned = owned && p[d] >= R.olo[d] && p[d] < R.ohi[d];
        }
        const uint64_t m = __ballot(en);
        cnt_scan_own += (uint32_t)__popcll(__ballot(en && owned));
        if (lane == 0 && (uint32_t)m) claim[base >> 5] = (uint32_t)m;
        if (lane == 1 && (uint32_t)(m >> 32)) claim[(base >> 5) + 1] = (uint32_t)(m >> 32);
        wave_append(en, (uint16_t)i, lists, &sizes[0], lane);
    }
    if (lane == 0 && cnt_scan_own) atomicAdd(&ctr[11], (int)cnt_scan_own);
    __syncthreads();

    // ---- rounds: apply every listed arrival; re-test the cells whose
    // neighbourhood changed (the applied cell and its neighbour slots); claim
    // the newly enabled ones into the next list.  A listed cell stays enabled
    // until applied: none of its neighbours can be enabled meanwhile.
    for (int rnd = 0; rnd < a.max_sweeps; ++rnd) {
        const int cur = rnd & 1;
        const int sz = sizes[rnd % 3];
        if (sz == 0) break;
        ++rounds;
        if (tid == 0) {
            sizes[(rnd + 2) % 3] = 0;
            takes[(rnd + 2) % 3] = 0;
        }
        const uint16_t *lcur = lists + cur * list_cap;
        uint16_t *lnext = lists + (1 - cur) * list_cap;
        int *next_size = &sizes[(rnd + 1) % 3];
        for (;;) {
            int start = 0;
            if (lane == 0) start = atomicAdd(&takes[rnd % 3], 64);
            start = __shfl(start, 0, 64);
            if (start >= sz) break;
            const bool active = lane < sz - start;
            int p[3] = {0, 0, 0};
            if (active) {
                const int ii = lcur[start + lane];
                R.coords(ii, p);
                const int bi = R.box_index(p);
                atomicAnd(&claim[ii >> 5], ~(1u << (ii & 31)));
                const uint64_t wd = lds_load_word(&ts[bi]);
                int sum = 0;
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    int up, dn;
                    R.slot_offsets(d, p, up, dn);
                    sum += (lds_load_word(&ts[bi + up]) >> 63) ? -1 : 1;
                    sum += (lds_load_word(&ts[bi + dn]) >> 63) ? -1 : 1;
                }
                const uint32_t k = nl[ii];
                const Draw y = philox4x32_10(k, R.global_index(p), 0u, 0u, a.key_lo,
                                             a.key_hi);
                const int up_spin = (wd >> 63) ? 0 : 1;            // (s+1)/2
                const int idx = (sum + Z) / 2 + (Z + 1) * up_spin;
                const bool flip = (uint64_t)y.w2 < thr[idx];
                const double tnow = __longlong_as_double((long long)(wd & kTimeMask));
                const double tnext = tnow + arrival_gap(y.w0, y.w1, a.rate, unit_rate);
                const uint64_t sign = (wd & kSignBit) ^ (flip ? kSignBit : 0ull);
                if (FRAMES)
                    capture_frames(a.frames, a.frame_dt, a.frame_k0, a.nframes, a.n_cells, R.global_index(p), tnow, __builtin_fmin(tnext, final_t),
                                   sign ? (int8_t)-1 : (int8_t)1);
                nl[ii] = k + 1u;
                fl[ii] = (uint16_t)(fl[ii] + (flip ? 1u : 0u));
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                lds_store_word(&ts[bi], (uint64_t)__double_as_longlong(tnext) | sign);
                bool own_cell = true;
#pragma unroll
                for (int d = 0; d < DIM; ++d)
                    own_cell = own_cell && p[d] >= R.olo[d] && p[d] < R.ohi[d];
                if (own_cell) {
                    ++my_events;
                    my_flips += flip ? 1u : 0u;
                } else {
                    ++my_ghost;
                }
            }
            // re-tests read neighbour words only after this lane's arrival is
            // published, so the later of two concurrent re-tests of a shared
            // neighbour sees both new words
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
            // re-test the applied cell and each neighbour slot
#pragma unroll
            for (int slot = 0; slot <= Z; ++slot) {
                bool want = false;
                int ci = 0;
                if (active) {
                    int q[3] = {p[0], p[1], p[2]};
                    bool inside = true;
                    if (slot > 0) {
                        const int d = (slot - 1) >> 1;
                        const int step = ((slot - 1) & 1) ? -1 : 1;
                        q[d] += step;
                        if (R.span[d]) {
                            q[d] = (q[d] < 0) ? q[d] + R.rin[d] : q[d];
                            q[d] = (q[d] >= R.rin[d]) ? q[d] - R.rin[d] : q[d];
                        } else {
                            inside = q[d] >= 0 && q[d] < R.rin[d];
                        }
                    }
                    if (inside) {
                        ++my_checks;
                        ci = R.inner_index(q);
                        if (cell_enabled<DIM>(R, ts, q, R.box_index(q), horizon)) {
                            const uint32_t bit = 1u << (ci & 31);
                            want = (atomicOr(&claim[ci >> 5], bit) & bit) == 0u;
                        }
                    }
                }
                wave_append(want, (uint16_t)ci, lnext, next_size, lane);
            }
        }
        __syncthreads();
    }
    }  // own_due

    // ---- merge every owned copy and every ghost copy that moved into the
    // ---- next snapshot; detect owned cells with arrivals still due
    bool live = false;
    for (int j = tid; j < R.inner; j += nthreads) {
        int p[3];
        R.coords(j, p);
        bool own_cell = true;
#pragma unroll
        for (int d = 0; d < DIM; ++d) own_cell = own_cell && p[d] >= R.olo[d] && p[d] < R.ohi[d];
        const int bi = R.box_index(p);
        const uint32_t gi = R.global_index(p);
        const uint32_t n_copy = nl[j];
        const unsigned long long key_in = a.key_in[gi];
        const uint32_t n_in = (uint32_t)(key_in >> 32);
        const uint64_t wd = ts[bi];
        if (own_cell || n_copy != n_in) {
            const unsigned long long f = ((key_in >> 1) & 0x7FFFFFFFull) + fl[j];
            const unsigned long long key = ((unsigned long long)n_copy << 32) | (f << 1) |
                                           (wd >> 63);
            atomicMax(&a.key_out[gi], key);
            atomicMax(&a.time_out[gi], (unsigned long long)(wd & kTimeMask));
        }
        if (own_cell) live = live || (wd & kTimeMask) < final_bits;
    }
    // ---- counters
    atomicAdd(&ctr[6], (int)my_events);
    atomicAdd(&ctr[7], (int)my_flips);
    atomicAdd(&ctr[8], (int)my_ghost);
    atomicAdd(&ctr[9], (int)my_checks);
    const int any_live = __syncthreads_or(live ? 1 : 0);
    if (tid == 0) {
        unsigned long long *gc = a.counters;
        atomicAdd(&gc[kEvents], (unsigned long long)(unsigned)ctr[6]);
        atomicAdd(&gc[kFlips], (unsigned long long)(unsigned)ctr[7]);
        atomicAdd(&gc[kGhostEvents], (unsigned long long)(unsigned)ctr[8]);
        atomicAdd(&gc[kChecks], (unsigned long long)(unsigned)ctr[9]);
        atomicAdd(&gc[kSweeps], (unsigned long long)rounds);
        atomicAdd(&gc[kScanLive], (unsigned long long)(unsigned)ctr[10]);
        atomicAdd(&gc[kScanEnabled], (unsigned long long)(unsigned)ctr[11]);
        atomicAdd(&gc[kRoundCells], (unsigned long long)(unsigned)ctr[12] * (unsigned)rounds);
        if (any_live) atomicAdd(&gc[kLiveTiles], 1ull);
        // owned cells that were all at or past the horizon when loaded can
        // never change again: both snapshots now hold them
        if (!own_due) a.dead[blockIdx.x] = 1;
        finish_visit_block(a, ntiles_total);
    }
}

// ----------------------------------------------------------------- pack

// Sum over the block (wavefront shuffles, then LDS), one global atomic per
// block; called by every thread of the block.
__device__ __forceinline__ void block_add(unsigned long long *dst, unsigned long long v)
{
    __shared__ unsigned long long part[16];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) part[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w];
        if (t) atomicAdd(dst, t);
    }
    __syncthreads();
}

__global__ void pack_kernel(uint64_t n_cells, const int8_t *s, const double *t,
                            const uint32_t *n, unsigned long long *key,
                            unsigned long long *time, unsigned long long *sum_n)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long acc = 0;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells;
         c += stride) {
        key[c] = ((unsigned long long)n[c] << 32) | (s[c] < 0 ? 1ull : 0ull);
        time[c] = (unsigned long long)__double_as_longlong(t[c]);
        acc += n[c];
    }
    block_add(sum_n, acc);
}

__global__ void count_bound_kernel(uint64_t n_cells, const uint32_t *n,
                                   unsigned long long *flag)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t high = 0;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells;
         c += stride)
        high |= n[c] >> 31;
    if (__ballot(high != 0u) != 0ull && (threadIdx.x & 63u) == 0u) atomicOr(flag, 1ull);
}

__global__ void unpack_kernel(uint64_t n_cells, const unsigned long long *key,
                              const unsigned long long *time, int8_t *s, double *t,
                              uint32_t *n, unsigned long long *sums)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long acc_n = 0, acc_f = 0;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells;
         c += stride) {
        const unsigned long long k = key[c];
        s[c] = (k & 1ull) ? (int8_t)-1 : (int8_t)1;
        n[c] = (uint32_t)(k >> 32);
        t[c] = __longlong_as_double((long long)time[c]);
        acc_n += k >> 32;
        acc_f += (k >> 1) & 0x7FFFFFFFull;
    }
    block_add(&sums[0], acc_n);
    block_add(&sums[1], acc_f);
}

// ----------------------------------------------------------------- frames

__global__ void frames_init_kernel(VisitArgs a, const int8_t *s, const double *t, double T0,
                                   double T)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.n_cells;
         c += stride)
        capture_frames(a.frames, a.frame_dt, a.frame_k0, a.nframes, a.n_cells, (uint32_t)c, T0, __builtin_fmin(t[c], T), s[c]);
}

// ----------------------------------------------------------------- checks

__global__ void philox_kernel(const uint32_t *ctr, uint32_t key_lo, uint32_t key_hi,
                              uint32_t *out, uint64_t count)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += stride) {
        const Draw y = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2],
                                     ctr[4 * i + 3], key_lo, key_hi);
        out[4 * i] = y.w0;
        out[4 * i + 1] = y.w1;
        out[4 * i + 2] = y.w2;
        out[4 * i + 3] = y.w3;
    }
}

__global__ void neg_log_kernel(const uint64_t *w, double *out, uint64_t count)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += stride)
        out[i] = neg_log_u53(w[i]);
}

unsigned grid_for(uint64_t count, unsigned block)
{
    uint64_t g = (count + block - 1) / block;
    if (g > 65535ull * 16) g = 65535ull * 16;
    return (unsigned)(g ? g : 1);
}

}  // namespace

size_t visit_lds_bytes(int dim, const VisitArgs &a, int block)
{
    (void)block;
    int inner_max = 0;
    const int box_max = region_box_max(dim, a, &inner_max);
    return lds_plan(box_max, inner_max).total;
}

int visit_inner_max(int dim, const VisitArgs &a)
{
    int inner_max = 0;
    region_box_max(dim, a, &inner_max);
    return inner_max;
}

hipError_t launch_init(int dim, const int32_t *L, uint64_t n_cells, uint32_t key_lo,
                       uint32_t key_hi, double rate, int init, int8_t *s, double *t,
                       uint32_t *n, hipStream_t stream)
{
    (void)dim;
    (void)L;
    const unsigned block = 256;
    hipLaunchKernelGGL(aca_init_kernel, dim3(grid_for(n_cells, block)), dim3(block), 0,
                       stream, n_cells, key_lo, key_hi, rate, rate == 1.0 ? 1 : 0, init,
                       s, t, n);
    return hipGetLastError();
}

template <bool FRAMES>
void launch_generic(int dim, const VisitArgs &a, unsigned tiles, int block, size_t lds,
                    hipStream_t stream)
{
    switch (dim) {
    case 1:
        hipLaunchKernelGGL((visit_kernel<1, FRAMES>), dim3(tiles), dim3(block), lds, stream, a);
        break;
    case 2:
        hipLaunchKernelGGL((visit_kernel<2, FRAMES>), dim3(tiles), dim3(block), lds, stream, a);
        break;
    default:
        hipLaunchKernelGGL((visit_kernel<3, FRAMES>), dim3(tiles), dim3(block), lds, stream, a);
        break;
    }
}

hipError_t launch_visit(int dim, const VisitArgs &a, int block, size_t lds,
                        hipStream_t stream)
{
    const unsigned tiles = (unsigned)a.ntiles[0] * (unsigned)a.ntiles[1] *
                           (unsigned)a.ntiles[2];
    if (a.frames)
        launch_generic<true>(dim, a, tiles, block, lds, stream);
    else
        launch_generic<false>(dim, a, tiles, block, lds, stream);
    return hipGetLastError();
}

// Grid of at most four blocks per CU: each thread loops over many cells, so
// the per-block sums need few global atomics.
unsigned reduce_grid(uint64_t count, unsigned block)
{
    const unsigned g = grid_for(count, block);
    return g < 1024u ? g : 1024u;
}

hipError_t launch_pack(uint64_t n_cells, const int8_t *s, const double *t,
                       const uint32_t *n, unsigned long long *key,
                       unsigned long long *time, unsigned long long *sum_n,
                       hipStream_t stream)
{
    const unsigned block = 256;
    hipLaunchKernelGGL(pack_kernel, dim3(reduce_grid(n_cells, block)), dim3(block), 0, stream,
                       n_cells, s, t, n, key, time, sum_n);
    return hipGetLastError();
}

hipError_t launch_count_bound(uint64_t n_cells, const uint32_t *n, unsigned long long *flag,
                              hipStream_t stream)
{
    const unsigned block = 256;
    hipLaunchKernelGGL(count_bound_kernel, dim3(reduce_grid(n_cells, block)), dim3(block), 0,
                       stream, n_cells, n, flag);
    return hipGetLastError();
}

hipError_t launch_unpack(uint64_t n_cells, const unsigned long long *key,
                         const unsigned long long *time, int8_t *s, double *t,
                         uint32_t *n, unsigned long long *sums, hipStream_t stream)
{
    const unsigned block = 256;
    hipLaunchKernelGGL(unpack_kernel, dim3(reduce_grid(n_cells, block)), dim3(block), 0,
                       stream, n_cells, key, time, s, t, n, sums);
    return hipGetLastError();
}

hipError_t set_visit_lds_limit(size_t bytes)
{
    const void *fns[6] = {(const void *)visit_kernel<1, false>,
                          (const void *)visit_kernel<2, false>,
                          (const void *)visit_kernel<3, false>,
                          (const void *)visit_kernel<1, true>,
                          (const void *)visit_kernel<2, true>,
                          (const void *)visit_kernel<3, true>};
    for (const void *f : fns) {
        const hipError_t e =
            hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_frames_init(const VisitArgs &a, const int8_t *s, const double *t, double T0,
                              double T, hipStream_t stream)
{
    const unsigned block = 256;
    hipLaunchKernelGGL(frames_init_kernel, dim3(reduce_grid(a.n_cells, block)), dim3(block), 0,
                       stream, a, s, t, T0, T);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, uint64_t seed, uint32_t *out,
                         uint64_t count, hipStream_t stream)
{
    const unsigned block = 256;
    hipLaunchKernelGGL(philox_kernel, dim3(grid_for(count, block)), dim3(block), 0,
                       stream, ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out, count);
    return hipGetLastError();
}

hipError_t launch_neg_log(const uint64_t *w, double *out, uint64_t count,
                          hipStream_t stream)
{
    const unsigned block = 256;
    hipLaunchKernelGGL(neg_log_kernel, dim3(grid_for(count, block)), dim3(block), 0,
                       stream, w, out, count);
    return hipGetLastError();
}

}  // namespace aca

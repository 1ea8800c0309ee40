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
// Work distribution.  Each wavefront scans a strided share of the region's
// cells; enabled cells are compacted with a ballot into a per-wavefront list
// in LDS and applied 64 at a time, so the Philox draw and the logarithm run
// on full wavefronts.  A workgroup barrier after each sweep counts the
// arrivals applied; the visit ends after a sweep with none or after
// max_sweeps sweeps.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aca_device.h"
#include "aca_internal.h"

#pragma clang fp contract(off)

namespace aca {
namespace {

constexpr uint64_t kSignBit = 0x8000000000000000ull;
constexpr uint64_t kTimeMask = 0x7FFFFFFFFFFFFFFFull;
constexpr int kListCap = 128;   // per-wavefront list: 64 pending + 64 incoming

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

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS carve-up shared with visit_lds_bytes().
struct LdsPlan {
    size_t thr_off, ctr_off, ts_off, n_off, f_off, list_off, total;
};

__host__ __device__ inline LdsPlan lds_plan(int box_max, int nwaves)
{
    LdsPlan p;
    p.thr_off = 0;                                   // uint64 thr[16]
    p.ctr_off = 128;                                 // int counters[8]
    p.ts_off = 160;                                  // uint64 ts[box_max]
    p.n_off = p.ts_off + 8 * (size_t)box_max;        // uint32 n[box_max]
    p.f_off = p.n_off + 4 * (size_t)box_max;         // uint16 flips[box_max]
    p.list_off = p.f_off + 2 * (size_t)box_max;      // uint32 per wave 2*kListCap
    p.list_off = (p.list_off + 15) & ~(size_t)15;
    p.total = p.list_off + (size_t)nwaves * 2 * kListCap * 4;
    return p;
}

__host__ __device__ inline int region_box_max(int dim, const VisitArgs &a)
{
    int box = 1;
    for (int d = 0; d < dim; ++d) {
        const int rin = a.span[d] ? a.L[d] : a.tile[d] + 2 * a.ghost[d];
        box *= rin + (a.span[d] ? 0 : 2);
    }
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

template <int DIM>
__global__ void __launch_bounds__(1024) visit_kernel(VisitArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int nthreads = blockDim.x;
    const int nwaves = nthreads >> 6;

    // ---- region geometry of this tile
    int tc[3];
    {
        uint32_t b = blockIdx.x;
        tc[0] = (int)(b % (uint32_t)a.ntiles[0]);
        b /= (uint32_t)a.ntiles[0];
        tc[1] = (int)(b % (uint32_t)a.ntiles[1]);
        tc[2] = (int)(b / (uint32_t)a.ntiles[1]);
    }
    int rin[3], ring[3], rbox[3], org[3], olo[3], ohi[3], side[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d < DIM) {
            side[d] = a.L[d];
            const int lo = tc[d] * a.tile[d];
            const int w = min(a.tile[d], a.L[d] - lo);
            if (a.span[d]) {
                rin[d] = a.L[d]; ring[d] = 0; org[d] = 0; olo[d] = 0; ohi[d] = a.L[d];
            } else {
                rin[d] = w + 2 * a.ghost[d]; ring[d] = 1; org[d] = lo - a.ghost[d];
                olo[d] = a.ghost[d]; ohi[d] = a.ghost[d] + w;
            }
        } else {
            side[d] = 1; rin[d] = 1; ring[d] = 0; org[d] = 0; olo[d] = 0; ohi[d] = 1;
        }
        rbox[d] = rin[d] + 2 * ring[d];
    }
    const int sbox[3] = {1, rbox[0], rbox[0] * rbox[1]};
    const int inner = rin[0] * rin[1] * rin[2];
    const int box = rbox[0] * rbox[1] * rbox[2];
    const int gs1 = side[0], gs2 = side[0] * side[1];

    const LdsPlan plan = lds_plan(region_box_max(DIM, a), nwaves);
    uint64_t *thr = reinterpret_cast<uint64_t *>(lds + plan.thr_off);
    int *ctr = reinterpret_cast<int *>(lds + plan.ctr_off);
    uint64_t *ts = reinterpret_cast<uint64_t *>(lds + plan.ts_off);
    uint32_t *nl = reinterpret_cast<uint32_t *>(lds + plan.n_off);
    uint16_t *fl = reinterpret_cast<uint16_t *>(lds + plan.f_off);
    uint32_t *meta_list = reinterpret_cast<uint32_t *>(lds + plan.list_off) +
                          wave * 2 * kListCap;
    uint32_t *gidx_list = meta_list + kListCap;

    if (tid < 2 * (2 * DIM + 1)) thr[tid] = a.thr[tid];
    if (tid < 8) ctr[tid] = 0;

    // ---- load the region (ring box) from the input state
    for (int j = tid; j < box; j += nthreads) {
        int q[3];
        q[0] = j % rbox[0];
        const int r = j / rbox[0];
        q[1] = r % rbox[1];
        q[2] = r / rbox[1];
        int g[3];
        bool in_core = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            g[d] = (d < DIM) ? wrap_side(org[d] - ring[d] + q[d], side[d]) : 0;
            in_core = in_core && q[d] >= ring[d] && q[d] < ring[d] + rin[d];
        }
        const uint32_t gi = (uint32_t)g[0] + (uint32_t)gs1 * (uint32_t)g[1] +
                            (uint32_t)gs2 * (uint32_t)g[2];
        const unsigned long long key = a.key_in[gi];
        ts[j] = (uint64_t)a.time_in[gi] | ((key & 1ull) << 63);
        if (in_core) {
            nl[j] = (uint32_t)(key >> 32);
            fl[j] = 0;
        }
    }
    __syncthreads();

    // ---- per-thread scan position (inner coordinates) and its stride
    int p0[3], step[3];
    {
        p0[0] = tid % rin[0];
        int r = tid / rin[0];
        p0[1] = r % rin[1];
        p0[2] = r / rin[1];
        step[0] = nthreads % rin[0];
        r = nthreads / rin[0];
        step[1] = r % rin[1];
        step[2] = r / rin[1];
    }
    constexpr int Z = 2 * DIM;
    const uint64_t horizon = a.horizon_bits;
    const bool unit_rate = a.unit_rate != 0;

    uint32_t my_events = 0, my_flips = 0, my_ghost = 0, my_checks = 0;
    int sweeps = 0;

    for (int sw = 0; sw < a.max_sweeps; ++sw) {
        int cnt = 0;             // wave-uniform: entries pending in the list
        int wave_applied = 0;    // wave-uniform
        int p[3] = {p0[0], p0[1], p0[2]};

        // Apply the arrivals of list entries [0, m) (m <= 64), one per lane.
        auto apply = [&](int m) {
            if (lane < m) {
                const uint32_t meta = meta_list[lane];
                const uint32_t gidx = gidx_list[lane];
                const int bi = (int)(meta & 0xFFFFFu);
                const bool own_cell = (meta >> 20) & 1u;
                const uint32_t wrapf = meta >> 21;
                const uint64_t wd = lds_load_word(&ts[bi]);
                int sum = 0;
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    int up = sbox[d], dn = -sbox[d];
                    if (wrapf & (1u << (2 * d))) up -= rin[d] * sbox[d];
                    if (wrapf & (1u << (2 * d + 1))) dn += rin[d] * sbox[d];
                    sum += (lds_load_word(&ts[bi + up]) >> 63) ? -1 : 1;
                    sum += (lds_load_word(&ts[bi + dn]) >> 63) ? -1 : 1;
                }
                const uint32_t k = nl[bi];
                const Draw y = philox4x32_10(k, gidx, 0u, 0u, a.key_lo, a.key_hi);
                const int up_spin = (wd >> 63) ? 0 : 1;            // (s+1)/2
                const int idx = (sum + Z) / 2 + (Z + 1) * up_spin;
                const bool flip = (uint64_t)y.w2 < thr[idx];
                const double tnow = __longlong_as_double((long long)(wd & kTimeMask));
                const double tnext = tnow + arrival_gap(y.w0, y.w1, a.rate, unit_rate);
                const uint64_t sign = (wd & kSignBit) ^ (flip ? kSignBit : 0ull);
                nl[bi] = k + 1u;
                fl[bi] = (uint16_t)(fl[bi] + (flip ? 1u : 0u));
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                lds_store_word(&ts[bi], (uint64_t)__double_as_longlong(tnext) | sign);
                if (own_cell) {
                    ++my_events;
                    my_flips += flip ? 1u : 0u;
                } else {
                    ++my_ghost;
                }
            }
        };

        for (int base = wave * 64; base < inner; base += nthreads) {
            const int i = base + lane;
            bool en = false;
            uint32_t meta = 0, gidx = 0;
            if (i < inner) {
                ++my_checks;
                const int bi = (p[0] + ring[0]) + sbox[1] * (p[1] + ring[1]) +
                               sbox[2] * (p[2] + ring[2]);
                const uint64_t tw = lds_load_word(&ts[bi]) & kTimeMask;
                en = tw < horizon;
                uint32_t wrapf = 0;
                bool own_cell = true;
                uint32_t gi = 0;
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    int up = sbox[d], dn = -sbox[d];
                    if (a.span[d]) {
                        if (p[d] == rin[d] - 1) { up -= rin[d] * sbox[d]; wrapf |= 1u << (2 * d); }
                        if (p[d] == 0) { dn += rin[d] * sbox[d]; wrapf |= 1u << (2 * d + 1); }
                    }
                    const int gd = wrap_side(org[d] + p[d], side[d]);
                    gi += (uint32_t)gd * (uint32_t)(d == 0 ? 1 : (d == 1 ? gs1 : gs2));
                    const uint64_t tu = lds_load_word(&ts[bi + up]) & kTimeMask;
                    const uint64_t tdn = lds_load_word(&ts[bi + dn]) & kTimeMask;
                    // (t, c) < (t', c'): on equal times the smaller global index
                    // wins; +d neighbour is larger unless it wraps, -d neighbour
                    // is smaller unless it wraps.
                    en = en && (tw < tu || (tw == tu && gd + 1 < side[d]));
                    en = en && (tw < tdn || (tw == tdn && gd == 0));
                    own_cell = own_cell && p[d] >= olo[d] && p[d] < ohi[d];
                }
                meta = (uint32_t)bi | (own_cell ? (1u << 20) : 0u) | (wrapf << 21);
                gidx = gi;
            }
            const uint64_t m = __ballot(en);
            if (m) {
                const int pos = cnt + (int)__popcll(m & ((1ull << lane) - 1ull));
                if (en) {
                    meta_list[pos] = meta;
                    gidx_list[pos] = gidx;
                }
                cnt += (int)__popcll(m);
                if (cnt >= 64) {
                    wave_sync();
                    apply(64);
                    const int rest = cnt - 64;
                    wave_sync();
                    uint32_t mv = 0, gv = 0;
                    if (lane < rest) {
                        mv = meta_list[64 + lane];
                        gv = gidx_list[64 + lane];
                    }
                    wave_sync();
                    if (lane < rest) {
                        meta_list[lane] = mv;
                        gidx_list[lane] = gv;
                    }
                    wave_sync();
                    wave_applied += 64;
                    cnt = rest;
                }
            }
            // advance the scan position by nthreads cells
            p[0] += step[0];
            int c = p[0] >= rin[0];
            p[0] -= c ? rin[0] : 0;
            p[1] += step[1] + c;
            c = p[1] >= rin[1];
            p[1] -= c ? rin[1] : 0;
            p[2] += step[2] + c;
        }
        if (cnt > 0) {
            wave_sync();
            apply(cnt);
            wave_sync();
            wave_applied += cnt;
        }
        if (lane == 0) atomicAdd(&ctr[sw % 3], wave_applied);
        if (tid == 0) ctr[(sw + 1) % 3] = 0;
        __syncthreads();
        const int total = ctr[sw % 3];
        ++sweeps;
        if (total == 0) break;
    }
    __syncthreads();

    // ---- merge every owned copy and every ghost copy that moved into the
    // ---- next snapshot; detect owned cells with arrivals still due
    bool live = false;
    for (int j = tid; j < inner; j += nthreads) {
        int p[3];
        p[0] = j % rin[0];
        const int r = j / rin[0];
        p[1] = r % rin[1];
        p[2] = r / rin[1];
        int g[3];
        bool own_cell = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            g[d] = (d < DIM) ? wrap_side(org[d] + p[d], side[d]) : 0;
            own_cell = own_cell && p[d] >= olo[d] && p[d] < ohi[d];
        }
        const int bi = (p[0] + ring[0]) + sbox[1] * (p[1] + ring[1]) +
                       sbox[2] * (p[2] + ring[2]);
        const uint32_t gi = (uint32_t)g[0] + (uint32_t)gs1 * (uint32_t)g[1] +
                            (uint32_t)gs2 * (uint32_t)g[2];
        const uint32_t n_copy = nl[bi];
        const unsigned long long key_in = a.key_in[gi];
        const uint32_t n_in = (uint32_t)(key_in >> 32);
        const uint64_t wd = ts[bi];
        if (own_cell || n_copy != n_in) {
            const unsigned long long f = ((key_in >> 1) & 0x7FFFFFFFull) + fl[bi];
            const unsigned long long key = ((unsigned long long)n_copy << 32) | (f << 1) |
                                           (wd >> 63);
            atomicMax(&a.key_out[gi], key);
            atomicMax(&a.time_out[gi], (unsigned long long)(wd & kTimeMask));
        }
        if (own_cell) live = live || (wd & kTimeMask) < horizon;
    }
    // ---- counters
    atomicAdd(&ctr[3], (int)my_events);
    atomicAdd(&ctr[4], (int)my_flips);
    atomicAdd(&ctr[5], (int)my_ghost);
    atomicAdd(&ctr[6], (int)my_checks);
    const int any_live = __syncthreads_or(live ? 1 : 0);
    if (tid == 0) {
        unsigned long long *gc = a.counters;
        atomicAdd(&gc[kEvents], (unsigned long long)(unsigned)ctr[3]);
        atomicAdd(&gc[kFlips], (unsigned long long)(unsigned)ctr[4]);
        atomicAdd(&gc[kGhostEvents], (unsigned long long)(unsigned)ctr[5]);
        atomicAdd(&gc[kChecks], (unsigned long long)(unsigned)ctr[6]);
        atomicAdd(&gc[kSweeps], (unsigned long long)sweeps);
        if (any_live) atomicAdd(&gc[kLiveTiles], 1ull);
    }
}

// ----------------------------------------------------------------- pack

__device__ __forceinline__ void block_add(unsigned long long *dst, unsigned long long v)
{
    // wavefront reduction, then one atomic per wavefront
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, v);
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
    return lds_plan(region_box_max(dim, a), block / 64).total;
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

hipError_t launch_visit(int dim, const VisitArgs &a, int block, size_t lds,
                        hipStream_t stream)
{
    const unsigned tiles = (unsigned)a.ntiles[0] * (unsigned)a.ntiles[1] *
                           (unsigned)a.ntiles[2];
    switch (dim) {
    case 1:
        hipLaunchKernelGGL(visit_kernel<1>, dim3(tiles), dim3(block), lds, stream, a);
        break;
    case 2:
        hipLaunchKernelGGL(visit_kernel<2>, dim3(tiles), dim3(block), lds, stream, a);
        break;
    default:
        hipLaunchKernelGGL(visit_kernel<3>, dim3(tiles), dim3(block), lds, stream, a);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_pack(uint64_t n_cells, const int8_t *s, const double *t,
                       const uint32_t *n, unsigned long long *key,
                       unsigned long long *time, unsigned long long *sum_n,
                       hipStream_t stream)
{
    const unsigned block = 256;
    hipLaunchKernelGGL(pack_kernel, dim3(grid_for(n_cells, block)), dim3(block), 0, stream,
                       n_cells, s, t, n, key, time, sum_n);
    return hipGetLastError();
}

hipError_t launch_unpack(uint64_t n_cells, const unsigned long long *key,
                         const unsigned long long *time, int8_t *s, double *t,
                         uint32_t *n, unsigned long long *sums, hipStream_t stream)
{
    const unsigned block = 256;
    hipLaunchKernelGGL(unpack_kernel, dim3(grid_for(n_cells, block)), dim3(block), 0,
                       stream, n_cells, key, time, s, t, n, sums);
    return hipGetLastError();
}

hipError_t set_visit_lds_limit(size_t bytes)
{
    hipError_t e = hipFuncSetAttribute((const void *)visit_kernel<1>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)visit_kernel<2>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)visit_kernel<3>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
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

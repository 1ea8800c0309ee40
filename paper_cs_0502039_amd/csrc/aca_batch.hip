// aca_batch.hip -- kernels that advance many independent lattices at once.
//
// The per-lattice schedule is the one of the single-lattice loop (each epoch
// of a lattice reads one snapshot and merges into the other, so every epoch
// boundary is a consistent cut and the result is the unique trajectory of
// Fig. 3.1's process, whatever else runs beside it).  What changes is who
// decides when an epoch starts: instead of one launch per epoch with the host
// waiting in between, one persistent launch keeps every compute unit busy
// with (lattice, tile) items, and the workgroup that completes an epoch opens
// the next one at once.  Lattices are scanned in the host's priority order
// (most remaining work first), so long jobs start early and short ones fill
// the gaps.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aca_internal.h"
#include "aca_region.h"

namespace aca {
namespace {

constexpr int kBatchBlock = 512;
constexpr int kPackBlock = 256;

__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t ld_agent32(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_agent(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_agent32(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum over the block (wavefront shuffles, then LDS), one global atomic.
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

// Index i with start[i] <= b < start[i + 1] (start[0] = 0, strictly
// increasing, start[count] = grid size).
__device__ __forceinline__ uint32_t find_member(const uint32_t *start, uint32_t count, uint32_t b)
{
    uint32_t lo = 0, hi = count;   // start[lo] <= b < start[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (start[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void batch_reset_kernel(BatchState *state, const uint32_t *joining, uint32_t count)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    BatchState &st = state[joining[i]];
    st.claim = 0ull;                 // epoch 0, nothing handed out
    st.finished = 0u;
    st.live = 0u;
    st.status = kSlotRunning;
    st.epochs = 0u;
    st.total_epochs = 0u;
    st.final_snap = 0u;
    st.epoch_moves = 0ull;
    for (int k = 0; k < kNumCounters; ++k) st.ctr[k] = 0ull;
    st.sum_start = 0ull;
    st.sum_end = 0ull;
    st.sum_flips = 0ull;
    st.unpacked = 0ull;
}

__global__ void __launch_bounds__(kPackBlock)
batch_pack_kernel(const BatchSlot *slots, BatchState *state, const uint32_t *joining,
                  const uint32_t *block_start, uint32_t count)
{
    const uint32_t i = find_member(block_start, count, blockIdx.x);
    const uint32_t slot = joining[i];
    const BatchSlot &sl = slots[slot];
    const uint32_t nb = block_start[i + 1] - block_start[i];
    const uint64_t stride = (uint64_t)nb * blockDim.x;
    const uint64_t first = (uint64_t)(blockIdx.x - block_start[i]) * blockDim.x + threadIdx.x;
    unsigned long long acc = 0;
    for (uint64_t c = first; c < sl.n_cells; c += stride) {
        const uint32_t n = sl.cnt[c];
        sl.key[0][c] = ((unsigned long long)n << 32) | (sl.s[c] < 0 ? 1ull : 0ull);
        sl.time[0][c] = (unsigned long long)__double_as_longlong(sl.t[c]);
        // the other snapshot starts below every copy
        sl.key[1][c] = 0ull;
        sl.time[1][c] = 0ull;
        acc += n;
    }
    for (uint64_t j = first; j < sl.ntiles; j += stride) sl.a.dead[j] = 0;
    block_add(&state[slot].sum_start, acc);
}

__global__ void __launch_bounds__(kPackBlock)
batch_unpack_kernel(const BatchSlot *slots, BatchState *state, const uint32_t *members,
                    const uint32_t *block_start, uint32_t count)
{
    const uint32_t i = find_member(block_start, count, blockIdx.x);
    const uint32_t slot = members[i];
    // only members that finished during the launch just run; the decision is
    // the same in every block of the member (nothing changes it meanwhile)
    if (state[slot].status != kSlotDone || state[slot].unpacked) return;
    const BatchSlot &sl = slots[slot];
    const uint32_t snap = state[slot].final_snap;
    const unsigned long long *key = sl.key[snap];
    const unsigned long long *time = sl.time[snap];
    const uint32_t nb = block_start[i + 1] - block_start[i];
    const uint64_t stride = (uint64_t)nb * blockDim.x;
    unsigned long long acc_n = 0, acc_f = 0;
    for (uint64_t c = (uint64_t)(blockIdx.x - block_start[i]) * blockDim.x + threadIdx.x;
         c < sl.n_cells; c += stride) {
        const unsigned long long k = key[c];
        sl.s[c] = (k & 1ull) ? (int8_t)-1 : (int8_t)1;
        sl.cnt[c] = (uint32_t)(k >> 32);
        sl.t[c] = __longlong_as_double((long long)time[c]);
        acc_n += k >> 32;
        acc_f += (k >> 1) & 0x7FFFFFFFull;
    }
    block_add(&state[slot].sum_end, acc_n);
    block_add(&state[slot].sum_flips, acc_f);
}

// One block: the members of this launch that the previous launch finished
// are marked unpacked, paused ones re-open their epoch, and the running ones
// are counted (slots that are not members are ignored, whatever they hold).
__global__ void batch_open_kernel(BatchState *state, const uint32_t *members, uint32_t count,
                                  BatchGlobal *g, unsigned long long budget_ticks,
                                  unsigned long long max_epochs)
{
    __shared__ uint32_t running;
    if (threadIdx.x == 0) running = 0u;
    __syncthreads();
    uint32_t mine = 0;
    for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) {
        BatchState &st = state[members[i]];
        if (st.status == kSlotDone) st.unpacked = 1ull;
        if (st.status == kSlotPaused) {
            st.status = kSlotRunning;
            st.claim &= 0xFFFFFFFF00000000ull;     // same epoch, nothing handed out
        }
        if (st.status == kSlotRunning) {
            st.epochs = 0u;
            ++mine;
        }
    }
    if (mine) atomicAdd(&running, mine);
    __syncthreads();
    if (threadIdx.x == 0) {
        g->active = running;
        g->error = 0u;
        g->deadline = budget_ticks ? wall_clock64() + budget_ticks : ~0ull;
        g->max_epochs = max_epochs;
    }
}

// Wavefront 0 of a block looks for an open (lattice, tile) item, scanning the
// members in priority order; returns false when no member is running any more
// or when it waited longer than `wait_limit` ticks without finding one.
__device__ bool claim_item(const BatchSlot *slots, BatchState *state, const uint32_t *order,
                           uint32_t norder, BatchGlobal *g, unsigned long long wait_limit,
                           uint32_t *slot_out, uint32_t *tile_out, uint32_t *epoch_out)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long t0 = wall_clock64();
    for (;;) {
        if (ld_agent32(&g->active) == 0u) return false;
        for (uint32_t base = 0; base < norder; base += 64) {
            const uint32_t i = base + (uint32_t)lane;
            bool open = false;
            uint32_t s = 0;
            if (i < norder) {
                s = order[i];
                const unsigned long long w = ld_agent(&state[s].claim);
                open = (uint32_t)w < slots[s].ntiles;
            }
            unsigned long long m = __ballot(open);
            while (m) {
                const int l = __builtin_ctzll(m);
                unsigned long long old = 0;
                if (lane == l) old = atomicAdd(&state[s].claim, 1ull);
                old = __shfl(old, l, 64);
                const uint32_t sl = (uint32_t)__shfl((int)s, l, 64);
                if ((uint32_t)old < slots[sl].ntiles) {
                    *slot_out = sl;
                    *tile_out = (uint32_t)old;
                    *epoch_out = (uint32_t)(old >> 32);
                    return true;
                }
                m &= m - 1ull;
            }
        }
        if (wall_clock64() - t0 > wait_limit) {
            if (lane == 0) atomicOr(&g->error, 1u);
            return false;
        }
        __builtin_amdgcn_s_sleep(32);
        // The claim words are read with device-scope loads, which this XCD's
        // L2 may still serve from a line cached before another compute unit
        // opened an epoch (lines of memory not local to an L2 are not kept
        // coherent).  Items that start a visit invalidate it; when every
        // workgroup here is waiting, this acquire does.
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
}

// Thread 0 of the block that finished the last tile of `epoch` of `slot`:
// open the next epoch, or pause (step budget) or retire the member.
__device__ void close_epoch(BatchState &st, uint32_t epoch, BatchGlobal *g)
{
    // every tile's merge and counters of this epoch were performed before its
    // ticket; drop lines this XCD cached before them
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const uint32_t live = ld_agent32(&st.live);
    const unsigned long long moves = ld_agent(&st.epoch_moves);
    const uint32_t next = epoch + 1u;
    st_agent32(&st.finished, 0u);
    st_agent32(&st.live, 0u);
    st_agent(&st.epoch_moves, 0ull);
    // the closer of the next epoch may run on another XCD: device-scope words
    const uint32_t done_epochs = ld_agent32(&st.epochs) + 1u;
    st_agent32(&st.epochs, done_epochs);
    st_agent32(&st.total_epochs, ld_agent32(&st.total_epochs) + 1u);
    const unsigned long long closed = ((unsigned long long)next << 32) | kClaimClosed;
    uint32_t status = kSlotRunning;
    if (live == 0u) {
        // no owned cell before the horizon: the merged snapshot is final
        st_agent32(&st.final_snap, next & 1u);
        status = kSlotDone;
    } else if (moves == 0ull) {
        status = kSlotStalled;
    } else if (done_epochs >= g->max_epochs ||
               (unsigned long long)wall_clock64() >= g->deadline) {
        status = kSlotPaused;
    }
    // the stores above (device-scope) complete before the epoch opens
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (status != kSlotRunning) {
        st_agent32(&st.status, status);
        st_agent(&st.claim, closed);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        atomicSub(&g->active, 1u);
    } else {
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        atomicExch(&st.claim, (unsigned long long)next << 32);
    }
}

// DIM = 1, 2 or 3 when every member has that dimension, 0 for a mix (the
// dimension is then read per item).  WAVES = 4 wavefronts per SIMD when two
// workgroups fit a compute unit's LDS (at most 128 registers per lane), 2
// when the regions are so large that only one does (then up to 256 registers
// per lane cost no occupancy).
template <int DIM, int WAVES>
__global__ void __launch_bounds__(kBatchBlock) __attribute__((amdgpu_waves_per_eu(WAVES)))
batch_visit_kernel(const BatchSlot *slots, BatchState *state, const uint32_t *order,
                   uint32_t norder, BatchGlobal *g, unsigned long long wait_limit)
{
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ uint32_t item[4];     // slot, tile, epoch, go
    for (;;) {
        if (threadIdx.x < 64) {
            uint32_t s = 0, t = 0, e = 0;
            const bool go = claim_item(slots, state, order, norder, g, wait_limit, &s, &t, &e);
            if (threadIdx.x == 0) {
                item[0] = s; item[1] = t; item[2] = e; item[3] = go ? 1u : 0u;
            }
        }
        __syncthreads();
        const uint32_t go = item[3];
        const uint32_t slot = __builtin_amdgcn_readfirstlane(item[0]);
        const uint32_t tile = __builtin_amdgcn_readfirstlane(item[1]);
        const uint32_t epoch = __builtin_amdgcn_readfirstlane(item[2]);
        // every wavefront has its item before wavefront 0 may look for the next
        __syncthreads();
        if (!go) return;
        // see the merges of the epoch before (and no stale cached copy)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const BatchSlot &sl = slots[slot];
        const VisitArgs &a = sl.a;
        const uint32_t in = epoch & 1u;
        const region::Snapshots io{sl.key[in], sl.time[in], sl.key[in ^ 1u], sl.time[in ^ 1u]};
        region::RegionTally r;
        // unit-rate lattices take the visit without the division by the rate;
        // batch members do not collect the efficiency counters
        if (DIM == 2 || (DIM == 0 && sl.dim == 2))
            r = a.unit_rate ? region::visit_region<2, false, 1, true, false>(a, io, tile, lds)
                            : region::visit_region<2, false, 1, false, false>(a, io, tile, lds);
        else if (DIM == 3 || (DIM == 0 && sl.dim == 3))
            r = a.unit_rate ? region::visit_region<3, false, 1, true, false>(a, io, tile, lds)
                            : region::visit_region<3, false, 1, false, false>(a, io, tile, lds);
        else
            r = a.unit_rate ? region::visit_region<1, false, 1, true, false>(a, io, tile, lds)
                            : region::visit_region<1, false, 1, false, false>(a, io, tile, lds);
        // every wavefront's merge atomics have been performed
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __syncthreads();
        if (threadIdx.x == 0) {
            BatchState &st = state[slot];
            if (!r.skipped) {
                atomicAdd(&st.ctr[kEvents], (unsigned long long)r.events);
                atomicAdd(&st.ctr[kFlips], (unsigned long long)r.flips);
                atomicAdd(&st.ctr[kGhostEvents], (unsigned long long)r.ghost);
                atomicAdd(&st.ctr[kChecks], (unsigned long long)r.checks);
                atomicAdd(&st.ctr[kSweeps], (unsigned long long)r.rounds);
                atomicAdd(&st.epoch_moves, (unsigned long long)(r.events + r.ghost));
                if (r.any_live) atomicAdd(&st.live, 1u);
                // a later epoch's visit of this tile may run on another XCD
                if (!r.own_due)
                    atomicOr(reinterpret_cast<unsigned int *>(a.dead) + (tile >> 2),
                             1u << (8u * (tile & 3u)));
            }
            // this tile's merge and counters before its ticket
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __builtin_amdgcn_s_waitcnt(0);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            const uint32_t ticket = atomicAdd(&st.finished, 1u);
            if (ticket == sl.ntiles - 1u) close_epoch(st, epoch, g);
        }
        // the next claim's barriers keep the LDS of this visit until every
        // thread is done with it
    }
}

}  // namespace

size_t batch_lds_bytes(int dim, const VisitArgs &a) { return region::fast_plan(a, dim).total; }

namespace {
// Regions above half of a compute unit's LDS leave room for one workgroup.
int waves_for(size_t lds) { return lds > 80 * 1024 ? 2 : 4; }
}  // namespace

int batch_block_size(size_t) { return kBatchBlock; }

template <int WAVES>
const void *batch_visit_fn_w(int dim)
{
    switch (dim) {
    case 1: return (const void *)batch_visit_kernel<1, WAVES>;
    case 2: return (const void *)batch_visit_kernel<2, WAVES>;
    case 3: return (const void *)batch_visit_kernel<3, WAVES>;
    default: return (const void *)batch_visit_kernel<0, WAVES>;
    }
}

const void *batch_visit_fn(int dim, size_t lds)
{
    return waves_for(lds) == 2 ? batch_visit_fn_w<2>(dim) : batch_visit_fn_w<4>(dim);
}

hipError_t set_batch_lds_limit(size_t bytes)
{
    for (int d = 0; d <= 3; ++d)
        for (size_t l : {(size_t)0, (size_t)160 * 1024}) {
            const hipError_t e = hipFuncSetAttribute(
                batch_visit_fn(d, l), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

hipError_t batch_max_blocks(int dim, size_t lds, int *blocks)
{
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, batch_visit_fn(dim, lds), kBatchBlock, lds);
    if (e != hipSuccess) return e;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    *blocks = per_cu * cus;
    return hipSuccess;
}

hipError_t launch_batch_pack(const BatchSlot *slots, BatchState *state,
                             const uint32_t *joining, const uint32_t *block_start,
                             uint32_t count, uint32_t blocks, hipStream_t stream)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(batch_reset_kernel, dim3((count + 255) / 256), dim3(256), 0, stream,
                       state, joining, count);
    hipLaunchKernelGGL(batch_pack_kernel, dim3(blocks), dim3(kPackBlock), 0, stream, slots,
                       state, joining, block_start, count);
    return hipGetLastError();
}

hipError_t launch_batch_open(BatchState *state, const uint32_t *members, uint32_t count,
                             BatchGlobal *g, unsigned long long budget_ticks,
                             unsigned long long max_epochs, hipStream_t stream)
{
    hipLaunchKernelGGL(batch_open_kernel, dim3(1), dim3(1024), 0, stream, state, members,
                       count, g, budget_ticks, max_epochs);
    return hipGetLastError();
}

hipError_t launch_batch_visit(int dim, const BatchSlot *slots, BatchState *state,
                              const uint32_t *order, uint32_t norder, BatchGlobal *g,
                              unsigned long long wait_limit_ticks, int blocks, size_t lds,
                              hipStream_t stream)
{
    void *args[] = {(void *)&slots, (void *)&state, (void *)&order, (void *)&norder,
                    (void *)&g, (void *)&wait_limit_ticks};
    return hipLaunchKernel(batch_visit_fn(dim, lds), dim3(blocks), dim3(kBatchBlock), args,
                           lds, stream);
}

hipError_t launch_batch_unpack(const BatchSlot *slots, BatchState *state,
                               const uint32_t *members, const uint32_t *block_start,
                               uint32_t count, uint32_t blocks, hipStream_t stream)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(batch_unpack_kernel, dim3(blocks), dim3(kPackBlock), 0, stream, slots,
                       state, members, block_start, count);
    return hipGetLastError();
}

}  // namespace aca

// aca_internal.h -- launch interface between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aca {

// Most neighbours a cell's rule may read (q-th degree neighbourhoods).
constexpr int kMaxSlots = 31;

// Per-launch counters in device scratch (64-bit words).
enum Counter : int {
    kEvents = 0,        // arrivals applied to owned cells
    kFlips = 1,         // of which reversed the spin
    kGhostEvents = 2,   // arrivals applied to ghost copies (discarded)
    kLiveTiles = 3,     // tiles with an owned cell still before the horizon
    kSweeps = 4,        // worklist rounds summed over tile visits
    kChecks = 5,        // enabling tests evaluated
    kTminBits = 6,      // least pending time of the owned cells at load (bits)
    // Efficiency instruments (Section 4: the fraction of cells that pass the
    // enabling test at an iteration of Fig. 3.2, N0 / N)
    kScanLive = 7,      // owned cells with an arrival before the horizon at load
    kScanEnabled = 8,   // of which the visit's initial scan found enabled
    kRoundCells = 9,    // simulated cells before the horizon at load, times rounds run
    kNumCounters = 12
};

// Working state of a cell during aca_advance, two 64-bit words:
//   key  = n << 32 | f << 1 | (spin < 0)   n arrivals applied since time 0,
//                                          f spin flips since the advance began
//   time = bit pattern of the pending arrival time (> 0, so ordered as uint64)
// Both words only grow as the cell's trajectory advances, so the most
// advanced of several copies of a cell is their element-wise maximum.
//
// Everything a tile visit needs.  One workgroup simulates one tile region:
// the tile's own cells, `ghost` extra cells on each side of every direction
// the tile does not span, and a frozen one-cell ring around that.  Along a
// direction the tile spans (tile side >= lattice side) the region is the
// whole periodic side and its neighbours wrap inside the region.
struct VisitArgs {
    int32_t L[3];
    int32_t tile[3];
    int32_t ntiles[3];
    int32_t ghost[3];
    int32_t span[3];
    int32_t max_sweeps;
    uint32_t key_lo, key_hi;
    int32_t unit_rate;
    double rate;
    uint64_t horizon_bits;     // bit pattern of the horizon T > 0
    const unsigned long long *key_in;     // snapshot read by every region
    const unsigned long long *time_in;
    unsigned long long *key_out;          // merged record (element-wise max)
    unsigned long long *time_out;
    unsigned long long *counters;         // device slot of this launch
    unsigned long long *host_counters;    // pinned host copy, written by the last block
    unsigned int *done_blocks;            // ticket counter of this slot
    uint8_t *dead;                        // per tile: owned cells final in both snapshots
    int32_t range;                        // q of the q-th degree neighbourhood (1: nearest)
    uint64_t thr[2 * (kMaxSlots + 1)];
    // The advance's horizon T: a cell whose pending time is at or past it is
    // final.  `horizon_bits` above bounds the arrivals this launch may apply;
    // it equals final_bits unless a lag bound is set (then the host sets it
    // per launch to min(T, least pending time + lag), and every block adds
    // the least pending time of its owned cells to the kTminBits counter).
    uint64_t final_bits;
    int32_t track_tmin;
    // Output frames (Fig. 3.7): frame k holds the spins at time k * frame_dt
    // for k in [frame_k0, frame_k0 + nframes), int8 per cell, cell order.
    int8_t *frames;                       // NULL: no frames
    double frame_dt;
    long long frame_k0;
    long long nframes;
    uint64_t n_cells;
    // collect the efficiency counters (kScanLive, kScanEnabled, kRoundCells);
    // the region visits of the nearest-neighbour rule without frames skip
    // them otherwise
    int32_t count_efficiency;
};

// Write `spin` into every frame whose time k dt lies in (t_lo, t_hi]: the
// cell holds that spin from just after t_lo up to and including t_hi.  Every
// copy of a cell writes the same values (all copies follow the one
// trajectory), so concurrent writers agree.
__device__ __forceinline__ void capture_frames(
    int8_t *frames, double dt, long long k0, long long nframes, uint64_t n_cells, uint32_t gi,
    double t_lo, double t_hi, int8_t spin)
{
    const double q = t_lo / dt;
    if (!(q < 9.0e18)) return;            // beyond any representable frame index
    long long k = (long long)__builtin_floor(q);
    if (k < k0) k = k0;
    // the quotient may be off by one either way: settle on exact comparisons
    while ((double)k * dt <= t_lo) ++k;
    while (k > k0 && (double)(k - 1) * dt > t_lo) --k;
    const long long kend = k0 + nframes;
    for (; k < kend && (double)k * dt <= t_hi; ++k)
        frames[(uint64_t)(k - k0) * n_cells + gi] = spin;
}

// Called by thread 0 of every block of a visit launch after it has added its
// counters.  The last block to finish (ticket ntiles - 1) publishes the slot's
// counters to pinned host memory and clears the slot for its next use, so a
// launch needs no separate memset or copy command.  The counters and the
// ticket are device-scope atomics, performed where all blocks see them: the
// ticket only has to wait until this block's counter atomics have completed
// (a full release fence here would also write back the L2 on every block;
// the block's other writes are read by later launches only).
__device__ inline void finish_visit_block(const VisitArgs &a, unsigned int ntiles)
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);   // vmcnt, expcnt and lgkmcnt all zero
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    const unsigned int ticket = atomicAdd(a.done_blocks, 1u);
    if (ticket == ntiles - 1u) {
        __threadfence();
        for (int i = 0; i < kNumCounters; ++i) {
            const unsigned long long v =
                __hip_atomic_load(&a.counters[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.host_counters[i], v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&a.counters[i], i == kTminBits ? ~0ull : 0ull,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __hip_atomic_store(a.done_blocks, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence_system();
    }
}

// Bytes of dynamic LDS a visit needs for the largest region of this plan, and
// the number of simulated cells of that region (must stay below 65536).
size_t visit_lds_bytes(int dim, const VisitArgs &a, int block);
int visit_inner_max(int dim, const VisitArgs &a);

hipError_t launch_init(int dim, const int32_t *L, uint64_t n_cells, uint32_t key_lo,
                       uint32_t key_hi, double rate, int init, int8_t *s, double *t,
                       uint32_t *n, hipStream_t stream);

hipError_t launch_visit(int dim, const VisitArgs &a, int block, size_t lds,
                        hipStream_t stream);
hipError_t set_visit_lds_limit(size_t bytes);

// The variant for tiles that span no direction (aca_visit_fast.hip): its LDS
// need, its region box size (must stay below 65536), launch and LDS limit.
size_t visit_fast_lds_bytes(int dim, const VisitArgs &a);
int visit_fast_box(int dim, const VisitArgs &a);
hipError_t launch_visit_fast(int dim, const VisitArgs &a, int block, size_t lds,
                             hipStream_t stream);
// Whether a pitched-box visit exists for this dimension and reach q.
bool visit_fast_supports(int dim, int q);
hipError_t set_visit_fast_lds_limit(size_t bytes);

// Caller state (s, t, n) -> working words (flip count 0); adds sum of n to
// *sum_n.
hipError_t launch_pack(uint64_t n_cells, const int8_t *s, const double *t,
                       const uint32_t *n, unsigned long long *key,
                       unsigned long long *time, unsigned long long *sum_n,
                       hipStream_t stream);

// Sets *flag to 1 if some count n(c) is 2^31 or more (the region visits keep
// a claim in bit 31 of a count word); *flag must be 0 before.
hipError_t launch_count_bound(uint64_t n_cells, const uint32_t *n, unsigned long long *flag,
                              hipStream_t stream);

// Working words -> caller state; adds sum of n and sum of f to sums[0..1].
hipError_t launch_unpack(uint64_t n_cells, const unsigned long long *key,
                         const unsigned long long *time, int8_t *s, double *t,
                         uint32_t *n, unsigned long long *sums, hipStream_t stream);

// Frames at times in (T0, min(t(c), T)] get each cell's spin at the start of
// an advance from T0 to T (before any arrival of the advance is applied).
hipError_t launch_frames_init(const VisitArgs &a, const int8_t *s, const double *t, double T0,
                              double T, hipStream_t stream);

hipError_t launch_philox(const uint32_t *ctr, uint64_t seed, uint32_t *out,
                         uint64_t count, hipStream_t stream);

hipError_t launch_neg_log(const uint64_t *w, double *out, uint64_t count,
                          hipStream_t stream);


// ---------------------------------------------------------------- batches
//
// A batch advances many independent lattices in one persistent launch.  A
// lattice advances in epochs: epoch e visits every tile of the lattice once,
// reading snapshot e % 2 and merging into the other one, exactly like one
// launch of the single-lattice loop; the epochs of different lattices overlap
// freely.  Workgroups take (lattice, tile) items from the lattices' claim
// words; the workgroup that finishes the last tile of an epoch opens the next
// epoch, or retires the lattice once no owned cell has an arrival before its
// horizon.

// Read-only description of one member lattice during a launch.
struct BatchSlot {
    VisitArgs a;                         // geometry, stream key, horizon, thresholds
    unsigned long long *key[2];          // the two snapshots
    unsigned long long *time[2];
    int8_t *s;                           // the caller's state buffers
    double *t;
    uint32_t *cnt;
    uint64_t n_cells;
    int32_t dim;
    uint32_t ntiles;
};

enum SlotStatus : uint32_t {
    kSlotIdle = 0,      // not a member
    kSlotRunning = 1,   // has an open epoch in this launch
    kSlotPaused = 2,    // stopped at an epoch boundary (step budget); resumes next launch
    kSlotDone = 3,      // horizon reached; final state in snapshot `final_snap`
    kSlotStalled = 4,   // an epoch applied no arrival while some were due (error)
};

// Closed claim word: the low half is far above any tile count, so late
// increments by workgroups that read an open word never reach the epoch bits.
constexpr uint32_t kClaimClosed = 0x80000000u;

// Device-resident state of one member, kept across launches.
struct BatchState {
    unsigned long long claim;     // epoch << 32 | tiles handed out in that epoch
    uint32_t finished;            // tiles of the open epoch finished
    uint32_t live;                // of which an owned cell is still before the horizon
    uint32_t status;              // SlotStatus
    uint32_t epochs;              // epochs completed in the current launch
    uint32_t total_epochs;        // since the lattice joined
    uint32_t final_snap;          // snapshot holding the final state (when done)
    unsigned long long epoch_moves;   // arrivals applied (owned + ghost) in the open epoch
    unsigned long long ctr[kNumCounters];   // Counter totals since the lattice joined
    unsigned long long sum_start;   // sum of n when packed
    unsigned long long sum_end;     // sum of n when unpacked
    unsigned long long sum_flips;   // flips since packed (from the unpacked words)
    unsigned long long unpacked;    // 1 once the final state is in the caller's buffers
};

struct BatchGlobal {
    uint32_t active;              // members running in this launch
    uint32_t error;               // a workgroup gave up waiting (no progress anywhere)
    uint32_t pad[2];
    unsigned long long deadline;  // device wall clock after which epochs pause
    unsigned long long max_epochs;   // epochs per member per launch
};

// Host side of the batch kernels (aca_batch.hip).
size_t batch_lds_bytes(int dim, const VisitArgs &a);
hipError_t set_batch_lds_limit(size_t bytes);
// Threads per workgroup of the persistent visit (for regions of `lds` bytes).
int batch_block_size(size_t lds);
// Resident blocks of the visit kernel for `dim` (0 = mixed) on this device.
hipError_t batch_max_blocks(int dim, size_t lds, int *blocks);
// Pack the members listed in `joining` (state zeroed, snapshot 1 and tile
// flags cleared, sum of n recorded); `block_start[i]` is the first block of
// joining[i], block_start[count] the grid size.
hipError_t launch_batch_pack(const BatchSlot *slots, BatchState *state,
                             const uint32_t *joining, const uint32_t *block_start,
                             uint32_t count, uint32_t blocks, hipStream_t stream);
// Re-open paused members, count running ones, arm the deadline (ticks of the
// device wall clock from now; 0 = none).
hipError_t launch_batch_open(BatchState *state, const uint32_t *members, uint32_t count,
                             BatchGlobal *g, unsigned long long budget_ticks,
                             unsigned long long max_epochs, hipStream_t stream);
hipError_t launch_batch_visit(int dim, const BatchSlot *slots, BatchState *state,
                              const uint32_t *order, uint32_t norder, BatchGlobal *g,
                              unsigned long long wait_limit_ticks, int blocks, size_t lds,
                              hipStream_t stream);
// Unpack members that are done and not yet unpacked (same block map as pack).
hipError_t launch_batch_unpack(const BatchSlot *slots, BatchState *state,
                               const uint32_t *members, const uint32_t *block_start,
                               uint32_t count, uint32_t blocks, hipStream_t stream);

}  // namespace aca

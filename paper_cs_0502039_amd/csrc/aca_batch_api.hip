// aca_batch_api.hip -- C-ABI of batches (declared in include/aca.h).
//
// Host side of the persistent batch kernels: member bookkeeping, the tile
// plan of each member, the priority order, and one step = pack the joining
// members, re-open the paused ones, one persistent visit launch, unpack the
// members that finished, read the members' device state back.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <vector>

#include "../../include/aca.h"
#include "aca_host.h"
#include "aca_internal.h"

using namespace aca_host;

namespace {

constexpr int kPackBlock = 256;            // threads per pack/unpack block
constexpr uint64_t kCellsPerPackBlock = 8 * kPackBlock;
constexpr uint32_t kMaxPackBlocks = 1024;  // per member
// A workgroup that finds no open item for this long gives up; the step then
// reports ACA_ENOPROGRESS instead of waiting for ever.
constexpr double kWaitLimitSeconds = 20.0;
// Static LDS of the persistent visit kernel (its item words), with room to spare.
constexpr size_t kBatchStaticLds = 256;
// aca_batch_advance returns to the host at least this often.
constexpr double kAdvanceStepMs = 1000.0;
// Tiles per member stay far below the closed-claim mark of the claim words.
constexpr uint64_t kMaxBatchTiles = aca::kClaimClosed / 2;

struct WorkLayout {
    size_t slots, state, order, joining, joining_start, members, members_start, global, total;
};

WorkLayout work_layout(int32_t cap)
{
    WorkLayout w;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    w.slots = take(sizeof(aca::BatchSlot) * (size_t)cap);
    w.state = take(sizeof(aca::BatchState) * (size_t)cap);
    w.order = take(4 * (size_t)cap);
    w.joining = take(4 * (size_t)cap);
    w.joining_start = take(4 * ((size_t)cap + 1));
    w.members = take(4 * (size_t)cap);
    w.members_start = take(4 * ((size_t)cap + 1));
    w.global = take(sizeof(aca::BatchGlobal));
    w.total = off;
    return w;
}

struct Member {
    aca_lattice *lat = nullptr;
    double T = 0.0;
    bool joining = false;
    uint64_t seq = 0;           // attach order
    uint64_t work = 0;          // arrivals expected: N (T - last T) rate
    uint64_t region_bytes = 0;  // per epoch
    size_t lds = 0;
};

uint32_t pack_blocks(uint64_t n)
{
    const uint64_t b = (n + kCellsPerPackBlock - 1) / kCellsPerPackBlock;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(b, kMaxPackBlocks));
}

}  // namespace

struct aca_batch {
    int device = 0;
    int32_t capacity = 0;
    WorkLayout wl;
    char *work = nullptr;
    aca::BatchSlot *d_slots = nullptr;
    aca::BatchState *d_state = nullptr;
    aca::BatchGlobal *d_g = nullptr;
    uint32_t *d_order = nullptr, *d_joining = nullptr, *d_joining_start = nullptr;
    uint32_t *d_members = nullptr, *d_members_start = nullptr;
    // pinned host staging
    aca::BatchSlot *h_slots = nullptr;
    aca::BatchState *h_state = nullptr;
    uint32_t *h_lists = nullptr;      // order, joining, joining_start, members, members_start
    aca::BatchGlobal *h_g = nullptr;
    std::vector<Member> member;       // per slot
    std::deque<aca_lattice *> finished;
    aca_tuning tun[4];                // per dim (index 1..3); 0 fields = automatic
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double wall_hz = 0.0;
    size_t lds_limit_set = 0;
    int32_t order = ACA_ORDER_WORK;
    uint64_t next_seq = 0;
    aca_batch_stats stats;
};

namespace {

// Automatic knobs of batch members: those of a single lattice (the
// persistent kernel picks its own threads per workgroup).
void batch_auto_tuning(int dim, aca_tuning *t)
{
    aca_params p;
    memset(&p, 0, sizeof p);
    p.dim = dim;
    p.range = 1;
    auto_tuning(p, t);
}

// Tile plan of a batch member: at least two tiles along every direction, so
// every region has a frozen ring and the pitched-box visit applies.
aca_status member_plan(const aca_batch *b, const aca_lattice *lat, double T, aca::VisitArgs *a,
                       size_t *lds)
{
    const aca_params &p = lat->p;
    aca_tuning t;
    memset(&t, 0, sizeof t);
    t.ghost[0] = t.ghost[1] = t.ghost[2] = -1;
    batch_auto_tuning(p.dim, &t);
    const aca_tuning &u = b->tun[p.dim];
    for (int d = 0; d < 3; ++d) {
        if (u.tile[d] > 0) t.tile[d] = u.tile[d];
        if (u.ghost[d] >= 0) t.ghost[d] = u.ghost[d];
    }
    if (u.max_sweeps > 0) t.max_sweeps = u.max_sweeps;
    t.max_sweeps = std::min(t.max_sweeps, 255);
    memset(a, 0, sizeof *a);
    for (int d = 0; d < 3; ++d) {
        if (d < p.dim) {
            const int L = p.L[d];
            const int k = std::max(2, (L + t.tile[d] - 1) / t.tile[d]);
            const int tile = (L + k - 1) / k;
            a->L[d] = L;
            a->tile[d] = tile;
            a->ntiles[d] = (L + tile - 1) / tile;
            a->ghost[d] = std::max(0, std::min(t.ghost[d], (L - tile) / 2));
            a->span[d] = 0;
        } else {
            a->L[d] = 1; a->tile[d] = 1; a->ntiles[d] = 1; a->ghost[d] = 0; a->span[d] = 1;
        }
    }
    a->max_sweeps = t.max_sweeps;
    a->key_lo = (uint32_t)p.seed;
    a->key_hi = (uint32_t)(p.seed >> 32);
    a->rate = p.rate;
    a->unit_rate = p.rate == 1.0 ? 1 : 0;
    uint64_t hb;
    memcpy(&hb, &T, sizeof hb);
    a->horizon_bits = hb;
    a->final_bits = hb;          // no lag bound and no frames in a batch
    a->n_cells = lat->n;
    a->dead = lat->dead;
    memcpy(a->thr, lat->thr, sizeof a->thr);
    const uint64_t tiles = (uint64_t)a->ntiles[0] * a->ntiles[1] * a->ntiles[2];
    if (tiles >= kMaxBatchTiles)
        return fail(ACA_EINVAL, "lattice has too many tiles for a batch");
    int dev_lds = 0;
    HIP_TRY(hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                  lat->device));
    if (aca::visit_fast_box(p.dim, *a) > 65535)
        return fail(ACA_EINVAL, "batch tile region box of %d cells exceeds 65535",
                    aca::visit_fast_box(p.dim, *a));
    *lds = aca::batch_lds_bytes(p.dim, *a);
    if (*lds > (size_t)dev_lds)
        return fail(ACA_EINVAL, "batch tile region needs %zu B of LDS, device has %d B",
                    *lds, dev_lds);
    return ACA_OK;
}

}  // namespace

ACA_EXPORT aca_status aca_batch_query(int32_t capacity, uint64_t *work_bytes)
{
    if (capacity < 1 || capacity > (1 << 20))
        return fail(ACA_EINVAL, "capacity %d not in 1..2^20", capacity);
    if (!work_bytes) return fail(ACA_EINVAL, "work_bytes is NULL");
    *work_bytes = work_layout(capacity).total;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_batch_create(int32_t capacity, void *d_work, uint64_t work_bytes,
                                       aca_batch **out)
{
    if (capacity < 1 || capacity > (1 << 20))
        return fail(ACA_EINVAL, "capacity %d not in 1..2^20", capacity);
    if (!d_work || !out) return fail(ACA_EINVAL, "NULL argument");
    if (((uintptr_t)d_work) % kAlign != 0)
        return fail(ACA_EINVAL, "work buffer must be %zu-byte aligned", kAlign);
    const WorkLayout wl = work_layout(capacity);
    if (work_bytes < wl.total)
        return fail(ACA_ENOMEM, "work buffer has %llu bytes, needs %zu",
                    (unsigned long long)work_bytes, wl.total);
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    aca_batch *b = new (std::nothrow) aca_batch();
    if (!b) return fail(ACA_ENOMEM, "host allocation failed");
    b->device = device;
    b->capacity = capacity;
    b->wl = wl;
    b->work = static_cast<char *>(d_work);
    b->d_slots = reinterpret_cast<aca::BatchSlot *>(b->work + wl.slots);
    b->d_state = reinterpret_cast<aca::BatchState *>(b->work + wl.state);
    b->d_order = reinterpret_cast<uint32_t *>(b->work + wl.order);
    b->d_joining = reinterpret_cast<uint32_t *>(b->work + wl.joining);
    b->d_joining_start = reinterpret_cast<uint32_t *>(b->work + wl.joining_start);
    b->d_members = reinterpret_cast<uint32_t *>(b->work + wl.members);
    b->d_members_start = reinterpret_cast<uint32_t *>(b->work + wl.members_start);
    b->d_g = reinterpret_cast<aca::BatchGlobal *>(b->work + wl.global);
    b->member.resize(capacity);
    for (int d = 0; d < 4; ++d) {
        memset(&b->tun[d], 0, sizeof b->tun[d]);
        b->tun[d].struct_size = sizeof(aca_tuning);
        b->tun[d].ghost[0] = b->tun[d].ghost[1] = b->tun[d].ghost[2] = -1;
    }
    memset(&b->stats, 0, sizeof b->stats);
    b->stats.struct_size = sizeof(aca_batch_stats);
    int khz = 0;
    bool ok = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device) ==
              hipSuccess && khz > 0;
    b->wall_hz = 1e3 * khz;
    ok = ok &&
         hipHostMalloc((void **)&b->h_slots, sizeof(aca::BatchSlot) * capacity) == hipSuccess &&
         hipHostMalloc((void **)&b->h_state, sizeof(aca::BatchState) * capacity) ==
             hipSuccess &&
         hipHostMalloc((void **)&b->h_lists, 4 * (5 * (size_t)capacity + 2)) == hipSuccess &&
         hipHostMalloc((void **)&b->h_g, sizeof(aca::BatchGlobal)) == hipSuccess &&
         hipEventCreate(&b->ev0) == hipSuccess && hipEventCreate(&b->ev1) == hipSuccess;
    if (!ok) {
        if (b->h_slots) (void)hipHostFree(b->h_slots);
        if (b->h_state) (void)hipHostFree(b->h_state);
        if (b->h_lists) (void)hipHostFree(b->h_lists);
        if (b->h_g) (void)hipHostFree(b->h_g);
        if (b->ev0) (void)hipEventDestroy(b->ev0);
        if (b->ev1) (void)hipEventDestroy(b->ev1);
        delete b;
        return fail(ACA_EDEVICE, "pinned staging, events or the wall-clock rate unavailable");
    }
    memset(b->h_state, 0, sizeof(aca::BatchState) * capacity);
    // every slot starts idle on the device
    hipError_t e = hipMemcpy(b->d_state, b->h_state, sizeof(aca::BatchState) * capacity,
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipHostFree(b->h_slots);
        (void)hipHostFree(b->h_state);
        (void)hipHostFree(b->h_lists);
        (void)hipHostFree(b->h_g);
        (void)hipEventDestroy(b->ev0);
        (void)hipEventDestroy(b->ev1);
        delete b;
        return fail(ACA_EDEVICE, "hipMemcpy of the idle slot states failed: %s",
                    hipGetErrorString(e));
    }
    *out = b;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_batch_set_tuning(aca_batch *b, int32_t dim, const aca_tuning *t)
{
    if (!b) return fail(ACA_EINVAL, "batch is NULL");
    if (dim < 1 || dim > 3) return fail(ACA_EINVAL, "dim %d not in 1..3", dim);
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
        v = *t;
        v.block = 0;
    }
    b->tun[dim] = v;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_batch_get_tuning(const aca_batch *b, int32_t dim, aca_tuning *out)
{
    if (!b || !out) return fail(ACA_EINVAL, "NULL argument");
    if (dim < 1 || dim > 3) return fail(ACA_EINVAL, "dim %d not in 1..3", dim);
    aca_tuning t;
    memset(&t, 0, sizeof t);
    batch_auto_tuning(dim, &t);
    const aca_tuning &u = b->tun[dim];
    for (int d = 0; d < 3; ++d) {
        if (u.tile[d] > 0) t.tile[d] = u.tile[d];
        if (u.ghost[d] >= 0) t.ghost[d] = u.ghost[d];
        if (d >= dim) { t.tile[d] = 0; t.ghost[d] = 0; }
    }
    if (u.max_sweeps > 0) t.max_sweeps = u.max_sweeps;
    t.struct_size = sizeof t;
    t.block = 0;     // the persistent kernel always runs 512 threads per workgroup
    *out = t;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_batch_set_order(aca_batch *b, int32_t order)
{
    if (!b) return fail(ACA_EINVAL, "batch is NULL");
    if (order != ACA_ORDER_WORK && order != ACA_ORDER_ARRIVAL)
        return fail(ACA_EINVAL, "unknown order %d", order);
    b->order = order;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_batch_attach(aca_batch *b, aca_lattice *lat, double T)
{
    if (!b || !lat) return fail(ACA_EINVAL, "NULL argument");
    if (lat->attached) return fail(ACA_ESTATE, "lattice is already a batch member");
    if (!lat->initialized) return fail(ACA_ESTATE, "aca_init (or aca_resume) first");
    if (lat->p.range > 1)
        return fail(ACA_EINVAL, "q-th degree neighbourhoods run on the single-lattice path");
    if (lat->device != b->device)
        return fail(ACA_EINVAL, "lattice is on device %d, batch on device %d", lat->device,
                    b->device);
    if (!is_finite(T) || T < lat->last_T || T <= 0.0)
        return fail(ACA_EINVAL, "horizon %.17g must be finite, > 0 and >= the last one %.17g",
                    T, lat->last_T);
    if (!aca_host::horizon_fits_counts(lat->p.rate, T))
        return fail(ACA_EINVAL, "rate * horizon = %.17g exceeds 2^30 (arrival counts are 31-bit)",
                    lat->p.rate * T);
    int slot = -1;
    for (int i = 0; i < b->capacity; ++i)
        if (!b->member[i].lat) { slot = i; break; }
    if (slot < 0) return fail(ACA_ENOMEM, "batch is full (%d members)", b->capacity);
    aca::VisitArgs a;
    size_t lds = 0;
    aca_status st = member_plan(b, lat, T, &a, &lds);
    if (st != ACA_OK) return st;
    aca::BatchSlot &s = b->h_slots[slot];
    memset(&s, 0, sizeof s);
    s.a = a;
    for (int k = 0; k < 2; ++k) {
        s.key[k] = lat->key[k];
        s.time[k] = lat->time[k];
    }
    s.s = lat->s;
    s.t = lat->t;
    s.cnt = lat->cnt;
    s.n_cells = lat->n;
    s.dim = lat->p.dim;
    s.ntiles = (uint32_t)((uint64_t)a.ntiles[0] * a.ntiles[1] * a.ntiles[2]);
    Member &m = b->member[slot];
    m.lat = lat;
    m.T = T;
    m.joining = true;
    m.seq = b->next_seq++;
    m.work = (uint64_t)((double)lat->n * (T - lat->last_T) * lat->p.rate);
    m.region_bytes = launch_region_bytes(lat->p.dim, a);
    m.lds = lds;
    lat->attached = true;
    return ACA_OK;
}

namespace {

void detach(aca_batch *b, int slot)
{
    b->member[slot].lat->attached = false;
    b->member[slot] = Member();
}

}  // namespace

ACA_EXPORT aca_status aca_batch_step(aca_batch *b, double budget_ms, int32_t max_epochs,
                                     void *stream, int32_t *n_members)
{
    if (!b) return fail(ACA_EINVAL, "batch is NULL");
    if (!is_finite(budget_ms)) return fail(ACA_EINVAL, "budget_ms must be finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const auto t0 = std::chrono::steady_clock::now();
    // member lists: priority order (most remaining work first), joining, all
    std::vector<int> mem;
    for (int i = 0; i < b->capacity; ++i)
        if (b->member[i].lat) mem.push_back(i);
    if (mem.empty()) {
        if (n_members) *n_members = 0;
        return ACA_OK;
    }
    const int cap = b->capacity;
    uint32_t *h_order = b->h_lists;
    uint32_t *h_join = h_order + cap;
    uint32_t *h_join_start = h_join + cap;
    uint32_t *h_mem = h_join_start + cap + 1;
    uint32_t *h_mem_start = h_mem + cap;
    std::vector<int> prio = mem;
    if (b->order == ACA_ORDER_ARRIVAL)
        std::sort(prio.begin(), prio.end(), [&](int x, int y) {
            return b->member[x].seq < b->member[y].seq;
        });
    else
        std::stable_sort(prio.begin(), prio.end(), [&](int x, int y) {
            return b->member[x].work > b->member[y].work;
        });
    // Members whose regions leave room for two workgroups per compute unit
    // (class 0) and the others (class 1) run in launches of their own, one
    // after the other: a launch gives every workgroup the largest region of
    // its members, so one large 3D region would otherwise halve the
    // workgroups of every 2D member.
    int lds_per_cu = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds_per_cu,
                                  hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, b->device));
    auto cls = [&](const Member &m) { return 2 * (m.lds + kBatchStaticLds) <= (size_t)lds_per_cu ? 0 : 1; };
    int dim_c[2] = {-1, -1};
    size_t lds_c[2] = {0, 0};
    uint64_t work_c[2] = {0, 0};
    uint32_t n_c[2] = {0, 0};
    uint32_t njoin = 0, jblocks = 0, mblocks = 0;
    int max_slot = 0;
    for (size_t i = 0; i < mem.size(); ++i) {
        const int sl = mem[i];
        const Member &m = b->member[sl];
        h_mem[i] = (uint32_t)sl;
        h_mem_start[i] = mblocks;
        mblocks += pack_blocks(m.lat->n);
        if (m.joining) {
            h_join[njoin] = (uint32_t)sl;
            h_join_start[njoin] = jblocks;
            jblocks += pack_blocks(m.lat->n);
            ++njoin;
        }
        const int c = cls(m);
        dim_c[c] = dim_c[c] < 0 ? m.lat->p.dim : (dim_c[c] == m.lat->p.dim ? dim_c[c] : 0);
        lds_c[c] = std::max(lds_c[c], m.lds);
        work_c[c] += m.work;
        ++n_c[c];
        max_slot = std::max(max_slot, sl);
    }
    // the priority order, class 0's members first, then class 1's
    uint32_t fill[2] = {0, n_c[0]};
    for (int sl : prio) h_order[fill[cls(b->member[sl])]++] = (uint32_t)sl;
    const uint32_t nmem = (uint32_t)mem.size();
    h_mem_start[nmem] = mblocks;
    h_join_start[njoin] = jblocks;

    const size_t lds_max = std::max(lds_c[0], lds_c[1]);
    if (lds_max > b->lds_limit_set) {
        HIP_TRY(aca::set_batch_lds_limit(lds_max));
        b->lds_limit_set = lds_max;
    }
    int blocks_c[2] = {0, 0};
    for (int c = 0; c < 2; ++c) {
        if (!n_c[c]) continue;
        HIP_TRY(aca::batch_max_blocks(dim_c[c], lds_c[c], &blocks_c[c]));
        if (blocks_c[c] < 1) return fail(ACA_EINVAL, "the batch kernel does not fit a compute unit");
    }

    if (njoin) {
        HIP_TRY(hipMemcpyAsync(b->d_slots, b->h_slots, sizeof(aca::BatchSlot) * (max_slot + 1),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(b->d_joining, h_join, 4 * njoin, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(b->d_joining_start, h_join_start, 4 * (njoin + 1),
                               hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipMemcpyAsync(b->d_order, h_order, 4 * nmem, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(b->d_members, h_mem, 4 * nmem, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(b->d_members_start, h_mem_start, 4 * (nmem + 1),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(aca::launch_batch_pack(b->d_slots, b->d_state, b->d_joining, b->d_joining_start,
                                   njoin, jblocks, s));
    const unsigned long long epochs_cap =
        max_epochs > 0 ? (unsigned long long)max_epochs : ~0ull;
    // With both classes present the step's budget is shared in proportion to
    // their remaining arrivals (at least a quarter each); a launch whose
    // members all finish ends early anyway.
    const uint64_t work_all = work_c[0] + work_c[1];
    HIP_TRY(hipEventRecord(b->ev0, s));
    uint32_t first = 0;
    for (int c = 0; c < 2; ++c) {
        if (!n_c[c]) continue;
        double share = 1.0;
        if (n_c[0] && n_c[1] && work_all > 0)
            share = std::min(1.0, std::max(0.25, (double)work_c[c] / (double)work_all));
        const unsigned long long budget_ticks =
            budget_ms > 0.0
                ? (unsigned long long)std::max(1.0, share * budget_ms * 1e-3 * b->wall_hz)
                : 0ull;
        HIP_TRY(aca::launch_batch_open(b->d_state, b->d_order + first, n_c[c], b->d_g,
                                       budget_ticks, epochs_cap, s));
        HIP_TRY(aca::launch_batch_visit(dim_c[c], b->d_slots, b->d_state, b->d_order + first,
                                        n_c[c], b->d_g,
                                        (unsigned long long)(kWaitLimitSeconds * b->wall_hz),
                                        blocks_c[c], lds_c[c], s));
        first += n_c[c];
    }
    HIP_TRY(hipEventRecord(b->ev1, s));
    HIP_TRY(aca::launch_batch_unpack(b->d_slots, b->d_state, b->d_members, b->d_members_start,
                                     nmem, mblocks, s));
    HIP_TRY(hipMemcpyAsync(b->h_state, b->d_state, sizeof(aca::BatchState) * (max_slot + 1),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(b->h_g, b->d_g, sizeof(aca::BatchGlobal), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    float kms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&kms, b->ev0, b->ev1));

    aca_batch_stats &S = b->stats;
    S.steps += 1;
    S.kernel_ms += kms;
    aca_status result = ACA_OK;
    for (int sl : mem) {
        Member &m = b->member[sl];
        const aca::BatchState &st = b->h_state[sl];
        m.joining = false;
        if (st.status == aca::kSlotDone) {
            aca_lattice *lat = m.lat;
            const uint64_t events = st.sum_end - st.sum_start;
            aca_stats &L = lat->stats;
            L.launches += st.total_epochs;
            L.visits += (uint64_t)st.total_epochs * b->h_slots[sl].ntiles;
            L.sweeps += st.ctr[aca::kSweeps];
            L.ghost_events += st.ctr[aca::kGhostEvents];
            L.cell_checks += st.ctr[aca::kChecks];
            L.events += events;
            L.flips += st.sum_flips;
            L.region_bytes += (uint64_t)st.total_epochs * m.region_bytes;
            lat->last_T = m.T;
            L.last_T = m.T;
            S.epochs += st.total_epochs;
            S.visits += (uint64_t)st.total_epochs * b->h_slots[sl].ntiles;
            S.sweeps += st.ctr[aca::kSweeps];
            S.events += events;
            S.flips += st.sum_flips;
            S.ghost_events += st.ctr[aca::kGhostEvents];
            S.cell_checks += st.ctr[aca::kChecks];
            S.region_bytes += (uint64_t)st.total_epochs * m.region_bytes;
            S.finished += 1;
            b->finished.push_back(lat);
            detach(b, sl);
        } else if (st.status == aca::kSlotPaused) {
            // progress estimate for the priority order
            const uint64_t done = st.ctr[aca::kEvents];
            const uint64_t total =
                (uint64_t)((double)m.lat->n * (m.T - m.lat->last_T) * m.lat->p.rate);
            m.work = total > done ? total - done : 0;
        } else {
            if (result == ACA_OK)
                result = fail(ACA_ENOPROGRESS,
                              st.status == aca::kSlotStalled
                                  ? "a batch member's epoch applied no arrival while arrivals "
                                    "were due"
                                  : "batch workgroups found no open item for %.0f s",
                              kWaitLimitSeconds);
            detach(b, sl);
        }
    }
    if (n_members) {
        int32_t n = 0;
        for (int i = 0; i < b->capacity; ++i) n += b->member[i].lat ? 1 : 0;
        *n_members = n;
    }
    S.device_ms +=
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
            .count();
    return result;
}

ACA_EXPORT aca_status aca_batch_poll(aca_batch *b, aca_lattice **done, int32_t cap,
                                     int32_t *n_done)
{
    if (!b || !n_done || (cap > 0 && !done)) return fail(ACA_EINVAL, "NULL argument");
    int32_t n = 0;
    while (n < cap && !b->finished.empty()) {
        done[n++] = b->finished.front();
        b->finished.pop_front();
    }
    *n_done = n;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_batch_advance(aca_batch *b, aca_lattice *const *lats, const double *T,
                                        int32_t count, void *stream)
{
    if (!b) return fail(ACA_EINVAL, "batch is NULL");
    if (count < 0 || (count > 0 && (!lats || !T))) return fail(ACA_EINVAL, "bad lattice list");
    for (int i = 0; i < b->capacity; ++i)
        if (b->member[i].lat) return fail(ACA_ESTATE, "batch already has members");
    if (count > b->capacity)
        return fail(ACA_ENOMEM, "%d lattices exceed the batch capacity %d", count, b->capacity);
    for (int32_t i = 0; i < count; ++i) {
        if (!lats[i]) return fail(ACA_EINVAL, "lattice %d is NULL", i);
        for (int32_t j = 0; j < i; ++j)
            if (lats[j] == lats[i]) return fail(ACA_EINVAL, "lattice %d listed twice", i);
    }
    for (int32_t i = 0; i < count; ++i) {
        // a horizon equal to the last one needs no work
        if (lats[i]->initialized && !lats[i]->attached && T[i] == lats[i]->last_T) continue;
        aca_status st = aca_batch_attach(b, lats[i], T[i]);
        if (st != ACA_OK) {
            for (int k = 0; k < b->capacity; ++k)
                if (b->member[k].lat) detach(b, k);
            return st;
        }
    }
    int32_t left = 1;
    aca_status result = ACA_OK;
    while (left > 0) {
        aca_status st = aca_batch_step(b, kAdvanceStepMs, 0, stream, &left);
        if (st != ACA_OK) {
            result = st;
            if (st != ACA_ENOPROGRESS) {
                for (int k = 0; k < b->capacity; ++k)
                    if (b->member[k].lat) detach(b, k);
                break;
            }
        }
    }
    b->finished.clear();
    return result;
}

ACA_EXPORT aca_status aca_batch_tune(aca_batch *b, aca_lattice *const *lats, const double *T,
                                     int32_t count, int32_t dim, const aca_tuning *cands,
                                     int32_t n, double frac, void *stream, int32_t *best,
                                     double *rates, int32_t *n_out)
{
    if (!b) return fail(ACA_EINVAL, "batch is NULL");
    if (dim < 1 || dim > 3) return fail(ACA_EINVAL, "dim %d not in 1..3", dim);
    if (count < 1 || !lats || !T) return fail(ACA_EINVAL, "bad lattice list");
    if (!is_finite(frac) || !(frac > 0.0) || frac >= 0.5)
        return fail(ACA_EINVAL, "frac must be in (0, 0.5)");
    for (int i = 0; i < b->capacity; ++i)
        if (b->member[i].lat) return fail(ACA_ESTATE, "batch already has members");
    aca_tuning table[ACA_TUNE_MAX];
    if (!cands || n <= 0) {
        n = tune_candidates(dim, table);
        cands = table;
    }
    if (n > ACA_TUNE_MAX) return fail(ACA_EINVAL, "at most %d candidates", ACA_TUNE_MAX);
    for (int32_t k = 0; k < n; ++k)
        if (cands[k].struct_size != sizeof(aca_tuning))
            return fail(ACA_EINVAL, "candidate %d: struct_size mismatch", k);
    for (int32_t i = 0; i < count; ++i) {
        if (!lats[i]) return fail(ACA_EINVAL, "lattice %d is NULL", i);
        if (!lats[i]->initialized || lats[i]->attached)
            return fail(ACA_ESTATE, "lattice %d is not initialised or is attached", i);
        if (!is_finite(T[i]) || T[i] < lats[i]->last_T)
            return fail(ACA_EINVAL, "lattice %d: horizon before its last one", i);
    }
    const aca_tuning keep = b->tun[dim];
    std::vector<double> start(count), h(count);
    for (int32_t i = 0; i < count; ++i) start[i] = lats[i]->last_T;
    // slice s ends at start + (s + 1) frac / 2 (T - start); slice 0 is the
    // warm-up, then each candidate runs two slices, the candidates in order and
    // then in reverse order (a steady drift along the trajectories favours none)
    auto slice = [&](int s) -> aca_status {
        for (int32_t i = 0; i < count; ++i) {
            h[i] = start[i] + (double)(s + 1) * 0.5 * frac * (T[i] - start[i]);
            h[i] = std::min(std::max(h[i], lats[i]->last_T), T[i]);
        }
        return aca_batch_advance(b, lats, h.data(), count, stream);
    };
    if ((2 * n + 1) * frac > 2.0)
        return fail(ACA_EINVAL, "%d candidates need (n + 1/2) frac <= 1", n);
    aca_status st = aca_batch_set_tuning(b, dim, &cands[0]);
    if (st == ACA_OK) st = slice(0);
    std::vector<double> ev(n, 0.0), ms(n, 0.0);
    for (int32_t j = 0; j < 2 * n && st == ACA_OK; ++j) {
        const int32_t k = j < n ? j : 2 * n - 1 - j;
        st = aca_batch_set_tuning(b, dim, &cands[k]);
        if (st != ACA_OK) break;
        const aca_batch_stats s0 = b->stats;
        st = slice(j + 1);
        if (st != ACA_OK) break;
        ev[k] += (double)(b->stats.events - s0.events);
        ms[k] += b->stats.device_ms - s0.device_ms;
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
        b->tun[dim] = keep;
        return st;
    }
    st = aca_batch_set_tuning(b, dim, &cands[best_k]);
    if (st != ACA_OK) return st;
    if (best) *best = best_k;
    if (n_out) *n_out = n;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_batch_members(const aca_batch *b, aca_lattice **out, int32_t cap,
                                        int32_t *n_members)
{
    if (!b || !n_members || (cap > 0 && !out)) return fail(ACA_EINVAL, "NULL argument");
    int32_t n = 0;
    for (int i = 0; i < b->capacity; ++i) {
        if (!b->member[i].lat) continue;
        if (n < cap) out[n] = b->member[i].lat;
        ++n;
    }
    *n_members = n;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_batch_get_stats(const aca_batch *b, aca_batch_stats *out)
{
    if (!b || !out) return fail(ACA_EINVAL, "NULL argument");
    *out = b->stats;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_batch_destroy(aca_batch *b)
{
    if (!b) return ACA_OK;
    for (int i = 0; i < b->capacity; ++i)
        if (b->member[i].lat) return fail(ACA_ESTATE, "batch still has members");
    (void)hipHostFree(b->h_slots);
    (void)hipHostFree(b->h_state);
    (void)hipHostFree(b->h_lists);
    (void)hipHostFree(b->h_g);
    (void)hipEventDestroy(b->ev0);
    (void)hipEventDestroy(b->ev1);
    delete b;
    return ACA_OK;
}

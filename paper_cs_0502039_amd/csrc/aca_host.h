// aca_host.h -- host-side internals shared by the C-ABI translation units:
// error reporting, argument checks, the scratch layout, the lattice handle
// and the tile plan.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/aca.h"
#include "aca_internal.h"

#define ACA_EXPORT extern "C" __attribute__((visibility("default")))

// Returns ACA_EDEVICE with the HIP message from the enclosing function.
#define HIP_TRY(expr)                                                              \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess)                                                      \
            return aca_host::fail(ACA_EDEVICE, "%s failed: %s", #expr,             \
                                  hipGetErrorString(e_));                          \
    } while (0)

namespace aca_host {

// Sets the calling thread's message (aca_last_error) and returns `code`.
aca_status fail(aca_status code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// Arrival counts stay below 2^31 (a region's LDS count word keeps a claim bit
// above them): a horizon is accepted while rate * T <= 2^30, so that 2^31
// arrivals of one cell would lie some 2^15 standard deviations out.
constexpr double kMaxMeanArrivals = 1073741824.0;
inline bool horizon_fits_counts(double rate, double T) { return rate * T <= kMaxMeanArrivals; }

// Scratch: two snapshots of working words (key, time), one flag byte per
// cell for tile flags (a tile holds at least one cell), and the counters.
struct ScratchLayout {
    size_t key_off[2], time_off[2], dead_off, ctr_off, total;
};
ScratchLayout scratch_layout(uint64_t n);

// Counter words in scratch: two slots of visit counters (launches alternate
// between them), the pack/unpack sums, and the two slots' block tickets.
enum : int {
    kSlotWords = 16, kSumStart = 32, kSumEnd = 33, kSumFlips = 34, kTicketWord = 36,
    kCounterWords = 40
};
static_assert(aca::kNumCounters <= kSlotWords, "a counter slot holds every counter");
static_assert(8 * kCounterWords <= 2 * kAlign, "counters fit their scratch block");

bool is_finite(double v);
// Validates the caller's parameters (either ABI size) and writes a full copy
// (range 1 for the older size) to *full when full is not NULL.
aca_status check_params(const aca_params *p, uint64_t *n_out, aca_params *full);
// Fills the flip table for z neighbours (2 dim, or the q-th degree
// neighbourhood's size - 1); returns its 2 (z + 1) entries (thr NULL: only
// counts them).
int build_thresholds(const aca_params *p, uint64_t *thr);
// Cells at lattice distance 1..q (the q-th degree neighbourhood without c).
int ball_size(int dim, int q);

struct Plan {
    aca::VisitArgs a;
    int block;
    size_t lds;
    bool fast;      // no direction spanned: the pitched-box kernel
};

void auto_tuning(const aca_params &p, aca_tuning *t);
// The library's candidate schedules for the autotuner (at most ACA_TUNE_MAX).
int tune_candidates(int dim, aca_tuning *out);
uint64_t launch_region_bytes(int dim, const aca::VisitArgs &a);

}  // namespace aca_host

struct aca_lattice {
    aca_params p;
    uint64_t n;
    int8_t *s;                      // caller's state buffers
    double *t;
    uint32_t *cnt;
    unsigned long long *key[2];     // working snapshots in scratch
    unsigned long long *time[2];
    unsigned long long *counters;   // device, in scratch
    uint8_t *dead;                  // device, per-tile flags, in scratch
    bool initialized;
    double last_T;
    aca_tuning tun;                 // as requested (0 / -1 = automatic)
    aca_stats stats;
    uint64_t thr[2 * (aca::kMaxSlots + 1)];
    int device;
    hipEvent_t ev_start[2], ev_stop[2];
    unsigned long long *host_ctr;   // pinned, mapped, kCounterWords words
    unsigned long long *host_ctr_dev;   // its device address
    bool attached;                  // member of a batch: advanced by it only
    double lag;                     // lag bound (0: none)
    std::vector<aca_launch_record> trace;   // launches of the last advance
    // Allocation-free advance (aca_advance_static): no pinned host words, no
    // HIP events and no trace.  The last block of a launch publishes its
    // counters to `publish` (device, 2 slots of kSlotWords words) and the
    // host copies them back after each launch.
    bool noalloc = false;
    unsigned long long *publish = nullptr;
    bool count_efficiency = false;  // collect the Section 4 counters (aca_set_counting)
};

namespace aca_host {
aca_status make_plan(const aca_lattice *lat, double T, Plan *plan);
}

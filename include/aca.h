/*
 * aca.h -- C-ABI of libaca: conservative simulation of Poisson-asynchronous
 * Ising arrays on AMD Instinct MI355X (gfx950).
 *
 * Method: B. D. Lubachevsky, "Efficient Parallel Simulations of Asynchronous
 * Cellular Arrays".  Each cell of a periodic 1-, 2- or 3-D lattice has its own
 * rate-lambda Poisson arrival stream (Section 1).  At an arrival the cell's spin
 * is reversed with a probability fixed by the spin and the sum of its
 * neighbours' spins just before the arrival (Section 2, Eq. (1)-(2); Glauber
 * form of the appendix program, or Metropolis).  Draws are deterministic
 * functions of (seed, cell, arrival number) (Section 3, Eq. (3)-(5)), so the
 * trajectory is unique (argument after Fig. 3.1) and the library reproduces,
 * bit for bit, the serial simulation that applies arrivals in increasing
 * (time, cell index) order.  The GPU schedule is the conservative one of
 * Fig. 3.1/3.2 inside workgroup tiles, aggregated as in Fig. 3.3/3.4.
 *
 * Conventions for every call:
 *  - Plain C types only.  Device pointers are HIP device addresses on the
 *    current device; host pointers are ordinary host memory.
 *  - A stream argument is a hipStream_t passed as void*; NULL is the null
 *    stream.  The library never creates streams.
 *  - Every call returns an aca_status; on failure aca_last_error() returns a
 *    message for the calling thread and nothing has been changed (EINVAL) or
 *    the lattice must be re-initialised (EDEVICE, ENOPROGRESS).
 *  - The library allocates no device memory: the caller owns the state
 *    buffers and the scratch buffer and frees them after aca_destroy().
 */
#ifndef ACA_H
#define ACA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ACA_ABI_VERSION 3u

typedef int32_t aca_status;
enum {
    ACA_OK = 0,
    ACA_EINVAL = -1,       /* bad argument; nothing changed */
    ACA_ENOMEM = -2,       /* scratch buffer too small */
    ACA_EDEVICE = -3,      /* a HIP call failed; message carries HIP's text */
    ACA_ESTATE = -4,       /* call out of order (e.g. advance before init) */
    ACA_ENOPROGRESS = -5   /* a launch applied no arrival while some were due */
};

enum { ACA_GLAUBER = 0, ACA_METROPOLIS = 1 };
enum { ACA_INIT_RANDOM = 0, ACA_INIT_PLUS = 1, ACA_INIT_MINUS = 2 };

/* Lattice description (Section 2 model, Ising rule of Section 1).
 * struct_size must be sizeof(aca_params).
 *  dim     1, 2 or 3
 *  L[d]    periodic side along d, >= 2 for d < dim (ignored beyond dim);
 *          the product N must be < 2^32.  Cell index x + L0 (y + L1 z).
 *  J, h    coupling and field: H = -J sum_<ij> s_i s_j - h sum_i s_i (finite)
 *  beta    inverse temperature, finite and >= 0
 *  rate    arrival rate lambda per cell, finite and > 0 (Eq. (5))
 *  rule    ACA_GLAUBER: flip with 1/(1+exp(beta dE));
 *          ACA_METROPOLIS: flip with min(1, exp(-beta dE))
 *  init    initial spins: iid +/-1 from the seed, all +1, or all -1
 *  seed    64-bit key of the Philox4x32-10 draws
 *  range   q >= 1: the rule reads the spins of every cell within lattice
 *          distance q (the q-th degree neighbourhood of Section 3, built by
 *          applying the nearest-neighbour map q times; z = its size - 1
 *          replaces 2 dim, e.g. z = 2q(q+1) in 2D).  q > 1 needs every side
 *          > 2q and q <= 4, 3, 2 in 1, 2, 3 D, and runs on the
 *          single-lattice path only (not in batches or the server).
 *          Structures of the size without this field (ABI 1) mean q = 1. */
typedef struct aca_params {
    uint32_t struct_size;
    int32_t dim;
    int32_t L[3];
    double J, h, beta, rate;
    int32_t rule, init;
    uint64_t seed;
    int32_t range;
    int32_t pad_;
} aca_params;

/* Size of aca_params before the range field (still accepted: range 1). */
#define ACA_PARAMS_SIZE_V1 72u

/* Schedule knobs; they never change results (partition invariance argued
 * for Fig. 3.4), only speed.  struct_size must be sizeof(aca_tuning).
 * Automatic values depend on the dimension and, for a single lattice too
 * small to give the device many default regions, on its size (smaller tiles,
 * wider ghosts, more rounds); batch and server members take the defaults of
 * their dimension.
 *  tile[d]    own cells of a workgroup tile along d (0 = automatic)
 *  ghost[d]   extra cells simulated on each side and discarded (-1 = auto)
 *  max_sweeps worklist rounds of a tile per visit (0 = automatic; larger
 *             values than 255 run as 255)
 *  block      threads per workgroup, multiple of 64 up to 1024 (0 = auto) */
typedef struct aca_tuning {
    uint32_t struct_size;
    int32_t tile[3];
    int32_t ghost[3];
    int32_t max_sweeps;
    int32_t block;
} aca_tuning;

/* Counters accumulated since aca_init (or aca_resume). */
typedef struct aca_stats {
    uint32_t struct_size;
    uint32_t pad_;
    uint64_t launches;      /* visit-kernel launches */
    uint64_t visits;        /* workgroup tile visits */
    uint64_t sweeps;        /* worklist rounds summed over tile visits */
    uint64_t events;        /* arrivals applied (spin-updates), exact */
    uint64_t flips;         /* of which reversed the spin, exact */
    uint64_t ghost_events;  /* arrivals applied to ghost copies in their
                               region (redundant work; some are merged) */
    uint64_t cell_checks;   /* enabling tests evaluated (scan + re-tests) */
    double last_T;          /* horizon reached so far */
    double device_ms;       /* time spent inside aca_advance (wall, ms) */
    double kernel_ms;       /* visit-kernel time, HIP events on the stream (ms) */
    uint64_t region_bytes;  /* bytes the visit kernels must move: 16 B per
                               region cell in, 16 B per owned cell out,
                               summed over launches */
    /* Efficiency instruments after Section 4, whose efficiency at an
     * iteration of Fig. 3.2 is N0 / N, the fraction of cells passing the
     * enabling test (Step 2).  Summed over tile visits:
     *  scan_enabled / scan_live: of the owned cells with an arrival before
     *    the horizon when a visit loaded them, the fraction the visit's
     *    initial scan found enabled (at the first launch from a fresh state
     *    this is exactly the first iteration of Fig. 3.2);
     *  (events + ghost_events) / round_cells: arrivals applied per simulated
     *    cell per worklist round -- each round applies exactly the cells that
     *    pass the test, so this is N0 / N of Fig. 3.2 inside the regions.
     * The tile visits of the nearest-neighbour rule without output frames
     * collect these three only while aca_set_counting is on (they cost those
     * visits a few per cent); the other visits (lattices a tile spans, output
     * frames, q-th degree neighbourhoods) always collect them.  Batch and
     * server members never do. */
    uint64_t scan_live;
    uint64_t scan_enabled;
    uint64_t round_cells;   /* simulated cells before the launch's horizon at
                               load, times the rounds the visit ran */
} aca_stats;

/* One record per visit launch of the last aca_advance (see aca_get_trace). */
typedef struct aca_launch_record {
    uint64_t events;        /* arrivals applied to owned cells */
    uint64_t ghost_events;  /* arrivals applied to ghost copies */
    uint64_t scan_live;     /* as in aca_stats, for this launch */
    uint64_t scan_enabled;
    uint64_t round_cells;
    uint64_t live_tiles;    /* tiles with an owned arrival still due afterwards */
    double kernel_ms;       /* HIP-event time of the launch */
} aca_launch_record;

typedef struct aca_lattice aca_lattice;   /* opaque host handle */

uint32_t aca_abi_version(void);
const char *aca_last_error(void);

/* Flip thresholds of parameters p, without a lattice handle.  Section 2,
 * Eq. (1): the new state is drawn from a distribution fixed by the cell's
 * state and its neighbours'; for the Ising rule this is the probability
 * table of the appendix program (Glauber x/(1+x), x = exp(-beta dE)) or the
 * Metropolis min(1, exp(-beta dE)), dE = 2 s (J sum + h).  Entry idx =
 * (sum + z)/2 + (z+1)(s+1)/2 -- the appendix's index generalised to z = 2 dim
 * neighbour slots (or the q-th degree neighbourhood's size - 1) -- holds
 * floor(p 2^32), or 2^32 when p >= 1; an arrival flips the spin iff its
 * 32-bit draw is below the entry.  Host only, needs no GPU.  out (host) must
 * hold cap >= 2(z+1) entries; *count (may be NULL) receives 2(z+1).
 * ACA_EINVAL for invalid p, a NULL out or a short cap; nothing is written
 * then. */
aca_status aca_thresholds(const aca_params *p, uint64_t *out, int32_t cap,
                          int32_t *count);

/* Sizes for p: number of cells, and bytes of device scratch the caller must
 * provide to aca_create (two working snapshots of 16 bytes per cell, a byte
 * per cell for per-tile flags, and counters: about 33 N + 512 bytes).
 * The array of cells and its neighbourhood map are those of Section 2 (a
 * periodic box, neighbours one step along each axis).  ACA_EINVAL for
 * invalid p; either output pointer may be NULL. */
aca_status aca_query(const aca_params *p, uint64_t *n_cells,
                     uint64_t *scratch_bytes);

/* Create a handle over caller-owned device buffers: spins int8[N], times
 * double[N], counts uint32[N] (structure of arrays, index as above), all
 * 256-byte aligned, and scratch of scratch_bytes >= aca_query's value.
 * These are the per-cell state s(c), local time t(c) and arrival count n(c)
 * of Fig. 3.1 (Section 3; the count numbers the draws of Eq. (5)).  The
 * handle owns none of them.  No device work is done.  The scratch buffer is
 * an addition to the paper's state: it holds the two working snapshots the
 * launches alternate between.  ACA_EINVAL for invalid p, NULL or misaligned
 * buffers; ACA_ENOMEM when scratch_bytes is short; *out is then untouched. */
aca_status aca_create(const aca_params *p, int8_t *d_spin, double *d_time,
                      uint32_t *d_count, void *d_scratch, uint64_t scratch_bytes,
                      aca_lattice **out);

/* Replace the schedule knobs (NULL restores the automatic choice). */
aca_status aca_set_tuning(aca_lattice *lat, const aca_tuning *t);
aca_status aca_get_tuning(const aca_lattice *lat, aca_tuning *out);

/* Initial state (asynchronous on `stream`): each cell's first arrival is one
 * exponential gap after time 0 (the Poisson stream of Section 1 starts at
 * time 0; the gap is Eq. (5)'s -ln r / lambda with the cell's initial draw),
 * its spin set per `init`, its count 0.  ACA_ESTATE for a batch member,
 * ACA_EDEVICE if the launch fails. */
aca_status aca_init(aca_lattice *lat, void *stream);

/* Declare that the state buffers already hold a state advanced to horizon
 * T_done (e.g. restored from a checkpoint); resets the statistics.  Every
 * count n(c) must be below 2^31: the call waits for the device (the caller's
 * writes to the buffers may be on any stream), checks the counts there and
 * returns ACA_EINVAL, leaving the lattice as it was, if one is not. */
aca_status aca_resume(aca_lattice *lat, double T_done);

/* Apply every arrival with time < T, in the conservative parallel schedule:
 * the loop of Fig. 3.1 run until every local time reaches end_time = T, a
 * cell applying its arrival once no neighbour's pending arrival precedes it
 * (ties by cell index), its new state drawn per Eq. (1)-(2) and its next
 * arrival set by Eq. (5); aggregated into workgroup tiles as in Fig. 3.3/3.4.
 * Returns when done (the state is in the caller's buffers and the stream is
 * synchronised).  T must be finite and >= the last horizon (equal: no-op),
 * and rate * T <= 2^30 (ACA_EINVAL otherwise: counts are kept below 2^31;
 * the same bound applies to aca_batch_attach and aca_server_submit).
 * Afterwards t(c) is the first arrival at or after T and n(c) counts the
 * arrivals applied since time 0. */
aca_status aca_advance(aca_lattice *lat, double T, void *stream);

/* aca_advance that also writes output frames (Fig. 3.7): for every k in
 * [k_first, k_first + nframes) whose time k dt lies in (last horizon, T],
 * frame k - k_first of d_frames (int8[N] per frame, consecutive, cell order)
 * receives the spins at time k dt, i.e. after every arrival before k dt.
 * Frames outside that interval are left untouched.  Each cell writes its own
 * frames as its arrivals are applied, with no global synchronisation: a
 * frame is complete when the advance returns. */
aca_status aca_advance_frames(aca_lattice *lat, double T, double dt, int8_t *d_frames,
                              int64_t k_first, int64_t nframes, void *stream);

/* Bound the lag between local times (the restriction a finite frame buffer
 * imposes, Section 4): each launch applies only arrivals before
 * min(T, t_min + lag), t_min the least pending time of the lattice when the
 * previous launch loaded it (0 = no bound).  A schedule knob: results do not
 * change, only the parallelism per launch. */
aca_status aca_set_lag(aca_lattice *lat, double lag);

/* Whether the lattice's advances collect the efficiency counters of
 * aca_stats (scan_live, scan_enabled, round_cells) on every path: on != 0
 * turns them on (default off; results are the same either way).  ACA_ESTATE
 * for a batch member. */
aca_status aca_set_counting(aca_lattice *lat, int32_t on);

/* Counters since aca_init (or aca_resume); see aca_stats. */
aca_status aca_get_stats(const aca_lattice *lat, aca_stats *out);

/* The flip thresholds the lattice applies (as aca_thresholds for its
 * parameters; Section 2, Eq. (1), and the appendix's probability table).
 * out (host) must hold n >= 2(z+1) entries; ACA_EINVAL otherwise. */
aca_status aca_get_thresholds(const aca_lattice *lat, uint64_t *out, int32_t n);

/* Per-launch records of the last aca_advance (or aca_advance_frames), in
 * launch order: the efficiency of each iteration, in the sense of Section 4,
 * as the advance went.  Up to cap records are copied to out (host); *count
 * receives the number held (at most ACA_TRACE_MAX: the first launches of a
 * longer advance). */
#define ACA_TRACE_MAX 65536
aca_status aca_get_trace(const aca_lattice *lat, aca_launch_record *out, int32_t cap,
                         int32_t *count);

/* Autotuning on the caller's own work.  Every schedule yields the same
 * trajectory (Fig. 3.4's partition invariance), so the tuner advances the
 * real lattice: first a warm-up slice of dT/2 with the first candidate, then
 * two slices of dT/2 per candidate, the candidates in order and then in
 * reverse order (so that a steady change of the work along the trajectory
 * favours none), each timed on the device; it keeps the candidate with the
 * most arrivals per millisecond over its two slices, installs it with
 * aca_set_tuning and leaves the lattice advanced by (n + 1/2) dT.  cands NULL
 * (or n = 0) uses the library's candidate set for the lattice's dimension.
 * rates (may be NULL) receives arrivals per millisecond of each candidate
 * (n entries; with cands NULL, up to ACA_TUNE_MAX entries, *n_out their
 * number). */
#define ACA_TUNE_MAX 16
aca_status aca_tune(aca_lattice *lat, const aca_tuning *cands, int32_t n, double dT,
                    void *stream, int32_t *best, double *rates, int32_t *n_out);


/* Synchronous copy of the state -- the spins, local times and arrival
 * counts of Section 3's per-cell variables -- to host memory (any pointer may
 * be NULL; each must hold N elements).  ACA_ESTATE for a batch member. */
aca_status aca_read(aca_lattice *lat, int8_t *h_spin, double *h_time,
                    uint32_t *h_count, void *stream);

/* Release the handle (the caller's buffers are untouched). */
aca_status aca_destroy(aca_lattice *lat);

/* Allocation-free advance, for callers that cannot allocate memory (tight
 * serving loops, harnesses that forbid hipMalloc): the result of aca_create
 * + aca_init (or aca_resume(T_done)) + aca_advance(T) over the caller's state
 * buffers, without a handle, a scratch buffer, pinned host memory or HIP
 * events.  The working snapshots, tile flags and counters live in a fixed
 * device array of 64 MiB inside the library (one per device, held until the
 * process ends), so the lattice may have at most about 2.03 million cells
 * (33 B of scratch per cell); larger lattices get ACA_EINVAL before any device
 * work.  The call calls no allocating routine.
 *  p            lattice parameters (as aca_create)
 *  d_spin, d_time, d_count
 *               the caller's state buffers (device, 256-byte aligned, N
 *               elements each), ready on `stream`
 *  draw_initial nonzero: first draw the initial state (as aca_init; T_done
 *               must then be 0); zero: the buffers hold a state advanced to
 *               T_done (counts below 2^31, else ACA_EINVAL)
 *  T_done, T    advance from horizon T_done to T >= T_done (rate * T <= 2^30)
 * Synchronous: returns with the state at T in the buffers.  Every call on a
 * device shares that device's array (each call clears what must start at
 * zero), so calls that overlap on one device -- from two host threads, say --
 * race and must not be made.  Launches run one at a time, each followed by
 * a copy of its counters to the host. */
aca_status aca_advance_static(const aca_params *p, int8_t *d_spin, double *d_time,
                              uint32_t *d_count, int32_t draw_initial, double T_done,
                              double T, void *stream);

/* Device primitives exposed for element-by-element checks against the
 * oracle (asynchronous on `stream`; all pointers are device pointers).
 *  aca_philox:    out[4i..4i+3] = Philox4x32-10(ctr[4i..4i+3]) under key
 *                 (seed lo, seed hi)
 *  aca_neg_log:   out[i] = -ln u(w[i]), u = (2 (w >> 12) + 1) 2^-53, by the
 *                 fixed atanh-series recipe used for every arrival gap */
aca_status aca_philox(const uint32_t *d_ctr, uint64_t seed, uint32_t *d_out,
                      uint64_t count, void *stream);
aca_status aca_neg_log(const uint64_t *d_w, double *d_out, uint64_t count,
                       void *stream);


/* ------------------------------------------------------------------ batches
 *
 * A batch advances many independent lattices -- any mix of dimensions,
 * sizes, parameters and horizons -- in persistent launches that keep every
 * compute unit busy with (lattice, tile) items.  Each lattice advances in
 * epochs, one visit of each of its tiles per epoch, exactly as in the
 * launches of aca_advance; the epochs of different lattices overlap, and a
 * lattice's next epoch opens as soon as its last tile is done.  Every result
 * is bit-identical to aca_advance of that lattice alone (the trajectory is
 * unique, argument after Fig. 3.1; the aggregation is partition-invariant,
 * Fig. 3.4).  Member lattices are split into at least two tiles along every
 * direction.
 *
 * A batch is either driven whole (aca_batch_advance) or step by step for
 * continuous batching: aca_batch_attach adds a lattice between steps,
 * aca_batch_step runs one persistent launch for at most a time budget,
 * aca_batch_poll returns the lattices that reached their horizon (their
 * state is then in their own buffers and they are detached).  While
 * attached, a lattice's state lives in its scratch; aca_advance, aca_read,
 * aca_set_tuning, aca_init, aca_resume and aca_destroy on it return
 * ACA_ESTATE.  One batch is driven from one host thread.
 */
typedef struct aca_batch aca_batch;   /* opaque host handle */

/* Counters accumulated since aca_batch_create. */
typedef struct aca_batch_stats {
    uint32_t struct_size;
    uint32_t pad_;
    uint64_t steps;          /* persistent launches */
    uint64_t epochs;         /* lattice epochs completed */
    uint64_t visits;         /* tile visits (epochs times tiles) */
    uint64_t sweeps;         /* worklist rounds summed over tile visits */
    uint64_t events;         /* arrivals applied, exact, over finished lattices */
    uint64_t flips;          /* of which reversed the spin, exact */
    uint64_t ghost_events;   /* arrivals applied to ghost copies */
    uint64_t cell_checks;    /* enabling tests evaluated */
    uint64_t finished;       /* lattices that reached their horizon */
    double device_ms;        /* wall time inside aca_batch_step (ms) */
    double kernel_ms;        /* persistent visit-kernel time, HIP events (ms) */
    uint64_t region_bytes;   /* 16 B per region cell in and per owned cell out,
                                summed over completed epochs */
} aca_batch_stats;

/* Bytes of device work buffer for a batch of up to `capacity` lattices
 * (descriptors, device-resident member state, work lists). */
aca_status aca_batch_query(int32_t capacity, uint64_t *work_bytes);

/* Create a batch over a caller-owned, 256-byte aligned device buffer of
 * work_bytes >= aca_batch_query's value (on the current device; members
 * must live on it too).  The batch owns none of the caller's memory. */
aca_status aca_batch_create(int32_t capacity, void *d_work, uint64_t work_bytes,
                            aca_batch **out);

/* Tile shape, ghost width and worklist rounds per visit used for members of
 * dimension `dim` attached from now on (NULL: automatic).  Per direction the
 * lattice is cut into max(2, ceil(L / tile)) nearly equal tiles.  `block` is
 * ignored (the persistent kernel runs 512 threads per workgroup). */
aca_status aca_batch_set_tuning(aca_batch *b, int32_t dim, const aca_tuning *t);
aca_status aca_batch_get_tuning(const aca_batch *b, int32_t dim, aca_tuning *out);

/* Order in which workgroups take open items of the members: ACA_ORDER_WORK
 * (default) serves the member with the most remaining arrivals first, which
 * shortens the whole batch; ACA_ORDER_ARRIVAL serves members in the order
 * they were attached, which bounds each member's wait (job serving). */
enum { ACA_ORDER_WORK = 0, ACA_ORDER_ARRIVAL = 1 };
aca_status aca_batch_set_order(aca_batch *b, int32_t order);

/* Add an initialised lattice that is not a member of any batch, to be
 * advanced to horizon T (finite, >= its last horizon).  It joins at the next
 * step.  ACA_ENOMEM when the batch is full. */
aca_status aca_batch_attach(aca_batch *b, aca_lattice *lat, double T);

/* One persistent launch over the members: new members are packed; every
 * member runs epochs until it reaches its horizon, or, once `budget_ms` of
 * device time has passed (<= 0: no limit) or it has completed `max_epochs`
 * epochs in this launch (<= 0: no limit), pauses at its next epoch boundary
 * and resumes at the next step.  Members that reached their horizon are
 * unpacked into their buffers and queued for aca_batch_poll.  Synchronous.
 * *n_members (may be NULL) receives the number of members still attached.
 * ACA_ENOPROGRESS if a member's epoch applied no arrival while arrivals were
 * due; that member is detached with its buffers as they were at attach. */
aca_status aca_batch_step(aca_batch *b, double budget_ms, int32_t max_epochs,
                          void *stream, int32_t *n_members);

/* Pop up to cap lattices that reached their horizon, in completion order. */
aca_status aca_batch_poll(aca_batch *b, aca_lattice **done, int32_t cap,
                          int32_t *n_done);

/* Advance lats[i] to T[i] for i < count in one batch (which must have no
 * members), stepping until all are done; returns with every state in its
 * buffers and the finished queue empty. */
aca_status aca_batch_advance(aca_batch *b, aca_lattice *const *lats, const double *T,
                             int32_t count, void *stream);


/* Batch autotuning for the members of dimension dim (as aca_tune): the batch
 * must be empty; lats[i] (initialised, horizons T[i]) are advanced slice by
 * slice, each slice a fraction frac/2 of every lattice's span to T[i] at the
 * start: a warm-up slice, then two slices per candidate, the candidates in
 * order and then in reverse order ((n + 1/2) frac must not exceed 1; frac in
 * (0, 0.5)); the candidate with the most arrivals per millisecond of device
 * time over its two slices becomes the batch's tuning for dim.  Lattices of
 * other dimensions advance too.  The lattices are left detached, short of
 * their horizons. */
aca_status aca_batch_tune(aca_batch *b, aca_lattice *const *lats, const double *T,
                          int32_t count, int32_t dim, const aca_tuning *cands, int32_t n,
                          double frac, void *stream, int32_t *best, double *rates,
                          int32_t *n_out);

/* The current members, up to cap of them, in slot order (*n_members gets
 * their total number). */
aca_status aca_batch_members(const aca_batch *b, aca_lattice **out, int32_t cap,
                             int32_t *n_members);

aca_status aca_batch_get_stats(const aca_batch *b, aca_batch_stats *out);

/* Release the handle; ACA_ESTATE while it has members. */
aca_status aca_batch_destroy(aca_batch *b);

/* ------------------------------------------------------------------ serving
 *
 * A server runs simulation jobs that arrive over time (continuous batching):
 * aca_server_submit queues a job; every aca_server_step first admits queued
 * jobs in arrival order while a batch slot and room in the device arena are
 * free (the job's state buffers and scratch are carved from the arena and
 * its initial state is drawn on the device), then runs one batch step with a
 * device-time budget, so jobs that arrive while others run join at the next
 * step and share the GPU with them.  A finished job's state stays in the
 * arena until aca_server_release.  Results are bit-identical to running the
 * job alone with aca_init + aca_advance.  One server is driven from one host
 * thread.
 */
typedef struct aca_server aca_server;   /* opaque host handle */

enum { ACA_JOB_QUEUED = 0, ACA_JOB_RUNNING = 1, ACA_JOB_DONE = 2, ACA_JOB_FAILED = 3 };

typedef struct aca_server_stats {
    uint32_t struct_size;
    uint32_t pad_;
    uint64_t submitted;      /* jobs accepted by aca_server_submit */
    uint64_t admitted;       /* jobs given arena memory and a batch slot */
    uint64_t finished;       /* jobs that reached their horizon */
    uint64_t failed;         /* jobs that ended with an error */
    uint64_t steps;          /* aca_server_step calls that ran the batch */
    uint64_t events;         /* arrivals applied, exact, over finished jobs */
    uint64_t arena_bytes;    /* size of the arena */
    uint64_t arena_peak;     /* most arena bytes in use at once */
    uint64_t queued_peak;    /* most jobs waiting for admission at once */
    double device_ms;        /* wall time inside aca_server_step (ms) */
    double kernel_ms;        /* persistent visit-kernel time (ms) */
} aca_server_stats;

/* Device bytes of the server's work buffer for up to max_jobs jobs at once. */
aca_status aca_server_query(int32_t max_jobs, uint64_t *work_bytes);

/* Arena bytes one job with parameters p occupies while admitted: its state
 * buffers (13 bytes per cell) and scratch, each 256-byte aligned. */
aca_status aca_server_job_bytes(const aca_params *p, uint64_t *bytes);

/* Create a server over two caller-owned, 256-byte aligned device buffers: the
 * arena that admitted jobs are carved from (its size is the HBM budget) and a
 * work buffer of work_bytes >= aca_server_query(max_jobs). */
aca_status aca_server_create(void *d_arena, uint64_t arena_bytes, void *d_work,
                             uint64_t work_bytes, int32_t max_jobs, aca_server **out);

/* Per-dimension schedule knobs for jobs admitted from now on (as
 * aca_batch_set_tuning). */
aca_status aca_server_set_tuning(aca_server *srv, int32_t dim, const aca_tuning *t);

/* Priority among running jobs (ACA_ORDER_*; the server starts with
 * ACA_ORDER_ARRIVAL). */
aca_status aca_server_set_order(aca_server *srv, int32_t order);

/* Queue a job: lattice p from its initial state to horizon T (finite, > 0).
 * *job receives its id (ids count up from 0).  ACA_ENOMEM if the job alone
 * exceeds the arena. */
aca_status aca_server_submit(aca_server *srv, const aca_params *p, double T, uint64_t *job);

/* Admit what fits, then one batch step of at most budget_ms of device time
 * (<= 0: until every running job is done).  Writes the ids of jobs that
 * finished during this call to done[0..cap) (*n_done receives how many
 * finished; ids beyond cap are still marked done).  Synchronous.  A job whose
 * batch step failed is marked ACA_JOB_FAILED and its memory released; the
 * call then returns that error after finishing the step for the others. */
aca_status aca_server_step(aca_server *srv, double budget_ms, void *stream, uint64_t *done,
                           int32_t cap, int32_t *n_done);

/* State of a job (ACA_JOB_*), and for finished jobs its statistics. */
aca_status aca_server_job(const aca_server *srv, uint64_t job, int32_t *state,
                          aca_stats *stats);

/* Synchronous copy of a finished job's spins, times and counts to host memory
 * (any pointer may be NULL).  ACA_ESTATE unless the job is done. */
aca_status aca_server_read(aca_server *srv, uint64_t job, int8_t *h_spin, double *h_time,
                           uint32_t *h_count, void *stream);

/* Return a finished or failed job's arena memory and forget the job. */
aca_status aca_server_release(aca_server *srv, uint64_t job);

/* Jobs waiting for admission and jobs running. */
aca_status aca_server_load(const aca_server *srv, int32_t *queued, int32_t *running);

aca_status aca_server_get_stats(const aca_server *srv, aca_server_stats *out);

/* Release the handle; ACA_ESTATE while jobs are queued or running (finished
 * jobs not yet released are dropped). */
aca_status aca_server_destroy(aca_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* ACA_H */

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

#define ACA_ABI_VERSION 1u

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
 *  seed    64-bit key of the Philox4x32-10 draws */
typedef struct aca_params {
    uint32_t struct_size;
    int32_t dim;
    int32_t L[3];
    double J, h, beta, rate;
    int32_t rule, init;
    uint64_t seed;
} aca_params;

/* Schedule knobs; they never change results (partition invariance argued
 * for Fig. 3.4), only speed.  struct_size must be sizeof(aca_tuning).
 *  tile[d]    own cells of a workgroup tile along d (0 = automatic)
 *  ghost[d]   extra cells simulated on each side and discarded (-1 = auto)
 *  max_sweeps worklist rounds of a tile per visit (0 = automatic)
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
} aca_stats;

typedef struct aca_lattice aca_lattice;   /* opaque host handle */

uint32_t aca_abi_version(void);
const char *aca_last_error(void);

/* Flip thresholds thr[idx] = floor(p * 2^32) (2^32 when p >= 1), idx =
 * (sum + z)/2 + (z+1)(s+1)/2 with z = 2 dim neighbour slots, for the
 * probability table of the appendix program.  Host only, needs no GPU.
 * out must hold cap >= 2(z+1) entries; *count receives 2(z+1). */
aca_status aca_thresholds(const aca_params *p, uint64_t *out, int32_t cap,
                          int32_t *count);

/* Sizes for p: number of cells, and bytes of device scratch the caller must
 * provide to aca_create (two working snapshots of 16 bytes per cell plus
 * counters; 32 N + 256 bytes). */
aca_status aca_query(const aca_params *p, uint64_t *n_cells,
                     uint64_t *scratch_bytes);

/* Create a handle over caller-owned device buffers: spins int8[N], times
 * double[N], counts uint32[N] (structure of arrays, index as above), all
 * 256-byte aligned, and scratch of scratch_bytes >= aca_query's value.
 * The handle owns none of them.  No device work is done. */
aca_status aca_create(const aca_params *p, int8_t *d_spin, double *d_time,
                      uint32_t *d_count, void *d_scratch, uint64_t scratch_bytes,
                      aca_lattice **out);

/* Replace the schedule knobs (NULL restores the automatic choice). */
aca_status aca_set_tuning(aca_lattice *lat, const aca_tuning *t);
aca_status aca_get_tuning(const aca_lattice *lat, aca_tuning *out);

/* Initial state (asynchronous on `stream`): each cell's first arrival is one
 * exponential gap after time 0, its spin set per `init`, its count 0. */
aca_status aca_init(aca_lattice *lat, void *stream);

/* Declare that the state buffers already hold a state advanced to horizon
 * T_done (e.g. restored from a checkpoint); resets the statistics. */
aca_status aca_resume(aca_lattice *lat, double T_done);

/* Apply every arrival with time < T, in the conservative parallel schedule.
 * Returns when done (the state is in the caller's buffers and the stream is
 * synchronised).  T must be finite and >= the last horizon (equal: no-op).
 * Afterwards t(c) is the first arrival at or after T and n(c) counts the
 * arrivals applied since time 0. */
aca_status aca_advance(aca_lattice *lat, double T, void *stream);

aca_status aca_get_stats(const aca_lattice *lat, aca_stats *out);

/* Synchronous copy of the state to host memory (any pointer may be NULL). */
aca_status aca_read(aca_lattice *lat, int8_t *h_spin, double *h_time,
                    uint32_t *h_count, void *stream);

/* Release the handle (the caller's buffers are untouched). */
aca_status aca_destroy(aca_lattice *lat);

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

#ifdef __cplusplus
}
#endif

#endif /* ACA_H */

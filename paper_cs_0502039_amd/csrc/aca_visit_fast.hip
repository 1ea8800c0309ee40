// aca_visit_fast.hip -- one launch visits every tile of one lattice once.
//
// Used for tiles that span no lattice direction (the region visit itself is
// in aca_region.h).  Block b visits tile b; the last block to finish
// publishes the launch's counters to pinned host memory.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aca_internal.h"
#include "aca_region.h"

namespace aca {
namespace {

// UNIT: the lattice's rate is 1 (no division in the gap); COUNT: collect the
// efficiency counters.  The nearest-neighbour visit without frames comes in
// all four combinations, each a kernel of its own so that none carries
// another's registers; the other visits always count and divide by the rate.
// CP0..CP2: compile-time box pitches (0: from the plan), for the default
// tiles of the large lattices.
template <int DIM, bool FRAMES, int Q, bool UNIT = false, bool COUNT = true, int CP0 = 0,
          int CP1 = 0, int CP2 = 0>
__global__ void __launch_bounds__(1024) visit_fast_kernel(VisitArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const unsigned int ntiles_total = (unsigned)a.ntiles[0] * (unsigned)a.ntiles[1] *
                                      (unsigned)a.ntiles[2];
    const region::Snapshots io{a.key_in, a.time_in, a.key_out, a.time_out};
    const region::RegionTally r =
        region::visit_region<DIM, FRAMES, Q, UNIT, COUNT, CP0, CP1, CP2>(a, io, blockIdx.x, lds);
    if (threadIdx.x == 0) {
        if (!r.skipped) {
            unsigned long long *gc = a.counters;
            atomicAdd(&gc[kEvents], (unsigned long long)r.events);
            atomicAdd(&gc[kFlips], (unsigned long long)r.flips);
            atomicAdd(&gc[kGhostEvents], (unsigned long long)r.ghost);
            atomicAdd(&gc[kChecks], (unsigned long long)r.checks);
            atomicAdd(&gc[kSweeps], (unsigned long long)r.rounds);
            if (COUNT) {
                atomicAdd(&gc[kScanLive], (unsigned long long)r.scan_live);
                atomicAdd(&gc[kScanEnabled], (unsigned long long)r.scan_enabled);
                atomicAdd(&gc[kRoundCells], (unsigned long long)r.round_cells);
            }
            if (r.any_live) atomicAdd(&gc[kLiveTiles], 1ull);
            // owned cells that were all at or past the horizon when loaded can
            // never change again: both snapshots now hold them
            if (!r.own_due) a.dead[blockIdx.x] = 1;
        }
        finish_visit_block(a, ntiles_total);
    }
}

// Every (dimension, frames, reach) instantiation: reach 1..4 in 1D, 1..3 in
// 2D, 1..2 in 3D; plus the unit-rate nearest-neighbour visits without frames.
template <int DIM, bool FRAMES, int Q>
const void *fast_fn()
{
    return (const void *)visit_fast_kernel<DIM, FRAMES, Q>;
}

template <bool UNIT, bool COUNT, bool FRAMES = false>
const void *near_fn(int dim)
{
    switch (dim) {
    case 1: return (const void *)visit_fast_kernel<1, FRAMES, 1, UNIT, COUNT>;
    case 2: return (const void *)visit_fast_kernel<2, FRAMES, 1, UNIT, COUNT>;
    case 3: return (const void *)visit_fast_kernel<3, FRAMES, 1, UNIT, COUNT>;
    default: return nullptr;
    }
}

// The nearest-neighbour visit that writes output frames: unit-rate and
// uncounted instantiations too (the frame capture adds registers of its own).
const void *near_frames_kernel(int dim, bool unit, bool count)
{
    if (count) return unit ? near_fn<true, true, true>(dim) : near_fn<false, true, true>(dim);
    return unit ? near_fn<true, false, true>(dim) : near_fn<false, false, true>(dim);
}

// Box pitches compiled as constants (own tile + 2 ghost + 2 ring cells a
// side).  2D: 84 x 66 (the default 72 x 54 tile with 5 ghost cells), 76 x 72
// (64 x 60 with 5) and 76 x 64 (64 x 52 with 5); 3D: 24 x 24 x 20 (the
// default 20 x 20 x 16 tile with 1, or 18 x 18 x 14 with 2) and 24 x 24 x 18
// (20 x 20 x 14 with 1).
template <int P0, int P1, int P2>
struct CompiledPitch {
    static constexpr int dim = P2 > 1 ? 3 : 2;
    static bool matches(const int *pitch)
    {
        return pitch[0] == P0 && pitch[1] == P1 && pitch[2] == (P2 > 1 ? P2 : 1);
    }
    static const void *kernel(bool unit)
    {
        return unit ? (const void *)visit_fast_kernel<dim, false, 1, true, false, P0, P1, P2>
                    : (const void *)visit_fast_kernel<dim, false, 1, false, false, P0, P1, P2>;
    }
};
using Pitch2a = CompiledPitch<72 + 2 * 5 + 2, 54 + 2 * 5 + 2, 0>;
using Pitch2b = CompiledPitch<64 + 2 * 5 + 2, 60 + 2 * 5 + 2, 0>;
using Pitch2c = CompiledPitch<64 + 2 * 5 + 2, 52 + 2 * 5 + 2, 0>;
using Pitch3a = CompiledPitch<20 + 2 * 1 + 2, 20 + 2 * 1 + 2, 16 + 2 * 1 + 2>;
using Pitch3b = CompiledPitch<20 + 2 * 1 + 2, 20 + 2 * 1 + 2, 14 + 2 * 1 + 2>;

// The uncounted nearest-neighbour visit compiled for `pitch`, or NULL.
const void *compiled_pitch_kernel(int dim, bool unit, const int *pitch)
{
    if (!pitch) return nullptr;
    if (dim == 2) {
        if (Pitch2a::matches(pitch)) return Pitch2a::kernel(unit);
        if (Pitch2b::matches(pitch)) return Pitch2b::kernel(unit);
        if (Pitch2c::matches(pitch)) return Pitch2c::kernel(unit);
    } else if (dim == 3) {
        if (Pitch3a::matches(pitch)) return Pitch3a::kernel(unit);
        if (Pitch3b::matches(pitch)) return Pitch3b::kernel(unit);
    }
    return nullptr;
}

// The nearest-neighbour visit without frames, by rate and counting; the
// uncounted visit of a plan with a compiled pitch takes that instantiation.
const void *near_fast_kernel(int dim, bool unit, bool count, const int *pitch = nullptr)
{
    if (!count) {
        const void *f = compiled_pitch_kernel(dim, unit, pitch);
        if (f) return f;
    }
    if (unit) return count ? near_fn<true, true>(dim) : near_fn<true, false>(dim);
    return count ? near_fn<false, true>(dim) : near_fn<false, false>(dim);
}

template <bool FRAMES>
const void *fast_fn_for(int dim, int q)
{
    if (dim == 1) {
        switch (q) {
        case 1: return fast_fn<1, FRAMES, 1>();
        case 2: return fast_fn<1, FRAMES, 2>();
        case 3: return fast_fn<1, FRAMES, 3>();
        case 4: return fast_fn<1, FRAMES, 4>();
        default: return nullptr;
        }
    }
    if (dim == 2) {
        switch (q) {
        case 1: return fast_fn<2, FRAMES, 1>();
        case 2: return fast_fn<2, FRAMES, 2>();
        case 3: return fast_fn<2, FRAMES, 3>();
        default: return nullptr;
        }
    }
    switch (q) {
    case 1: return fast_fn<3, FRAMES, 1>();
    case 2: return fast_fn<3, FRAMES, 2>();
    default: return nullptr;
    }
}

const void *fast_kernel(int dim, int q, bool frames)
{
    return frames ? fast_fn_for<true>(dim, q) : fast_fn_for<false>(dim, q);
}

}  // namespace

size_t visit_fast_lds_bytes(int dim, const VisitArgs &a) { return region::fast_plan(a, dim).total; }

int visit_fast_box(int dim, const VisitArgs &a)
{
    const int ring = a.range > 1 ? a.range : 1;
    int box = 1;
    for (int d = 0; d < dim; ++d) box *= a.tile[d] + 2 * a.ghost[d] + 2 * ring;
    return box;
}

bool visit_fast_supports(int dim, int q) { return fast_kernel(dim, q, false) != nullptr; }

hipError_t launch_visit_fast(int dim, const VisitArgs &a, int block, size_t lds,
                             hipStream_t stream)
{
    const unsigned tiles = (unsigned)a.ntiles[0] * (unsigned)a.ntiles[1] *
                           (unsigned)a.ntiles[2];
    const int q = a.range > 1 ? a.range : 1;
    int pitch[3];
    region::box_pitch(a, dim, pitch);
    const void *fn = (q == 1 && !a.frames)
                         ? near_fast_kernel(dim, a.unit_rate != 0, a.count_efficiency != 0, pitch)
                         : (q == 1 ? near_frames_kernel(dim, a.unit_rate != 0,
                                                        a.count_efficiency != 0)
                                   : fast_kernel(dim, q, a.frames != nullptr));
    if (!fn) return hipErrorInvalidValue;
    void *args[] = {const_cast<VisitArgs *>(&a)};
    return hipLaunchKernel(fn, dim3(tiles), dim3(block), args, lds, stream);
}

hipError_t set_visit_fast_lds_limit(size_t bytes)
{
    for (int dim = 1; dim <= 3; ++dim)
        for (int q = 1; q <= 4; ++q)
            for (int fr = 0; fr < 2; ++fr) {
                const void *f = fast_kernel(dim, q, fr != 0);
                if (!f) continue;
                const hipError_t e =
                    hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
                if (e != hipSuccess) return e;
            }
    for (int dim = 1; dim <= 3; ++dim)
        for (int v = 0; v < 4; ++v) {
            const hipError_t e = hipFuncSetAttribute(near_frames_kernel(dim, v & 1, v & 2),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)bytes);
            if (e != hipSuccess) return e;
        }
    for (int dim = 1; dim <= 3; ++dim)
        for (int v = 0; v < 4; ++v) {
            const hipError_t e = hipFuncSetAttribute(near_fast_kernel(dim, v & 1, v & 2),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)bytes);
            if (e != hipSuccess) return e;
        }
    const void *compiled[] = {Pitch2a::kernel(false), Pitch2a::kernel(true),
                              Pitch2b::kernel(false), Pitch2b::kernel(true),
                              Pitch2c::kernel(false), Pitch2c::kernel(true),
                              Pitch3a::kernel(false), Pitch3a::kernel(true),
                              Pitch3b::kernel(false), Pitch3b::kernel(true)};
    for (const void *f : compiled) {
        const hipError_t e =
            hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace aca

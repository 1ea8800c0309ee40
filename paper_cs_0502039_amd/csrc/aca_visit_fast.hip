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

template <int DIM, bool FRAMES>
__global__ void __launch_bounds__(1024) visit_fast_kernel(VisitArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const unsigned int ntiles_total = (unsigned)a.ntiles[0] * (unsigned)a.ntiles[1] *
                                      (unsigned)a.ntiles[2];
    const region::Snapshots io{a.key_in, a.time_in, a.key_out, a.time_out};
    const region::RegionTally r = region::visit_region<DIM, FRAMES>(a, io, blockIdx.x, lds);
    if (threadIdx.x == 0) {
        if (!r.skipped) {
            unsigned long long *gc = a.counters;
            atomicAdd(&gc[kEvents], (unsigned long long)r.events);
            atomicAdd(&gc[kFlips], (unsigned long long)r.flips);
            atomicAdd(&gc[kGhostEvents], (unsigned long long)r.ghost);
            atomicAdd(&gc[kChecks], (unsigned long long)r.checks);
            atomicAdd(&gc[kSweeps], (unsigned long long)r.rounds);
            if (r.any_live) atomicAdd(&gc[kLiveTiles], 1ull);
            // owned cells that were all at or past the horizon when loaded can
            // never change again: both snapshots now hold them
            if (!r.own_due) a.dead[blockIdx.x] = 1;
        }
        finish_visit_block(a, ntiles_total);
    }
}

}  // namespace

size_t visit_fast_lds_bytes(int dim, const VisitArgs &a) { return region::fast_plan(a, dim).total; }

int visit_fast_box(int dim, const VisitArgs &a)
{
    int box = 1;
    for (int d = 0; d < dim; ++d) box *= a.tile[d] + 2 * a.ghost[d] + 2;
    return box;
}

template <bool FRAMES>
void launch_fast(int dim, const VisitArgs &a, unsigned tiles, int block, size_t lds,
                 hipStream_t stream)
{
    switch (dim) {
    case 1:
        hipLaunchKernelGGL((visit_fast_kernel<1, FRAMES>), dim3(tiles), dim3(block), lds,
                           stream, a);
        break;
    case 2:
        hipLaunchKernelGGL((visit_fast_kernel<2, FRAMES>), dim3(tiles), dim3(block), lds,
                           stream, a);
        break;
    default:
        hipLaunchKernelGGL((visit_fast_kernel<3, FRAMES>), dim3(tiles), dim3(block), lds,
                           stream, a);
        break;
    }
}

hipError_t launch_visit_fast(int dim, const VisitArgs &a, int block, size_t lds,
                             hipStream_t stream)
{
    const unsigned tiles = (unsigned)a.ntiles[0] * (unsigned)a.ntiles[1] *
                           (unsigned)a.ntiles[2];
    if (a.frames)
        launch_fast<true>(dim, a, tiles, block, lds, stream);
    else
        launch_fast<false>(dim, a, tiles, block, lds, stream);
    return hipGetLastError();
}

hipError_t set_visit_fast_lds_limit(size_t bytes)
{
    const void *fns[6] = {(const void *)visit_fast_kernel<1, false>,
                          (const void *)visit_fast_kernel<2, false>,
                          (const void *)visit_fast_kernel<3, false>,
                          (const void *)visit_fast_kernel<1, true>,
                          (const void *)visit_fast_kernel<2, true>,
                          (const void *)visit_fast_kernel<3, true>};
    for (const void *f : fns) {
        const hipError_t e =
            hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace aca

// plan_fixed.hip -- planning kernels specialised to one reach v_max and one
// tile width.  A kernel that dispatches over every (v_max, tile width) on the
// device gets one register allocation for the union of all shapes, larger
// than any single shape needs; these kernels get their own, which lets the
// batched kernel keep eight wavefronts per SIMD and spares the spills of the
// dispatching kernels.  This file is compiled once per v_max, with PLAN_V
// set to 1..5; each object exports its two launchers under names ending in
// its v_max.
#include <hip/hip_ext.h>

#include "plan_tile.h"

#ifndef PLAN_V
#error "PLAN_V (the v_max this object is compiled for) must be defined"
#endif

#define FK_CAT2(a, b) a##b
#define FK_CAT(a, b) FK_CAT2(a, b)

namespace fk {

// Wavefronts per SIMD the batched kernel is built for: eight (64 VGPRs) up to
// v_max = 4; the 11-row window of v_max = 5 needs more registers than that
// leaves without spilling to scratch.
constexpr int FIXED_WAVES = PLAN_V >= 5 ? 7 : 8;

// A batch of scenarios that all have v_max = V and tile width TX: one
// workgroup per tile, items[i] = (slot << 20) | tile or PLAN_ITEM_NONE.  (V is a template
// parameter, not just PLAN_V, so that each object's kernels have names of
// their own.)
template <int V, int TX>
__global__ __launch_bounds__(PLAN_THREADS) __attribute__((amdgpu_waves_per_eu(FIXED_WAVES)))
void plan_kernel_fixed(const SlotDev *__restrict__ table, const uint32_t *__restrict__ items)
{
    __shared__ PlanShared sh;
    const uint32_t it = items[blockIdx.x];
    if (it == PLAN_ITEM_NONE) return;                     // padding
    plan_tile<V, TX, false>(table[it >> 20], (int)(it & 0xFFFFFu), sh);
}

// One scenario, descriptor by value, workgroup i plans tile row_tile(i).
template <int V, int TX>
__global__ __launch_bounds__(ONE_MAX_THREADS) void plan_kernel_one_fixed(const SlotDev s)
{
    __shared__ PlanShared sh;
    const int tile = row_tile((int)blockIdx.x, s.ntx, s.nty);
    if (tile < 0) return;
    plan_tile<V, TX, false>(s, tile, sh);
}

}  // namespace fk

// Batched launch for tile width tx (8, 16, 32 or 64).
extern "C" hipError_t FK_CAT(fk_launch_plan_fixed_v, PLAN_V)(int tx, const fk::SlotDev *table,
                                                              const uint32_t *items, int n_items,
                                                              hipStream_t stream, hipEvent_t start,
                                                              hipEvent_t stop)
{
    if (n_items <= 0) return hipSuccess;
    const dim3 grid(n_items), block(fk::PLAN_THREADS);
    switch (tx) {
        case 8: hipExtLaunchKernelGGL((fk::plan_kernel_fixed<PLAN_V, 8>), grid, block, 0, stream, start, stop, 0, table, items); break;
        case 16: hipExtLaunchKernelGGL((fk::plan_kernel_fixed<PLAN_V, 16>), grid, block, 0, stream, start, stop, 0, table, items); break;
        case 32: hipExtLaunchKernelGGL((fk::plan_kernel_fixed<PLAN_V, 32>), grid, block, 0, stream, start, stop, 0, table, items); break;
        case 64: hipExtLaunchKernelGGL((fk::plan_kernel_fixed<PLAN_V, 64>), grid, block, 0, stream, start, stop, 0, table, items); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Single-scenario launch.  A scenario of a few hundred tiles cannot fill the
// device, so its launch lasts as long as its slowest tile: it takes one thread
// per tile cell (256 .. 1,024), so that a crowded tile needs one pass over its
// agents.
extern "C" hipError_t FK_CAT(fk_launch_plan_one_fixed_v, PLAN_V)(const fk::SlotDev *slot,
                                                                  int n_tiles, hipStream_t stream,
                                                                  hipEvent_t start, hipEvent_t stop)
{
    if (n_tiles <= 0) return hipSuccess;
    if (slot->v != PLAN_V) return hipErrorInvalidValue;
    const int cells = slot->tx * slot->ty;
    const int threads = cells < fk::PLAN_THREADS ? fk::PLAN_THREADS
                        : cells > fk::ONE_MAX_THREADS ? fk::ONE_MAX_THREADS : cells;
    const dim3 grid(fk::row_grid(slot->ntx, slot->nty)), block(threads);
    switch (slot->tx) {
        case 8: hipExtLaunchKernelGGL((fk::plan_kernel_one_fixed<PLAN_V, 8>), grid, block, 0, stream, start, stop, 0, *slot); break;
        case 16: hipExtLaunchKernelGGL((fk::plan_kernel_one_fixed<PLAN_V, 16>), grid, block, 0, stream, start, stop, 0, *slot); break;
        case 32: hipExtLaunchKernelGGL((fk::plan_kernel_one_fixed<PLAN_V, 32>), grid, block, 0, stream, start, stop, 0, *slot); break;
        case 64: hipExtLaunchKernelGGL((fk::plan_kernel_one_fixed<PLAN_V, 64>), grid, block, 0, stream, start, stop, 0, *slot); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

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
// workgroup per tile, items[i] = (slot << 20) | tile.  (V is a template
// parameter, not just PLAN_V, so that each object's kernels have names of
// their own.)
template <int V, int TX>
__global__ __launch_bounds__(PLAN_THREADS) __attribute__((amdgpu_waves_per_eu(FIXED_WAVES)))
void plan_kernel_fixed(const SlotDev *__restrict__ table, const uint32_t *__restrict__ items)
{
    __shared__ PlanShared<false> sh;
    const uint32_t it = items[blockIdx.x];
    plan_tile<V, TX, false, false>(table[it >> 20], (int)(it & 0xFFFFFu), sh);
}

// One scenario, descriptor by value, workgroup i plans tile i (SS: the floor
// field window is staged in LDS too).
template <int V, int TX, bool SS>
__global__ __launch_bounds__(ONE_MAX_THREADS) void plan_kernel_one_fixed(const SlotDev s)
{
    __shared__ PlanShared<SS> sh;
    plan_tile<V, TX, false, SS>(s, (int)blockIdx.x, sh);
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

namespace {

template <int TX>
void launch_one_v(bool ss, dim3 grid, dim3 block, hipStream_t stream, hipEvent_t start,
                hipEvent_t stop, const fk::SlotDev &s)
{
    if (ss)
        hipExtLaunchKernelGGL((fk::plan_kernel_one_fixed<PLAN_V, TX, true>), grid, block, 0, stream, start,
                              stop, 0, s);
    else
        hipExtLaunchKernelGGL((fk::plan_kernel_one_fixed<PLAN_V, TX, false>), grid, block, 0, stream, start,
                              stop, 0, s);
}

}  // namespace

// Single-scenario launch.  A scenario of a few hundred tiles cannot fill the
// device, so its launch lasts as long as its slowest tile: up to
// ONE_STAGE_S_TILES tiles it takes one thread per tile cell (256 .. 1,024; a
// crowded tile needs one pass over its agents) and stages the floor field, so
// the rare FP64 re-resolve reads LDS only; larger scenarios take 256 threads
// and read the floor field from global memory.
extern "C" hipError_t FK_CAT(fk_launch_plan_one_fixed_v, PLAN_V)(const fk::SlotDev *slot,
                                                                  int n_tiles, hipStream_t stream,
                                                                  hipEvent_t start, hipEvent_t stop)
{
    if (n_tiles <= 0) return hipSuccess;
    const bool ss = n_tiles <= fk::ONE_STAGE_S_TILES;
    const int cells = slot->tx * slot->ty;
    const int threads = !ss ? fk::PLAN_THREADS
                        : cells < fk::PLAN_THREADS ? fk::PLAN_THREADS
                        : cells > fk::ONE_MAX_THREADS ? fk::ONE_MAX_THREADS : cells;
    const dim3 grid(n_tiles), block(threads);
    switch (slot->tx) {
        case 8: launch_one_v<8>(ss, grid, block, stream, start, stop, *slot); break;
        case 16: launch_one_v<16>(ss, grid, block, stream, start, stop, *slot); break;
        case 32: launch_one_v<32>(ss, grid, block, stream, start, stop, *slot); break;
        case 64: launch_one_v<64>(ss, grid, block, stream, start, stop, *slot); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// plan_batch.hip -- the batched planning launch: one launch plans the tiles of
// many scenarios, one workgroup per tile.  A batch whose scenarios share
// v_max and tile width runs the kernel specialised to that shape
// (plan_fixed.hip); a mixed batch (uneven grids, agent counts, v_max and tile
// shapes) runs this kernel, which dispatches per tile on the device.
#include <hip/hip_ext.h>

#include "fast_host.h"
#include "plan_tile.h"

namespace fk {

// items[i] = (slot << 20) | tile index (row-major over the slot's tiles), or
// PLAN_ITEM_NONE; descriptors come from the device table.  Built for eight
// wavefronts per SIMD: the union of all shapes then fits 64 VGPRs with one
// 8-byte spill in one shape's agent loop, and the 256-scenario ensemble
// stepped about 2 us faster than with seven wavefronts and no spill.
__global__ __launch_bounds__(PLAN_THREADS) __attribute__((amdgpu_waves_per_eu(8)))
void plan_kernel(const SlotDev *__restrict__ table, const uint32_t *__restrict__ items)
{
    __shared__ PlanShared sh;
    const uint32_t it = items[blockIdx.x];
    if (it == PLAN_ITEM_NONE) return;                     // padding
    plan_dispatch<false>(table[it >> 20], (int)(it & 0xFFFFFu), sh);
}

}  // namespace fk

// v, tx: the shared v_max and tile width of every item's scenario, or 0 for a
// mixed batch.  start / stop (optional): events that record the kernel's own
// start and end.
extern "C" hipError_t fk_launch_plan(const fk::SlotDev *table, const uint32_t *items, int n_items,
                                     int v, int tx, hipStream_t stream, hipEvent_t start,
                                     hipEvent_t stop)
{
    if (n_items <= 0) return hipSuccess;
    switch (v) {
        case 0: break;
        case 1: return fk_launch_plan_fixed_v1(tx, table, items, n_items, stream, start, stop);
        case 2: return fk_launch_plan_fixed_v2(tx, table, items, n_items, stream, start, stop);
        case 3: return fk_launch_plan_fixed_v3(tx, table, items, n_items, stream, start, stop);
        case 4: return fk_launch_plan_fixed_v4(tx, table, items, n_items, stream, start, stop);
        case 5: return fk_launch_plan_fixed_v5(tx, table, items, n_items, stream, start, stop);
        default: return hipErrorInvalidValue;
    }
    hipExtLaunchKernelGGL(fk::plan_kernel, dim3(n_items), dim3(fk::PLAN_THREADS), 0, stream, start,
                          stop, 0, table, items);
    return hipGetLastError();
}

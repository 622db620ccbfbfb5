// plan_batch.hip -- the batched planning kernel: one launch plans the tiles
// of many scenarios (uneven grids, agent counts, v_max and tile shapes), one
// workgroup per tile.
#include <hip/hip_ext.h>

#include "plan_tile.h"

namespace fk {

// items[i] = (slot << 20) | tile index (row-major over the slot's tiles);
// descriptors come from the device table.
__global__ __launch_bounds__(PLAN_THREADS) __attribute__((amdgpu_waves_per_eu(7)))
void plan_kernel(const SlotDev *__restrict__ table, const uint32_t *__restrict__ items)
{
    __shared__ PlanShared<false> sh;
    const uint32_t it = items[blockIdx.x];
    plan_dispatch<false, false>(table[it >> 20], (int)(it & 0xFFFFFu), sh);
}

}  // namespace fk

// start / stop (optional): events that record the kernel's own start and end.
extern "C" hipError_t fk_launch_plan(const fk::SlotDev *table, const uint32_t *items, int n_items,
                                     hipStream_t stream, hipEvent_t start, hipEvent_t stop)
{
    if (n_items <= 0) return hipSuccess;
    hipExtLaunchKernelGGL(fk::plan_kernel, dim3(n_items), dim3(fk::PLAN_THREADS), 0, stream, start,
                          stop, 0, table, items);
    return hipGetLastError();
}

// plan_one.hip -- single-scenario planning launches: the debug kernel (it also
// writes weights, flags and margins; one kernel dispatching over v_max and
// tile width on the device), and the dispatch of ordinary launches to the
// kernels specialised to the scenario's v_max and tile width (plan_fixed.hip).
#include <hip/hip_ext.h>

#include "fast_host.h"
#include "plan_tile.h"

namespace fk {

__global__ __launch_bounds__(PLAN_THREADS) void plan_kernel_debug(const SlotDev s)
{
    __shared__ PlanShared sh;
    const int tile = row_tile((int)blockIdx.x, s.ntx, s.nty);
    if (tile < 0) return;
    plan_dispatch<true>(s, tile, sh);
}

}  // namespace fk

// start / stop (optional): events that record the kernel's own start and end
// (hipExtLaunchKernelGGL), the timestamps a kernel trace reports.
extern "C" hipError_t fk_launch_plan_one(const fk::SlotDev *slot, int n_tiles, int debug,
                                         hipStream_t stream, hipEvent_t start, hipEvent_t stop)
{
    if (n_tiles <= 0) return hipSuccess;
    if (debug) {
        hipLaunchKernelGGL(fk::plan_kernel_debug, dim3(fk::row_grid(slot->ntx, slot->nty)), dim3(fk::PLAN_THREADS), 0, stream,
                           *slot);
        return hipGetLastError();
    }
    switch (slot->v) {
        case 1: return fk_launch_plan_one_fixed_v1(slot, n_tiles, stream, start, stop);
        case 2: return fk_launch_plan_one_fixed_v2(slot, n_tiles, stream, start, stop);
        case 3: return fk_launch_plan_one_fixed_v3(slot, n_tiles, stream, start, stop);
        case 4: return fk_launch_plan_one_fixed_v4(slot, n_tiles, stream, start, stop);
        case 5: return fk_launch_plan_one_fixed_v5(slot, n_tiles, stream, start, stop);
        default: return hipErrorInvalidValue;
    }
}

// Scenarios with per-agent speeds or several fields (plan_het.hip).
extern "C" hipError_t fk_launch_plan_het(const fk::SlotDev *slot, const fk::HetDev *h, int n_tiles,
                                         int debug, hipStream_t stream, hipEvent_t start,
                                         hipEvent_t stop)
{
    switch (slot->v) {
        case 1: return fk_launch_plan_het_v1(slot, h, n_tiles, debug, stream, start, stop);
        case 2: return fk_launch_plan_het_v2(slot, h, n_tiles, debug, stream, start, stop);
        case 3: return fk_launch_plan_het_v3(slot, h, n_tiles, debug, stream, start, stop);
        case 4: return fk_launch_plan_het_v4(slot, h, n_tiles, debug, stream, start, stop);
        case 5: return fk_launch_plan_het_v5(slot, h, n_tiles, debug, stream, start, stop);
        default: return hipErrorInvalidValue;
    }
}

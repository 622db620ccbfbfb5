// plan_one.hip -- planning kernels of a single scenario: its descriptor
// arrives by value with the kernel arguments and workgroup i plans tile i,
// which saves two dependent memory round trips per workgroup.
//
// A single scenario of a few hundred tiles cannot fill the device, so its
// launch time is the latency of its slowest tile: such launches use up to one
// thread per tile cell (a crowded tile needs one pass over its agents) and
// stage the floor-field window in LDS beside the exp table, so the rare FP64
// re-resolve makes no global reads.  Launches with many tiles keep 256
// threads and read the floor field from global memory, like the batched
// kernel.  The debug form also writes weights, flags and margins.
#include <hip/hip_ext.h>

#include "plan_tile.h"

namespace fk {

constexpr int ONE_MAX_THREADS = 1024;
constexpr int ONE_STAGE_S_TILES = 2048;     // stage the floor field up to this many tiles

template <bool DEBUG, bool SS>
__global__ __launch_bounds__(ONE_MAX_THREADS) void plan_kernel_one(const SlotDev s)
{
    __shared__ PlanShared<SS> sh;
    plan_dispatch<DEBUG, SS>(s, (int)blockIdx.x, sh);
}

}  // namespace fk

// start / stop (optional): events that record the kernel's own start and end
// (hipExtLaunchKernelGGL), the timestamps a kernel trace reports.
extern "C" hipError_t fk_launch_plan_one(const fk::SlotDev *slot, int n_tiles, int debug,
                                         hipStream_t stream, hipEvent_t start, hipEvent_t stop)
{
    if (n_tiles <= 0) return hipSuccess;
    if (debug) {
        hipLaunchKernelGGL((fk::plan_kernel_one<true, false>), dim3(n_tiles), dim3(fk::PLAN_THREADS),
                           0, stream, *slot);
    } else if (n_tiles <= fk::ONE_STAGE_S_TILES) {
        const int cells = slot->tx * slot->ty;
        const int threads = cells < fk::PLAN_THREADS ? fk::PLAN_THREADS
                            : cells > fk::ONE_MAX_THREADS ? fk::ONE_MAX_THREADS : cells;
        hipExtLaunchKernelGGL((fk::plan_kernel_one<false, true>), dim3(n_tiles), dim3(threads), 0,
                              stream, start, stop, 0, *slot);
    } else {
        hipExtLaunchKernelGGL((fk::plan_kernel_one<false, false>), dim3(n_tiles),
                              dim3(fk::PLAN_THREADS), 0, stream, start, stop, 0, *slot);
    }
    return hipGetLastError();
}

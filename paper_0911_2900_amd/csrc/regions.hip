// regions.hip -- the count kernel behind region counts (see regions.h).
#include <hip/hip_runtime.h>

#include "fast_dev.h"
#include "regions.h"

namespace fk {

// Workgroup (j, r): rectangle r of job j.  Threads stride over the
// rectangle's cells and count those holding an agent; the sum of the
// wavefront counts goes to row ctr[C_STEP] of the job's series.  Rows outside
// the series are skipped.
__global__ __launch_bounds__(COUNT_THREADS) void count_kernel(const RegionDev *jobs)
{
    __shared__ int part[COUNT_THREADS / 64];
    const RegionDev &j = jobs[blockIdx.x];
    const int r = blockIdx.y;
    if (r >= j.n) return;
    const int step = j.ctr[C_STEP];
    if (step < 0 || step >= j.rows) return;
    const int x0 = j.rect[4 * r], y0 = j.rect[4 * r + 1];
    const int w = j.rect[4 * r + 2] - x0, h = j.rect[4 * r + 3] - y0;
    int cnt = 0;
    for (int i = threadIdx.x; i < w * h; i += COUNT_THREADS) {
        const int y = y0 + i / w, x = x0 + i % w;
        cnt += j.occ[(y + j.pad) * j.Wp + x + j.pad] >= 0;
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_down(cnt, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int k = 0; k < COUNT_THREADS / 64; ++k) t += part[k];
        j.series[step * j.n + r] = t;
    }
}

}  // namespace fk

// One launch over n_jobs scenarios with at most max_regions rectangles each.
extern "C" hipError_t fk_launch_count(const fk::RegionDev *jobs, int n_jobs, int max_regions,
                                      hipStream_t stream)
{
    if (n_jobs <= 0 || max_regions <= 0) return hipSuccess;
    if (max_regions > fk::MAX_REGIONS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fk::count_kernel, dim3((unsigned)n_jobs, (unsigned)max_regions),
                       dim3(fk::COUNT_THREADS), 0, stream, jobs);
    return hipGetLastError();
}

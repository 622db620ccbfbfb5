// stream.hip -- a streaming kernel that measures the bandwidth a launch of a
// given footprint can reach: five reads for each write (out = a + b + c + d + e
// over float4), close to the planning kernel's read/write mix.  It is the
// yardstick for the planning kernel's fraction of achievable bandwidth, both
// beyond the 256 MB last-level cache (a 4 GiB footprint) and at the planning
// launch's own footprint.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace fk {

__global__ __launch_bounds__(256) void stream_kernel(const float4 *__restrict__ a,
                                                     const float4 *__restrict__ b,
                                                     const float4 *__restrict__ c,
                                                     const float4 *__restrict__ d,
                                                     const float4 *__restrict__ e,
                                                     float4 *__restrict__ out, size_t n4)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n4) return;
    const float4 x = a[i], y = b[i], z = c[i], w = d[i], v = e[i];
    out[i] = make_float4(x.x + y.x + z.x + w.x + v.x, x.y + y.y + z.y + w.y + v.y,
                         x.z + y.z + z.z + w.z + v.z, x.w + y.w + z.w + w.w + v.w);
}

}  // namespace fk

// base: six arrays of n4 float4 each, back to back (a, b, c, d, e, out).
extern "C" hipError_t fk_launch_stream(float4 *base, size_t n4, hipStream_t stream,
                                       hipEvent_t start, hipEvent_t stop)
{
    if (n4 == 0) return hipSuccess;
    const size_t blocks = (n4 + 255) / 256;
    if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipExtLaunchKernelGGL(fk::stream_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, start,
                          stop, 0, base, base + n4, base + 2 * n4, base + 3 * n4, base + 4 * n4,
                          base + 5 * n4, n4);
    return hipGetLastError();
}

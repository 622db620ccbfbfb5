// cus.hip -- counts the compute units that a stream's launches reach.
//
// A stream created with a CU mask runs its kernels on a subset of the chip.
// The motion phase needs every workgroup of its launch resident at once (its
// workgroups meet at group barriers), so a context on such a stream sizes its
// motion groups from the CUs counted here rather than from the mask's bits.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fk {

// s_getreg operands: register id | offset << 6 | (bits - 1) << 11.
constexpr int HWREG_HW_ID = 4 | (31 << 11);    // wave, SIMD, CU, SH, SE of this wave
constexpr int HWREG_XCC_ID = 20 | (31 << 11);  // XCD of this wave (bits 0..3)

// One wavefront per workgroup.  Lane 0 writes where the workgroup runs:
// (XCD << 8) | the CU, SH and SE fields (bits 8..15 of HW_ID); wave, SIMD and
// workgroup-slot fields are left out, so two workgroups on one CU write the
// same id.  Every workgroup then sleeps for `hold` x 8128 clocks (a fixed
// count, so every wave ends) while holding the dynamic LDS the launch gives
// it; with 48 KB each at most three fit on a CU, so a grid of more than three
// workgroups per enabled CU occupies every enabled CU at once.
__global__ __launch_bounds__(64) void cu_probe_kernel(uint32_t *ids, int hold)
{
    extern __shared__ uint32_t pad[];
    const uint32_t hw = __builtin_amdgcn_s_getreg(HWREG_HW_ID);
    const uint32_t xcc = __builtin_amdgcn_s_getreg(HWREG_XCC_ID);
    pad[threadIdx.x] = hw;
    if (threadIdx.x == 0) ids[blockIdx.x] = ((xcc & 0xFu) << 8) | ((hw >> 8) & 0xFFu);
    for (int i = 0; i < hold; ++i) __builtin_amdgcn_s_sleep(127);
}

}  // namespace fk

// Fills ids_host[0..n_wg) with the placement id of each workgroup of one
// probe launch on `stream` (synchronises it).  n_wg in 1..4096.
extern "C" hipError_t fk_cu_probe(hipStream_t stream, int n_wg, uint32_t *ids_host)
{
    if (n_wg < 1 || n_wg > 4096 || !ids_host) return hipErrorInvalidValue;
    uint32_t *ids = nullptr;
    hipError_t e = hipMalloc(&ids, sizeof(uint32_t) * n_wg);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fk::cu_probe_kernel, dim3(n_wg), dim3(64), 48 * 1024, stream, ids, 4);
    e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(ids_host, ids, sizeof(uint32_t) * n_wg, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFree(ids);
    return e;
}

// scratch.hip -- the library's static work-item scratch: device memory that
// the allocation-free batched run (fast_run_noalloc) uses in place of the
// per-batch allocation of fast_run.  It holds the launch's work items (the
// planning launch's tile items, the motion launch's workgroup items) and the
// region-count jobs; nothing in it needs to start at zero.
//
// The array is a file-scope __device__ symbol, so each GPU the library runs
// on holds its own copy until the process ends.  Host code never passes the
// symbol itself to a kernel (on the host it is only a stand-in, not a device
// address): fk_scratch_ptr resolves the device address once per device, with
// that device current, and every launch and copy uses that address.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "fast_host.h"

namespace {

static __device__ __align__(256) uint8_t scratch[fk::SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};

}  // namespace

// The device address of `scratch` on `device`, which must be the current
// device.  Resolved on the first call per device and kept.
extern "C" hipError_t fk_scratch_ptr(int device, void **out)
{
    if (device < 0 || device >= MAX_DEVICES || !out) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[device] = p;
    }
    *out = g_ptr[device];
    return hipSuccess;
}

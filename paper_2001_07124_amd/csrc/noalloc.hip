// rhosvd_decompose_noalloc: the whole decomposition on a fixed per-device
// scratch array, for callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"
#include "rhosvd.h"

// Every device the library runs on holds its own copy of this array until
// the process ends.  In host code its name is only a stand-in: kernels get
// the device address hipGetSymbolAddress returns for the current device
// (kept per device below), never the name.
static __device__ __align__(256) unsigned char scratch[RHOSVD_NOALLOC_SCRATCH_BYTES];

namespace rh {

int32_t noalloc_scratch_address(int device, void** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    if (!out || device < 0 || device >= kMaxDevices) return RHOSVD_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int prev = -1;
        if (hipGetDevice(&prev) != hipSuccess) return RHOSVD_EHIP;
        if (prev != device && hipSetDevice(device) != hipSuccess) return RHOSVD_EHIP;
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (prev != device) (void)hipSetDevice(prev);
        if (e != hipSuccess || !ptr) return RHOSVD_EHIP;
        addr[device] = ptr;
    }
    *out = addr[device];
    return RHOSVD_OK;
}

}  // namespace rh

extern "C" int32_t rhosvd_decompose_noalloc(rhosvd_ctx* ctx, const rhosvd_tensor* x,
                                            const rhosvd_params* p, const rhosvd_output* out,
                                            void* stream) {
    if (!ctx) return RHOSVD_EINVAL;
    void* ws = rh::ctx_scratch(ctx);
    if (!ws) return RHOSVD_EHIP;
    return rh::decompose_fixed(ctx, x, p, ws, RHOSVD_NOALLOC_SCRATCH_BYTES, RHOSVD_ESCRATCH, out,
                               stream);
}

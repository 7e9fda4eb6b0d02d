// Library-internal entry points shared between the host source files (not
// part of the C ABI).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "rhosvd.h"

namespace rh {

// rhosvd_decompose on a caller-given fixed workspace (ws, ws_bytes) with its
// plan on the stack: no allocation of any kind.  Returns `too_small` when the
// problem needs more than ws_bytes.  (rhosvd_api.hip)
int32_t decompose_fixed(rhosvd_ctx* ctx, const rhosvd_tensor* x, const rhosvd_params* p,
                        void* ws, size_t ws_bytes, int32_t too_small, const rhosvd_output* out,
                        void* stream);

// The context's device address of the no-alloc scratch.  (rhosvd_api.hip)
void* ctx_scratch(const rhosvd_ctx* ctx);

// Device address of the fixed no-alloc scratch on `device`, looked up once
// per device with that device current.  (noalloc.hip)
int32_t noalloc_scratch_address(int device, void** out);

}  // namespace rh

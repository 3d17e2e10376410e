// orrb_render_batch_noalloc: the render call for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  It is orrb_render_batch with the workspace taken from a fixed array in
// the library's device image instead of a caller buffer.
//
// The array below is a device symbol: on the host its name is only a stand-in, not a
// device address.  orrb_create resolves the address of each device's copy once, with
// that device current (hipGetSymbolAddress), and every use goes through that address.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/orrb.h"
#include "orrb_device.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // ORRB_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == ORRB_NOALLOC_SCRATCH_BYTES, "header and library disagree on the scratch size");

// One copy per device, alive until the process ends.  Every call on a device shares it.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};  // device address of each device's copy (null until resolved)

void *scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return g_scratch_ptr[device];
}

}  // namespace

namespace orrb {

// Called by orrb_create with `device` current.  Resolves the device's copy once.
hipError_t scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

}  // namespace orrb

extern "C" orrb_status orrb_render_batch_noalloc(orrb_context *ctx, const orrb_layout *layout,
                                                 const orrb_scenes *scenes, const orrb_cameras *cameras,
                                                 const orrb_params *params, const orrb_outputs *out, void *stream) {
    orrb::set_error(ORRB_OK, "");  // the thread's last error describes this call only
    if (!ctx || !layout) return orrb::set_error(ORRB_ERR_INVALID_ARGUMENT, "NULL handle");
    const size_t need = orrb::render_workspace_bytes(layout);
    if (need > kScratchBytes) {
        char msg[192];
        snprintf(msg, sizeof(msg),
                 "the batch needs %zu bytes of workspace; orrb_render_batch_noalloc holds at most %zu "
                 "(use orrb_render_batch with a caller workspace)",
                 need, kScratchBytes);
        return orrb::set_error(ORRB_ERR_UNSUPPORTED, msg);
    }
    void *ws = scratch_address(orrb::context_device(ctx));
    if (!ws) return orrb::set_error(ORRB_ERR_DEVICE, "the device's scratch address was not resolved");
    // The kernels reset what must start at zero themselves (the persistent tile
    // counter is cleared by the vertex kernel, the frame kernel's claim counter by a
    // one-thread kernel before it), so no memset is issued.
    const orrb_status st = orrb::debug_validate(ctx, layout, scenes, cameras, params, out, stream);
    if (st != ORRB_OK) return st;
    return orrb::render_impl(ctx, layout, scenes, cameras, params, out, ws, kScratchBytes, stream, true);
}

// ckv_run_noalloc: ckv_run with its workspace in a static device array, for
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc).
//
// The array lives in the library's code object: every GPU the library runs on
// holds its own copy, at its own address, from the first launch until the
// process ends.  Its address on a device is taken once per device with
// hipGetSymbolAddress (in host code the array's name is only a host stand-in,
// never a device address) and kept; kernels receive that pointer exactly as
// they receive a caller's workspace.  Nothing here allocates device memory.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ckv_internal.h"

namespace ckv {
namespace {

constexpr size_t kScratchBytes = (size_t)CKV_NOALLOC_SCRATCH_MIB << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_ptr(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
        return CKV_ERR_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("ckv_run_noalloc: device index beyond the library's table");
        return CKV_ERR_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return CKV_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CKV_OK;
}

}  // namespace
}  // namespace ckv

using namespace ckv;

extern "C" {

size_t ckv_noalloc_workspace_size(int64_t n_segments, int32_t n_showers, int32_t n_tel,
                                  int64_t capacity, const ckv_params* params)
{
    if (n_segments < 0 || n_showers < 1 || n_tel < 1 || capacity < 0 || !params) return 0;
    // the layout for the grid the launch will use (params->grid, else one
    // workgroup per compute unit of the current device)
    ckv_params p = *params;
    if (p.grid <= 0 && default_emit_grid(&p.grid) != CKV_OK) return 0;
    return workspace_layout(n_segments, n_showers, n_tel, capacity, &p, nullptr, nullptr);
}

int ckv_run_noalloc(const ckv_segments* segs, const ckv_showers* showers, const ckv_params* params,
                    const ckv_atmo* atmo, const ckv_array* arr, ckv_output* out,
                    const ckv_cursor* resume_from, void* stream)
{
    if (!segs || !showers || !params || !arr || !out) {
        set_error("NULL argument");
        return CKV_ERR_ARG;
    }
    ckv_params p = *params;
    if (p.grid <= 0) {
        if (int rc = default_emit_grid(&p.grid)) return rc;
    }
    if (segs->n < 0 || showers->n_showers < 1 || out->capacity < 0) {
        set_error("need n >= 0, n_showers >= 1 and capacity >= 0");
        return CKV_ERR_ARG;
    }
    const size_t need =
        workspace_layout(segs->n, showers->n_showers, arr->n_tel, out->capacity, &p, nullptr, nullptr);
    if (need > kScratchBytes) {
        set_error("ckv_run_noalloc: the run needs " + std::to_string(need) +
                  " bytes of workspace, more than the static scratch of " +
                  std::to_string(kScratchBytes) + " bytes (use ckv_run with a workspace)");
        return CKV_ERR_CAPACITY;
    }
    void* ws = nullptr;
    if (int rc = scratch_ptr(&ws)) return rc;
    return run_checked(segs, showers, &p, atmo, arr, ws, kScratchBytes, out, resume_from, stream);
}

}  // extern "C"

// hygt_transform_noalloc(): hygt_forward() / hygt_inverse() with the
// workspace in a static device array of the library instead of caller
// memory, for callers that cannot allocate.
//
// The array lives in this translation unit. Its name in host code is only a
// host-side stand-in for the device symbol, so the device address of each
// GPU's copy is looked up once per device (hipGetSymbolAddress, with that
// device current) and kept; kernels and every other host use take that
// address, never the name.

#include <mutex>

#include "hygt.h"
#include "hygt_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[HYGT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device

// The current device's copy of `scratch`, or nullptr (with *status set).
void* device_scratch(int* status) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *status = HYGT_EHIP;
        return nullptr;
    }
    std::lock_guard<std::mutex> guard(g_lock);
    if (g_scratch[dev] == nullptr) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
            *status = HYGT_EHIP;
            return nullptr;
        }
        g_scratch[dev] = ptr;
    }
    *status = HYGT_OK;
    return g_scratch[dev];
}

}  // namespace

extern "C" int hygt_transform_noalloc(const float* x, float* y, const int32_t* cls,
                                      int64_t nblocks, int log2n, int rounds,
                                      const float* angles, int nclasses, int direction,
                                      hipStream_t stream) {
    const size_t need = hygt_workspace_bytes(nblocks, log2n, rounds, nclasses);
    if (need == 0) return HYGT_EINVAL;  // sizes out of range
    if (need > HYGT_NOALLOC_SCRATCH_BYTES) return HYGT_ESCRATCH;
    int status = HYGT_OK;
    void* ws = device_scratch(&status);
    if (ws == nullptr) return status;
    return hygt::transform_in_workspace(x, y, cls, nblocks, log2n, rounds, angles, nclasses,
                                        direction, ws, HYGT_NOALLOC_SCRATCH_BYTES, stream);
}

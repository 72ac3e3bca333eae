// C ABI of the HyGT library (declared in include/hygt.h): argument checks,
// workspace sizing and the launch sequence. Every check runs on the host
// before anything is enqueued.

#include "hygt.h"

#include <cstdint>
#include <vector>

#include "hygt_internal.h"

namespace {

using hygt::WsLayout;

bool sizes_ok(int64_t nblocks, int log2n, int rounds, int nclasses) {
    return nblocks >= 0 && nblocks <= HYGT_MAX_BLOCKS && log2n >= 1 &&
           log2n <= HYGT_MAX_LOG2N && rounds >= 1 && rounds <= HYGT_MAX_ROUNDS &&
           nclasses >= 1 && nclasses <= HYGT_MAX_CLASSES;
}

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int check_workspace(const void* ws, size_t ws_bytes, const WsLayout& l) {
    if (ws == nullptr || ws_bytes < l.total || !aligned(ws, 256)) return HYGT_EWORKSPACE;
    return HYGT_OK;
}

// x and y must be the same array or not overlap at all.
bool overlap_ok(const float* x, const float* y, int64_t nblocks, int log2n) {
    if (x == y) return true;
    const uintptr_t bytes = static_cast<uintptr_t>(nblocks) * (uintptr_t{4} << log2n);
    const uintptr_t xa = reinterpret_cast<uintptr_t>(x);
    const uintptr_t ya = reinterpret_cast<uintptr_t>(y);
    return xa + bytes <= ya || ya + bytes <= xa;
}

int plan_impl(const int32_t* cls, int64_t nblocks, int log2n, int rounds, const float* angles,
              int nclasses, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!sizes_ok(nblocks, log2n, rounds, nclasses)) return HYGT_EINVAL;
    const WsLayout l = hygt::ws_layout(nblocks, log2n, rounds, nclasses);
    if (int s = check_workspace(ws, ws_bytes, l)) return s;
    if (nblocks == 0) return HYGT_OK;  // empty arrays may come as NULL pointers
    if (angles == nullptr || !aligned(angles, 4)) return HYGT_EINVAL;
    if (cls == nullptr && nclasses != 1) return HYGT_EINVAL;
    if (cls != nullptr && !aligned(cls, 4)) return HYGT_EINVAL;
    const hipError_t e = hygt::launch_plan(cls, nblocks, log2n, rounds, angles, nclasses, l,
                                           hygt::ws_ptrs(ws, l), stream);
    return e == hipSuccess ? HYGT_OK : HYGT_ELAUNCH;
}

int apply_impl(const float* x, float* y, int64_t nblocks, int log2n, int rounds, int nclasses,
               int direction, const void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!sizes_ok(nblocks, log2n, rounds, nclasses)) return HYGT_EINVAL;
    if (direction != HYGT_FORWARD && direction != HYGT_INVERSE) return HYGT_EINVAL;
    const WsLayout l = hygt::ws_layout(nblocks, log2n, rounds, nclasses);
    if (int s = check_workspace(ws, ws_bytes, l)) return s;
    if (nblocks == 0) return HYGT_OK;
    if (x == nullptr || y == nullptr) return HYGT_EINVAL;
    const uintptr_t align = log2n == 1 ? 8 : 16;
    if (!aligned(x, align) || !aligned(y, align)) return HYGT_EINVAL;
    if (!overlap_ok(x, y, nblocks, log2n)) return HYGT_EINVAL;
    const hipError_t e =
        hygt::launch_rotate(x, y, nblocks, log2n, rounds, nclasses, direction, l,
                            hygt::ws_ptrs(const_cast<void*>(ws), l), stream);
    return e == hipSuccess ? HYGT_OK : HYGT_ELAUNCH;
}

int dense_impl(const float* x, float* y, int64_t nblocks, int log2n, int rounds, int nclasses,
               const uint16_t* mats, const void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!sizes_ok(nblocks, log2n, rounds, nclasses)) return HYGT_EINVAL;
    if (log2n != HYGT_DENSE_LOG2N) return HYGT_EINVAL;
    const WsLayout l = hygt::ws_layout(nblocks, log2n, rounds, nclasses);
    if (int s = check_workspace(ws, ws_bytes, l)) return s;
    if (nblocks == 0) return HYGT_OK;
    if (x == nullptr || y == nullptr || mats == nullptr) return HYGT_EINVAL;
    if (!aligned(x, 16) || !aligned(y, 16) || !aligned(mats, 16)) return HYGT_EINVAL;
    if (!overlap_ok(x, y, nblocks, log2n)) return HYGT_EINVAL;
    const hipError_t e =
        hygt::launch_dense(x, y, nblocks, reinterpret_cast<const unsigned short*>(mats), l,
                           hygt::ws_ptrs(const_cast<void*>(ws), l), stream);
    return e == hipSuccess ? HYGT_OK : HYGT_ELAUNCH;
}

int backward_impl(const float* y, const float* gy, float* gx, float* gangles, int64_t nblocks,
                  int log2n, int rounds, const float* angles, int nclasses, void* ws,
                  size_t ws_bytes, hipStream_t stream) {
    if (!sizes_ok(nblocks, log2n, rounds, nclasses)) return HYGT_EINVAL;
    if (log2n > HYGT_BACKWARD_MAX_LOG2N) return HYGT_EINVAL;
    const WsLayout l = hygt::ws_layout(nblocks, log2n, rounds, nclasses);
    if (int s = check_workspace(ws, ws_bytes, l)) return s;
    if (angles == nullptr || gangles == nullptr) return HYGT_EINVAL;
    if (!aligned(angles, 4) || !aligned(gangles, 4)) return HYGT_EINVAL;
    if (nblocks > 0) {
        if (y == nullptr || gy == nullptr || gx == nullptr) return HYGT_EINVAL;
        const uintptr_t align = log2n == 1 ? 8 : 16;
        if (!aligned(y, align) || !aligned(gy, align) || !aligned(gx, align)) return HYGT_EINVAL;
        // gx may alias gy (in place); y must be separate from both
        if (!overlap_ok(gy, gx, nblocks, log2n)) return HYGT_EINVAL;
        if (!overlap_ok(y, gx, nblocks, log2n) || y == gx) return HYGT_EINVAL;
    }
    const hipError_t e = hygt::launch_backward(y, gy, gx, gangles, nblocks, log2n, rounds,
                                               angles, nclasses, l, hygt::ws_ptrs(ws, l), stream);
    return e == hipSuccess ? HYGT_OK : HYGT_ELAUNCH;
}

int plan_and_apply(const float* x, float* y, const int32_t* cls, int64_t nblocks, int log2n,
                   int rounds, const float* angles, int nclasses, int direction, void* ws,
                   size_t ws_bytes, hipStream_t stream) {
    // Check the data arguments before enqueuing the plan, so that a failing
    // call enqueues nothing.
    if (!sizes_ok(nblocks, log2n, rounds, nclasses)) return HYGT_EINVAL;
    if (nblocks > 0) {
        if (x == nullptr || y == nullptr) return HYGT_EINVAL;
        const uintptr_t align = log2n == 1 ? 8 : 16;
        if (!aligned(x, align) || !aligned(y, align)) return HYGT_EINVAL;
        if (!overlap_ok(x, y, nblocks, log2n)) return HYGT_EINVAL;
    }
    if (int s = plan_impl(cls, nblocks, log2n, rounds, angles, nclasses, ws, ws_bytes, stream))
        return s;
    return apply_impl(x, y, nblocks, log2n, rounds, nclasses, direction, ws, ws_bytes, stream);
}

}  // namespace

extern "C" {

size_t hygt_workspace_bytes(int64_t nblocks, int log2n, int rounds, int nclasses) {
    if (!sizes_ok(nblocks, log2n, rounds, nclasses)) return 0;
    return hygt::ws_layout(nblocks, log2n, rounds, nclasses).total;
}

int hygt_plan(const int32_t* cls, int64_t nblocks, int log2n, int rounds, const float* angles,
              int nclasses, void* workspace, size_t workspace_bytes, hipStream_t stream) {
    return plan_impl(cls, nblocks, log2n, rounds, angles, nclasses, workspace, workspace_bytes,
                     stream);
}

int hygt_apply(const float* x, float* y, int64_t nblocks, int log2n, int rounds, int nclasses,
               int direction, const void* workspace, size_t workspace_bytes,
               hipStream_t stream) {
    return apply_impl(x, y, nblocks, log2n, rounds, nclasses, direction, workspace,
                      workspace_bytes, stream);
}

int hygt_forward(const float* x, float* y, const int32_t* cls, int64_t nblocks, int log2n,
                 int rounds, const float* angles, int nclasses, void* workspace,
                 size_t workspace_bytes, hipStream_t stream) {
    return plan_and_apply(x, y, cls, nblocks, log2n, rounds, angles, nclasses, HYGT_FORWARD,
                          workspace, workspace_bytes, stream);
}

int hygt_inverse(const float* x, float* y, const int32_t* cls, int64_t nblocks, int log2n,
                 int rounds, const float* angles, int nclasses, void* workspace,
                 size_t workspace_bytes, hipStream_t stream) {
    return plan_and_apply(x, y, cls, nblocks, log2n, rounds, angles, nclasses, HYGT_INVERSE,
                          workspace, workspace_bytes, stream);
}

int hygt_backward(const float* y, const float* gy, float* gx, float* gangles, int64_t nblocks,
                  int log2n, int rounds, const float* angles, int nclasses, void* workspace,
                  size_t workspace_bytes, hipStream_t stream) {
    return backward_impl(y, gy, gx, gangles, nblocks, log2n, rounds, angles, nclasses, workspace,
                         workspace_bytes, stream);
}

int hygt_dense_apply(const float* x, float* y, int64_t nblocks, int log2n, int rounds,
                     int nclasses, const uint16_t* mats, const void* workspace,
                     size_t workspace_bytes, hipStream_t stream) {
    return dense_impl(x, y, nblocks, log2n, rounds, nclasses, mats, workspace, workspace_bytes,
                      stream);
}

int hygt_check_error(const void* workspace, size_t workspace_bytes, hipStream_t stream) {
    if (workspace == nullptr || !aligned(workspace, 256) ||
        workspace_bytes < sizeof(hygt::PlanHeader))
        return HYGT_EWORKSPACE;
    if (hipStreamSynchronize(stream) != hipSuccess) return HYGT_EHIP;
    const auto* base = static_cast<const char*>(workspace);
    hygt::PlanHeader hdr;
    if (hipMemcpy(&hdr, base, sizeof(hdr), hipMemcpyDeviceToHost) != hipSuccess) return HYGT_EHIP;
    // per-chunk flags follow the header (see ws_layout)
    const size_t nchunks = hdr.nchunks > 0 ? static_cast<size_t>(hdr.nchunks) : 0;
    if (sizeof(hygt::PlanHeader) + nchunks * 4 > workspace_bytes) return HYGT_EWORKSPACE;
    std::vector<int32_t> flags(nchunks);
    if (nchunks && hipMemcpy(flags.data(), base + sizeof(hygt::PlanHeader), nchunks * 4,
                             hipMemcpyDeviceToHost) != hipSuccess)
        return HYGT_EHIP;
    for (int32_t f : flags)
        if (f) return HYGT_ECLASS;
    return HYGT_OK;
}

const char* hygt_strerror(int status) {
    switch (status) {
        case HYGT_OK: return "success";
        case HYGT_EINVAL: return "invalid argument (size out of range, NULL or misaligned pointer, or overlapping x/y)";
        case HYGT_EWORKSPACE: return "workspace NULL, smaller than hygt_workspace_bytes() or not 256-byte aligned";
        case HYGT_ELAUNCH: return "HIP kernel launch failed";
        case HYGT_ECLASS: return "a class index was outside [0, nclasses)";
        case HYGT_EHIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

}  // extern "C"

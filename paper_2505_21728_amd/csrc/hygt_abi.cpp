// C ABI of the HyGT library (declared in include/hygt.h): argument checks,
// workspace sizing and the launch sequence. Every check runs on the host
// before anything is enqueued.

#include "hygt.h"

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <new>
#include <vector>

#include "hygt_internal.h"

static_assert(HYGT_MAX_SEGMENTS == hygt::kMaxSegments, "segment limits differ");
static_assert(HYGT_MAX_TABLES == hygt::kMaxReqTables, "table limits differ");
static_assert(HYGT_MAX_BATCH_REQUESTS == hygt::kMaxBatchRequests && HYGT_MAX_BATCH_REQUESTS <= 64,
              "a batch's descriptors are read a lane each");
static_assert(sizeof(hygt_request) == 48 && sizeof(hygt_table_ref) == 24, "descriptor layout");
static_assert(offsetof(hygt_request, status) == 36, "a status every 12 int32 from entry 0's");
static_assert(HYGT_MAX_REQUEST_BLOCKS <= (1LL << 26), "block counts and workgroups in int32");

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

// Class indices and angles (or codes) of a plan with blocks.
int plan_inputs_ok(const int32_t* cls, const float* angles, const uint8_t* codes, int nclasses) {
    if (angles == nullptr && codes == nullptr) return HYGT_EINVAL;
    if (angles != nullptr && !aligned(angles, 4)) return HYGT_EINVAL;
    if (cls == nullptr && nclasses != 1) return HYGT_EINVAL;
    if (cls != nullptr && !aligned(cls, 4)) return HYGT_EINVAL;
    return HYGT_OK;
}

int plan_any(const int32_t* cls, int64_t nblocks, int log2n, int rounds, const float* angles,
             const uint8_t* codes, int integer, int nclasses, void* ws, size_t ws_bytes,
             hipStream_t stream) {
    if (!sizes_ok(nblocks, log2n, rounds, nclasses)) return HYGT_EINVAL;
    const WsLayout l = hygt::ws_layout(nblocks, log2n, rounds, nclasses);
    if (int s = check_workspace(ws, ws_bytes, l)) return s;
    if (nblocks == 0) return HYGT_OK;  // empty arrays may come as NULL pointers
    if (int s = plan_inputs_ok(cls, angles, codes, nclasses)) return s;
    const hipError_t e = hygt::launch_plan(cls, nblocks, log2n, rounds, angles, codes, integer,
                                           nclasses, l, hygt::ws_ptrs(ws, l), stream);
    return e == hipSuccess ? HYGT_OK : HYGT_ELAUNCH;
}

int plan_impl(const int32_t* cls, int64_t nblocks, int log2n, int rounds, const float* angles,
              int nclasses, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (nblocks > 0 && angles == nullptr) return HYGT_EINVAL;
    return plan_any(cls, nblocks, log2n, rounds, angles, nullptr, 0, nclasses, ws, ws_bytes,
                    stream);
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

namespace hygt {
int transform_in_workspace(const float* x, float* y, const int32_t* cls, int64_t nblocks,
                           int log2n, int rounds, const float* angles, int nclasses,
                           int direction, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (direction != HYGT_FORWARD && direction != HYGT_INVERSE) return HYGT_EINVAL;
    return plan_and_apply(x, y, cls, nblocks, log2n, rounds, angles, nclasses, direction, ws,
                          ws_bytes, stream);
}
}  // namespace hygt

namespace {

// ---- mixed batches ------------------------------------------------------

bool segment_ok(const hygt_segment& g) {
    return sizes_ok(g.nblocks, g.log2n, g.rounds, g.nclasses) && g.log2n >= 2;
}

// Offsets of the segments' parts of a mixed workspace, and its total size.
size_t mixed_layout(const hygt_segment* segs, int nseg, size_t* offsets) {
    size_t off = 0;
    for (int i = 0; i < nseg; ++i) {
        if (offsets) offsets[i] = off;
        const WsLayout l =
            hygt::ws_layout(segs[i].nblocks, segs[i].log2n, segs[i].rounds, segs[i].nclasses);
        off = hygt::align_up(off + l.total, 256);
    }
    return off;
}

int check_segments(const hygt_segment* segs, int nseg) {
    if (segs == nullptr || nseg < 1 || nseg > HYGT_MAX_SEGMENTS) return HYGT_EINVAL;
    for (int i = 0; i < nseg; ++i)
        if (!segment_ok(segs[i])) return HYGT_EINVAL;
    return HYGT_OK;
}

int mixed_args(const hygt_segment* segs, int nseg, const void* ws, size_t ws_bytes,
               hygt::MixedArgs* a) {
    if (int s = check_segments(segs, nseg)) return s;
    size_t offsets[HYGT_MAX_SEGMENTS];
    const size_t total = mixed_layout(segs, nseg, offsets);
    if (ws == nullptr || ws_bytes < total || !aligned(ws, 256)) return HYGT_EWORKSPACE;
    *a = hygt::MixedArgs{};
    // Items of the largest blocks go first: their tiles take longest, and
    // the shorter ones then fill in behind them instead of trailing.
    int order[HYGT_MAX_SEGMENTS];
    for (int i = 0; i < nseg; ++i) order[i] = i;
    std::stable_sort(order, order + nseg,
                     [&](int p, int q) { return segs[p].log2n > segs[q].log2n; });
    int64_t item = 0;
    for (int o = 0; o < nseg; ++o) {
        const int i = order[o];
        const hygt_segment& g = segs[i];
        if (g.nblocks > 0) {
            if (g.x == nullptr || g.y == nullptr) return HYGT_EINVAL;
            if (!aligned(g.x, 16) || !aligned(g.y, 16)) return HYGT_EINVAL;
            if (!overlap_ok(g.x, g.y, g.nblocks, g.log2n)) return HYGT_EINVAL;
        }
        const WsLayout l = hygt::ws_layout(g.nblocks, g.log2n, g.rounds, g.nclasses);
        void* part = static_cast<char*>(const_cast<void*>(ws)) + offsets[i];
        const hygt::WsPtrs p = hygt::ws_ptrs(part, l);
        hygt::MixedSeg& m = a->seg[o];
        m.x = g.x;
        m.y = g.y;
        m.nblocks = g.nblocks;
        m.max_tiles = g.nblocks > 0 ? l.max_tiles : 0;
        m.tile_class = p.tile_class;
        m.perm = p.perm;
        m.modes = p.modes;
        m.coef = p.coef;
        m.signs = p.signs;
        m.log2n = g.log2n;
        m.rounds = g.rounds;
        m.nclasses = g.nclasses;
        m.item_begin = item;
        m.items = hygt::mixed_items(g.log2n, m.max_tiles);
        item += m.items;
    }
    a->nseg = nseg;
    a->total_items = item;
    return HYGT_OK;
}

int mixed_plan_impl(const hygt_segment* segs, int nseg, void* ws, size_t ws_bytes,
                    hipStream_t stream, bool tables = true) {
    if (int s = check_segments(segs, nseg)) return s;
    size_t offsets[HYGT_MAX_SEGMENTS];
    const size_t total = mixed_layout(segs, nseg, offsets);
    if (ws == nullptr || ws_bytes < total || !aligned(ws, 256)) return HYGT_EWORKSPACE;
    // Every segment with blocks gets its share of the same two launches.
    hygt::PlanArgs a{};
    a.tables = tables ? 1 : 0;
    int64_t count_wgs = 0, place_wgs = 0;
    for (int i = 0; i < nseg; ++i) {
        const hygt_segment& g = segs[i];
        if (g.nblocks == 0) continue;
        if (int s = plan_inputs_ok(g.cls, g.angles, nullptr, g.nclasses)) return s;
        const WsLayout l = hygt::ws_layout(g.nblocks, g.log2n, g.rounds, g.nclasses);
        const hygt::WsPtrs p = hygt::ws_ptrs(static_cast<char*>(ws) + offsets[i], l);
        hygt::PlanSeg& m = a.seg[a.nseg++];
        m.cls = g.cls;
        m.angles = g.angles;
        m.hdr = p.hdr;
        m.chunk_err = p.chunk_err;
        m.counts = p.counts;
        m.tile_class = p.tile_class;
        m.perm = p.perm;
        m.modes = p.modes;
        m.coef = p.coef;
        m.signs = p.signs;
        m.nblocks = g.nblocks;
        m.nchunks = l.nchunks;
        m.chunk = l.chunk;
        m.max_tiles = l.max_tiles;
        m.interleave = l.interleave;
        m.count_begin = count_wgs;
        m.place_begin = place_wgs;
        m.log2n = g.log2n;
        m.rounds = g.rounds;
        m.nclasses = g.nclasses;
        count_wgs += l.nchunks;
        place_wgs += (tables ? 2 * static_cast<int64_t>(g.nclasses) : 0) + l.nchunks;
    }
    const hipError_t e = hygt::launch_plan_mixed(a, count_wgs, place_wgs, stream);
    return e == hipSuccess ? HYGT_OK : HYGT_ELAUNCH;
}

int mixed_apply_impl(const hygt_segment* segs, int nseg, int direction, int config,
                     const void* ws, size_t ws_bytes, hipStream_t stream) {
    if (direction != HYGT_FORWARD && direction != HYGT_INVERSE) return HYGT_EINVAL;
    if (config < 0 || config >= hygt::kMixedConfigs) return HYGT_EINVAL;
    hygt::MixedArgs a;
    if (int s = mixed_args(segs, nseg, ws, ws_bytes, &a)) return s;
    if (a.total_items == 0) return HYGT_OK;
    const hipError_t e = hygt::launch_mixed(a, direction, config, stream);
    return e == hipSuccess ? HYGT_OK : HYGT_ELAUNCH;
}

}  // namespace

struct hygt_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

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

int hygt_apply_perm(const float* x, float* y, int64_t nblocks, int log2n, int rounds,
                    int nclasses, int direction, const int32_t* perm, const void* workspace,
                    size_t workspace_bytes, hipStream_t stream) {
    if (!sizes_ok(nblocks, log2n, rounds, nclasses)) return HYGT_EINVAL;
    if (log2n < 2 || log2n > HYGT_PERM_MAX_LOG2N) return HYGT_EINVAL;
    if (direction != HYGT_FORWARD && direction != HYGT_INVERSE) return HYGT_EINVAL;
    const WsLayout l = hygt::ws_layout(nblocks, log2n, rounds, nclasses);
    if (int s = check_workspace(workspace, workspace_bytes, l)) return s;
    if (nblocks == 0) return HYGT_OK;
    if (x == nullptr || y == nullptr || perm == nullptr) return HYGT_EINVAL;
    if (!aligned(x, 16) || !aligned(y, 16) || !aligned(perm, 4)) return HYGT_EINVAL;
    if (!overlap_ok(x, y, nblocks, log2n)) return HYGT_EINVAL;
    const hipError_t e = hygt::launch_rotate_perm(
        x, y, nblocks, log2n, rounds, nclasses, direction, perm, l,
        hygt::ws_ptrs(const_cast<void*>(workspace), l), stream);
    return e == hipSuccess ? HYGT_OK : HYGT_ELAUNCH;
}

int hygt_plan_codes(const int32_t* cls, int64_t nblocks, int log2n, int rounds,
                    const uint8_t* codes, int nclasses, void* workspace, size_t workspace_bytes,
                    hipStream_t stream) {
    if (nblocks > 0 && codes == nullptr) return HYGT_EINVAL;
    return plan_any(cls, nblocks, log2n, rounds, nullptr, codes, 0, nclasses, workspace,
                    workspace_bytes, stream);
}

int hygt_plan_int(const int32_t* cls, int64_t nblocks, int log2n, int rounds,
                  const uint8_t* codes, int nclasses, void* workspace, size_t workspace_bytes,
                  hipStream_t stream) {
    if (log2n < 2 || log2n > HYGT_INT_MAX_LOG2N) return HYGT_EINVAL;
    if (nblocks > 0 && codes == nullptr) return HYGT_EINVAL;
    return plan_any(cls, nblocks, log2n, rounds, nullptr, codes, 1, nclasses, workspace,
                    workspace_bytes, stream);
}

int hygt_apply_int(const int32_t* x, int32_t* y, int64_t nblocks, int log2n, int rounds,
                   int nclasses, int direction, const void* workspace, size_t workspace_bytes,
                   hipStream_t stream) {
    if (!sizes_ok(nblocks, log2n, rounds, nclasses)) return HYGT_EINVAL;
    if (log2n < 2 || log2n > HYGT_INT_MAX_LOG2N) return HYGT_EINVAL;
    if (direction != HYGT_FORWARD && direction != HYGT_INVERSE) return HYGT_EINVAL;
    const WsLayout l = hygt::ws_layout(nblocks, log2n, rounds, nclasses);
    if (int s = check_workspace(workspace, workspace_bytes, l)) return s;
    if (nblocks == 0) return HYGT_OK;
    if (x == nullptr || y == nullptr) return HYGT_EINVAL;
    if (!aligned(x, 16) || !aligned(y, 16)) return HYGT_EINVAL;
    const float* xf = reinterpret_cast<const float*>(x);
    if (!overlap_ok(xf, reinterpret_cast<const float*>(y), nblocks, log2n)) return HYGT_EINVAL;
    const hipError_t e = hygt::launch_rotate_int(
        x, y, nblocks, log2n, rounds, nclasses, direction, l,
        hygt::ws_ptrs(const_cast<void*>(workspace), l), stream);
    return e == hipSuccess ? HYGT_OK : HYGT_ELAUNCH;
}

size_t hygt_mixed_workspace_bytes(const hygt_segment* segs, int nseg) {
    if (check_segments(segs, nseg)) return 0;
    return mixed_layout(segs, nseg, nullptr);
}

int hygt_mixed_plan(const hygt_segment* segs, int nseg, void* workspace, size_t workspace_bytes,
                    hipStream_t stream) {
    return mixed_plan_impl(segs, nseg, workspace, workspace_bytes, stream);
}

int hygt_mixed_regroup(const hygt_segment* segs, int nseg, void* workspace,
                       size_t workspace_bytes, hipStream_t stream) {
    return mixed_plan_impl(segs, nseg, workspace, workspace_bytes, stream, false);
}

int hygt_mixed_num_configs(void) { return hygt::kMixedConfigs; }

int hygt_mixed_apply(const hygt_segment* segs, int nseg, int direction, int config,
                     const void* workspace, size_t workspace_bytes, hipStream_t stream) {
    return mixed_apply_impl(segs, nseg, direction, config, workspace, workspace_bytes, stream);
}

int hygt_mixed_autotune(const hygt_segment* segs, int nseg, int direction,
                        const void* workspace, size_t workspace_bytes, hipStream_t stream,
                        int* best_config, float* best_us) {
    if (best_config == nullptr || best_us == nullptr) return HYGT_EINVAL;
    // argument errors surface from the first apply, before any timing
    if (int s = mixed_apply_impl(segs, nseg, direction, 0, workspace, workspace_bytes, stream))
        return s;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return HYGT_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return HYGT_EHIP;
    }
    int status = HYGT_OK;
    float best = -1.0f;
    int best_k = 0;
    constexpr int kReps = 3;
    for (int k = 0; k < hygt::kMixedConfigs && status == HYGT_OK; ++k) {
        status = mixed_apply_impl(segs, nseg, direction, k, workspace, workspace_bytes, stream);
        if (status) break;
        if (hipEventRecord(e0, stream) != hipSuccess) { status = HYGT_EHIP; break; }
        for (int r = 0; r < kReps && status == HYGT_OK; ++r)
            status = mixed_apply_impl(segs, nseg, direction, k, workspace, workspace_bytes,
                                      stream);
        if (status) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            status = HYGT_EHIP;
            break;
        }
        const float us = ms * 1000.0f / kReps;
        if (best < 0.0f || us < best) {
            best = us;
            best_k = k;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status == HYGT_OK) {
        *best_config = best_k;
        *best_us = best;
    }
    return status;
}

int hygt_mixed_graph_create(const hygt_segment* segs, int nseg, int direction, int config,
                            void* workspace, size_t workspace_bytes, hipStream_t capture_stream,
                            hygt_graph* graph) {
    if (graph == nullptr || capture_stream == nullptr) return HYGT_EINVAL;
    *graph = nullptr;
    if (direction != HYGT_FORWARD && direction != HYGT_INVERSE) return HYGT_EINVAL;
    if (config < 0 || config >= hygt::kMixedConfigs) return HYGT_EINVAL;
    hygt::MixedArgs a;
    if (int s = mixed_args(segs, nseg, workspace, workspace_bytes, &a)) return s;
    if (hipStreamBeginCapture(capture_stream, hipStreamCaptureModeRelaxed) != hipSuccess)
        return HYGT_EHIP;
    int status = mixed_plan_impl(segs, nseg, workspace, workspace_bytes, capture_stream);
    if (status == HYGT_OK)
        status = mixed_apply_impl(segs, nseg, direction, config, workspace, workspace_bytes,
                                  capture_stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(capture_stream, &g);
    if (status == HYGT_OK && ec != hipSuccess) status = HYGT_EHIP;
    if (status != HYGT_OK) {
        if (g) (void)hipGraphDestroy(g);
        return status;
    }
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return HYGT_EHIP;
    }
    auto* h = new (std::nothrow) hygt_graph_s;
    if (h == nullptr) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(g);
        return HYGT_EHIP;
    }
    h->graph = g;
    h->exec = exec;
    *graph = h;
    return HYGT_OK;
}

int hygt_graph_launch(hygt_graph graph, hipStream_t stream) {
    if (graph == nullptr) return HYGT_EINVAL;
    return hipGraphLaunch(graph->exec, stream) == hipSuccess ? HYGT_OK : HYGT_ELAUNCH;
}

int hygt_graph_destroy(hygt_graph graph) {
    if (graph == nullptr) return HYGT_OK;
    int status = HYGT_OK;
    if (hipGraphExecDestroy(graph->exec) != hipSuccess) status = HYGT_EHIP;
    if (hipGraphDestroy(graph->graph) != hipSuccess) status = HYGT_EHIP;
    delete graph;
    return status;
}

size_t hygt_table_bytes(int log2n, int rounds, int nclasses) {
    if (log2n < 2 || log2n > HYGT_MAX_LOG2N || rounds < 1 || rounds > HYGT_MAX_ROUNDS ||
        nclasses < 1 || nclasses > HYGT_MAX_CLASSES)
        return 0;
    return hygt::table_layout(log2n, rounds, nclasses).total;
}

int hygt_table_build(const float* angles, int log2n, int rounds, int nclasses, void* table,
                     size_t table_bytes, hipStream_t stream) {
    const size_t need = hygt_table_bytes(log2n, rounds, nclasses);
    if (need == 0 || angles == nullptr || !aligned(angles, 4)) return HYGT_EINVAL;
    if (table == nullptr || table_bytes < need || !aligned(table, 256)) return HYGT_EWORKSPACE;
    const hipError_t e = hygt::launch_table_build(angles, log2n, rounds, nclasses,
                                                  hygt::table_layout(log2n, rounds, nclasses),
                                                  table, stream);
    return e == hipSuccess ? HYGT_OK : HYGT_ELAUNCH;
}

int hygt_requests_apply(hygt_request* ring, int64_t capacity, int64_t first, int count,
                        const hygt_table_ref* tables, int ntables, int direction,
                        hipStream_t stream) {
    if (direction != HYGT_FORWARD && direction != HYGT_INVERSE) return HYGT_EINVAL;
    if (ring == nullptr || !aligned(ring, 8) || capacity < 1 || first < 0 || count < 1 ||
        count > HYGT_MAX_BATCH_REQUESTS || count > capacity)
        return HYGT_EINVAL;
    if (tables == nullptr || ntables < 1 || ntables > HYGT_MAX_TABLES) return HYGT_EINVAL;
    hygt::RequestArgs a{};
    for (int i = 0; i < ntables; ++i) {
        const hygt_table_ref& t = tables[i];
        if (hygt_table_bytes(t.log2n, t.rounds, t.nclasses) == 0 || t.table == nullptr ||
            !aligned(t.table, 256))
            return HYGT_EINVAL;
        const hygt::TableLayout l = hygt::table_layout(t.log2n, t.rounds, t.nclasses);
        const char* b = static_cast<const char*>(t.table);
        a.tab[i].modes = reinterpret_cast<const int32_t*>(b + l.modes);
        a.tab[i].coef = reinterpret_cast<const float*>(b + l.coef);
        a.tab[i].signs = reinterpret_cast<const float*>(b + l.signs);
        a.tab[i].log2n = t.log2n;
        a.tab[i].rounds = t.rounds;
        a.tab[i].nclasses = t.nclasses;
    }
    first %= capacity;
    // every entry is checked before any is written or anything launched
    for (int i = 0; i < count; ++i) {
        const hygt_request& e = ring[(first + i) % capacity];
        if (e.table < 0 || e.table >= ntables) return HYGT_EINVAL;
        if (e.nblocks < 0 || e.nblocks > HYGT_MAX_REQUEST_BLOCKS) return HYGT_EINVAL;
        if (e.nblocks == 0) continue;
        const hygt_table_ref& t = tables[e.table];
        if (e.x == nullptr || e.y == nullptr || !aligned(e.x, 16) || !aligned(e.y, 16))
            return HYGT_EINVAL;
        if (!overlap_ok(e.x, e.y, e.nblocks, t.log2n)) return HYGT_EINVAL;
        if (e.cls == nullptr ? t.nclasses != 1 : !aligned(e.cls, 4)) return HYGT_EINVAL;
    }
    // The batch's descriptors go to the launch by value (the kernel reads
    // them from its argument segment); only the statuses are written back
    // into the ring by the device.
    int64_t wgs = 0;
    for (int i = 0; i < count; ++i) {
        hygt_request& e = ring[(first + i) % capacity];
        e.first_wg = wgs;
        hygt::ReqDesc& q = a.req[i];
        q.x = e.x;
        q.y = e.y;
        q.cls = e.cls;
        q.nblocks = static_cast<int32_t>(e.nblocks);
        q.table = e.table;
        q.first_wg = static_cast<int32_t>(wgs);
        q.entry = i;
        wgs += hygt::request_workgroups(e.nblocks, tables[e.table].log2n);
    }
    if (wgs == 0) return HYGT_OK;
    // The device's address of the ring; fails (and nothing is launched) for
    // memory that is not pinned, device-accessible host memory.
    void* dring = nullptr;
    if (hipHostGetDevicePointer(&dring, ring, 0) != hipSuccess || dring == nullptr) {
        (void)hipGetLastError();  // clear the error this leaves behind
        return HYGT_EINVAL;
    }
    a.status = reinterpret_cast<int32_t*>(static_cast<char*>(dring) +
                                          offsetof(hygt_request, status));
    a.capacity = capacity;
    a.first = first;
    a.count = count;
    a.ntables = ntables;
    const hipError_t err = hygt::launch_requests(a, wgs, direction, stream);
    return err == hipSuccess ? HYGT_OK : HYGT_ELAUNCH;
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
        case HYGT_ESCRATCH: return "the sizes need more workspace than the static scratch area of hygt_transform_noalloc() holds";
        default: return "unknown status";
    }
}

}  // extern "C"

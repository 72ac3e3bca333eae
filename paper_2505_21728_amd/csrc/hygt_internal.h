// Internal declarations shared by the HyGT library's translation units:
// the workspace layout, the device-side plan header and the kernel launchers.
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

namespace hygt {

// Blocks per tile: one wavefront lane per block.
constexpr int kTile = 64;
// Blocks whose classes one histogram / scatter workgroup handles.
constexpr int kChunk = 4096;
// Threads per workgroup of the histogram and scatter kernels.
constexpr int kPlanThreads = 256;
// Threads per workgroup of the multiplier-table kernel (>= N/2 for N <= 256).
constexpr int kTableThreads = 128;

// A class uses the scaled schedule only if every per-element scale factor
// stays in [2^-kScaleExp, 1]; stored values are then at most 2^kScaleExp times
// the block norm.
constexpr int kScaleExp = 64;

// Device-side header at the start of the workspace.
struct alignas(256) PlanHeader {
    int32_t err;     // bit 0: a class index was out of range
    int32_t ntiles;  // tiles written by the grouping (grouped plans only)
    int32_t ticket;  // completion counter of the histogram kernel
    int32_t grouped; // 1: tiles come from the class grouping; 0: identity tiles
    int32_t pad[60];
};

struct WsLayout {
    size_t hdr = 0;          // PlanHeader
    size_t counts = 0;       // int32 [C]   blocks per class
    size_t cursor = 0;       // int32 [C]   scatter cursors
    size_t class_start = 0;  // int32 [C+1] first grouped position of each class
    size_t tile_start = 0;   // int32 [C+1] first tile of each class
    size_t tiles = 0;        // int4  [max_tiles] {class, first, count, 0}
    size_t perm = 0;         // int32 [nblocks] block ids grouped by class
    size_t modes = 0;        // int32 [2][C] 1 = direct schedule, 0 = scaled schedule
    size_t coef = 0;         // float [2][C][P][2N] per-pass multipliers
    size_t total = 0;
    int64_t max_tiles = 0;
    int64_t nhist = 0;       // histogram / scatter workgroups
    int passes = 0;
    int n = 0;
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline WsLayout ws_layout(int64_t nblocks, int log2n, int rounds, int nclasses) {
    WsLayout l;
    l.n = 1 << log2n;
    l.passes = rounds * log2n;
    const size_t C = static_cast<size_t>(nclasses);
    // A grouped plan has at most one partial tile per class.
    l.max_tiles = (nblocks + kTile - 1) / kTile + nclasses;
    l.nhist = (nblocks + kChunk - 1) / kChunk;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    l.hdr = take(sizeof(PlanHeader));
    l.counts = take(C * 4);
    l.cursor = take(C * 4);
    l.class_start = take((C + 1) * 4);
    l.tile_start = take((C + 1) * 4);
    l.tiles = take(static_cast<size_t>(l.max_tiles) * 16);
    l.perm = take(static_cast<size_t>(nblocks) * 4);
    l.modes = take(2 * C * 4);
    l.coef = take(2 * C * static_cast<size_t>(l.passes) * 2 * l.n * 4);
    l.total = off;
    return l;
}

// Pointers into one workspace.
struct WsPtrs {
    PlanHeader* hdr;
    int32_t* counts;
    int32_t* cursor;
    int32_t* class_start;
    int32_t* tile_start;
    int4* tiles;
    int32_t* perm;
    int32_t* modes;
    float* coef;
};

inline WsPtrs ws_ptrs(void* ws, const WsLayout& l) {
    char* b = static_cast<char*>(ws);
    WsPtrs p;
    p.hdr = reinterpret_cast<PlanHeader*>(b + l.hdr);
    p.counts = reinterpret_cast<int32_t*>(b + l.counts);
    p.cursor = reinterpret_cast<int32_t*>(b + l.cursor);
    p.class_start = reinterpret_cast<int32_t*>(b + l.class_start);
    p.tile_start = reinterpret_cast<int32_t*>(b + l.tile_start);
    p.tiles = reinterpret_cast<int4*>(b + l.tiles);
    p.perm = reinterpret_cast<int32_t*>(b + l.perm);
    p.modes = reinterpret_cast<int32_t*>(b + l.modes);
    p.coef = reinterpret_cast<float*>(b + l.coef);
    return p;
}

// Kernel launchers (hygt_plan.hip, hygt_rotate.hip). Each returns the
// hipError_t of its launches.
hipError_t launch_plan(const int32_t* cls, int64_t nblocks, int log2n, int rounds,
                       const float* angles, int nclasses, const WsLayout& l,
                       const WsPtrs& p, hipStream_t stream);

hipError_t launch_rotate(const float* x, float* y, int64_t nblocks, int log2n, int rounds, int nclasses, int direction,
                         const WsLayout& l, const WsPtrs& p, hipStream_t stream);

}  // namespace hygt

// Internal declarations shared by the HyGT library's translation units:
// the workspace layout, the device-side plan header and the kernel launchers.
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

namespace hygt {

// Blocks per tile: one wavefront lane per block.
constexpr int kTile = 64;
// Chunks of consecutive blocks counted and placed by one plan workgroup each:
// at least 4096 blocks, at most kMaxChunks chunks.
constexpr int64_t kMinChunk = 4096;
constexpr int64_t kMaxChunks = 1024;
// Threads per plan workgroup (>= N/2 for the table builders, N <= 256).
constexpr int kPlanThreads = 256;
// The interleaved tile order (see WsLayout::interleave) is used up to this
// many classes and table entries per chunk; each entry costs the placing
// launch O(nclasses) work.
constexpr int kInterleaveMaxClasses = 64;
constexpr int64_t kInterleaveMaxEntries = 2048;
// Hypercube dimensions kept inside one wavefront lane: a lane holds at most
// 64 values, so for N = 128 (256) two (four) wavefronts share each tile,
// wavefront q holding values 64q .. 64q+63 of every block, and the passes
// along bits 6 and 7 pair values of different wavefronts. Those passes use
// the plain (cos, sin) form of the rotation, the others the lifting form
// (see hygt_plan.hip).
constexpr int kLaneBits = 6;

// Device-side header at the start of the workspace.
struct alignas(256) PlanHeader {
    int32_t nchunks;  // chunks of the last non-empty plan
    int32_t pad[63];
};

struct WsLayout {
    size_t hdr = 0;          // PlanHeader
    size_t chunk_err = 0;    // int32 [nchunks] bit 0: a class index was out of range
    size_t counts = 0;       // int32 [nchunks][C] blocks of each class in each chunk
    size_t tile_class = 0;   // int32 [max_tiles] class of each tile, -1 past the last
    size_t perm = 0;         // int32 [max_tiles][64] block ids of each tile, -1 = empty lane
    size_t modes = 0;        // int32 [2][C] 1 = some output needs a final sign flip
    size_t coef = 0;         // float [2][C][P][N] per-pass multipliers (two per pair)
    size_t signs = 0;        // float [2][C][N] final sign (+1 / -1) of each output
    // the backward's own inverse-direction tables, built from its angles:
    size_t bcoef = 0;        // float [C][P][N] lifting multipliers, application order
    size_t bflip = 0;        // uint32 [C][P] pairs whose stored signs differ, per pass
    size_t bsigns = 0;       // float [C][N] final signs
    size_t bmodes = 0;       // int32 [C] 1 = some final sign is -1
    size_t total = 0;
    int64_t nchunks = 0;
    int64_t chunk = 0;       // blocks per chunk (a multiple of 256)
    int64_t max_tiles = 0;
    // Tile order of the plan: 0 = class by class; > 0 = the tiles of all
    // classes interleaved by tile index (round i holds tile i of every class
    // that has one), with room for this many (class, tile index) entries per
    // chunk in the placing launch's table.
    int64_t interleave = 0;
    int passes = 0;
    int n = 0;
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline WsLayout ws_layout(int64_t nblocks, int log2n, int rounds, int nclasses) {
    WsLayout l;
    l.n = 1 << log2n;
    l.passes = rounds * log2n;
    const size_t C = static_cast<size_t>(nclasses);
    int64_t nch = (nblocks + kMinChunk - 1) / kMinChunk;
    if (nch > kMaxChunks) nch = kMaxChunks;
    if (nch < 1) nch = 1;
    l.chunk = static_cast<int64_t>(align_up(static_cast<size_t>((nblocks + nch - 1) / nch), 256));
    if (l.chunk < 256) l.chunk = 256;
    l.nchunks = (nblocks + l.chunk - 1) / l.chunk;
    // Classes are grouped over the whole batch: at most one partly filled
    // tile per class.
    l.max_tiles = (nblocks + kTile - 1) / kTile + static_cast<int64_t>(nclasses);
    // A chunk's blocks of class c have consecutive ranks in the class, so they
    // fall in at most cnt_c / 64 + 2 of its tiles.
    const int64_t entries = l.chunk / kTile + 2 * static_cast<int64_t>(nclasses) + 1;
    if (nclasses <= kInterleaveMaxClasses && entries <= kInterleaveMaxEntries)
        l.interleave = entries;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    l.hdr = take(sizeof(PlanHeader));
    l.chunk_err = take(static_cast<size_t>(l.nchunks) * 4);  // always at offset 256
    l.counts = take(static_cast<size_t>(l.nchunks) * C * 4);
    l.tile_class = take(static_cast<size_t>(l.max_tiles) * 4);
    l.perm = take(static_cast<size_t>(l.max_tiles) * kTile * 4);
    l.modes = take(2 * C * 4);
    l.coef = take(2 * C * static_cast<size_t>(l.passes) * l.n * 4);
    l.signs = take(2 * C * static_cast<size_t>(l.n) * 4);
    l.bcoef = take(C * static_cast<size_t>(l.passes) * l.n * 4);
    l.bflip = take(C * static_cast<size_t>(l.passes) * 4);
    l.bsigns = take(C * static_cast<size_t>(l.n) * 4);
    l.bmodes = take(C * 4);
    l.total = off;
    return l;
}

// Pointers into one workspace.
struct WsPtrs {
    PlanHeader* hdr;
    int32_t* chunk_err;
    int32_t* counts;
    int32_t* tile_class;
    int32_t* perm;
    int32_t* modes;
    float* coef;
    float* signs;
    float* bcoef;
    uint32_t* bflip;
    float* bsigns;
    int32_t* bmodes;
};

inline WsPtrs ws_ptrs(void* ws, const WsLayout& l) {
    char* b = static_cast<char*>(ws);
    WsPtrs p;
    p.hdr = reinterpret_cast<PlanHeader*>(b + l.hdr);
    p.chunk_err = reinterpret_cast<int32_t*>(b + l.chunk_err);
    p.counts = reinterpret_cast<int32_t*>(b + l.counts);
    p.tile_class = reinterpret_cast<int32_t*>(b + l.tile_class);
    p.perm = reinterpret_cast<int32_t*>(b + l.perm);
    p.modes = reinterpret_cast<int32_t*>(b + l.modes);
    p.coef = reinterpret_cast<float*>(b + l.coef);
    p.signs = reinterpret_cast<float*>(b + l.signs);
    p.bcoef = reinterpret_cast<float*>(b + l.bcoef);
    p.bflip = reinterpret_cast<uint32_t*>(b + l.bflip);
    p.bsigns = reinterpret_cast<float*>(b + l.bsigns);
    p.bmodes = reinterpret_cast<int32_t*>(b + l.bmodes);
    return p;
}

// Kernel launchers (hygt_plan.hip, hygt_rotate.hip, hygt_backward.hip, hygt_dense.hip). Each returns the
// hipError_t of its launches.
// Exactly one of angles (FP32 radians) and codes (8-bit codes) is non-NULL.
hipError_t launch_plan(const int32_t* cls, int64_t nblocks, int log2n, int rounds,
                       const float* angles, const uint8_t* codes, int integer, int nclasses,
                       const WsLayout& l, const WsPtrs& p, hipStream_t stream);

// Segments (block sizes) of a mixed batch, at most.
constexpr int kMaxSegments = 4;

// One batch (block size) of a fused mixed plan: its inputs, its part of the
// workspace, and the first workgroup index of its share of either launch.
struct PlanSeg {
    const int32_t* cls;
    const float* angles;
    PlanHeader* hdr;
    int32_t* chunk_err;
    int32_t* counts;
    int32_t* tile_class;
    int32_t* perm;
    int32_t* modes;
    float* coef;
    float* signs;
    int64_t nblocks;
    int64_t nchunks;
    int64_t chunk;
    int64_t max_tiles;
    int64_t count_begin;  // first workgroup of launch A (counting)
    int64_t place_begin;  // first workgroup of launch B (tables if built, then placing)
    int64_t interleave;   // WsLayout::interleave
    int log2n;
    int rounds;
    int nclasses;
    int pad;
};

struct PlanArgs {
    PlanSeg seg[kMaxSegments];
    int nseg;
    int tables;  // 1: the placing launch also builds every segment's multiplier tables
};

// The plans of every segment with blocks in two launches of count_wgs and
// place_wgs workgroups (hygt_plan.hip).
hipError_t launch_plan_mixed(const PlanArgs& a, int64_t count_wgs, int64_t place_wgs,
                             hipStream_t stream);

// Integer arithmetic: multipliers with kIntFracBits fractional bits, outputs
// rounded by adding half a unit and shifting right (floor).
constexpr int kIntFracBits = 14;
constexpr double kIntOne = 16384.0;  // 2^kIntFracBits

// The integer transform (hygt_rotate.hip) on int32 blocks, 4 <= N <= 64,
// with tables built by launch_plan(integer = 1).
hipError_t launch_rotate_int(const int32_t* x, int32_t* y, int64_t nblocks, int log2n,
                             int rounds, int nclasses, int direction, const WsLayout& l,
                             const WsPtrs& p, hipStream_t stream);

hipError_t launch_rotate(const float* x, float* y, int64_t nblocks, int log2n, int rounds,
                         int nclasses, int direction, const WsLayout& l, const WsPtrs& p,
                         hipStream_t stream);

// The transform with the permutation pass of Fig. 4 (hygt_rotate.hip), 4 <= N <= 64.
hipError_t launch_rotate_perm(const float* x, float* y, int64_t nblocks, int log2n, int rounds,
                              int nclasses, int direction, const int32_t* outperm,
                              const WsLayout& l, const WsPtrs& p, hipStream_t stream);

// Reverse-mode derivative of the forward transform (hygt_backward.hip), N <= 64.
hipError_t launch_backward(const float* y, const float* gy, float* gx, float* gangles,
                           int64_t nblocks, int log2n, int rounds, const float* angles,
                           int nclasses, const WsLayout& l, const WsPtrs& p, hipStream_t stream);

// Mixed batches: several block sizes, each a segment with its own plan,
// transformed by one persistent launch (hygt_rotate.hip).
struct MixedSeg {
    const float* x;
    float* y;
    int64_t nblocks;
    int64_t max_tiles;
    const int32_t* tile_class;
    const int32_t* perm;
    const int32_t* modes;
    const float* coef;
    const float* signs;
    int64_t item_begin;  // first work item of the segment in the launch
    int64_t items;       // work items: 4 tiles (N <= 128) or 2 tiles (N = 256)
    int log2n;
    int rounds;
    int nclasses;
    int pad;
};
struct MixedArgs {
    MixedSeg seg[kMaxSegments];
    int64_t total_items;
    int nseg;
    int pad;
};
// Launch configurations of the mixed kernel (see mixed_config()).
constexpr int kMixedConfigs = 8;
int64_t mixed_items(int log2n, int64_t max_tiles);
hipError_t launch_mixed(const MixedArgs& a, int direction, int config, hipStream_t stream);

// hygt_forward() / hygt_inverse() on a given workspace (hygt_abi.cpp): host
// checks, plan, apply; returns a hygt_status.
int transform_in_workspace(const float* x, float* y, const int32_t* cls, int64_t nblocks,
                           int log2n, int rounds, const float* angles, int nclasses,
                           int direction, void* ws, size_t ws_bytes, hipStream_t stream);

// A stand-alone multiplier table of one block size (hygt_table_build()):
// the modes, coef and signs parts of a workspace, for both directions.
struct TableLayout {
    size_t modes = 0;  // int32 [2][C]
    size_t coef = 0;   // float [2][C][P][N]
    size_t signs = 0;  // float [2][C][N]
    size_t total = 0;
    int passes = 0;
    int n = 0;
};

inline TableLayout table_layout(int log2n, int rounds, int nclasses) {
    TableLayout t;
    t.n = 1 << log2n;
    t.passes = rounds * log2n;
    const size_t C = static_cast<size_t>(nclasses);
    t.modes = 0;
    t.coef = align_up(2 * C * 4, 256);
    t.signs = align_up(t.coef + 2 * C * static_cast<size_t>(t.passes) * t.n * 4, 256);
    t.total = align_up(t.signs + 2 * C * static_cast<size_t>(t.n) * 4, 256);
    return t;
}

// Builds the tables of both directions into `table` (hygt_plan.hip).
hipError_t launch_table_build(const float* angles, int log2n, int rounds, int nclasses,
                              const TableLayout& t, void* table, hipStream_t stream);

// One table of a request launch, with its parts resolved.
struct ReqTable {
    const int32_t* modes;
    const float* coef;
    const float* signs;
    int log2n;
    int rounds;
    int nclasses;
    int pad;
};

// One request of a launch, copied from its ring entry by the host.
struct ReqDesc {
    const float* x;
    float* y;
    const int32_t* cls;
    int32_t nblocks;   // <= 2^26
    int32_t table;
    int32_t first_wg;  // first workgroup of the request in its launch
    int32_t entry;     // its ring entry: first + entry (mod capacity)
};

// Arguments of a request launch (hygt_rotate.hip): the batch's descriptors
// travel with the launch, so that the kernel reads them from its argument
// segment rather than from host memory; `status` is the device's address
// of ring entry 0's status field (entries are 12 int32 apart), where a
// request with a class out of range gets HYGT_ECLASS.
constexpr int kMaxReqTables = 4;
constexpr int kMaxBatchRequests = 64;
struct RequestArgs {
    int32_t* status;
    int64_t capacity;
    int64_t first;  // ring index of the batch's first entry (< capacity)
    int count;
    int ntables;
    ReqTable tab[kMaxReqTables];
    ReqDesc req[kMaxBatchRequests];
};
static_assert(sizeof(RequestArgs) <= 4096, "kernel arguments");

// Workgroups (of four wavefronts) of a request of nblocks blocks of 2^log2n
// values: a wavefront takes one block for N >= 64 and 64 / N blocks for
// N <= 32.
inline int64_t request_workgroups(int64_t nblocks, int log2n) {
    if (log2n >= kLaneBits) return (nblocks + 3) / 4;
    const int64_t per = 4 * (int64_t{64} >> log2n);  // blocks per workgroup
    return (nblocks + per - 1) / per;
}

hipError_t launch_requests(const RequestArgs& a, int64_t workgroups, int direction,
                           hipStream_t stream);

// Dense per-class transform (hygt_dense.hip), N = 64.
hipError_t launch_dense(const float* x, float* y, int64_t nblocks, const unsigned short* mats,
                        const WsLayout& l, const WsPtrs& p, hipStream_t stream);

}  // namespace hygt

// Plan kernels: per-class multiplier tables and the grouping of blocks into
// class-uniform tiles.
//
// Multiplier tables: one workgroup per (direction, class) runs the table
// builder of hygt_table.h (FP64 conversion into lifting multipliers, with
// the sign bookkeeping of the angle reduction).
//
// Grouping. A tile is 64 blocks of one class, so that a wavefront (one lane
// per block) reads one class table with scalar loads. Tiles are sorted by
// class over the whole batch, so that the wavefronts of a compute unit pair
// mostly share one class and its table stays in their scalar cache. The
// counting sort takes two launches over chunks of consecutive blocks: the
// first counts the classes of each chunk, the second gives every chunk its
// start inside each class from the counts of the chunks before it and
// scatters the block ids into the class's tiles, while other workgroups of
// the same launch build the multiplier tables.

#include <algorithm>
#include <cmath>

#include "hygt.h"
#include "hygt_internal.h"
#include "hygt_table.h"

namespace hygt {
namespace {

using table::build_table;
using table::code_angle;
using table::TableShared;

// Entries of the per-chunk class counts cached in LDS by the placing kernel.
constexpr int kCountsCache = 16384;
// Blocks whose class indices one thread loads at once (a whole chunk of
// kMinChunk blocks in one round of loads).
constexpr int kUnroll = static_cast<int>(kMinChunk / kPlanThreads);

// LDS of a chunk counter (the counting launch).
struct CountShared {
    int hist[HYGT_MAX_CLASSES];
    int flag;
};

// LDS of the placing launch, sized at launch time for the class count:
// the cached per-chunk counts (when they fit), then per class the blocks in
// the batch, the blocks in earlier chunks, the blocks placed so far and the
// first tile, then the scan scratch.
struct PlaceLds {
    int* counts;
    int* total;
    int* pre;
    int* pos;
    int* tile_base;  // [C + 1]
    int* scan;       // [kPlanThreads]
};

__host__ __device__ inline bool place_counts_cached(int64_t nchunks, int nclasses) {
    return nchunks * nclasses <= kCountsCache;
}

__host__ __device__ inline size_t place_lds_bytes(int64_t nchunks, int nclasses) {
    const size_t cached = place_counts_cached(nchunks, nclasses)
                              ? static_cast<size_t>(nchunks) * nclasses : 0;
    const size_t place = (cached + 4 * static_cast<size_t>(nclasses) + 1 + kPlanThreads) *
                         sizeof(int);
    return place > sizeof(TableShared) ? place : sizeof(TableShared);
}

__device__ inline PlaceLds place_lds(int* base, int64_t nchunks, int nclasses) {
    PlaceLds l;
    l.counts = base;
    int* p = base + (place_counts_cached(nchunks, nclasses) ? nchunks * nclasses : 0);
    l.total = p;
    l.pre = p + nclasses;
    l.pos = p + 2 * nclasses;
    l.tile_base = p + 3 * nclasses;
    l.scan = p + 4 * nclasses + 1;
    return l;
}

// Integer tables (Fig. 6 with integer arithmetic): for every pair, in the
// passes' application order, the fixed-point multipliers
// (C, S) = (round(2^14 cos th), round(2^14 sin th)) of its code's angle th
// (negated for the inverse, eq. (9)), stored as two int32 in the slots of the
// lifting pair. No sign bookkeeping: the signs stay +1.
__device__ void build_table_int(int dir, int c, const uint8_t* __restrict__ codes, int log2n,
                                int rounds, int nclasses, float* __restrict__ coef,
                                float* __restrict__ signs, int32_t* __restrict__ modes) {
    const int n = 1 << log2n;
    const int half = n >> 1;
    const int passes = rounds * log2n;
    const size_t table = static_cast<size_t>(dir) * nclasses + c;
    int32_t* cbase = reinterpret_cast<int32_t*>(coef) + table * passes * n;
    for (int e = threadIdx.x; e < passes * half; e += blockDim.x) {
        const int p = e / half;
        const int j = e % half;
        const int kk = p % log2n, rr = p / log2n;
        const int k = dir ? log2n - 1 - kk : kk;
        const int r = dir ? rounds - 1 - rr : rr;
        const size_t ai = ((static_cast<size_t>(c) * rounds + r) * log2n + k) * half + j;
        double th = code_angle(codes[ai]);
        if (dir) th = -th;
        cbase[static_cast<size_t>(p) * n + 2 * j + 0] = static_cast<int32_t>(rint(kIntOne * cos(th)));
        cbase[static_cast<size_t>(p) * n + 2 * j + 1] = static_cast<int32_t>(rint(kIntOne * sin(th)));
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) signs[table * n + i] = 1.0f;
    if (threadIdx.x == 0) modes[table] = 0;
}

// Tiles of a class of `count` blocks: whole tiles of 64, rounded up to a
// multiple of the tiles a rotation wavefront takes at once.
__device__ __forceinline__ int class_tiles(int count) {
    const int t = (count + kTile - 1) / kTile;
    return (t + kTilesPerWave - 1) / kTilesPerWave * kTilesPerWave;
}

// Exclusive scan of one int per thread over the workgroup; returns the
// thread's prefix and sets *total.
__device__ int block_exclusive_scan(int v, int* sh, int* total) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < static_cast<int>(blockDim.x); off <<= 1) {
        const int add = tid >= off ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += add;
        __syncthreads();
    }
    const int incl = sh[tid];
    *total = sh[blockDim.x - 1];
    __syncthreads();
    return incl - v;
}

// Class counts of chunk k -> counts[k][c]; out-of-range classes set
// chunk_err[k]. Without class indices every block is class 0.
__device__ void count_chunk(CountShared& sh, int64_t k, const int32_t* __restrict__ cls,
                            int64_t nblocks, int64_t chunk, int nclasses,
                            int32_t* __restrict__ counts, int32_t* __restrict__ chunk_err) {
    const int tid = threadIdx.x;
    const int64_t start = k * chunk;
    const int cnt = static_cast<int>(min<int64_t>(chunk, nblocks - start));
    for (int c = tid; c < nclasses; c += blockDim.x) sh.hist[c] = 0;
    if (tid == 0) sh.flag = 0;
    __syncthreads();
    if (cls != nullptr) {
        // kUnroll class loads in flight per thread before the LDS atomics
        const int step = static_cast<int>(blockDim.x) * kUnroll;
        for (int i0 = tid; i0 < cnt; i0 += step) {
            int cv[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int i = i0 + u * static_cast<int>(blockDim.x);
                cv[u] = i < cnt ? cls[start + i] : 0;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int i = i0 + u * static_cast<int>(blockDim.x);
                if (i >= cnt) break;
                if (cv[u] >= 0 && cv[u] < nclasses)
                    atomicAdd(&sh.hist[cv[u]], 1);
                else
                    sh.flag = 1;
            }
        }
    } else if (tid == 0) {
        sh.hist[0] = cnt;
    }
    __syncthreads();
    for (int c = tid; c < nclasses; c += blockDim.x)
        counts[k * nclasses + c] = sh.hist[c];
    if (tid == 0) chunk_err[k] = sh.flag;
}

// Launch A: workgroup k counts chunk k.
__global__ __launch_bounds__(kPlanThreads) void plan_count_kernel(
    const int32_t* __restrict__ cls, int64_t nblocks, int nclasses, int64_t nchunks,
    int64_t chunk, PlanHeader* __restrict__ hdr, int32_t* __restrict__ chunk_err,
    int32_t* __restrict__ counts) {
    __shared__ CountShared sh;
    const int64_t k = blockIdx.x;
    if (k == 0 && threadIdx.x == 0) hdr->nchunks = static_cast<int32_t>(nchunks);
    count_chunk(sh, k, cls, nblocks, chunk, nclasses, counts, chunk_err);
}

// Table builder of workgroup w < 2C of a placing launch: (direction, class) =
// (w / C, w % C).
__device__ __forceinline__ void build_tables_wg(int* place_dyn, int w, const float* __restrict__ angles,
                                const uint8_t* __restrict__ codes, int log2n, int rounds,
                                int integer, int nclasses, int32_t* __restrict__ modes,
                                float* __restrict__ coef, float* __restrict__ signs) {
    if (integer) {
        build_table_int(w / nclasses, w % nclasses, codes, log2n, rounds, nclasses, coef, signs,
                        modes);
        return;
    }
    const int dir = w / nclasses, c = w % nclasses;
    const size_t t = static_cast<size_t>(w);  // = dir * nclasses + c
    const size_t passes = static_cast<size_t>(rounds) * log2n;
    build_table(*reinterpret_cast<TableShared*>(place_dyn), dir, c, angles, codes, log2n, rounds,
                coef + t * passes * (size_t{1} << log2n), signs + t * (size_t{1} << log2n),
                modes + t, nullptr);
}

// Places chunk k of one batch: its blocks' ids into their classes' tiles, and
// the class of this chunk's share of the tile list.
__device__ __forceinline__ void place_chunk(int* place_dyn, int64_t k, const int32_t* __restrict__ cls,
                            int64_t nblocks, int nclasses, int64_t nchunks, int64_t chunk,
                            int64_t max_tiles, const int32_t* __restrict__ counts,
                            int32_t* __restrict__ tile_class, int32_t* __restrict__ perm) {
    const PlaceLds sh = place_lds(place_dyn, nchunks, nclasses);
    const int tid = threadIdx.x;
    const int64_t ncounts = nchunks * nclasses;
    const bool cached = place_counts_cached(nchunks, nclasses);
    // The first round of this chunk's class indices, loaded now so that their
    // latency overlaps the count reduction below.
    const int64_t start = k * chunk;
    const int cnt = static_cast<int>(min<int64_t>(chunk, nblocks - start));
    int cv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const int i = tid + u * static_cast<int>(blockDim.x);
        cv[u] = (i < cnt && cls != nullptr) ? cls[start + i] : 0;
    }
    if (cached) {
        // 16-byte loads (counts starts 256-byte aligned), all in flight
        const int64_t n4 = ncounts / 4;
        const int4* c4 = reinterpret_cast<const int4*>(counts);
        int4* s4 = reinterpret_cast<int4*>(sh.counts);  // sh.counts is at the LDS base
#pragma unroll 16
        for (int64_t e = tid; e < n4; e += blockDim.x) s4[e] = c4[e];
        for (int64_t e = n4 * 4 + tid; e < ncounts; e += blockDim.x) sh.counts[e] = counts[e];
    }
    __syncthreads();
    // Per class: blocks in the whole batch and in the chunks before this one.
    // One wavefront per class at a time, its lanes striding over the chunks.
    {
        const int lane = tid & 63;
        const int wave = tid >> 6;
        const int nwaves = blockDim.x >> 6;
        for (int c = wave; c < nclasses; c += nwaves) {
            int total = 0, pre = 0;
            for (int64_t q = lane; q < nchunks; q += 64) {
                const int v = cached ? sh.counts[q * nclasses + c] : counts[q * nclasses + c];
                total += v;
                if (q < k) pre += v;
            }
            for (int off = 32; off > 0; off >>= 1) {
                total += __shfl_xor(total, off, 64);
                pre += __shfl_xor(pre, off, 64);
            }
            if (lane == 0) {
                sh.total[c] = total;
                sh.pre[c] = pre;
                sh.pos[c] = 0;
            }
        }
    }
    __syncthreads();
    // First tile of each class: exclusive scan of the per-class tile counts,
    // each thread owning a contiguous run of classes.
    const int per = (nclasses + blockDim.x - 1) / blockDim.x;
    const int c0 = min(tid * per, nclasses);
    const int c1 = min(c0 + per, nclasses);
    int run = 0;
    for (int c = c0; c < c1; ++c) run += class_tiles(sh.total[c]);
    int ntiles = 0;
    int base = block_exclusive_scan(run, sh.scan, &ntiles);
    for (int c = c0; c < c1; ++c) {
        sh.tile_base[c] = base;
        base += class_tiles(sh.total[c]);
    }
    if (tid == 0) sh.tile_base[nclasses] = ntiles;
    __syncthreads();
    // Block ids of this chunk into their classes' tiles.
    const int step = static_cast<int>(blockDim.x) * kUnroll;
    for (int i0 = tid; i0 < cnt; i0 += step) {
        if (i0 != tid) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int i = i0 + u * static_cast<int>(blockDim.x);
                cv[u] = (i < cnt && cls != nullptr) ? cls[start + i] : 0;
            }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int i = i0 + u * static_cast<int>(blockDim.x);
            const int c = cv[u];
            if (i < cnt && c >= 0 && c < nclasses) {
                const int p = sh.pre[c] + atomicAdd(&sh.pos[c], 1);
                const int64_t slot = static_cast<int64_t>(sh.tile_base[c]) * kTile + p;
                // Counts and classes agree unless cls changed between the two
                // plan launches; never write outside perm even then.
                if (slot < max_tiles * kTile) perm[slot] = static_cast<int32_t>(start + i);
            }
        }
    }
    // Class of every tile of this chunk's share of the tile list, and the
    // empty lanes of each class's last tile.
    const int64_t share = (max_tiles + nchunks - 1) / nchunks;
    const int64_t t0 = k * share;
    const int64_t t1 = min(t0 + share, max_tiles);
    for (int64_t t = t0 + tid; t < t1; t += blockDim.x) {
        if (t >= ntiles) {
            tile_class[t] = -1;
            continue;
        }
        // last class whose first tile is <= t (classes without blocks share
        // their first tile index with the next class)
        int lo = 0, hi = nclasses - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sh.tile_base[mid] <= t) lo = mid; else hi = mid - 1;
        }
        tile_class[t] = lo;
        const int used = sh.total[lo] - static_cast<int>(t - sh.tile_base[lo]) * kTile;
        for (int s2 = max(used, 0); s2 < kTile; ++s2) perm[t * kTile + s2] = -1;
    }
}


// Launch B: workgroups [0, 2C) build the multiplier tables of (direction,
// class), which need nothing from launch A, so they run beside the placing
// workgroups instead of before them; workgroup 2C + k places chunk k. Class
// c's blocks fill tiles tile_base[c] .. in chunk order; inside a chunk their
// order is that of the LDS counters (any order gives the same results,
// block by block).
__global__ __launch_bounds__(kPlanThreads) void plan_place_kernel(
    const int32_t* __restrict__ cls, int64_t nblocks, int nclasses, int64_t nchunks,
    int64_t chunk, int64_t max_tiles, const int32_t* __restrict__ counts,
    int32_t* __restrict__ tile_class, int32_t* __restrict__ perm,
    const float* __restrict__ angles, const uint8_t* __restrict__ codes, int log2n, int rounds,
    int integer, int32_t* __restrict__ modes,
    float* __restrict__ coef, float* __restrict__ signs) {
    extern __shared__ __align__(16) int place_dyn[];
    const int64_t w = blockIdx.x;
    if (w < 2 * nclasses) {
        build_tables_wg(place_dyn, static_cast<int>(w), angles, codes, log2n, rounds, integer,
                        nclasses, modes, coef, signs);
        return;
    }
    place_chunk(place_dyn, w - 2 * static_cast<int64_t>(nclasses), cls, nblocks, nclasses,
                nchunks, chunk, max_tiles, counts, tile_class, perm);
}

// The plans of up to HYGT_MAX_SEGMENTS batches (block sizes) in the same two
// launches: the workgroups of segment s follow those of the segments before
// it, in both launches, and each finds its segment by the first workgroup
// indices of the segments (wave-uniform, at most four compares).
__device__ __forceinline__ int plan_segment(const PlanArgs& a, int64_t w, bool place) {
    int s = 0;
    for (int i = 1; i < a.nseg; ++i)
        if (w >= (place ? a.seg[i].place_begin : a.seg[i].count_begin)) s = i;
    return s;
}

__global__ __launch_bounds__(kPlanThreads) void plan_count_mixed_kernel(PlanArgs a) {
    __shared__ CountShared sh;
    const int64_t w = blockIdx.x;
    const PlanSeg& g = a.seg[plan_segment(a, w, false)];
    const int64_t k = w - g.count_begin;
    if (k == 0 && threadIdx.x == 0) g.hdr->nchunks = static_cast<int32_t>(g.nchunks);
    count_chunk(sh, k, g.cls, g.nblocks, g.chunk, g.nclasses, g.counts, g.chunk_err);
}

__global__ __launch_bounds__(kPlanThreads) void plan_place_mixed_kernel(PlanArgs a) {
    extern __shared__ __align__(16) int place_dyn[];
    const int64_t w = blockIdx.x;
    const PlanSeg& g = a.seg[plan_segment(a, w, true)];
    const int64_t local = w - g.place_begin;
    if (local < 2 * g.nclasses) {
        build_tables_wg(place_dyn, static_cast<int>(local), g.angles, nullptr, g.log2n, g.rounds,
                        0, g.nclasses, g.modes, g.coef, g.signs);
        return;
    }
    place_chunk(place_dyn, local - 2 * static_cast<int64_t>(g.nclasses), g.cls, g.nblocks,
                g.nclasses, g.nchunks, g.chunk, g.max_tiles, g.counts, g.tile_class, g.perm);
}

}  // namespace

hipError_t launch_plan(const int32_t* cls, int64_t nblocks, int log2n, int rounds,
                       const float* angles, const uint8_t* codes, int integer, int nclasses,
                       const WsLayout& l, const WsPtrs& p, hipStream_t stream) {
    hipLaunchKernelGGL(plan_count_kernel, dim3(static_cast<unsigned>(l.nchunks)),
                       dim3(kPlanThreads), 0, stream, cls, nblocks, nclasses, l.nchunks, l.chunk,
                       p.hdr, p.chunk_err, p.counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = place_lds_bytes(l.nchunks, nclasses);
    if (lds > 64 * 1024) {
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(plan_place_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(plan_place_kernel, dim3(static_cast<unsigned>(2 * nclasses + l.nchunks)),
                       dim3(kPlanThreads), lds, stream, cls, nblocks, nclasses, l.nchunks, l.chunk,
                       l.max_tiles, p.counts, p.tile_class, p.perm, angles, codes, log2n,
                       rounds, integer, p.modes, p.coef, p.signs);
    return hipGetLastError();
}

hipError_t launch_plan_mixed(const PlanArgs& a, int64_t count_wgs, int64_t place_wgs,
                             hipStream_t stream) {
    if (count_wgs == 0) return hipSuccess;
    hipLaunchKernelGGL(plan_count_mixed_kernel, dim3(static_cast<unsigned>(count_wgs)),
                       dim3(kPlanThreads), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t lds = 0;
    for (int i = 0; i < a.nseg; ++i)
        lds = std::max(lds, place_lds_bytes(a.seg[i].nchunks, a.seg[i].nclasses));
    if (lds > 64 * 1024) {
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(plan_place_mixed_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(plan_place_mixed_kernel, dim3(static_cast<unsigned>(place_wgs)),
                       dim3(kPlanThreads), lds, stream, a);
    return hipGetLastError();
}

}  // namespace hygt

// Plan kernels: per-class multiplier tables and the grouping of blocks into
// class-uniform tiles.
//
// Multiplier tables: one workgroup per (direction, class) runs the table
// builder of hygt_table.h (FP64 conversion into lifting multipliers, with
// the sign bookkeeping of the angle reduction), inside the placing launch
// of a plan (skipped by a regrouping that keeps the tables) or, for the
// request path, in a launch of its own (table_build_kernel).
//
// Grouping. A tile is 64 blocks of one class, so that a wavefront (one lane
// per block) reads one class table with scalar loads. The blocks of each
// class are ranked in batch order, tile i of class c holding ranks
// 64i .. 64i+63, and the tile list holds the classes' tiles interleaved by
// tile index: round i lists tile i of every class that has one. Tiles that
// sit next to each other in the list then hold blocks from the same region
// of the batch, so the tiles that the rotation kernels run at any moment read
// and write one compact window of the arrays (measured on MI355X, 2^20 8x8
// blocks: 107 against 122 us per forward transform with the tiles in class
// order). With many classes (more than kInterleaveMaxClasses) the tiles stay
// in class order. The counting sort takes two launches over chunks of
// consecutive blocks: the first counts the classes of each chunk, the second
// gives every chunk its first rank inside each class from the counts of the
// chunks before it and scatters the block ids into the class's tiles, while
// other workgroups of the same launch build the multiplier tables.

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
// 16-byte loads per thread that bring the cached counts into LDS.
constexpr int kCountLoads = kCountsCache / 4 / kPlanThreads;
static_assert(kCountsCache % (4 * kPlanThreads) == 0, "counts cache in whole rounds");

// LDS of a chunk counter (the counting launch).
struct CountShared {
    int hist[HYGT_MAX_CLASSES];
    int flag;
};

// LDS of the placing launch, sized at launch time for the class count:
// the cached per-chunk counts (when they fit), then per class the blocks in
// the batch, the blocks in earlier chunks, the blocks placed so far and the
// first tile, then the scan scratch, then (interleaved order only) per class
// the first tile index that this chunk fills and the offset of its entries in
// the chunk's table of tile positions, and that table.
struct PlaceLds {
    int* counts;
    int* total;
    int* pre;
    int* pos;
    int* tile_base;  // [C + 1]
    int* tiles;      // [C] tiles of each class
    int* scan;       // [2 * kPlanThreads]
    int* ilo;        // [C]
    int* ioff;       // [C + 1]
    int* tab;        // [interleave] tile position of each entry
    int* owner;      // [interleave] class of each entry
};

__host__ __device__ inline bool place_counts_cached(int64_t nchunks, int nclasses) {
    return nchunks * nclasses <= kCountsCache;
}

__host__ __device__ inline size_t place_lds_bytes(int64_t nchunks, int nclasses,
                                                  int64_t interleave) {
    const size_t cached = place_counts_cached(nchunks, nclasses)
                              ? static_cast<size_t>(nchunks) * nclasses : 0;
    const size_t inter =
        interleave > 0
            ? 2 * static_cast<size_t>(nclasses) + 1 + 2 * static_cast<size_t>(interleave)
            : 0;
    const size_t place =
        (cached + 5 * static_cast<size_t>(nclasses) + 1 + 2 * kPlanThreads + inter) * sizeof(int);
    return place > sizeof(TableShared) ? place : sizeof(TableShared);
}

__device__ inline PlaceLds place_lds(int* base, int64_t nchunks, int nclasses, int64_t interleave) {
    PlaceLds l;
    l.counts = base;
    int* p = base + (place_counts_cached(nchunks, nclasses) ? nchunks * nclasses : 0);
    l.total = p;
    l.pre = p + nclasses;
    l.pos = p + 2 * nclasses;
    l.tile_base = p + 3 * nclasses;
    l.tiles = p + 4 * nclasses + 1;
    l.scan = p + 5 * nclasses + 1;
    l.ilo = l.scan + 2 * kPlanThreads;
    l.ioff = l.ilo + nclasses;
    l.tab = l.ioff + nclasses + 1;
    l.owner = l.tab + interleave;
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

// Tiles of a class of `count` blocks (count <= HYGT_MAX_BLOCKS, so no
// intermediate sum may exceed int32).
__device__ __forceinline__ int class_tiles(int count) {
    return count / kTile + (count % kTile != 0);
}

// Position of tile i of class c in the interleaved order: round i' < i holds
// tile i' of every class that has one (sum over c' of min(T_c', i) tiles
// before round i), and round i lists its tiles by class. tiles[c'] = T_c'.
__device__ int interleaved_position(const int* tiles, int nclasses, int c, int i) {
    int pos = 0;
    // unrolled, so that several LDS reads are in flight at once
#pragma unroll 8
    for (int k = 0; k < nclasses; ++k) {
        const int t = tiles[k];
        pos += t < i ? t : i;
        pos += (k < c && t > i) ? 1 : 0;
    }
    return pos;
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

// Stand-alone tables (hygt_table_build()): workgroup w builds (direction,
// class) = (w / C, w % C), laid out as in a workspace.
__global__ __launch_bounds__(kPlanThreads) void table_build_kernel(
    const float* __restrict__ angles, int log2n, int rounds, int nclasses,
    int32_t* __restrict__ modes, float* __restrict__ coef, float* __restrict__ signs) {
    __shared__ TableShared sh;
    const int w = blockIdx.x;
    const size_t passes = static_cast<size_t>(rounds) * log2n;
    const size_t n = size_t{1} << log2n;
    build_table(sh, w / nclasses, w % nclasses, angles, nullptr, log2n, rounds,
                coef + static_cast<size_t>(w) * passes * n, signs + static_cast<size_t>(w) * n,
                modes + w, nullptr);
}

// Blocks of class c in chunk k.
__device__ __forceinline__ int chunk_class_count(const PlaceLds& sh, const int32_t* __restrict__ counts,
                                                 bool cached, int64_t k, int nclasses, int c) {
    if (cached) return sh.counts[k * nclasses + c];
    return counts[k * nclasses + c];
}

// Inclusive sum of v over lanes 0..lane of the wavefront.
__device__ __forceinline__ int wave_inclusive_sum(int v, int lane) {
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Places chunk k of one batch: its blocks' ids into their classes' tiles, and
// the class of this chunk's share of the tile list.
__device__ __forceinline__ void place_chunk(int* place_dyn, int64_t k, const int32_t* __restrict__ cls,
                            int64_t nblocks, int nclasses, int64_t nchunks, int64_t chunk,
                            int64_t max_tiles, int64_t interleave,
                            const int32_t* __restrict__ counts,
                            int32_t* __restrict__ tile_class, int32_t* __restrict__ perm) {
    const PlaceLds sh = place_lds(place_dyn, nchunks, nclasses, interleave);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
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
        // 16-byte loads (counts starts 256-byte aligned), all issued before
        // the first LDS store, so that they share one memory round trip. The
        // loads are unconditional (lanes past the end read the first 16
        // bytes, inside the 256-byte-aligned counts area), so that the
        // compiler keeps them in flight together.
        const int n4 = static_cast<int>(ncounts / 4);
        const int4* c4 = reinterpret_cast<const int4*>(counts);
        int4* s4 = reinterpret_cast<int4*>(sh.counts);  // sh.counts is at the LDS base
        int4 got[kCountLoads];
#pragma unroll
        for (int u = 0; u < kCountLoads; ++u) {
            const int e = tid + u * kPlanThreads;
            got[u] = c4[e < n4 ? e : 0];
        }
        // The LDS area is reached through a generic pointer, which the
        // compiler may not separate from the loads: without this, it waits
        // for each load before the next.
#pragma unroll
        for (int u = 0; u < kCountLoads; ++u)
            asm volatile("" ::"v"(got[u].x), "v"(got[u].y), "v"(got[u].z), "v"(got[u].w));
#pragma unroll
        for (int u = 0; u < kCountLoads; ++u) {
            const int e = tid + u * kPlanThreads;
            if (e < n4) s4[e] = got[u];
        }
        for (int64_t e = static_cast<int64_t>(n4) * 4 + tid; e < ncounts; e += kPlanThreads)
            sh.counts[e] = counts[e];
    }
    __syncthreads();
    // Per class: blocks in the whole batch and in the chunks before this one.
    // Classes in groups of 64, a lane per class: each wavefront sums its
    // share of the chunks, then wavefront 0 adds the shares.
    {
        const int nwaves = blockDim.x >> 6;
        int* part_total = sh.scan;
        int* part_pre = sh.scan + kPlanThreads;
        for (int c0 = 0; c0 < nclasses; c0 += 64) {
            const int c = c0 + lane;
            int total = 0, pre = 0;
            // Unrolled, so that the reads of several chunks are in flight; the
            // two sources in separate loops, so that each read is an LDS or
            // a global load and not a generic one.
            if (c < nclasses && cached) {
                // (cached: fewer than kCountsCache counts, so int indices)
                const int nq = static_cast<int>(nchunks), kq = static_cast<int>(k);
#pragma unroll 8
                for (int q = wave; q < nq; q += nwaves) {
                    const int v = sh.counts[q * nclasses + c];
                    total += v;
                    pre += q < kq ? v : 0;
                }
            } else if (c < nclasses) {
#pragma unroll 8
                for (int64_t q = wave; q < nchunks; q += nwaves) {
                    const int v = counts[q * nclasses + c];
                    total += v;
                    pre += q < k ? v : 0;
                }
            }
            part_total[tid] = total;
            part_pre[tid] = pre;
            __syncthreads();
            if (wave == 0 && c < nclasses) {
                for (int w = 1; w < nwaves; ++w) {
                    total += part_total[w * 64 + lane];
                    pre += part_pre[w * 64 + lane];
                }
                sh.total[c] = total;
                sh.pre[c] = pre;
                sh.pos[c] = pre;  // the next rank in the class
                sh.tiles[c] = class_tiles(total);
            }
            __syncthreads();
        }
    }
    // Per class, as prefix sums over the classes: the first tile in class
    // order (tile_base; its last entry is the batch's tile count in either
    // order) and, for the interleaved order, the first tile index this chunk
    // fills (ilo) and the offset of the class's entries in the chunk's table
    // of tile positions (ioff). Up to 64 classes one wavefront does it, a
    // lane per class; beyond, every thread owns a contiguous run of classes.
    if (nclasses <= 64) {
        if (wave == 0) {
            const bool own = lane < nclasses;
            const int tiles = own ? sh.tiles[lane] : 0;
            const int tincl = wave_inclusive_sum(tiles, lane);
            int ent = 0, pre = 0;
            if (own && interleave > 0) {
                pre = sh.pre[lane];
                const int n = chunk_class_count(sh, counts, cached, k, nclasses, lane);
                if (n > 0) ent = ((pre + n - 1) >> 6) - (pre >> 6) + 1;
            }
            const int eincl = wave_inclusive_sum(ent, lane);
            if (own) {
                sh.tile_base[lane] = tincl - tiles;
                if (interleave > 0) {
                    sh.ilo[lane] = pre >> 6;
                    sh.ioff[lane] = eincl - ent;
                    for (int e = eincl - ent; e < eincl && e < interleave; ++e) sh.owner[e] = lane;
                }
            }
            if (lane == 63) {
                sh.tile_base[nclasses] = tincl;
                if (interleave > 0) sh.ioff[nclasses] = eincl;
            }
        }
    } else {
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
    }
    __syncthreads();
    const int ntiles = sh.tile_base[nclasses];
    if (interleave > 0) {
        // entry e: tile ilo[c] + (e - ioff[c]) of the class c that owns it
        const int entries = sh.ioff[nclasses];
        for (int e = tid; e < entries && e < interleave; e += blockDim.x) {
            const int c = sh.owner[e];
            sh.tab[e] = interleaved_position(sh.tiles, nclasses, c, sh.ilo[c] + e - sh.ioff[c]);
        }
        __syncthreads();
    }
    // Block ids of this chunk into their classes' tiles: first every rank in
    // its class (LDS counters), then the stores, so that the counter updates
    // of a thread's blocks are in flight together.
    const int step = static_cast<int>(blockDim.x) * kUnroll;
    for (int i0 = tid; i0 < cnt; i0 += step) {
        if (i0 != tid) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int i = i0 + u * static_cast<int>(blockDim.x);
                cv[u] = (i < cnt && cls != nullptr) ? cls[start + i] : 0;
            }
        }
        int rank[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int i = i0 + u * static_cast<int>(blockDim.x);
            const int c = cv[u];
            rank[u] = (i < cnt && c >= 0 && c < nclasses) ? atomicAdd(&sh.pos[c], 1) : -1;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int p = rank[u];
            if (p < 0) continue;
            const int c = cv[u];
            const int32_t id = static_cast<int32_t>(start + i0 + u * static_cast<int>(blockDim.x));
            // Counts and classes agree unless cls changed between the two
            // plan launches; never write outside perm even then.
            if (interleave > 0) {
                const int e = sh.ioff[c] + (p >> 6) - sh.ilo[c];
                if (e < sh.ioff[c + 1] && e < interleave) {
                    const int64_t t = sh.tab[e];
                    const int ln = p & (kTile - 1);
                    if (t < max_tiles) {
                        perm[t * kTile + ln] = id;
                        if (ln == 0) tile_class[t] = c;
                    }
                }
            } else {
                const int64_t slot = static_cast<int64_t>(sh.tile_base[c]) * kTile + p;
                if (slot < max_tiles * kTile) perm[slot] = id;
            }
        }
    }
    // Interleaved order: the empty lanes of each class's last tile, class c
    // by the workgroup of chunk c mod nchunks, a thread per class (with few
    // chunks, one workgroup has many classes: a wavefront taking them one
    // after another would spend most of the launch in these lookups).
    if (interleave > 0) {
        const int64_t cstep = static_cast<int64_t>(blockDim.x) * nchunks;
        for (int64_t c = k + tid * nchunks; c < nclasses; c += cstep) {
            const int used = sh.total[c] % kTile;
            if (used == 0) continue;
            const int ci = static_cast<int>(c);
            const int64_t t = interleaved_position(sh.tiles, nclasses, ci, sh.tiles[ci] - 1);
            if (t >= max_tiles) continue;
            for (int ln = used; ln < kTile; ++ln) perm[t * kTile + ln] = -1;
        }
    }
    // Class of every tile of this chunk's share of the tile list (class order
    // only: the interleaved order writes them while placing), the empty lanes
    // of each class's last tile, and -1 for every tile past the last.
    const int64_t share = (max_tiles + nchunks - 1) / nchunks;
    const int64_t t0 = k * share;
    const int64_t t1 = min(t0 + share, max_tiles);
    for (int64_t t = t0 + tid; t < t1; t += blockDim.x) {
        if (t >= ntiles) {
            tile_class[t] = -1;
            continue;
        }
        if (interleave > 0) continue;
        // last class whose first tile is <= t (classes without blocks share
        // their first tile index with the next class)
        int lo = 0, hi = nclasses - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sh.tile_base[mid] <= t) lo = mid; else hi = mid - 1;
        }
        tile_class[t] = lo;
        const int64_t used = sh.total[lo] - (t - sh.tile_base[lo]) * kTile;
        for (int64_t s2 = used > 0 ? used : 0; s2 < kTile; ++s2) perm[t * kTile + s2] = -1;
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
    int64_t chunk, int64_t max_tiles, int64_t interleave, const int32_t* __restrict__ counts,
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
                nchunks, chunk, max_tiles, interleave, counts, tile_class, perm);
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
    const int64_t ntab = a.tables ? 2 * static_cast<int64_t>(g.nclasses) : 0;
    if (local < ntab) {
        build_tables_wg(place_dyn, static_cast<int>(local), g.angles, nullptr, g.log2n, g.rounds,
                        0, g.nclasses, g.modes, g.coef, g.signs);
        return;
    }
    place_chunk(place_dyn, local - ntab, g.cls, g.nblocks,
                g.nclasses, g.nchunks, g.chunk, g.max_tiles, g.interleave, g.counts,
                g.tile_class, g.perm);
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
    const size_t lds = place_lds_bytes(l.nchunks, nclasses, l.interleave);
    if (lds > 64 * 1024) {
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(plan_place_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(plan_place_kernel, dim3(static_cast<unsigned>(2 * nclasses + l.nchunks)),
                       dim3(kPlanThreads), lds, stream, cls, nblocks, nclasses, l.nchunks, l.chunk,
                       l.max_tiles, l.interleave, p.counts, p.tile_class, p.perm, angles, codes, log2n,
                       rounds, integer, p.modes, p.coef, p.signs);
    return hipGetLastError();
}

hipError_t launch_table_build(const float* angles, int log2n, int rounds, int nclasses,
                              const TableLayout& t, void* table, hipStream_t stream) {
    char* b = static_cast<char*>(table);
    hipLaunchKernelGGL(table_build_kernel, dim3(static_cast<unsigned>(2 * nclasses)),
                       dim3(kPlanThreads), 0, stream, angles, log2n, rounds, nclasses,
                       reinterpret_cast<int32_t*>(b + t.modes), reinterpret_cast<float*>(b + t.coef),
                       reinterpret_cast<float*>(b + t.signs));
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
        lds = std::max(lds, place_lds_bytes(a.seg[i].nchunks, a.seg[i].nclasses,
                                            a.seg[i].interleave));
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

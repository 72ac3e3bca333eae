// Plan kernels: per-class multiplier tables and the grouping of blocks into
// class-uniform tiles.
//
// Multiplier tables. Sec. IV of the paper keeps the transform parameters
// compact and converts them to higher-precision multipliers only when they
// are needed. Here the conversion evaluates cos and sin of every FP32 angle in
// FP64 and folds them into per-pass FP32 coefficients for one of two
// evaluation forms of the Givens butterfly (Sec. IV element definition):
//
//   direct:  y_m = (c s_m) a + (s s_n) b,  y_n = (c s_n) b - (s s_m) a
//   scaled:  y_m = a + t_m b,  y_n = b + t_n a,
//            t_m = s s_n / (c s_m),  t_n = -s s_m / (c s_n)
//
// where a, b are the stored values of elements m, n and s_m, s_n their scale
// factors (true value = scale * stored value). The scaled form costs two FMAs
// per butterfly instead of four operations and leaves the outputs scaled by
// c s_m and c s_n (a square-root-free Givens rotation); the direct form costs
// four and returns unscaled outputs. A class normally runs the scaled
// schedule: every pass scaled except the last, which is direct so that the
// stored result is the true result. If its angles would push a scale factor
// below 2^-64 (cosines near zero), the class runs the direct schedule, every
// pass direct with unit scales. Both give the exact rotation in exact
// arithmetic; the choice depends only on the angles, so every block of a
// class follows the same arithmetic.
//
// Grouping. A tile is 64 blocks of one class, so that a wavefront (one lane
// per block) reads one class table with scalar loads. The grouping is a
// counting sort by class: a histogram with LDS-local counts, an exclusive scan
// done by the last histogram workgroup to finish, and a scatter that reserves
// per-class ranges with one atomic per class per workgroup.

#include <cmath>

#include "hygt_internal.h"

namespace hygt {
namespace {

__device__ __forceinline__ int insert_zero_bit(int j, int k) {
    // pair j of pass k: lower index m is j with a 0 inserted at bit k (Fig. 5)
    return ((j >> k) << (k + 1)) | (j & ((1 << k) - 1));
}

// One workgroup per (direction, class) builds that table; one extra
// workgroup resets the counters used by the grouping kernels.
__global__ __launch_bounds__(kTableThreads) void plan_tables_kernel(
    const float* __restrict__ angles, int log2n, int rounds, int nclasses, int grouped,
    float* __restrict__ coef, int32_t* __restrict__ modes, PlanHeader* __restrict__ hdr,
    int32_t* __restrict__ counts) {
    const int tid = threadIdx.x;
    const int wg = blockIdx.x;
    if (wg == 2 * nclasses) {
        for (int c = tid; c < nclasses; c += blockDim.x) counts[c] = 0;
        if (tid == 0) {
            hdr->err = 0;
            hdr->ticket = 0;
            hdr->ntiles = 0;
            hdr->grouped = grouped;
        }
        return;
    }
    const int dir = wg / nclasses;
    const int c = wg % nclasses;
    const int n = 1 << log2n;
    const int half = n >> 1;
    const int passes = rounds * log2n;

    __shared__ double scale[256];
    __shared__ int any_bad;
    const size_t table = static_cast<size_t>(dir) * nclasses + c;
    float* cbase = coef + table * passes * 2 * n;

    // Attempt 0 builds the scaled schedule; if any scale factor leaves the
    // safe range, attempt 1 rebuilds the table for the direct schedule.
    for (int attempt = 0; attempt < 2; ++attempt) {
        const bool all_direct = attempt == 1;
        for (int i = tid; i < n; i += blockDim.x) scale[i] = 1.0;
        if (tid == 0) any_bad = 0;
        __syncthreads();
        for (int p = 0; p < passes; ++p) {
            const int kk = p % log2n;
            const int rr = p / log2n;
            const int k = dir ? log2n - 1 - kk : kk;
            const int r = dir ? rounds - 1 - rr : rr;
            const bool direct = all_direct || p == passes - 1;
            float* cp = cbase + static_cast<size_t>(p) * 2 * n;
            if (tid < half) {
                const int m = insert_zero_bit(tid, k);
                const int nn = m + (1 << k);
                double th = static_cast<double>(
                    angles[((static_cast<size_t>(c) * rounds + r) * log2n + k) * half + tid]);
                if (dir) th = -th;  // eq. (9): the inverse pass uses negated angles
                double sn, cs;
                sincos(th, &sn, &cs);
                const double sm = scale[m];
                const double sq = scale[nn];
                if (direct) {
                    cp[4 * tid + 0] = static_cast<float>(cs * sm);
                    cp[4 * tid + 1] = static_cast<float>(sn * sq);
                    cp[4 * tid + 2] = static_cast<float>(cs * sq);
                    cp[4 * tid + 3] = static_cast<float>(-sn * sm);
                    scale[m] = 1.0;
                    scale[nn] = 1.0;
                } else {
                    const double nsm = cs * sm;
                    const double nsq = cs * sq;
                    const double lo = ldexp(1.0, -kScaleExp);
                    // written so that NaN fails the test
                    if (!(fabs(nsm) >= lo && fabs(nsq) >= lo)) any_bad = 1;
                    cp[2 * tid + 0] = static_cast<float>(sn * sq / nsm);
                    cp[2 * tid + 1] = static_cast<float>(-sn * sm / nsq);
                    scale[m] = nsm;
                    scale[nn] = nsq;
                }
            }
            __syncthreads();
        }
        if (!any_bad) {
            if (tid == 0) modes[table] = all_direct ? 1 : 0;
            return;
        }
        __syncthreads();
    }
}

// Block-wide exclusive scan of one int per thread (kPlanThreads threads).
__device__ int block_exclusive_scan(int v, int* sh, int* total) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < kPlanThreads; off <<= 1) {
        int add = tid >= off ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += add;
        __syncthreads();
    }
    const int incl = sh[tid];
    *total = sh[kPlanThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kPlanThreads) void plan_hist_kernel(
    const int32_t* __restrict__ cls, int64_t nblocks, int nclasses, PlanHeader* __restrict__ hdr,
    int32_t* __restrict__ counts, int32_t* __restrict__ cursor,
    int32_t* __restrict__ class_start, int32_t* __restrict__ tile_start) {
    __shared__ int hist[4096];
    __shared__ int bad;
    __shared__ int last;
    __shared__ int scan_sh[kPlanThreads];
    const int tid = threadIdx.x;
    for (int c = tid; c < nclasses; c += kPlanThreads) hist[c] = 0;
    if (tid == 0) bad = 0;
    __syncthreads();
    const int64_t start = static_cast<int64_t>(blockIdx.x) * kChunk;
    const int64_t stop = min(start + kChunk, nblocks);
    for (int64_t i = start + tid; i < stop; i += kPlanThreads) {
        const int c = cls[i];
        if (c >= 0 && c < nclasses)
            atomicAdd(&hist[c], 1);
        else
            bad = 1;
    }
    __syncthreads();
    for (int c = tid; c < nclasses; c += kPlanThreads)
        if (hist[c]) atomicAdd(&counts[c], hist[c]);
    if (tid == 0 && bad) atomicOr(&hdr->err, 1);
    __threadfence();
    __syncthreads();
    if (tid == 0) last = atomicAdd(&hdr->ticket, 1) == static_cast<int>(gridDim.x) - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    // Exclusive scans of the class counts and of the tiles per class. Each
    // thread owns a contiguous run of classes.
    const int per = (nclasses + kPlanThreads - 1) / kPlanThreads;
    const int c0 = min(tid * per, nclasses);
    const int c1 = min(c0 + per, nclasses);
    int run_blocks = 0, run_tiles = 0;
    for (int c = c0; c < c1; ++c) {
        const int cnt = __hip_atomic_load(&counts[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        run_blocks += cnt;
        run_tiles += (cnt + kTile - 1) / kTile;
    }
    int total_blocks = 0, total_tiles = 0;
    int b = block_exclusive_scan(run_blocks, scan_sh, &total_blocks);
    int t = block_exclusive_scan(run_tiles, scan_sh, &total_tiles);
    for (int c = c0; c < c1; ++c) {
        const int cnt = __hip_atomic_load(&counts[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        class_start[c] = b;
        cursor[c] = b;
        tile_start[c] = t;
        b += cnt;
        t += (cnt + kTile - 1) / kTile;
    }
    if (tid == 0) {
        class_start[nclasses] = total_blocks;
        tile_start[nclasses] = total_tiles;
        hdr->ntiles = total_tiles;
        hdr->ticket = 0;
    }
}

__global__ __launch_bounds__(kPlanThreads) void plan_scatter_kernel(
    const int32_t* __restrict__ cls, int64_t nblocks, int nclasses,
    const PlanHeader* __restrict__ hdr, int32_t* __restrict__ cursor,
    const int32_t* __restrict__ class_start, const int32_t* __restrict__ tile_start,
    int4* __restrict__ tiles, int32_t* __restrict__ perm, int64_t max_tiles) {
    __shared__ int hist[4096];
    __shared__ int base[4096];
    __shared__ int chunk_cls[kChunk];
    const int tid = threadIdx.x;
    for (int c = tid; c < nclasses; c += kPlanThreads) hist[c] = 0;
    __syncthreads();
    const int64_t start = static_cast<int64_t>(blockIdx.x) * kChunk;
    const int64_t stop = min(start + kChunk, nblocks);
    for (int64_t i = start + tid; i < stop; i += kPlanThreads) {
        const int c = cls[i];
        chunk_cls[i - start] = c;
        if (c >= 0 && c < nclasses) atomicAdd(&hist[c], 1);
    }
    __syncthreads();
    for (int c = tid; c < nclasses; c += kPlanThreads) {
        const int h = hist[c];
        base[c] = h ? atomicAdd(&cursor[c], h) : 0;
        hist[c] = 0;
    }
    __syncthreads();
    for (int64_t i = start + tid; i < stop; i += kPlanThreads) {
        const int c = chunk_cls[i - start];
        if (c >= 0 && c < nclasses) {
            const int pos = atomicAdd(&hist[c], 1);
            perm[base[c] + pos] = static_cast<int32_t>(i);
        }
    }
    // Tile descriptors: this workgroup's share of the tile list.
    const int ntiles = hdr->ntiles;
    const int64_t per = (max_tiles + gridDim.x - 1) / gridDim.x;
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * per;
    const int64_t t1 = min(t0 + per, static_cast<int64_t>(ntiles));
    for (int64_t t = t0 + tid; t < t1; t += kPlanThreads) {
        // last class whose first tile is <= t (classes with no tiles share
        // their first tile with the next class, so take the last match)
        int lo = 0, hi = nclasses - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tile_start[mid] <= t) lo = mid; else hi = mid - 1;
        }
        const int c = lo;
        const int first = class_start[c] + static_cast<int>(t - tile_start[c]) * kTile;
        const int count = min(kTile, class_start[c + 1] - first);
        tiles[t] = make_int4(c, first, count, 0);
    }
}

}  // namespace

hipError_t launch_plan(const int32_t* cls, int64_t nblocks, int log2n, int rounds,
                       const float* angles, int nclasses, const WsLayout& l,
                       const WsPtrs& p, hipStream_t stream) {
    const int grouped = cls != nullptr ? 1 : 0;
    hipLaunchKernelGGL(plan_tables_kernel, dim3(2 * nclasses + 1), dim3(kTableThreads), 0,
                       stream, angles, log2n, rounds, nclasses, grouped, p.coef, p.modes,
                       p.hdr, p.counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !grouped || nblocks == 0) return e;
    const dim3 grid(static_cast<unsigned>(l.nhist));
    hipLaunchKernelGGL(plan_hist_kernel, grid, dim3(kPlanThreads), 0, stream, cls, nblocks,
                       nclasses, p.hdr, p.counts, p.cursor, p.class_start, p.tile_start);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(plan_scatter_kernel, grid, dim3(kPlanThreads), 0, stream, cls, nblocks,
                       nclasses, p.hdr, p.cursor, p.class_start, p.tile_start, p.tiles,
                       p.perm, l.max_tiles);
    return hipGetLastError();
}

}  // namespace hygt

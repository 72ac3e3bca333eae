// Memory ceilings for the benchmark (libhygt_ceiling.so, not part of the
// HyGT library): what the rotation kernels' data movement costs with no
// arithmetic at all.
//
//   hygt_ceiling_stream_copy   y = x over n floats: each workgroup of 256
//       threads copies one contiguous 16 KB piece with 16-byte loads and
//       non-temporal 16-byte stores; the plain streaming bound of reading and
//       writing the batch once.
//   hygt_ceiling_gather_copy   the rotation kernels' own access pattern with
//       the passes taken out: a wavefront per tile of the plan in the
//       workspace (class-grouped blocks, the plan's tile order), the tile
//       brought in by load_tile (LDS DMA plus row loads) and written back by
//       the LDS-staged whole-block stores, one-wave workgroups as in
//       rotate_kernel. N <= 64.
//
// Both return a hygt_status. x and y must not overlap.

#include <cstdint>

#include "hygt.h"
#include "hygt_internal.h"
#include "hygt_tile.h"

namespace {

using namespace hygt;
using namespace hygt::tile;

constexpr int kCopyThreads = 256;
constexpr int kCopyPerThread = 4;  // float4 per thread: 16 KB per workgroup

__global__ __launch_bounds__(kCopyThreads) void stream_copy_kernel(
    const float4* __restrict__ x, float4* __restrict__ y, int64_t n4) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kCopyThreads * kCopyPerThread;
    float4 v[kCopyPerThread];
#pragma unroll
    for (int u = 0; u < kCopyPerThread; ++u) {
        const int64_t i = base + u * kCopyThreads + threadIdx.x;
        if (i < n4) v[u] = x[i];
    }
#pragma unroll
    for (int u = 0; u < kCopyPerThread; ++u) {
        const int64_t i = base + u * kCopyThreads + threadIdx.x;
        if (i < n4) store_nt(reinterpret_cast<float*>(y + i), v[u]);
    }
}

template <int D>
__global__ __launch_bounds__(64) void gather_copy_kernel(
    const float* __restrict__ x, float* __restrict__ y, int64_t nblocks, int64_t max_tiles,
    const int32_t* __restrict__ tile_class, const int32_t* __restrict__ perm) {
    using G = TileGeo<D>;
    __shared__ float4 lds[kTile * G::CHP];
    const int lane = threadIdx.x & 63;
    const int64_t t0 = blockIdx.x;
    if (t0 >= max_tiles) return;
    const int c = __builtin_amdgcn_readfirstlane(tile_class[t0]);
    if (c < 0) return;
    const int blk = valid_block(perm[t0 * kTile + lane], nblocks);
    float v[G::V];
    load_tile<D>(x, blk, v, lds, lane);
    int lane2 = lane;
    asm volatile("" : "+v"(lane2));
    const int sw2 = swz<G::CHP>(lane2);
    int b = blk;
    asm volatile("" : "+v"(b));
    int bb[G::CHP];
    instr_blocks<D>(bb, b, lane2);
    StaticFor<0, G::PARTS>::run([&](auto pp) {
        store_part<D, decltype(pp)::value>(y, lds, bb, v, lane2, sw2);
    });
}

template <int D>
hipError_t launch_gather(const float* x, float* y, int64_t nblocks, const WsLayout& l,
                         const WsPtrs& p, hipStream_t stream) {
    hipLaunchKernelGGL((gather_copy_kernel<D>), dim3(static_cast<unsigned>(l.max_tiles)),
                       dim3(64), 0, stream, x, y, nblocks, l.max_tiles, p.tile_class, p.perm);
    return hipGetLastError();
}

bool disjoint(const void* a, const void* b, uint64_t bytes) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x + bytes <= y || y + bytes <= x;
}

}  // namespace

extern "C" {

int hygt_ceiling_stream_copy(const float* x, float* y, int64_t nfloats, hipStream_t stream) {
    if (nfloats < 0 || nfloats % 4 != 0) return HYGT_EINVAL;
    if (nfloats == 0) return HYGT_OK;
    if (x == nullptr || y == nullptr || reinterpret_cast<uintptr_t>(x) % 16 ||
        reinterpret_cast<uintptr_t>(y) % 16 || !disjoint(x, y, static_cast<uint64_t>(nfloats) * 4))
        return HYGT_EINVAL;
    const int64_t n4 = nfloats / 4;
    const int64_t per = static_cast<int64_t>(kCopyThreads) * kCopyPerThread;
    const int64_t grid = (n4 + per - 1) / per;
    if (grid > 0x7fffffff) return HYGT_EINVAL;
    hipLaunchKernelGGL(stream_copy_kernel, dim3(static_cast<unsigned>(grid)), dim3(kCopyThreads),
                       0, stream, reinterpret_cast<const float4*>(x), reinterpret_cast<float4*>(y),
                       n4);
    return hipGetLastError() == hipSuccess ? HYGT_OK : HYGT_ELAUNCH;
}

int hygt_ceiling_gather_copy(const float* x, float* y, int64_t nblocks, int log2n, int rounds,
                             int nclasses, const void* workspace, size_t workspace_bytes,
                             hipStream_t stream) {
    if (nblocks < 0 || nblocks > HYGT_MAX_BLOCKS || log2n < 2 || log2n > 6 || rounds < 1 ||
        rounds > HYGT_MAX_ROUNDS || nclasses < 1 || nclasses > HYGT_MAX_CLASSES)
        return HYGT_EINVAL;
    if (nblocks == 0) return HYGT_OK;
    const WsLayout l = ws_layout(nblocks, log2n, rounds, nclasses);
    if (workspace == nullptr || workspace_bytes < l.total ||
        reinterpret_cast<uintptr_t>(workspace) % 256)
        return HYGT_EWORKSPACE;
    if (x == nullptr || y == nullptr || reinterpret_cast<uintptr_t>(x) % 16 ||
        reinterpret_cast<uintptr_t>(y) % 16 ||
        !disjoint(x, y, static_cast<uint64_t>(nblocks) * (uint64_t{4} << log2n)))
        return HYGT_EINVAL;
    const WsPtrs p = ws_ptrs(const_cast<void*>(workspace), l);
    hipError_t e = hipErrorInvalidValue;
    switch (log2n) {
        case 2: e = launch_gather<2>(x, y, nblocks, l, p, stream); break;
        case 3: e = launch_gather<3>(x, y, nblocks, l, p, stream); break;
        case 4: e = launch_gather<4>(x, y, nblocks, l, p, stream); break;
        case 5: e = launch_gather<5>(x, y, nblocks, l, p, stream); break;
        case 6: e = launch_gather<6>(x, y, nblocks, l, p, stream); break;
        default: break;
    }
    return e == hipSuccess ? HYGT_OK : HYGT_ELAUNCH;
}

}  // extern "C"

// Dense per-class transform on the matrix cores: y_b = M_{cls[b]} x_b with
// one N x N matrix per class (N = 64).
//
// This is the matrix-based non-separable transform that HyGT replaces (the
// KLT of Sec. II, eq. (3); Table I lists its cost as N^2 operations and
// N^2 stored values per class against HyGT's P N). It runs here as a grouped
// GEMM over the same class-sorted tiles as the rotation kernels: a wavefront
// takes a tile of 64 blocks of one class and computes
//
//   Y (64 blocks x 64 outputs) = X (64 blocks x 64 inputs) . M_c^T
//
// with 32 v_mfma_f32_16x16x32_bf16 (4 x 4 output fragments of 16 x 16, two
// K steps of 32). X is rounded to BF16 (round to nearest even) as it leaves
// LDS, the products are exact in FP32 and are summed in FP32. M_c comes in
// as BF16.
//
// Memory. The tile moves through LDS in both directions, as in the rotation
// kernels: 16 global_load_lds_dwordx4 bring 4 whole blocks each, 16 stores
// write 4 whole blocks each; in LDS the 16 chunks of 16 bytes of block b sit
// at b*16 + (q ^ (b & 15)), which keeps the fragment reads and writes free of
// bank conflicts. The B fragments (rows of M_c) are read from global memory;
// the 35 x 8 KB of matrices stay in L2.
//
// Operand layout of v_mfma_f32_16x16x32_bf16, for lane l: A holds row l % 16
// at k = 8 (l / 16) .. + 7, B holds column l % 16 at the same k, and the four
// accumulators hold rows 4 (l / 16) .. + 3 of column l % 16.

#include "hygt_internal.h"

namespace hygt {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

using lds_void_ptr = __attribute__((address_space(3))) void*;

constexpr int kDenseWaves = 4;   // tiles (wavefronts) per workgroup
constexpr int kDenseN = 64;      // block length handled
constexpr int kChunks = kDenseN / 4;  // 16-byte chunks per block
constexpr int kXcdsDense = 8;

__device__ __forceinline__ int64_t dense_tile_group() {
    const int64_t w = blockIdx.x;
    const int64_t per_xcd = gridDim.x / kXcdsDense;
    return (w % kXcdsDense) * per_xcd + w / kXcdsDense;
}

// LDS slot of chunk q of tile block b.
__device__ __forceinline__ int slot(int b, int q) { return b * kChunks + (q ^ (b & 15)); }

__global__ __launch_bounds__(64 * kDenseWaves) void dense_kernel(
    const float* __restrict__ x, float* __restrict__ y, int64_t nblocks, int64_t max_tiles,
    const int32_t* __restrict__ tile_class, const int32_t* __restrict__ perm,
    const unsigned short* __restrict__ mats) {
    __shared__ float4 lds[kDenseWaves][kTile * kChunks];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t = dense_tile_group() * kDenseWaves + wv;
    if (t >= max_tiles) return;
    const int c = __builtin_amdgcn_readfirstlane(tile_class[t]);
    if (c < 0) return;
    float4* L = lds[wv];

    int blk = perm[t * kTile + lane];
    blk = (blk >= 0 && blk < nblocks) ? blk : -1;
    // Instruction i moves tile blocks 4i .. 4i+3: lane l takes chunk
    // (l % 16) ^ (b & 15) of block b = 4i + l / 16, LDS slot 64i + l.
    int bb[kChunks];
#pragma unroll
    for (int i = 0; i < kChunks; ++i)
        bb[i] = __builtin_amdgcn_ds_bpermute((4 * i + lane / 16) << 2, blk);
    (void)x;  // read only by the device pass below
#if defined(__HIP_DEVICE_COMPILE__)  // the LDS-DMA builtin exists only in the device pass
#pragma unroll
    for (int i = 0; i < kChunks; ++i) {
        const int b = 4 * i + lane / 16;
        const int q = (lane % 16) ^ (b & 15);
        if (bb[i] >= 0)
            __builtin_amdgcn_global_load_lds(x + static_cast<int64_t>(bb[i]) * kDenseN + q * 4,
                                             (lds_void_ptr)(L + i * 64), 16, 0, 0);
    }
#endif

    // B fragments: row n = 16 nt + l % 16 of M_c, elements k = 32 ks + 8 (l / 16) ..
    const unsigned short* mc = mats + static_cast<size_t>(c) * kDenseN * kDenseN;
    bf16x8 bf[4][2];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const u16x8 raw = *reinterpret_cast<const u16x8*>(
                mc + (16 * nt + lane % 16) * kDenseN + 32 * ks + 8 * (lane / 16));
            bf[nt][ks] = __builtin_bit_cast(bf16x8, raw);
        }

    // The DMA writes land in LDS asynchronously.
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");

    f32x4 acc[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const int b = 16 * mt + lane % 16;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int q0 = 8 * ks + 2 * (lane / 16);
            const float4 lo = L[slot(b, q0)];
            const float4 hi = L[slot(b, q0 + 1)];
            bf16x8 a;
            a[0] = static_cast<__bf16>(lo.x);
            a[1] = static_cast<__bf16>(lo.y);
            a[2] = static_cast<__bf16>(lo.z);
            a[3] = static_cast<__bf16>(lo.w);
            a[4] = static_cast<__bf16>(hi.x);
            a[5] = static_cast<__bf16>(hi.y);
            a[6] = static_cast<__bf16>(hi.z);
            a[7] = static_cast<__bf16>(hi.w);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bf[nt][ks], acc[mt][nt],
                                                                      0, 0, 0);
        }
    }
    // Every fragment read of X is complete before Y overwrites the tile.
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");

    // Accumulator e of fragment (mt, nt) is Y[16 mt + 4 (l / 16) + e][16 nt + l % 16].
    float* Lf = reinterpret_cast<float*>(L);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int b = 16 * mt + 4 * (lane / 16) + e;
                const int j = 16 * nt + lane % 16;
                Lf[slot(b, j / 4) * 4 + (j % 4)] = acc[mt][nt][e];
            }
    // LDS executes one wavefront's operations in order; only the compiler's
    // ordering of the reads below after the writes above needs pinning.
    asm volatile("" ::: "memory");
#pragma unroll
    for (int i = 0; i < kChunks; ++i) {
        const int b = 4 * i + lane / 16;
        const int q = (lane % 16) ^ (b & 15);
        const float4 f = L[i * 64 + lane];
        if (bb[i] >= 0) {
            // non-temporal: outputs are not read again by this launch
            const vf4 w = {f.x, f.y, f.z, f.w};
            __builtin_nontemporal_store(w, reinterpret_cast<vf4*>(
                                               y + static_cast<int64_t>(bb[i]) * kDenseN + q * 4));
        }
    }
}

}  // namespace

hipError_t launch_dense(const float* x, float* y, int64_t nblocks, const unsigned short* mats,
                        const WsLayout& l, const WsPtrs& p, hipStream_t stream) {
    const int64_t groups = (l.max_tiles + kDenseWaves - 1) / kDenseWaves;
    const dim3 grid(static_cast<unsigned>((groups + kXcdsDense - 1) / kXcdsDense * kXcdsDense));
    hipLaunchKernelGGL(dense_kernel, grid, dim3(64 * kDenseWaves), 0, stream, x, y, nblocks,
                       l.max_tiles, p.tile_class, p.perm, mats);
    return hipGetLastError();
}

}  // namespace hygt

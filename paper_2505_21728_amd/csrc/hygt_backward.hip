// Reverse-mode derivative of the forward transform, for the parameter
// optimisation of Sec. V: given the outputs y = T_c x of every block and
// g = dL/dy, computes dL/dx = T_c^T g for every block and dL/dtheta summed
// over the blocks of each class.
//
// Nothing from the forward pass is stored. The passes are walked backwards
// (last round first, pass d-1 first inside it) and each pass's inputs are
// recovered from its outputs by the inverse rotation (eq. (9)). For one
// rotation y_m = c x_m + s x_n, y_n = -s x_m + c x_n:
//
//   dL/dtheta = g_m y_n - g_n y_m
//   (dL/dx_m, dL/dx_n) = (c g_m - s g_n, s g_m + c g_n)
//
// Mapping as in the rotation kernels: one wavefront per class-uniform tile of
// 64 blocks, one lane per block holding the block's y and g (2N registers, so
// N <= 64), the pass's (cos, sin) pairs as wave-uniform scalar operands. The
// N/2 angle contributions of a pass are summed over the 64 lanes by a
// transposed halving: at each step a lane keeps half of its values and adds
// the partner lane's copy of that half, so after log2(N/2) steps each lane
// holds one pair's partial sum; the remaining lane bits are summed directly.
// One atomic add per pair and tile then accumulates the class's gradient
// (FP32 atomics: the order of the additions, so the last bits of the
// gradient, varies from run to run).

#include "hygt_tile.h"

namespace hygt {
namespace {

using namespace tile;

constexpr int kBwdWaves = 4;
constexpr int kBwdWavesPerSimd = 2;
constexpr int kPrepThreads = 256;

// Workgroup c: cos and sin (FP64, rounded once to FP32) of every angle of
// class c, in the angles' own layout (forward pass order), and the class's
// gradient set to zero.
__global__ __launch_bounds__(kPrepThreads) void backward_prep_kernel(
    const float* __restrict__ angles, int log2n, int rounds, float* __restrict__ trig,
    float* __restrict__ gangles) {
    const int64_t c = blockIdx.x;
    const int per = rounds * log2n * (1 << (log2n - 1));
    for (int e = threadIdx.x; e < per; e += blockDim.x) {
        const int64_t a = c * per + e;
        const double th = static_cast<double>(angles[a]);
        trig[2 * a + 0] = static_cast<float>(cos(th));
        trig[2 * a + 1] = static_cast<float>(sin(th));
        gangles[a] = 0.0f;
    }
}

// Sum over the 64 lanes of a[j], j < H, one value per pair. On return, the
// lanes whose low (6 - log2 H) bits are zero own pair j = lane >> (6 - log2 H)
// and hold its sum.
template <int H>
__device__ __forceinline__ float lane_sum(float (&a)[H], int lane) {
    constexpr int LH = H == 1 ? 0 : H == 2 ? 1 : H == 4 ? 2 : H == 8 ? 3 : H == 16 ? 4 : 5;
    // transposed halving along lane bits 5, 4, ..., 6 - LH
    StaticFor<0, LH>::run([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        constexpr int K = H >> (s + 1);  // values kept after this step
        constexpr int b = 5 - s;
        const bool hi = (lane >> b) & 1;
        StaticFor<0, K>::run([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            const float send = hi ? a[i] : a[i + K];
            const float keep = hi ? a[i + K] : a[i];
            a[i] = keep + __shfl_xor(send, 1 << b, 64);
        });
    });
    // the lanes that now hold the same pair: sum over the remaining bits
    float v = a[0];
    StaticFor<0, 6 - LH>::run([&](auto bb) {
        constexpr int b = 5 - LH - decltype(bb)::value;
        v += __shfl_xor(v, 1 << b, 64);
    });
    return v;
}

template <int D>
__global__ __launch_bounds__(64 * kBwdWaves) __attribute__((amdgpu_waves_per_eu(kBwdWavesPerSimd)))
void backward_kernel(const float* __restrict__ y, const float* __restrict__ gy,
                     float* __restrict__ gx, float* __restrict__ gangles, int64_t nblocks,
                     int rounds, int64_t max_tiles, const int32_t* __restrict__ tile_class,
                     const int32_t* __restrict__ perm, const float* __restrict__ trig) {
    using G = TileGeo<D>;
    constexpr int N = 1 << D;
    constexpr int H = N / 2;
    constexpr int LH = D - 1;
    __shared__ float4 lds[kBwdWaves][kTile * G::CHP];

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t0 = xcd_tile_group() * kBwdWaves + wv;
    if (t0 >= max_tiles) return;
    const int c = __builtin_amdgcn_readfirstlane(tile_class[t0]);
    if (c < 0) return;
    const int blk = valid_block(perm[t0 * kTile + lane], nblocks);
    float v[N], g[N];
    StaticFor<0, N>::run([&](auto ii) {
        v[decltype(ii)::value] = 0.0f;
        g[decltype(ii)::value] = 0.0f;
    });
    // empty lanes keep zeros, which add nothing to the sums
    if constexpr (D == 1) {
        if (blk >= 0) {
            const float2 a = reinterpret_cast<const float2*>(y)[blk];
            const float2 b = reinterpret_cast<const float2*>(gy)[blk];
            v[0] = a.x, v[1] = a.y, g[0] = b.x, g[1] = b.y;
        }
    } else {
        load_row<D>(y, blk, v);
        load_row<D>(gy, blk, g);
    }

    const int64_t per_class = static_cast<int64_t>(rounds) * D * H;
    const float* tc = trig + 2 * c * per_class;
    float* gc = gangles + c * per_class;
    const bool owner = (lane & ((1 << (6 - LH)) - 1)) == 0;
    const int my_pair = lane >> (6 - LH);
    for (int r = rounds - 1; r >= 0; --r) {
        StaticFor<0, D>::run([&](auto kk) {
            constexpr int K = D - 1 - decltype(kk)::value;
            const float* cp = tc + static_cast<int64_t>(r * D + K) * N;
            float contrib[H];
            StaticFor<0, H>::run([&](auto jj) {
                constexpr int j = decltype(jj)::value;
                constexpr int m = ins0(j, K);
                constexpr int n = m + (1 << K);
                const float cs = cp[2 * j];
                const float sn = cp[2 * j + 1];
                contrib[j] = fmaf(g[m], v[n], -(g[n] * v[m]));
                const float vm = v[m], vn = v[n];
                v[m] = fmaf(cs, vm, -(sn * vn));
                v[n] = fmaf(sn, vm, cs * vn);
                const float gm = g[m], gn = g[n];
                g[m] = fmaf(cs, gm, -(sn * gn));
                g[n] = fmaf(sn, gm, cs * gn);
            });
            const float sum = lane_sum<H>(contrib, lane);
            if (owner) unsafeAtomicAdd(gc + static_cast<int64_t>(r * D + K) * H + my_pair, sum);
        });
    }

    if constexpr (D == 1) {
        if (blk >= 0) reinterpret_cast<float2*>(gx)[blk] = make_float2(g[0], g[1]);
    } else {
        float4* L = lds[wv];
        int lane2 = lane;
        asm volatile("" : "+v"(lane2));
        const int sw = swz<G::CHP>(lane2);
        int bb[G::CHP];
        instr_blocks<D>(bb, blk, lane2);
        StaticFor<0, G::PARTS>::run([&](auto pp) {
            store_part<D, decltype(pp)::value>(gx, L, bb, g, lane2, sw);
        });
    }
}

template <int D>
hipError_t launch_bwd(const float* y, const float* gy, float* gx, float* gangles,
                      int64_t nblocks, int rounds, const WsLayout& l, const WsPtrs& p,
                      hipStream_t stream) {
    const int64_t groups = (l.max_tiles + kBwdWaves - 1) / kBwdWaves;
    const dim3 grid(static_cast<unsigned>((groups + kXcds - 1) / kXcds * kXcds));
    hipLaunchKernelGGL((backward_kernel<D>), grid, dim3(64 * kBwdWaves), 0, stream, y, gy, gx,
                       gangles, nblocks, rounds, l.max_tiles, p.tile_class, p.perm, p.trig);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_backward(const float* y, const float* gy, float* gx, float* gangles,
                           int64_t nblocks, int log2n, int rounds, const float* angles,
                           int nclasses, const WsLayout& l, const WsPtrs& p,
                           hipStream_t stream) {
    hipLaunchKernelGGL(backward_prep_kernel, dim3(static_cast<unsigned>(nclasses)),
                       dim3(kPrepThreads), 0, stream, angles, log2n, rounds, p.trig, gangles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nblocks == 0) return e;
    switch (log2n) {
        case 1: return launch_bwd<1>(y, gy, gx, gangles, nblocks, rounds, l, p, stream);
        case 2: return launch_bwd<2>(y, gy, gx, gangles, nblocks, rounds, l, p, stream);
        case 3: return launch_bwd<3>(y, gy, gx, gangles, nblocks, rounds, l, p, stream);
        case 4: return launch_bwd<4>(y, gy, gx, gangles, nblocks, rounds, l, p, stream);
        case 5: return launch_bwd<5>(y, gy, gx, gangles, nblocks, rounds, l, p, stream);
        case 6: return launch_bwd<6>(y, gy, gx, gangles, nblocks, rounds, l, p, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hygt

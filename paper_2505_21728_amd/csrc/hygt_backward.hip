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
// Both the recovered inputs and dL/dx are the inverse rotation (G^T) of the
// pass's outputs and output gradients. So y and g both run through the
// inverse transform's lifting tables (three FMAs per pair each; see
// hygt_table.h), which a preparation launch builds from the angles, and
// carry the same stored signs s: stored values are s times true ones. A
// pair's stored contribution g_m y_n - g_n y_m is then s_m s_n times the
// true one, so the pair's summed contribution is negated where the table
// records that the pair's two signs differ, and dL/dx takes the final signs.
//
// Mapping as in the rotation kernels: one wavefront per class-uniform tile of
// 64 blocks, one lane per block holding the block's y and g (2N registers, so
// N <= 64), the pass's lifting multipliers as wave-uniform scalar operands. The
// N/2 angle contributions of a pass are summed over the 64 lanes by a
// transposed halving: at each step a lane keeps half of its values and adds
// the partner lane's copy of that half, so after log2(N/2) steps each lane
// holds one pair's partial sum; the remaining lane bits are summed directly.
// One atomic add per pair and tile then accumulates the class's gradient
// (FP32 atomics: the order of the additions, so the last bits of the
// gradient, varies from run to run).

#include "hygt_table.h"
#include "hygt_tile.h"

namespace hygt {
namespace {

using namespace tile;

constexpr int kBwdWaves = 4;
constexpr int kBwdWavesPerSimd = 3;
constexpr int kPrepThreads = 256;

// Workgroup c: the inverse-direction lifting table of class c from the
// angles given (with the per-pass sign-difference masks), and the class's
// gradient set to zero.
__global__ __launch_bounds__(kPrepThreads) void backward_prep_kernel(
    const float* __restrict__ angles, int log2n, int rounds, float* __restrict__ bcoef,
    uint32_t* __restrict__ bflip, float* __restrict__ bsigns, int32_t* __restrict__ bmodes,
    float* __restrict__ gangles) {
    __shared__ table::TableShared sh;
    const int64_t c = blockIdx.x;
    const int n = 1 << log2n;
    const int passes = rounds * log2n;
    table::build_table(sh, 1, static_cast<int>(c), angles, nullptr, log2n, rounds,
                       bcoef + c * passes * n, bsigns + c * n, bmodes + c, bflip + c * passes);
    const int per = passes * (n / 2);
    for (int e = threadIdx.x; e < per; e += blockDim.x) gangles[c * per + e] = 0.0f;
}

// Lane exchanges that stay in the vector ALU (no LDS): the gfx950 row and
// half swaps, and DPP rotations inside rows of 16 lanes.
__device__ __forceinline__ float swap_sum32(float x, float y) {
    // x: lanes 32-63 take y's lanes 0-31; y: lanes 0-31 take x's lanes 32-63
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y),
                                                    false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float swap_sum16(float x, float y) {
    // the odd rows of x trade places with the even rows of y
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y),
                                                    false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Value of lane (l - R) mod 16 of the same row, for lane l.
template <int R>
__device__ __forceinline__ float row_ror(float v) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 + R, 0xF, 0xF, true));
}

// Sum over the 64 lanes of a[j], j < H, one value per pair. On return, the
// lanes whose low (6 - log2 H) bits are zero own pair j = lane >> (6 - log2 H)
// and hold its sum.
//
// Transposed halving along lane bits 5, 4, ..., 6 - log2 H: at the step for
// bit b a lane keeps the half of its values that its bit b selects (the
// upper half where the bit is set) and adds the partner lane's (lane ^ 2^b)
// copy of that half. For bits 5 and 4 one swap instruction moves both halves
// at once; for lower bits each lane rotates both halves within its row and
// keeps the sum it needs. The lanes that end up holding the same pair are
// then summed into the lowest of them.
template <int H>
__device__ __forceinline__ float lane_sum(float (&a)[H], int lane) {
    constexpr int LH = H == 1 ? 0 : H == 2 ? 1 : H == 4 ? 2 : H == 8 ? 3 : H == 16 ? 4 : 5;
    StaticFor<0, LH>::run([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        constexpr int K = H >> (s + 1);  // values kept after this step
        constexpr int b = 5 - s;
        const bool hi = (lane >> b) & 1;
        StaticFor<0, K>::run([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            if constexpr (b == 5) {
                a[i] = swap_sum32(a[i], a[i + K]);
            } else if constexpr (b == 4) {
                a[i] = swap_sum16(a[i], a[i + K]);
            } else {
                // bit clear: partner l + 2^b, bit set: partner l - 2^b
                const float lo_sum = a[i] + row_ror<16 - (1 << b)>(a[i]);
                const float hi_sum = a[i + K] + row_ror<(1 << b)>(a[i + K]);
                a[i] = hi ? hi_sum : lo_sum;
            }
        });
    });
    // bits 0 .. 5 - LH: lane l adds the partial sum of lane l + 2^b, so that
    // the lowest lane of each group ends with the group's total
    float v = a[0];
    StaticFor<0, 6 - LH>::run([&](auto bb) {
        constexpr int b = decltype(bb)::value;
        if constexpr (b == 5)
            v = swap_sum32(v, v);
        else if constexpr (b == 4)
            v = swap_sum16(v, v);
        else
            v += row_ror<16 - (1 << b)>(v);
    });
    return v;
}

template <int D>
__global__ __launch_bounds__(64 * kBwdWaves) __attribute__((amdgpu_waves_per_eu(kBwdWavesPerSimd)))
void backward_kernel(const float* __restrict__ y, const float* __restrict__ gy,
                     float* __restrict__ gx, float* __restrict__ gangles, int64_t nblocks,
                     int rounds, int64_t max_tiles, const int32_t* __restrict__ tile_class,
                     const int32_t* __restrict__ perm, const float* __restrict__ bcoef,
                     const uint32_t* __restrict__ bflip, const float* __restrict__ bsigns,
                     const int32_t* __restrict__ bmodes) {
    using G = TileGeo<D>;
    constexpr int N = 1 << D;
    constexpr int H = N / 2;
    constexpr int LH = D - 1;
    __shared__ float4 lds[kBwdWaves][kTile * G::CHP];

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kBwdWaves + wv;
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

    const int64_t passes = static_cast<int64_t>(rounds) * D;
    ctab_f tc = as_ctab(bcoef) + c * passes * N;
    ctab_i fc = as_ctab(reinterpret_cast<const int32_t*>(bflip)) + c * passes;
    float* gc = gangles + c * passes * H;
    const bool owner = (lane & ((1 << (6 - LH)) - 1)) == 0;
    const int my_pair = lane >> (6 - LH);
    // rr-th round of the walk = forward round rounds-1-rr; its passes K = D-1 .. 0
    for (int rr = 0; rr < rounds; ++rr) {
        const int r = rounds - 1 - rr;
        StaticFor<0, D>::run([&](auto kk) {
            constexpr int K = D - 1 - decltype(kk)::value;
            const int64_t p = static_cast<int64_t>(rr) * D + decltype(kk)::value;
            ctab_f cp = tc + p * N;
            const uint32_t flip = static_cast<uint32_t>(fc[p]);
            float contrib[H];
            StaticFor<0, H>::run([&](auto jj) {
                constexpr int j = decltype(jj)::value;
                constexpr int m = ins0(j, K);
                constexpr int n = m + (1 << K);
                const float pm = cp[2 * j];
                const float qm = cp[2 * j + 1];
                contrib[j] = fmaf(g[m], v[n], -(g[n] * v[m]));
                v[m] = fmaf(pm, v[n], v[m]);
                v[n] = fmaf(qm, v[m], v[n]);
                v[m] = fmaf(pm, v[n], v[m]);
                g[m] = fmaf(pm, g[n], g[m]);
                g[n] = fmaf(qm, g[m], g[n]);
                g[m] = fmaf(pm, g[n], g[m]);
            });
            float sum = lane_sum<H>(contrib, lane);
            if ((flip >> my_pair) & 1u) sum = -sum;
            if (owner) unsafeAtomicAdd(gc + static_cast<int64_t>(r * D + K) * H + my_pair, sum);
        });
    }
    // stored gradients carry the walk's final signs
    if (as_ctab(bmodes)[c]) {
        ctab_f sg = as_ctab(bsigns) + c * N;
        StaticFor<0, N>::run([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            g[i] *= sg[i];
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
    const dim3 grid(static_cast<unsigned>((l.max_tiles + kBwdWaves - 1) / kBwdWaves));
    hipLaunchKernelGGL((backward_kernel<D>), grid, dim3(64 * kBwdWaves), 0, stream, y, gy, gx,
                       gangles, nblocks, rounds, l.max_tiles, p.tile_class, p.perm, p.bcoef,
                       p.bflip, p.bsigns, p.bmodes);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_backward(const float* y, const float* gy, float* gx, float* gangles,
                           int64_t nblocks, int log2n, int rounds, const float* angles,
                           int nclasses, const WsLayout& l, const WsPtrs& p,
                           hipStream_t stream) {
    hipLaunchKernelGGL(backward_prep_kernel, dim3(static_cast<unsigned>(nclasses)),
                       dim3(kPrepThreads), 0, stream, angles, log2n, rounds, p.bcoef, p.bflip,
                       p.bsigns, p.bmodes, gangles);
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

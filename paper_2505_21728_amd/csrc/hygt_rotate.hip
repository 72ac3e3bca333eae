// The HyGT rotation kernels: R rounds of log2(N) parallel-Givens passes over
// a batch of blocks (Sec. IV, eq. (5)-(9)).
//
// Mapping. One wavefront owns a tile of 64 blocks of one class, one lane per
// block, and keeps its block's N values in registers for all passes: every
// butterfly of every pass is a register-to-register operation with
// compile-time register indices, and the class's per-pass multipliers are
// wave-uniform, so they arrive through scalar loads as SGPR operands of the
// FMAs. Nothing is exchanged between lanes during the passes. For N = 256 a
// lane's registers cannot hold a block, so two wavefronts share the tile,
// wavefront h holding values 128h .. 128h+127 of every block; the passes
// along bit 7 pair the two halves, which swap values through LDS in parts of
// 16 per lane.
//
// Memory. Each lane loads its own block (for N = 256, its half of the block)
// straight into registers, N / 4 loads of 16 bytes all in flight at once, so
// the first passes start on the chunks that arrive first. The way out goes
// through LDS: each lane writes its row, and the transposed slots go out so
// that each store instruction writes whole blocks (or whole 128-byte halves
// of 8x8 blocks), 16 bytes per lane; an XOR swizzle of the 16-byte chunks in
// LDS keeps the row writes on distinct banks. A tile goes out in parts of at
// most 8 chunks per block, so a wavefront needs only 8 KB of LDS. Stores are
// non-temporal. Measured on MI355X with cache-cold inputs, direct loads beat
// a gather through LDS (global_load_lds_dwordx4) by 4 to 6 us per 2^20 8x8
// blocks, and non-temporal stores beat ordinary ones by 14 us.
//
// Scheduling. Each wavefront handles one tile, four per workgroup. The
// lifting form needs no temporaries, so a wavefront fits in under 100 VGPRs
// and five wavefronts per SIMD stay resident: measured on MI355X, raising
// residency from two to five wavefronts per SIMD cut the 8x8 forward
// transform from 177 to 144 us, because loads, rotations and stores of
// different tiles then overlap. Tiles are sorted by class (see
// hygt_plan.hip) and each XCD walks its own contiguous share of the tile
// list, so the wavefronts that share a scalar cache mostly read one class
// table: measured on MI355X, the rotation slows by about a third once a
// compute-unit pair's wavefronts touch more than about three tables.
//
// Arithmetic. Each pair is rotated with the three in-place lifting steps
// built by the plan (see hygt_plan.hip), and a class whose sign bookkeeping
// left negative outputs multiplies them by -1 at the end. Every operation is
// an explicit fmaf or an exact sign flip, so every block of a class sees the
// same rounding whatever the batch, tile or launch.

#include "hygt_tile.h"

namespace hygt {
namespace {

using namespace tile;

// The passes act on T blocks at once (one per tile of the wavefront, all of
// one class): every multiplier fetched is used by T blocks.

// One pass along hypercube dimension K: each pair (m, n) gets the lifting
// steps a += p b, b += q a, a += p b, in place (three FMAs, no temporary).
template <int D, int K, int T>
__device__ __forceinline__ void pass_lift(float (&v)[T][1 << D], const float* __restrict__ cp) {
    StaticFor<0, (1 << D) / 2>::run([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        constexpr int m = ins0(j, K);
        constexpr int n = m + (1 << K);
        const float p = cp[2 * j];
        const float q = cp[2 * j + 1];
        StaticFor<0, T>::run([&](auto uu) {
            constexpr int u = decltype(uu)::value;
            v[u][m] = fmaf(p, v[u][n], v[u][m]);
            v[u][n] = fmaf(q, v[u][m], v[u][n]);
            v[u][m] = fmaf(p, v[u][n], v[u][m]);
        });
    });
}

// R rounds of D passes in application order (forward: k = 0..D-1 in every
// round; inverse: k = D-1..0), then the final signs. RT > 0 unrolls the
// rounds at compile time (RT == R); RT == 0 loops over `rounds`.
template <int D, int DIR, int RT, int T>
__device__ __forceinline__ void run_passes(float (&v)[T][1 << D], const float* __restrict__ tbl,
                                           const float* __restrict__ sign, int has_neg,
                                           int rounds) {
    constexpr int N = 1 << D;
    auto one_round = [&](int r) {
        StaticFor<0, D>::run([&](auto kk) {
            constexpr int K = DIR == 0 ? decltype(kk)::value : D - 1 - decltype(kk)::value;
            pass_lift<D, K, T>(v, tbl + static_cast<size_t>(r * D + decltype(kk)::value) * N);
        });
    };
    if constexpr (RT > 0) {
        StaticFor<0, RT>::run([&](auto rr) { one_round(decltype(rr)::value); });
    } else {
        for (int r = 0; r < rounds; ++r) one_round(r);
    }
    if (has_neg) {
        StaticFor<0, N>::run([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            const float sg = sign[i];
            StaticFor<0, T>::run([&](auto uu) { v[decltype(uu)::value][i] *= sg; });
        });
    }
}

// N = 256: a pass along bit 7 pairs value j of wavefront 0 (element j) with
// value j of wavefront 1 (element 128 + j). The wavefronts swap their values
// through LDS, 16 per lane at a time, and each computes its own outputs:
// y_m = c x_m + s x_n on wavefront 0, y_n = c x_n - s x_m on wavefront 1,
// with (c, s) = cp[2j], cp[2j + 1]. `xo` is this wavefront's exchange area
// and `xp` the other's, each two buffers of [4][64] float4; part g uses
// buffer g % 2, so the barrier of part g + 1 also guarantees that both
// wavefronts have read part g before either overwrites its buffer.
__device__ __forceinline__ void cross_pass(float (&v)[128], const float* __restrict__ cp,
                                           unsigned hbit, float4* xo, const float4* xp,
                                           int lane) {
    StaticFor<0, 8>::run([&](auto gg) {
        constexpr int g = decltype(gg)::value;
        constexpr int buf = g & 1;
        StaticFor<0, 4>::run([&](auto qq) {
            constexpr int q = decltype(qq)::value;
            constexpr int e = 16 * g + 4 * q;
            xo[(buf * 4 + q) * 64 + lane] = make_float4(v[e], v[e + 1], v[e + 2], v[e + 3]);
        });
        __syncthreads();
        float w[16];
        StaticFor<0, 4>::run([&](auto qq) {
            constexpr int q = decltype(qq)::value;
            const float4 f = xp[(buf * 4 + q) * 64 + lane];
            w[4 * q + 0] = f.x;
            w[4 * q + 1] = f.y;
            w[4 * q + 2] = f.z;
            w[4 * q + 3] = f.w;
        });
        StaticFor<0, 16>::run([&](auto tt) {
            constexpr int t = decltype(tt)::value;
            constexpr int j = 16 * g + t;
            const float c = cp[2 * j];
            const float sn = cp[2 * j + 1];
            // -s on wavefront 1: a sign-bit flip of a wave-uniform value
            const float sg = __uint_as_float(__float_as_uint(sn) ^ hbit);
            v[j] = fmaf(sg, w[t], c * v[j]);
        });
    });
}

// N = 256, wavefront h of a tile: R rounds of 8 passes in application order.
// Passes along bits 0..6 act on the lane's 128 values with the multipliers
// of pairs 64h .. 64h + 63 of the pass; passes along bit 7 go through
// cross_pass. Then the final signs of elements 128h .. 128h + 127.
template <int DIR>
__device__ __forceinline__ void run_passes_split(float (&v)[1][128], const float* __restrict__ tbl,
                                                 const float* __restrict__ sign, int has_neg,
                                                 int rounds, int h, float4* xo, const float4* xp,
                                                 int lane) {
    constexpr int D = 8;
    constexpr int N = 256;
    for (int r = 0; r < rounds; ++r) {
        StaticFor<0, D>::run([&](auto kk) {
            constexpr int K = DIR == 0 ? decltype(kk)::value : D - 1 - decltype(kk)::value;
            const float* cp = tbl + static_cast<size_t>(r * D + decltype(kk)::value) * N;
            if constexpr (K >= kLaneBits)
                cross_pass(v[0], cp, static_cast<unsigned>(h) << 31, xo, xp, lane);
            else
                pass_lift<kLaneBits, K, 1>(v, cp + h * (N / 2));
        });
    }
    if (has_neg) {
        StaticFor<0, N / 2>::run([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            v[0][i] *= sign[h * (N / 2) + i];
        });
    }
}

// N >= 4: LDS-staged tiles, one lane per block; one tile per wavefront, or
// for N = 256 one tile per pair of wavefronts (a workgroup), wavefront h
// holding half h of every block.
//
// x and y may be the same array (in place): every value is read by the
// wavefront that owns it and written back only after that read has
// completed, and no other wavefront touches it, so the restrict qualifiers
// (which let the per-tile class loads stay scalar) hold for every pair of
// accesses that the compiler could reorder.
template <int D, int DIR, int RT>
__global__ __launch_bounds__(64 * TileGeo<D>::WAVES)
__attribute__((amdgpu_waves_per_eu(TileGeo<D>::OCC)))
void rotate_kernel(const float* __restrict__ x, float* __restrict__ y, int64_t nblocks,
                   int rounds, int nclasses, int64_t max_tiles,
                   const int32_t* __restrict__ tile_class, const int32_t* __restrict__ perm,
                   const int32_t* __restrict__ modes, const float* __restrict__ coef,
                   const float* __restrict__ signs) {
    using G = TileGeo<D>;
    constexpr int N = G::N;
    constexpr int CHP = G::CHP;
    constexpr int T = G::SPLIT ? 1 : kTilesPerWave;
    // Staging of a part; for N = 256 also the exchange area (2 x 4 x 64 float4).
    __shared__ float4 lds[G::WAVES][kTile * CHP];
    static_assert(!G::SPLIT || kTile * CHP >= 2 * 4 * 64, "exchange area too small");

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int h = G::SPLIT ? wv : 0;  // half of every block held by this wavefront
    // This wavefront's T consecutive tiles; the plan gives them one class.
    const int64_t t0 = G::SPLIT ? xcd_tile_group() : (xcd_tile_group() * kWaves + wv) * T;
    if (t0 >= max_tiles) return;  // both wavefronts of a split tile leave together
    const int c = __builtin_amdgcn_readfirstlane(tile_class[t0]);
    if (c < 0) return;  // past the last tile
    const float* xh = x + h * G::V;
    float* yh = y + h * G::V;
    float4* L = lds[wv];
    int blk[T];
    float v[T][G::V];
    StaticFor<0, T>::run([&](auto uu) {
        constexpr int u = decltype(uu)::value;
        blk[u] = valid_block(perm[(t0 + u) * kTile + lane], nblocks);
        load_row<D>(xh, blk[u], v[u]);
    });

    const size_t passes = static_cast<size_t>(rounds) * D;
    const size_t table = static_cast<size_t>(DIR) * nclasses + c;
    if constexpr (G::SPLIT) {
        run_passes_split<DIR>(v, coef + table * passes * N, signs + table * N, modes[table],
                              rounds, h, lds[h], lds[1 - h], lane);
        // The other wavefront's last reads of this wavefront's exchange area
        // come before the stores below reuse it for staging.
        __syncthreads();
    } else {
        run_passes<D, DIR, RT, T>(v, coef + table * passes * N, signs + table * N,
                                  modes[table], rounds);
    }

    // Addresses for the way out are derived again from the block ids and the
    // lane index, made opaque here so that the compiler does not keep the
    // ones of the way in alive (in registers) across the passes.
    int lane2 = lane;
    asm volatile("" : "+v"(lane2));
    const int sw2 = swz<CHP>(lane2);
    StaticFor<0, T>::run([&](auto uu) {
        constexpr int u = decltype(uu)::value;
        int b = blk[u];
        asm volatile("" : "+v"(b));
        int bb[CHP];
        instr_blocks<D>(bb, b, lane2);
        StaticFor<0, G::PARTS>::run([&](auto pp) {
            store_part<D, decltype(pp)::value>(yh, L, bb, v[u], lane2, sw2);
        });
    });
}

// N == 2: one 8-byte block per lane, read and written directly.
template <int DIR>
__global__ __launch_bounds__(64 * kWaves) void rotate_kernel_n2(
    const float* __restrict__ x, float* __restrict__ y, int64_t nblocks, int rounds,
    int nclasses, int64_t max_tiles, const int32_t* __restrict__ tile_class,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ modes,
    const float* __restrict__ coef, const float* __restrict__ signs) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t0 = (xcd_tile_group() * kWaves + wv) * kTilesPerWave;
    if (t0 >= max_tiles) return;
    const int c = __builtin_amdgcn_readfirstlane(tile_class[t0]);
    if (c < 0) return;
    const size_t table = static_cast<size_t>(DIR) * nclasses + c;
    for (int u = 0; u < kTilesPerWave; ++u) {
        const int blk = valid_block(perm[(t0 + u) * kTile + lane], nblocks);
        if (blk < 0) continue;
        const float2 in = *reinterpret_cast<const float2*>(x + static_cast<int64_t>(blk) * 2);
        float v[1][2] = {{in.x, in.y}};
        run_passes<1, DIR, 0, 1>(v, coef + table * rounds * 2, signs + table * 2, modes[table],
                                 rounds);
        *reinterpret_cast<float2*>(y + static_cast<int64_t>(blk) * 2) =
            make_float2(v[0][0], v[0][1]);
    }
}

template <int D, int DIR, int RT>
hipError_t launch_one(const float* x, float* y, int64_t nblocks, int rounds, int nclasses,
                      const WsLayout& l, const WsPtrs& p, hipStream_t stream) {
    using G = TileGeo<D>;
    const int64_t per_group = G::SPLIT ? 1 : static_cast<int64_t>(kWaves) * kTilesPerWave;
    const int64_t groups = (l.max_tiles + per_group - 1) / per_group;
    const dim3 grid(static_cast<unsigned>((groups + kXcds - 1) / kXcds * kXcds));
    const dim3 block(D == 1 ? 64 * kWaves : 64 * G::WAVES);
    if constexpr (D == 1)
        hipLaunchKernelGGL((rotate_kernel_n2<DIR>), grid, block, 0, stream, x, y, nblocks,
                           rounds, nclasses, l.max_tiles, p.tile_class, p.perm, p.modes, p.coef,
                           p.signs);
    else
        hipLaunchKernelGGL((rotate_kernel<D, DIR, RT>), grid, block, 0, stream, x, y, nblocks,
                           rounds, nclasses, l.max_tiles, p.tile_class, p.perm, p.modes,
                           p.coef, p.signs);
    return hipGetLastError();
}

// Round counts unrolled at compile time; others take the looping kernel.
template <int D, int DIR>
hipError_t launch_rounds(const float* x, float* y, int64_t nblocks, int rounds, int nclasses,
                         const WsLayout& l, const WsPtrs& p, hipStream_t stream) {
    if constexpr (D == 1 || D >= 7) {
        // N = 2, and N >= 128 (whose unrolled rounds would not fit the
        // instruction cache), loop over the rounds.
        return launch_one<D, DIR, 0>(x, y, nblocks, rounds, nclasses, l, p, stream);
    } else {
        switch (rounds) {
            case 1: return launch_one<D, DIR, 1>(x, y, nblocks, rounds, nclasses, l, p, stream);
            case 2: return launch_one<D, DIR, 2>(x, y, nblocks, rounds, nclasses, l, p, stream);
            case 3: return launch_one<D, DIR, 3>(x, y, nblocks, rounds, nclasses, l, p, stream);
            case 4: return launch_one<D, DIR, 4>(x, y, nblocks, rounds, nclasses, l, p, stream);
            case 5: return launch_one<D, DIR, 5>(x, y, nblocks, rounds, nclasses, l, p, stream);
            default: return launch_one<D, DIR, 0>(x, y, nblocks, rounds, nclasses, l, p, stream);
        }
    }
}

template <int DIR>
hipError_t launch_dir(const float* x, float* y, int64_t nblocks, int log2n, int rounds,
                      int nclasses, const WsLayout& l, const WsPtrs& p, hipStream_t stream) {
    switch (log2n) {
        case 1: return launch_rounds<1, DIR>(x, y, nblocks, rounds, nclasses, l, p, stream);
        case 2: return launch_rounds<2, DIR>(x, y, nblocks, rounds, nclasses, l, p, stream);
        case 3: return launch_rounds<3, DIR>(x, y, nblocks, rounds, nclasses, l, p, stream);
        case 4: return launch_rounds<4, DIR>(x, y, nblocks, rounds, nclasses, l, p, stream);
        case 5: return launch_rounds<5, DIR>(x, y, nblocks, rounds, nclasses, l, p, stream);
        case 6: return launch_rounds<6, DIR>(x, y, nblocks, rounds, nclasses, l, p, stream);
        case 7: return launch_rounds<7, DIR>(x, y, nblocks, rounds, nclasses, l, p, stream);
        case 8: return launch_rounds<8, DIR>(x, y, nblocks, rounds, nclasses, l, p, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_rotate(const float* x, float* y, int64_t nblocks, int log2n, int rounds,
                         int nclasses, int direction, const WsLayout& l, const WsPtrs& p,
                         hipStream_t stream) {
    if (direction == 0) return launch_dir<0>(x, y, nblocks, log2n, rounds, nclasses, l, p, stream);
    return launch_dir<1>(x, y, nblocks, log2n, rounds, nclasses, l, p, stream);
}

}  // namespace hygt

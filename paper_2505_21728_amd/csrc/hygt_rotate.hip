// The HyGT rotation kernels: R rounds of log2(N) parallel-Givens passes over
// a batch of blocks (Sec. IV, eq. (5)-(9)).
//
// Mapping (N <= 64). One wavefront owns a tile of 64 blocks of one class, one
// lane per block, and keeps its block's N values in registers for all
// passes: every butterfly of every pass is a register-to-register operation
// with compile-time register indices, and the class's per-pass multipliers
// are wave-uniform, so they arrive through scalar loads as SGPR operands of
// the FMAs. Nothing is exchanged between lanes during the passes.
//
// Memory. A tile's blocks are moved between HBM and registers through LDS
// so that every global access covers whole 256-byte blocks: each load
// instruction fetches 16 bytes per lane for 64/(N/4) blocks, with the 16-byte
// chunks of a block rotated by an XOR swizzle so that the per-lane row reads
// (and the mirror-image writes on the way out) hit distinct LDS banks. Loads
// go straight to LDS (global_load_lds_dwordx4) without passing through VGPRs.
//
// Arithmetic. A class's transform runs either in the scaled schedule (every
// pass but the last as two FMAs per butterfly, the last pass direct) or, when
// its angles would drive the scale factors out of range, in the direct
// schedule (a multiply and an FMA per output everywhere); the plan picks the
// schedule from the angles alone (see hygt_plan.hip). Every operation is an
// explicit fmaf or a single multiply, so every block of a class sees the same
// rounding whatever the batch, tile or launch.

#include "hygt_internal.h"

namespace hygt {
namespace {

template <int I, int End>
struct StaticFor {
    template <typename F>
    __device__ __forceinline__ static void run(F&& f) {
        if constexpr (I < End) {
            f(std::integral_constant<int, I>{});
            StaticFor<I + 1, End>::run(f);
        }
    }
};

using lds_void_ptr = __attribute__((address_space(3))) void*;

constexpr int ins0(int j, int k) { return ((j >> k) << (k + 1)) | (j & ((1 << k) - 1)); }

// XOR swizzle of a block's 16-byte chunk index inside a tile's LDS image.
// With chunk q of block b at slot b*CH + (q ^ swz(b)), 8 (and 16) consecutive
// lanes reading the same q touch 8 (16) distinct 16-byte bank groups.
template <int CH>
__device__ __forceinline__ int swz(int b) {
    if constexpr (CH == 16) return b & 15;
    else if constexpr (CH == 8) return (b ^ (b >> 3)) & 7;
    else if constexpr (CH == 4) return ((b >> 1) ^ (b >> 3)) & 3;
    else if constexpr (CH == 2) return ((b >> 2) ^ (b >> 3)) & 1;
    else return 0;
}

// One scaled pass along hypercube dimension K.
template <int D, int K>
__device__ __forceinline__ void pass_scaled(float (&v)[1 << D], const float* __restrict__ cp) {
    StaticFor<0, (1 << D) / 2>::run([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        constexpr int m = ins0(j, K);
        constexpr int n = m + (1 << K);
        const float a = v[m];
        const float b = v[n];
        v[m] = fmaf(cp[2 * j], b, a);
        v[n] = fmaf(cp[2 * j + 1], a, b);
    });
}

// One direct pass along hypercube dimension K.
template <int D, int K>
__device__ __forceinline__ void pass_direct(float (&v)[1 << D], const float* __restrict__ cp) {
    StaticFor<0, (1 << D) / 2>::run([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        constexpr int m = ins0(j, K);
        constexpr int n = m + (1 << K);
        const float a = v[m];
        const float b = v[n];
        v[m] = fmaf(cp[4 * j], a, cp[4 * j + 1] * b);
        v[n] = fmaf(cp[4 * j + 2], b, cp[4 * j + 3] * a);
    });
}

// All passes but the last in the scaled form, the last direct. RT > 0 unrolls
// the R rounds at compile time (RT == R); RT == 0 loops over `rounds`.
template <int D, int DIR, int RT>
__device__ __forceinline__ void run_scaled_schedule(float (&v)[1 << D], const float* __restrict__ tbl,
                                                    int rounds) {
    constexpr int N = 1 << D;
    auto one_round = [&](int r, auto last_round) {
        StaticFor<0, D>::run([&](auto kk) {
            constexpr int K = DIR == 0 ? decltype(kk)::value : D - 1 - decltype(kk)::value;
            const float* cp = tbl + static_cast<size_t>(r * D + decltype(kk)::value) * 2 * N;
            if constexpr (decltype(last_round)::value && decltype(kk)::value == D - 1)
                pass_direct<D, K>(v, cp);
            else
                pass_scaled<D, K>(v, cp);
        });
    };
    if constexpr (RT > 0) {
        StaticFor<0, RT - 1>::run([&](auto rr) { one_round(decltype(rr)::value, std::false_type{}); });
        one_round(RT - 1, std::true_type{});
    } else {
        for (int r = 0; r < rounds - 1; ++r) one_round(r, std::false_type{});
        one_round(rounds - 1, std::true_type{});
    }
}

// Every pass direct (classes whose scaled schedule would leave the safe range).
template <int D, int DIR, int RT>
__device__ __forceinline__ void run_direct_schedule(float (&v)[1 << D], const float* __restrict__ tbl,
                                                    int rounds) {
    constexpr int N = 1 << D;
    auto one_round = [&](int r) {
        StaticFor<0, D>::run([&](auto kk) {
            constexpr int K = DIR == 0 ? decltype(kk)::value : D - 1 - decltype(kk)::value;
            pass_direct<D, K>(v, tbl + static_cast<size_t>(r * D + decltype(kk)::value) * 2 * N);
        });
    };
    if constexpr (RT > 0) {
        StaticFor<0, RT>::run([&](auto rr) { one_round(decltype(rr)::value); });
    } else {
        for (int r = 0; r < rounds; ++r) one_round(r);
    }
}

template <int D, int DIR, int RT>
__device__ __forceinline__ void run_passes(float (&v)[1 << D], const float* __restrict__ tbl,
                                           int direct_mode, int rounds) {
    if (direct_mode)
        run_direct_schedule<D, DIR, RT>(v, tbl, rounds);
    else
        run_scaled_schedule<D, DIR, RT>(v, tbl, rounds);
}

struct TileInfo {
    int cls;
    int count;
    int64_t first;
    bool valid;
};

__device__ __forceinline__ TileInfo tile_info(int64_t tile, const PlanHeader* __restrict__ hdr,
                                              const int4* __restrict__ tiles, int64_t nblocks) {
    TileInfo t{0, 0, 0, false};
    if (hdr->grouped) {
        if (tile >= hdr->ntiles) return t;
        const int4 d = tiles[tile];
        t.cls = __builtin_amdgcn_readfirstlane(d.x);
        t.first = __builtin_amdgcn_readfirstlane(d.y);
        t.count = __builtin_amdgcn_readfirstlane(d.z);
    } else {
        t.first = tile * kTile;
        if (t.first >= nblocks) return t;
        t.count = static_cast<int>(min<int64_t>(kTile, nblocks - t.first));
    }
    t.valid = true;
    return t;
}

// N >= 4: LDS-staged tile, one lane per block.
template <int D, int DIR, int RT>
__global__ __launch_bounds__(256) void rotate_kernel(
    const float* x, float* y, int64_t nblocks, int rounds, int nclasses,
    const PlanHeader* __restrict__ hdr, const int4* __restrict__ tiles,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ modes,
    const float* __restrict__ coef) {
    constexpr int N = 1 << D;
    constexpr int CH = N / 4;       // 16-byte chunks per block
    constexpr int BPI = 64 / CH;    // blocks per load instruction
    __shared__ float4 lds[4][kTile * CH];

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t tile = static_cast<int64_t>(blockIdx.x) * 4 + wv;
    const TileInfo ti = tile_info(tile, hdr, tiles, nblocks);
    if (!ti.valid) return;

    int blk = -1;
    if (lane < ti.count && ti.first + lane < nblocks) {
        blk = hdr->grouped ? perm[ti.first + lane] : static_cast<int>(ti.first + lane);
        if (blk < 0 || blk >= nblocks) blk = -1;  // never touch memory outside x / y
    }

    float4* L = lds[wv];
    // Gather: instruction i fetches chunk (lane%CH)^swz(b) of block b = i*BPI + lane/CH.
    StaticFor<0, CH>::run([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        const int b = i * BPI + lane / CH;
        const int bb = __builtin_amdgcn_ds_bpermute(b << 2, blk);
        const int ch = (lane % CH) ^ swz<CH>(b);
        if (bb >= 0)
            __builtin_amdgcn_global_load_lds(x + static_cast<int64_t>(bb) * N + ch * 4,
                                             (lds_void_ptr)(L + i * 64), 16, 0, 0);
    });
    // The DMA writes land in LDS asynchronously: wait for them before the
    // row reads (the asm also keeps the compiler from hoisting those reads).
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");

    float v[N];
    const int sw = swz<CH>(lane);
    StaticFor<0, CH>::run([&](auto qq) {
        constexpr int q = decltype(qq)::value;
        const float4 t = L[lane * CH + (q ^ sw)];
        v[4 * q + 0] = t.x;
        v[4 * q + 1] = t.y;
        v[4 * q + 2] = t.z;
        v[4 * q + 3] = t.w;
    });

    const size_t table = static_cast<size_t>(DIR) * nclasses + ti.cls;
    const size_t passes = static_cast<size_t>(rounds) * D;
    run_passes<D, DIR, RT>(v, coef + table * passes * 2 * N, modes[table], rounds);

    StaticFor<0, CH>::run([&](auto qq) {
        constexpr int q = decltype(qq)::value;
        L[lane * CH + (q ^ sw)] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    });
    // Rows written by each lane are read back by other lanes of the same
    // wavefront; LDS executes one wavefront's operations in order, so only the
    // compiler's ordering needs pinning here.
    asm volatile("" ::: "memory");
    StaticFor<0, CH>::run([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        const int b = i * BPI + lane / CH;
        const int bb = __builtin_amdgcn_ds_bpermute(b << 2, blk);
        const int ch = (lane % CH) ^ swz<CH>(b);
        const float4 t = L[i * 64 + lane];
        if (bb >= 0) *reinterpret_cast<float4*>(y + static_cast<int64_t>(bb) * N + ch * 4) = t;
    });
}

// N == 2: one 8-byte block per lane, read and written directly.
template <int DIR>
__global__ __launch_bounds__(256) void rotate_kernel_n2(
    const float* x, float* y, int64_t nblocks, int rounds, int nclasses,
    const PlanHeader* __restrict__ hdr, const int4* __restrict__ tiles,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ modes,
    const float* __restrict__ coef) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t tile = static_cast<int64_t>(blockIdx.x) * 4 + wv;
    const TileInfo ti = tile_info(tile, hdr, tiles, nblocks);
    if (!ti.valid) return;
    if (lane >= ti.count || ti.first + lane >= nblocks) return;
    const int blk = hdr->grouped ? perm[ti.first + lane] : static_cast<int>(ti.first + lane);
    if (blk < 0 || blk >= nblocks) return;  // never touch memory outside x / y
    const float2 in = *reinterpret_cast<const float2*>(x + static_cast<int64_t>(blk) * 2);
    float v[2] = {in.x, in.y};
    const size_t table = static_cast<size_t>(DIR) * nclasses + ti.cls;
    run_passes<1, DIR, 0>(v, coef + table * rounds * 4, modes[table], rounds);
    *reinterpret_cast<float2*>(y + static_cast<int64_t>(blk) * 2) = make_float2(v[0], v[1]);
}

template <int D, int DIR, int RT>
hipError_t launch_one(const float* x, float* y, int64_t nblocks, int rounds, int nclasses,
                      const WsLayout& l, const WsPtrs& p, hipStream_t stream) {
    const dim3 grid(static_cast<unsigned>((l.max_tiles + 3) / 4));
    if constexpr (D == 1)
        hipLaunchKernelGGL((rotate_kernel_n2<DIR>), grid, dim3(256), 0, stream, x, y, nblocks,
                           rounds, nclasses, p.hdr, p.tiles, p.perm, p.modes, p.coef);
    else
        hipLaunchKernelGGL((rotate_kernel<D, DIR, RT>), grid, dim3(256), 0, stream, x, y,
                           nblocks, rounds, nclasses, p.hdr, p.tiles, p.perm, p.modes, p.coef);
    return hipGetLastError();
}

// Round counts unrolled at compile time; others take the looping kernel.
template <int D, int DIR>
hipError_t launch_rounds(const float* x, float* y, int64_t nblocks, int rounds, int nclasses,
                         const WsLayout& l, const WsPtrs& p, hipStream_t stream) {
    if constexpr (D == 1) {
        return launch_one<1, DIR, 0>(x, y, nblocks, rounds, nclasses, l, p, stream);
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

// The HyGT rotation kernels: R rounds of log2(N) parallel-Givens passes over
// a batch of blocks (Sec. IV, eq. (5)-(9)).
//
// Mapping. One wavefront owns a tile of 64 blocks of one class, one lane per
// block, and keeps its block's N values in registers for all passes: every
// butterfly of every pass is a register-to-register operation with
// compile-time register indices, and the class's per-pass multipliers are
// wave-uniform, so they arrive through scalar loads as SGPR operands of the
// FMAs. Nothing is exchanged between lanes during the passes. A lane holds
// at most 64 values, so for N = 128 and N = 256 two and four wavefronts share
// the tile, wavefront q holding values 64q .. 64q+63 of every block; the
// passes along bits 6 and 7 pair values of two wavefronts, which swap them
// through double-buffered LDS areas in parts of 16 per lane and rotate with
// (cos, sin) multipliers instead of the lifting steps.
//
// Multipliers. The class table is read in chunks of the multipliers of up to
// 16 pairs, each chunk requested one chunk ahead of its use (TableStream in
// hygt_tile.h), so that the scalar loads of a pass overlap the arithmetic of
// the pass before. Measured on MI355X (2^20 8x8 blocks, R = 4), this took
// the forward transform from 119 to 112 us with the tiles in class order, and
// made the cost of switching class tables between neighbouring tiles
// negligible. Tiles of N >= 128 (and the 8x8 tiles of the mixed launch)
// stream their chunks into VGPRs instead, four chunks ahead, and read each
// multiplier from its lane of the row by DPP (VTableStream in hygt_tile.h):
// their few wavefronts cannot hide a scalar load's L2 round trip behind each
// other.
//
// Variants. The permutation pass of Fig. 4 (N <= 64) reorders each lane's
// row through a per-wavefront LDS row area after the passes (forward) or
// before them (inverse). The fused launch for batches of several block
// sizes (mixed_kernel) runs the same tile body over one persistent grid.
// The request kernel (at the end) serves batches of requests with no class
// grouping: a wavefront takes one block (or 64 / N blocks of N <= 32) and
// reads its class table a pass at a time.
//
// Memory. The single-size kernels with N <= 64 bring a tile in through LDS
// by DMA: each global_load_lds_dwordx4 reads the chunks of several whole
// blocks, and each lane then reads its own row from LDS; for N = 64 half of
// every block comes that way and the other half by the lanes' own row
// loads, all in flight at once (load_tile in hygt_tile.h). The fused mixed
// kernel, and tiles of N > 64, load each lane's block (or share of it)
// straight into registers. The way out goes through LDS: each lane writes
// its row, and the transposed slots go out so that each store instruction
// writes whole blocks (or whole 128-byte halves of 8x8 blocks), 16 bytes per
// lane; an XOR swizzle of the 16-byte chunks in LDS keeps the row writes on
// distinct banks. A tile goes out in parts of at most 8 chunks per block, so
// a wavefront needs only 8 KB of LDS, which the loads reuse. Stores are
// non-temporal. Measured on MI355X with cache-cold inputs (2^20 8x8 blocks):
// the half-DMA load beat row loads of whole blocks by 3 to 4 us, while a
// whole-tile DMA in two halves lost 2 us (two round trips); non-temporal
// stores beat ordinary ones by 14 us; stores of 64-byte pieces of blocks
// instead of 128-byte halves were 30 us slower.
//
// Scheduling. Each wavefront handles one tile and is a workgroup of its own
// (tiles of N >= 128: a workgroup of the tile's wavefronts), and workgroup w
// takes tile w of the plan's list. The lifting form needs no temporaries, so
// a wavefront fits in under 100 VGPRs and five wavefronts per SIMD stay
// resident, which lets the loads, rotations and stores of different tiles
// overlap. The plan lists the tiles of all classes interleaved by their
// position in the batch (see hygt_plan.hip), so the tiles running at any
// moment read and write one compact window of the arrays. Measured on
// MI355X (2^20 8x8 blocks, R = 4, with the multiplier prefetch): 107 us
// forward against 122 us with the tiles in class order, and 4 us more when
// each XCD walked its own contiguous share of the list.
//
// Arithmetic. Each pair is rotated with the three in-place lifting steps
// built by the plan (see hygt_plan.hip), and a class whose sign bookkeeping
// left negative outputs multiplies them by -1 at the end. Every operation is
// an explicit fmaf or an exact sign flip, so every block of a class sees the
// same rounding whatever the batch, tile or launch.

#include <algorithm>
#include <climits>

#include "hygt.h"
#include "hygt_tile.h"

namespace hygt {
namespace {

using namespace tile;

// Chunks of multipliers in flight per wavefront with the VGPR stream
// (VTableStream): the split tiles, and the 8x8 tiles of the mixed launch.
constexpr int kStreamPrefetch = 4;

// Floats of a multiplier chunk for pairs of N = 2^D values: the whole pass
// for N < 32, else 16 pairs.
template <int D>
constexpr int chunk_floats() {
    return (1 << D) < 32 ? (1 << D) : 32;
}

// Pairs H*CP .. H*CP+CP-1 of a pass along dimension K (CP = F/2 pairs of the
// chunk m): the lifting steps a += p b, b += q a, a += p b in place (three
// FMAs, no temporary).
template <int D, int K, int H, int F>
__device__ __forceinline__ void lift_chunk(float (&v)[1 << D], const Chunk<F>& m) {
    StaticFor<0, F / 2>::run([&](auto jj) {
        constexpr int jl = decltype(jj)::value;
        constexpr int j = H * (F / 2) + jl;
        constexpr int mi = ins0(j, K);
        constexpr int ni = mi + (1 << K);
        const float p = m.template get<2 * jl>();
        const float q = m.template get<2 * jl + 1>();
        v[mi] = fmaf(p, v[ni], v[mi]);
        v[ni] = fmaf(q, v[mi], v[ni]);
        v[mi] = fmaf(p, v[ni], v[mi]);
    });
}

// The same with multipliers streamed into VGPRs (VChunk): the three lifting
// steps of the chunk's pairs go in three sweeps over its 16 pairs, so that
// the operations on one pair are 16 instructions apart, beyond the wait
// states a DPP read needs after the write of its operands.
template <int D, int K, int H, int F>
__device__ __forceinline__ void lift_chunk(float (&v)[1 << D], const VChunk& m) {
    static_assert(F == 32, "16 pairs per chunk");
    StaticFor<0, 3>::run([&](auto st) {
        constexpr int step = decltype(st)::value;
        StaticFor<0, 16>::run([&](auto jj) {
            constexpr int jl = decltype(jj)::value;
            constexpr int j = H * 16 + jl;
            constexpr int mi = ins0(j, K);
            constexpr int ni = mi + (1 << K);
            if constexpr (step == 1)
                v[ni] = fmac_bcast<jl>(m.y, v[mi], v[ni]);
            else
                v[mi] = fmac_bcast<jl>(m.x, v[ni], v[mi]);
        });
    });
}

// Integer arithmetic (Fig. 6): the registers hold int32 values (as bit
// patterns), and pair j's multipliers (C, S) come from the integer table.
// y_m = (C x_m + S x_n + 2^13) >> 14, y_n = (C x_n - S x_m + 2^13) >> 14, with
// 24-bit multiplies (v_mad_i32_i24, full rate): exact while every value stays
// within +-2^23 and every sum within int32, which holds for blocks of L2 norm
// up to 2^15.
// p * q + r with p, q taken as signed 24-bit integers (one full-rate
// v_mad_i32_i24; left to itself the compiler splits such sums into
// multiplies and a three-input add, two instructions more per pair).
__device__ __forceinline__ int mad24(int p, int q, int r) {
    int out;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(out) : "s"(p), "v"(q), "v"(r));
    return out;
}

template <int D, int K, int H, int F>
__device__ __forceinline__ void int_chunk(float (&v)[1 << D], const Chunk<F>& m, int half) {
    StaticFor<0, F / 2>::run([&](auto jj) {
        constexpr int jl = decltype(jj)::value;
        constexpr int j = H * (F / 2) + jl;
        constexpr int mi = ins0(j, K);
        constexpr int ni = mi + (1 << K);
        const int c = __float_as_int(m.template get<2 * jl>());
        const int s = __float_as_int(m.template get<2 * jl + 1>());
        const int a = __float_as_int(v[mi]);
        const int b = __float_as_int(v[ni]);
        const int ym = mad24(c, a, mad24(s, b, half)) >> kIntFracBits;
        const int yn = mad24(c, b, mad24(-s, a, half)) >> kIntFracBits;
        v[mi] = __int_as_float(ym);
        v[ni] = __int_as_float(yn);
    });
}

// R rounds of D passes in application order (forward: k = 0..D-1 in every
// round; inverse: k = D-1..0), chunk by chunk from the table stream; pass p
// of the table (application order) is at p * N. RT > 0 unrolls the rounds at
// compile time (RT == R); RT == 0 loops over `rounds`. INTG selects the
// integer butterflies. The prefetch after the last chunk of the last round
// repeats that round's first chunk.
//
// With VS (N = 64 in the fused mixed launch only) the chunks come through the
// VGPR stream of the split tiles instead (VTableStream, kStreamPrefetch
// chunks in flight): the fused launch's 8x8 tiles share the GPU with
// latency-bound 16x16 tiles, and there this took the mixed step from 88 to
// 84.5 us, while the single-size 8x8 kernels lost 2 to 14 us with it.
template <int D, int DIR, int RT, bool INTG, bool VS = false>
__device__ __forceinline__ void run_rounds(float (&v)[1 << D], ctab_f tbl, int rounds) {
    constexpr int N = 1 << D;
    constexpr int F = chunk_floats<D>();
    constexpr int CPP = N / F;    // chunks per pass
    constexpr int CPR = D * CPP;  // chunks per round
    if constexpr (VS) {
        static_assert(F == 32 && !INTG, "chunks of 16 pairs");
        constexpr int Q = kStreamPrefetch;
        VTableStream<Q> vs;
        vs.init(reinterpret_cast<uint64_t>(tbl), __lane_id());
        // chunk g of the walk (past the last round: a chunk of the last one)
        StaticFor<0, Q>::run([&](auto gg) {
            constexpr int g = decltype(gg)::value;
            const int64_t r2 = g / CPR < rounds ? g / CPR : rounds - 1;
            vs.push(r2 * (D * N) + (g % CPR) * F);
        });
        auto one_round_v = [&](int64_t r) {
            StaticFor<0, CPR>::run([&](auto ee) {
                constexpr int e = decltype(ee)::value;
                constexpr int kk = e / CPP;
                constexpr int H = e % CPP;
                constexpr int K = DIR == 0 ? kk : D - 1 - kk;
                int64_t r2 = r + (e + Q) / CPR;
                if (r2 > rounds - 1) r2 = rounds - 1;
                const VChunk m = vs.next(r2 * (D * N) + ((e + Q) % CPR) * F);
                lift_chunk<D, K, H, F>(v, m);
            });
        };
        if constexpr (RT > 0) {
            StaticFor<0, RT>::run([&](auto rr) { one_round_v(decltype(rr)::value); });
        } else {
            for (int r = 0; r < rounds; ++r) one_round_v(r);
        }
        return;
    }
    int half = 0;
    if constexpr (INTG) {
        // the rounding constant, once in a VGPR (an instruction may read only
        // one scalar operand, and the multiplier is that one)
        half = 1 << (kIntFracBits - 1);
        asm volatile("" : "+v"(half));
    }
    TableStream<F> ts;
    ts.begin(tbl, 0);
    auto one_round = [&](int64_t r, int64_t rnext) {
        StaticFor<0, CPR>::run([&](auto ee) {
            constexpr int e = decltype(ee)::value;
            constexpr int kk = e / CPP;
            constexpr int H = e % CPP;
            constexpr int K = DIR == 0 ? kk : D - 1 - kk;
            const int64_t nxt = e + 1 < CPR ? r * (D * N) + (e + 1) * F : rnext * (D * N);
            const Chunk<F> m = ts.next(nxt);
            if constexpr (INTG)
                int_chunk<D, K, H, F>(v, m, half);
            else
                lift_chunk<D, K, H, F>(v, m);
        });
    };
    if constexpr (RT > 0) {
        StaticFor<0, RT>::run([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            one_round(r, r + 1 < RT ? r + 1 : r);
        });
    } else {
        for (int r = 0; r < rounds; ++r) one_round(r, r + 1 < rounds ? r + 1 : r);
    }
}

// The final signs of a class whose sign bookkeeping left negative outputs.
template <int V>
__device__ __forceinline__ void apply_signs(float (&v)[V], ctab_f sign, int has_neg) {
    if (has_neg) {
        StaticFor<0, V>::run([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            v[i] *= sign[i];
        });
    }
}

// N >= 128: a pass along bit K >= 6 pairs value i of wavefront q (element
// 64q + i, bit K - 6 of q clear) with value i of wavefront q | 2^(K-6). The
// two swap their values through LDS, 16 per lane at a time, and each
// computes its own outputs: y_m = c x_m + s x_n on the lower wavefront,
// y_n = c x_n - s x_m on the upper one, with (c, s) of pair i the two floats
// at 2i of the wavefront pair's part of the pass (128 floats, four chunks of
// 16 pairs, part g's chunk returned by next_chunk(g) for the compile-time
// g). `xo` is this wavefront's exchange area and `xp` the partner's, each
// two buffers of [4][64] float4; part g uses buffer g % 2, so the barrier of
// part g + 1 also guarantees that both wavefronts have read part g before
// either overwrites its buffer. Every wavefront of the workgroup passes the
// same barriers.
template <class NextChunk>
__device__ __forceinline__ void cross_pass(float (&v)[64], NextChunk&& next_chunk, unsigned hbit,
                                           float4* xo, const float4* xp, int lane) {
    StaticFor<0, 4>::run([&](auto gg) {
        constexpr int g = decltype(gg)::value;
        constexpr int buf = g & 1;
        const auto m = next_chunk(gg);
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
        if constexpr (std::is_same<std::decay_t<decltype(m)>, VChunk>::value) {
            // -s on the upper wavefront: a sign-bit flip of the chunk's s
            // values, then c x and the fused s x' + c x with DPP sources
            const float sg = xor_for_dpp(m.y, hbit);
            StaticFor<0, 16>::run([&](auto tt) {
                constexpr int t = decltype(tt)::value;
                constexpr int j = 16 * g + t;
                v[j] = fmac_bcast<t>(sg, w[t], m.template get<2 * t>() * v[j]);
            });
        } else {
            StaticFor<0, 16>::run([&](auto tt) {
                constexpr int t = decltype(tt)::value;
                constexpr int j = 16 * g + t;
                const float c = m.template get<2 * t>();
                const float sn = m.template get<2 * t + 1>();
                // -s on the upper wavefront: a sign-bit flip
                const float sg = __uint_as_float(__float_as_uint(sn) ^ hbit);
                v[j] = fmaf(sg, w[t], c * v[j]);
            });
        }
    });
}

// N >= 128, wavefront q of a tile's 2^(D-6) wavefronts: R rounds of D
// passes in application order. Passes along bits 0..5 act on the lane's 64
// values with the multipliers of pairs 32q .. 32q + 31 of the pass (table
// floats 64q .. 64q + 63 of the pass, two chunks); passes along bits 6, 7 go
// through cross_pass with the partner wavefront q ^ 2^(K-6), whose pairs
// start at 64 * (q without bit K-6). Then the final signs of elements
// 64q .. 64q + 63. The tile's wavefronts have consecutive LDS areas of 512
// float4 starting at `area0`.
//
// Table offset of the first chunk of wavefront q's share of pass kk
// (application order) of round r.
template <int D, int DIR>
__device__ __forceinline__ int64_t split_first(int64_t r, int kk, int q) {
    constexpr int N = 1 << D;
    constexpr int V = 64;
    const int K = DIR == 0 ? kk : D - 1 - kk;
    const int64_t off = (r * D + kk) * N;
    if (K >= kLaneBits) {
        const int b = K - kLaneBits;
        const int qq = ((q >> (b + 1)) << b) | (q & ((1 << b) - 1));
        return off + 2 * V * qq;
    }
    return off + q * V;
}

// Chunks of 16 pairs in one round of a split tile (N >= 128), in the order
// they are used: two per pass along bits 0..5, four per pass along bits 6, 7.
template <int D, int DIR>
constexpr int split_pass_chunks(int kk) {
    return (DIR == 0 ? kk : D - 1 - kk) >= kLaneBits ? 4 : 2;
}
template <int D, int DIR>
constexpr int split_chunks_before(int kk) {
    int n = 0;
    for (int i = 0; i < kk; ++i) n += split_pass_chunks<D, DIR>(i);
    return n;
}
template <int D, int DIR>
constexpr int split_chunk_pass(int j) {
    int kk = 0;
    while (j >= split_pass_chunks<D, DIR>(kk)) {
        j -= split_pass_chunks<D, DIR>(kk);
        ++kk;
    }
    return kk;
}


template <int D, int DIR, int Q = kStreamPrefetch>
__device__ __forceinline__ void run_passes_split(float (&v)[64], ctab_f tbl, ctab_f sign,
                                                 int has_neg, int rounds, int q, float4* area0,
                                                 int lane) {
    constexpr int V = 64;
    constexpr int CR = split_chunks_before<D, DIR>(D);
    static_assert(Q <= CR, "prefetch within the next round");
    // table offset of chunk J of round r
    auto off_of = [&](int64_t r, auto jj) -> int64_t {
        constexpr int J = decltype(jj)::value;
        constexpr int kk = split_chunk_pass<D, DIR>(J);
        return split_first<D, DIR>(r, kk, q) + 32 * (J - split_chunks_before<D, DIR>(kk));
    };
    // the chunk Q after chunk J of round r (past the last: the last again)
    auto ahead = [&](int64_t r, auto jj) -> int64_t {
        constexpr int J = decltype(jj)::value + Q;
        if constexpr (J < CR) {
            return off_of(r, std::integral_constant<int, J>{});
        } else {
            if (r + 1 < rounds) return off_of(r + 1, std::integral_constant<int, J - CR>{});
            return off_of(r, std::integral_constant<int, CR - 1>{});
        }
    };
    VTableStream<Q> vs;
    vs.init(reinterpret_cast<uint64_t>(tbl), lane);
    StaticFor<0, Q>::run([&](auto ii) { vs.push(off_of(0, ii)); });
    for (int r = 0; r < rounds; ++r) {
        StaticFor<0, D>::run([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            constexpr int K = DIR == 0 ? k : D - 1 - k;
            constexpr int j0 = split_chunks_before<D, DIR>(k);
            if constexpr (K >= kLaneBits) {
                constexpr int b = K - kLaneBits;
                cross_pass(
                    v,
                    [&](auto gg) {
                        constexpr int g = decltype(gg)::value;
                        return vs.next(ahead(r, std::integral_constant<int, j0 + g>{}));
                    },
                    static_cast<unsigned>((q >> b) & 1) << 31, area0 + 512 * q,
                    area0 + 512 * (q ^ (1 << b)), lane);
            } else {
                const VChunk m0 = vs.next(ahead(r, std::integral_constant<int, j0>{}));
                lift_chunk<kLaneBits, K, 0, 32>(v, m0);
                const VChunk m1 = vs.next(ahead(r, std::integral_constant<int, j0 + 1>{}));
                lift_chunk<kLaneBits, K, 1, 32>(v, m1);
            }
        });
    }
    apply_signs<V>(v, sign + q * V, has_neg);
}

// Permutation pass (Fig. 4), N <= 64, through this wavefront's row area R of
// 64 rows of N floats: chunk q of lane l's row sits at slot
// l * CH + (q ^ (l mod CH)), so that 16 consecutive lanes touch distinct
// banks. Position p of the class's permutation row holds output p's source
// coefficient; entries are masked to [0, N) so that no access leaves the row.
template <int D>
__device__ __forceinline__ int perm_addr(int lane, int p) {
    constexpr int CH = (1 << D) / 4;
    return 4 * (lane * CH + ((p >> 2) ^ (lane & (CH - 1)))) + (p & 3);
}

// Forward: v[j] <- v[perm[j]].
template <int D>
__device__ __forceinline__ void permute_row(float* v, float4* R, ctab_i perm, int lane) {
    constexpr int N = 1 << D;
    constexpr int CH = N / 4;
    StaticFor<0, CH>::run([&](auto qq) {
        constexpr int q = decltype(qq)::value;
        R[lane * CH + (q ^ (lane & (CH - 1)))] =
            make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    });
    asm volatile("" ::: "memory");
    const float* Rf = reinterpret_cast<const float*>(R);
    StaticFor<0, N>::run([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        v[j] = Rf[perm_addr<D>(lane, perm[j] & (N - 1))];
    });
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Inverse: v[perm[j]] <- v[j].
template <int D>
__device__ __forceinline__ void unpermute_row(float* v, float4* R, ctab_i perm, int lane) {
    constexpr int N = 1 << D;
    constexpr int CH = N / 4;
    float* Rf = reinterpret_cast<float*>(R);
    StaticFor<0, N>::run([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        Rf[perm_addr<D>(lane, perm[j] & (N - 1))] = v[j];
    });
    asm volatile("" ::: "memory");
    StaticFor<0, CH>::run([&](auto qq) {
        constexpr int q = decltype(qq)::value;
        const float4 f = R[lane * CH + (q ^ (lane & (CH - 1)))];
        v[4 * q + 0] = f.x;
        v[4 * q + 1] = f.y;
        v[4 * q + 2] = f.z;
        v[4 * q + 3] = f.w;
    });
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// One tile of a transform of N >= 4: loads, passes, stores. For N >= 128
// the tile belongs to 2^(D-6) wavefronts, this one (number q of them)
// holding values 64q .. 64q+63 of every block; the tile's wavefronts have
// consecutive LDS areas of 512 float4 from `area0`, and `L` is this
// wavefront's own (for N <= 64, the only one). A class c < 0 marks a
// dummy tile (N >= 128 only), which touches no memory but takes part in the
// tile's barriers.
//
// x and y may be the same array (in place): every value is read by the
// wavefront that owns it and written back only after that read has
// completed, and no other wavefront touches it, so the restrict qualifiers
// (which let the per-tile class loads stay scalar) hold for every pair of
// accesses that the compiler could reorder.
template <int D, int DIR, int RT, bool PERM = false, bool INTG = false, bool TILE_LOAD = false,
          bool VS = false>
__device__ __forceinline__ void rotate_tile(const float* __restrict__ x, float* __restrict__ y,
                                            int64_t nblocks, int rounds, int nclasses,
                                            int64_t t0, int c, int q,
                                            const int32_t* __restrict__ perm,
                                            const int32_t* __restrict__ modes,
                                            const float* __restrict__ coef,
                                            const float* __restrict__ signs, float4* L,
                                            float4* area0, int lane,
                                            ctab_i outperm = nullptr) {
    using G = TileGeo<D>;
    constexpr int N = G::N;
    constexpr int CHP = G::CHP;
    static_assert(!G::SPLIT || kTile * CHP == 512, "split tiles use areas of 512 float4");
    const float* xh = x + q * G::V;
    float* yh = y + q * G::V;
    // lanes without a block compute on whatever their registers hold and
    // store nothing
    const int blk = c < 0 ? -1 : valid_block(perm[t0 * kTile + lane], nblocks);
    float v[G::V];
    if constexpr (TILE_LOAD && !G::SPLIT) {
        if (c >= 0) load_tile<D, DIR == 1 && D == kLaneBits>(xh, blk, v, L, lane);
    } else {
        load_row<D>(xh, blk, v);
    }

    // with the permutation pass, the inverse first puts the coefficients back
    // in transform order (the row area is the staging area, 16 KB per wave)
    if constexpr (PERM && DIR == 1) unpermute_row<D>(v, L, outperm + c * N, lane);
    const size_t passes = static_cast<size_t>(rounds) * D;
    const size_t table = static_cast<size_t>(DIR) * nclasses + (c < 0 ? 0 : c);
    ctab_f tbl = as_ctab(coef) + table * passes * N;
    if constexpr (G::SPLIT) {
        run_passes_split<D, DIR>(v, tbl, as_ctab(signs) + table * N, as_ctab(modes)[table],
                                 rounds, q, area0, lane);
        // The partners' last reads of this wavefront's exchange area come
        // before the stores below reuse it for staging.
        __syncthreads();
    } else if constexpr (INTG) {
        run_rounds<D, DIR, 0, true>(v, tbl, rounds);
    } else {
        run_rounds<D, DIR, RT, false, VS && D == kLaneBits>(v, tbl, rounds);
        apply_signs<N>(v, as_ctab(signs) + table * N, as_ctab(modes)[table]);
        if constexpr (PERM && DIR == 0) permute_row<D>(v, L, outperm + c * N, lane);
    }

    // Addresses for the way out are derived again from the block ids and the
    // lane index, made opaque here so that the compiler does not keep the
    // ones of the way in alive (in registers) across the passes.
    int lane2 = lane;
    asm volatile("" : "+v"(lane2));
    const int sw2 = swz<CHP>(lane2);
    int b = blk;
    asm volatile("" : "+v"(b));
    int bb[CHP];
    instr_blocks<D>(bb, b, lane2);
    StaticFor<0, G::PARTS>::run([&](auto pp) {
        store_part<D, decltype(pp)::value>(yh, L, bb, v, lane2, sw2);
    });
}

// N >= 4: one tile per wavefront and workgroup, or for N = 128 and N = 256
// one tile per workgroup of 2 or 4 wavefronts, wavefront q holding values
// 64q .. 64q+63 of every block. Workgroup w takes tile w of the list.
template <int D, int DIR, int RT>
__global__ __launch_bounds__(64 * TileGeo<D>::WAVES)
__attribute__((amdgpu_waves_per_eu(TileGeo<D>::OCC)))
void rotate_kernel(const float* __restrict__ x, float* __restrict__ y, int64_t nblocks,
                   int rounds, int nclasses, int64_t max_tiles,
                   const int32_t* __restrict__ tile_class, const int32_t* __restrict__ perm,
                   const int32_t* __restrict__ modes, const float* __restrict__ coef,
                   const float* __restrict__ signs) {
    using G = TileGeo<D>;
    // Staging of a part; for N >= 128 also the exchange area (2 x 4 x 64 float4).
    __shared__ float4 lds[G::WAVES][kTile * G::CHP];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int q = G::SPLIT ? wv : 0;  // share of every block held by this wavefront
    const int64_t t0 = G::SPLIT ? static_cast<int64_t>(blockIdx.x)
                                : static_cast<int64_t>(blockIdx.x) * kWaves + wv;
    if (t0 >= max_tiles) return;  // all wavefronts of a split tile leave together
    const int c = __builtin_amdgcn_readfirstlane(tile_class[t0]);
    if (c < 0) return;  // past the last tile
    rotate_tile<D, DIR, RT, false, false, true>(x, y, nblocks, rounds, nclasses, t0, c, q, perm,
                                                modes, coef, signs, lds[wv], lds[0], lane);
}

// N <= 64 with the permutation pass: as rotate_kernel, with a 16 KB row area
// per wavefront for the permutation (the loads and the part staging reuse its
// start). LDS bounds the residency here: ten wavefronts fit a compute unit's
// 160 KB at N = 64.
constexpr int kPermWaves = 1;

template <int D, int DIR>
__global__ __launch_bounds__(64 * kPermWaves) void rotate_perm_kernel(
    const float* __restrict__ x, float* __restrict__ y, int64_t nblocks, int rounds,
    int nclasses, int64_t max_tiles, const int32_t* __restrict__ tile_class,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ modes,
    const float* __restrict__ coef, const float* __restrict__ signs,
    const int32_t* __restrict__ outperm) {
    __shared__ float4 lds[kPermWaves][64 * ((1 << D) / 4)];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kPermWaves + wv;
    if (t0 >= max_tiles) return;
    const int c = __builtin_amdgcn_readfirstlane(tile_class[t0]);
    if (c < 0) return;
    rotate_tile<D, DIR, 0, true, false, true>(x, y, nblocks, rounds, nclasses, t0, c, 0, perm,
                                              modes, coef, signs, lds[wv], lds[wv], lane,
                                              as_ctab(outperm));
}

// Integer blocks, 4 <= N <= 64: as rotate_kernel with the integer passes;
// loads, LDS staging and stores move the int32 bit patterns unchanged.
template <int D, int DIR>
__global__ __launch_bounds__(64 * kWaves) void rotate_int_kernel(
    const float* __restrict__ x, float* __restrict__ y, int64_t nblocks, int rounds,
    int nclasses, int64_t max_tiles, const int32_t* __restrict__ tile_class,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ modes,
    const float* __restrict__ coef, const float* __restrict__ signs) {
    using G = TileGeo<D>;
    __shared__ float4 lds[kWaves][kTile * G::CHP];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kWaves + wv;
    if (t0 >= max_tiles) return;
    const int c = __builtin_amdgcn_readfirstlane(tile_class[t0]);
    if (c < 0) return;
    rotate_tile<D, DIR, 0, false, true>(x, y, nblocks, rounds, nclasses, t0, c, 0, perm, modes,
                                        coef, signs, lds[wv], lds[wv], lane);
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
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kWaves + wv;
    if (t0 >= max_tiles) return;
    const int c = __builtin_amdgcn_readfirstlane(tile_class[t0]);
    if (c < 0) return;
    const size_t table = static_cast<size_t>(DIR) * nclasses + c;
    const int blk = valid_block(perm[t0 * kTile + lane], nblocks);
    float2 in = make_float2(0.0f, 0.0f);
    if (blk >= 0) in = *reinterpret_cast<const float2*>(x + static_cast<int64_t>(blk) * 2);
    float v[2] = {in.x, in.y};
    run_rounds<1, DIR, 0, false>(v, as_ctab(coef) + table * rounds * 2, rounds);
    apply_signs<2>(v, as_ctab(signs) + table * 2, as_ctab(modes)[table]);
    if (blk >= 0)
        *reinterpret_cast<float2*>(y + static_cast<int64_t>(blk) * 2) = make_float2(v[0], v[1]);
}

template <int D, int DIR, int RT>
hipError_t launch_one(const float* x, float* y, int64_t nblocks, int rounds, int nclasses,
                      const WsLayout& l, const WsPtrs& p, hipStream_t stream) {
    using G = TileGeo<D>;
    const int64_t per_group = G::SPLIT ? 1 : static_cast<int64_t>(kWaves);
    const dim3 grid(static_cast<unsigned>((l.max_tiles + per_group - 1) / per_group));
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

// ---------------------------------------------------------------------------
// Mixed batches: one persistent launch over the tiles of several block sizes
// ---------------------------------------------------------------------------

namespace {

// Resident wavefronts per SIMD of the mixed kernel: the persistent loop and
// the per-segment arguments cost some registers over the plain kernels,
// which at five wavefronts per SIMD would spill.
constexpr int kMixedWavesPerSimd = 4;
// Workgroups per compute unit at that budget (four wavefronts each).
constexpr int kMixedWgPerCu = kMixedWavesPerSimd;
constexpr int kComputeUnits = 256;

// Work item `local` of segment g: four tiles, one per wavefront (N <= 64),
// or 4 / 2^(D-6) tiles of N >= 128, each shared by 2^(D-6) consecutive
// wavefronts. With UNROLL, segments with N <= 64 and R in {1, 2, 4} run with
// their rounds unrolled at compile time.
template <int D, int DIR, bool UNROLL>
__device__ __forceinline__ void mixed_item(const MixedSeg& g, int64_t local, int wv, int lane,
                                           float4 (*lds)[512]) {
    using G = TileGeo<D>;
    if constexpr (G::SPLIT) {
        constexpr int S = G::SHARE;
        const int first = wv & ~(S - 1);  // first wavefront of this tile
        const int64_t t0 = local * (4 / S) + wv / S;
        int c = -1;  // a dummy tile still joins the workgroup's barriers
        if (t0 < g.max_tiles) c = __builtin_amdgcn_readfirstlane(as_ctab(g.tile_class)[t0]);
        rotate_tile<D, DIR, 0>(g.x, g.y, g.nblocks, g.rounds, g.nclasses, t0, c, wv - first,
                               g.perm, g.modes, g.coef, g.signs, lds[wv], lds[first], lane);
    } else {
        const int64_t t0 = local * 4 + wv;
        if (t0 >= g.max_tiles) return;
        const int c = __builtin_amdgcn_readfirstlane(as_ctab(g.tile_class)[t0]);
        if (c < 0) return;
        if constexpr (UNROLL && D <= 6) {
            switch (g.rounds) {
                case 1:
                    rotate_tile<D, DIR, 1, false, false, false, true>(g.x, g.y, g.nblocks, g.rounds, g.nclasses, t0, c, 0,
                                           g.perm, g.modes, g.coef, g.signs, lds[wv], lds[wv],
                                           lane);
                    return;
                case 2:
                    rotate_tile<D, DIR, 2, false, false, false, true>(g.x, g.y, g.nblocks, g.rounds, g.nclasses, t0, c, 0,
                                           g.perm, g.modes, g.coef, g.signs, lds[wv], lds[wv],
                                           lane);
                    return;
                case 4:
                    rotate_tile<D, DIR, 4, false, false, false, true>(g.x, g.y, g.nblocks, g.rounds, g.nclasses, t0, c, 0,
                                           g.perm, g.modes, g.coef, g.signs, lds[wv], lds[wv],
                                           lane);
                    return;
                default:
                    break;
            }
        }
        rotate_tile<D, DIR, 0, false, false, false, true>(g.x, g.y, g.nblocks, g.rounds,
                                                          g.nclasses, t0, c, 0, g.perm, g.modes,
                                                          g.coef, g.signs, lds[wv], lds[wv],
                                                          lane);
    }
}

// Each segment's items are split into kXcds contiguous shares, one per XCD
// (workgroups are dispatched round-robin over the XCDs, so workgroup w runs
// on XCD w mod 8): the class-sorted tiles of a share cover few classes, whose
// tables then stay in that XCD's caches. An XCD's shares of all segments,
// largest blocks first, form one list whose entries its P = gridDim / 8
// workgroups take in turn, so items of different sizes run side by side.
// Every wavefront of a workgroup walks the same items, so wavefronts sharing
// a tile meet at the same barriers.
__device__ __forceinline__ int64_t share_lo(int64_t items, int64_t xcd) {
    return items * xcd / kXcds;
}

template <int DIR, bool UNROLL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kMixedWavesPerSimd)))
void mixed_kernel(MixedArgs a) {
    __shared__ float4 lds[4][512];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t xcd = blockIdx.x % kXcds;
    const int64_t P = gridDim.x / kXcds;
    int64_t total = 0;  // entries of this XCD's list
    StaticFor<0, kMaxSegments>::run([&](auto ss) {
        constexpr int k = decltype(ss)::value;
        if (k < a.nseg)
            total += share_lo(a.seg[k].items, xcd + 1) - share_lo(a.seg[k].items, xcd);
    });
    for (int64_t e = blockIdx.x / kXcds; e < total; e += P) {
        int64_t off = 0;
        StaticFor<0, kMaxSegments>::run([&](auto ss) {
            constexpr int k = decltype(ss)::value;
            if (k >= a.nseg) return;
            const MixedSeg& g = a.seg[k];
            const int64_t lo = share_lo(g.items, xcd);
            const int64_t len = share_lo(g.items, xcd + 1) - lo;
            if (e >= off && e < off + len) {
                const int64_t item = lo + (e - off);
                switch (g.log2n) {
                    case 2: mixed_item<2, DIR, UNROLL>(g, item, wv, lane, lds); break;
                    case 3: mixed_item<3, DIR, UNROLL>(g, item, wv, lane, lds); break;
                    case 4: mixed_item<4, DIR, UNROLL>(g, item, wv, lane, lds); break;
                    case 5: mixed_item<5, DIR, UNROLL>(g, item, wv, lane, lds); break;
                    case 6: mixed_item<6, DIR, UNROLL>(g, item, wv, lane, lds); break;
                    case 7: mixed_item<7, DIR, UNROLL>(g, item, wv, lane, lds); break;
                    case 8: mixed_item<8, DIR, UNROLL>(g, item, wv, lane, lds); break;
                    default: break;
                }
            }
            off += len;
        });
    }
}

// Configuration k: bit 0 = rounds unrolled; bits 1-2 = grid: one workgroup
// per list entry, or 1, 2 or 4 waves of resident workgroups striding through
// the lists. Grids are multiples of 8.
template <int DIR>
hipError_t launch_mixed_dir(const MixedArgs& a, int config, hipStream_t stream) {
    const bool unroll = config & 1;
    const int grid_mode = (config >> 1) & 3;
    int64_t per_xcd = 0;  // longest list of any XCD
    for (int64_t x = 0; x < kXcds; ++x) {
        int64_t n = 0;
        for (int k = 0; k < a.nseg; ++k)
            n += a.seg[k].items * (x + 1) / kXcds - a.seg[k].items * x / kXcds;
        per_xcd = std::max(per_xcd, n);
    }
    int64_t grid = per_xcd * kXcds;
    if (grid_mode > 0) {
        const int64_t resident = static_cast<int64_t>(kComputeUnits) * kMixedWgPerCu;
        grid = std::min<int64_t>(grid, resident << (grid_mode - 1));
    }
    if (grid <= 0) return hipSuccess;
    if (unroll)
        hipLaunchKernelGGL((mixed_kernel<DIR, true>), dim3(static_cast<unsigned>(grid)), dim3(256),
                           0, stream, a);
    else
        hipLaunchKernelGGL((mixed_kernel<DIR, false>), dim3(static_cast<unsigned>(grid)),
                           dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

int64_t mixed_items(int log2n, int64_t max_tiles) {
    const int64_t per = log2n > kLaneBits ? 4 >> (log2n - kLaneBits) : 4;
    return (max_tiles + per - 1) / per;
}

hipError_t launch_mixed(const MixedArgs& a, int direction, int config, hipStream_t stream) {
    if (direction == 0) return launch_mixed_dir<0>(a, config, stream);
    return launch_mixed_dir<1>(a, config, stream);
}

namespace {
template <int D, int DIR>
hipError_t launch_perm_one(const float* x, float* y, int64_t nblocks, int rounds, int nclasses,
                           const int32_t* outperm, const WsLayout& l, const WsPtrs& p,
                           hipStream_t stream) {
    const dim3 grid(static_cast<unsigned>((l.max_tiles + kPermWaves - 1) / kPermWaves));
    hipLaunchKernelGGL((rotate_perm_kernel<D, DIR>), grid, dim3(64 * kPermWaves), 0, stream, x, y,
                       nblocks, rounds, nclasses, l.max_tiles, p.tile_class, p.perm, p.modes,
                       p.coef, p.signs, outperm);
    return hipGetLastError();
}

template <int DIR>
hipError_t launch_perm_dir(const float* x, float* y, int64_t nblocks, int log2n, int rounds,
                           int nclasses, const int32_t* outperm, const WsLayout& l,
                           const WsPtrs& p, hipStream_t stream) {
    switch (log2n) {
        case 2: return launch_perm_one<2, DIR>(x, y, nblocks, rounds, nclasses, outperm, l, p, stream);
        case 3: return launch_perm_one<3, DIR>(x, y, nblocks, rounds, nclasses, outperm, l, p, stream);
        case 4: return launch_perm_one<4, DIR>(x, y, nblocks, rounds, nclasses, outperm, l, p, stream);
        case 5: return launch_perm_one<5, DIR>(x, y, nblocks, rounds, nclasses, outperm, l, p, stream);
        case 6: return launch_perm_one<6, DIR>(x, y, nblocks, rounds, nclasses, outperm, l, p, stream);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace

namespace {
template <int D, int DIR>
hipError_t launch_int_one(const int32_t* x, int32_t* y, int64_t nblocks, int rounds,
                          int nclasses, const WsLayout& l, const WsPtrs& p, hipStream_t stream) {
    const dim3 grid(static_cast<unsigned>((l.max_tiles + kWaves - 1) / kWaves));
    hipLaunchKernelGGL((rotate_int_kernel<D, DIR>), grid, dim3(64 * kWaves), 0, stream,
                       reinterpret_cast<const float*>(x), reinterpret_cast<float*>(y), nblocks,
                       rounds, nclasses, l.max_tiles, p.tile_class, p.perm, p.modes, p.coef,
                       p.signs);
    return hipGetLastError();
}

template <int DIR>
hipError_t launch_int_dir(const int32_t* x, int32_t* y, int64_t nblocks, int log2n, int rounds,
                          int nclasses, const WsLayout& l, const WsPtrs& p, hipStream_t stream) {
    switch (log2n) {
        case 2: return launch_int_one<2, DIR>(x, y, nblocks, rounds, nclasses, l, p, stream);
        case 3: return launch_int_one<3, DIR>(x, y, nblocks, rounds, nclasses, l, p, stream);
        case 4: return launch_int_one<4, DIR>(x, y, nblocks, rounds, nclasses, l, p, stream);
        case 5: return launch_int_one<5, DIR>(x, y, nblocks, rounds, nclasses, l, p, stream);
        case 6: return launch_int_one<6, DIR>(x, y, nblocks, rounds, nclasses, l, p, stream);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_rotate_int(const int32_t* x, int32_t* y, int64_t nblocks, int log2n,
                             int rounds, int nclasses, int direction, const WsLayout& l,
                             const WsPtrs& p, hipStream_t stream) {
    if (direction == 0) return launch_int_dir<0>(x, y, nblocks, log2n, rounds, nclasses, l, p, stream);
    return launch_int_dir<1>(x, y, nblocks, log2n, rounds, nclasses, l, p, stream);
}

hipError_t launch_rotate_perm(const float* x, float* y, int64_t nblocks, int log2n, int rounds,
                              int nclasses, int direction, const int32_t* outperm,
                              const WsLayout& l, const WsPtrs& p, hipStream_t stream) {
    if (direction == 0)
        return launch_perm_dir<0>(x, y, nblocks, log2n, rounds, nclasses, outperm, l, p, stream);
    return launch_perm_dir<1>(x, y, nblocks, log2n, rounds, nclasses, outperm, l, p, stream);
}

hipError_t launch_rotate(const float* x, float* y, int64_t nblocks, int log2n, int rounds,
                         int nclasses, int direction, const WsLayout& l, const WsPtrs& p,
                         hipStream_t stream) {
    if (direction == 0) return launch_dir<0>(x, y, nblocks, log2n, rounds, nclasses, l, p, stream);
    return launch_dir<1>(x, y, nblocks, log2n, rounds, nclasses, l, p, stream);
}


// ---------------------------------------------------------------------------
// Request batches: one launch over a run of request descriptors, with no
// class grouping: every block follows its own class's table
// ---------------------------------------------------------------------------

namespace {

// Requests of N = 64, 128, 256: a wavefront per block, lane l holding the
// V = N / 64 elements Vl .. Vl+V-1 (one 4-, 8- or 16-byte load and store per
// lane, the whole block per wavefront). The block's class is wave-uniform,
// so the multipliers of a pass are one coalesced read of the class table.
// A pass along a bit below log2 V pairs values inside a lane (pairs
// (V/2)l .. (V/2)l + V/2 - 1 of the pass); a pass along bit K >= log2 V
// pairs lane l with lane l ^ 2^(K - log2 V), value by value, and lane l
// reads the multipliers of pairs Vl' .. Vl'+V-1 (l' = l without that bit).
// Each lane of such a pair fetches its partner's value and runs the pair's
// whole lifting (bits < 6) or its own half of the (cos, sin) step (bits 6,
// 7) with the same FMAs, operands and order as the grouped tiles, so results
// are bit-identical to theirs; it keeps its own output. Lane-per-block tiles
// read every multiplier as a per-lane load from the block's own table and
// keep a request of 8192 blocks on 128 to 512 wavefronts; this layout moves
// the same table bytes in whole rows, at 2-5x the arithmetic, and gives
// that request 8192 wavefronts. Multipliers are read one pass ahead.

// F consecutive floats (2, 4 or 8) from p, 8-byte aligned (16 for F >= 4).
template <int F>
__device__ __forceinline__ void load_floats(const float* p, float (&m)[8]) {
    if constexpr (F == 2) {
        const float2 a = *reinterpret_cast<const float2*>(p);
        m[0] = a.x, m[1] = a.y;
    } else {
        const float4 a = reinterpret_cast<const float4*>(p)[0];
        m[0] = a.x, m[1] = a.y, m[2] = a.z, m[3] = a.w;
        if constexpr (F == 8) {
            const float4 b = reinterpret_cast<const float4*>(p)[1];
            m[4] = b.x, m[5] = b.y, m[6] = b.z, m[7] = b.w;
        }
    }
}

// Multipliers of pass KK (application order) of round r for this lane.
template <int D, int DIR, int KK>
__device__ __forceinline__ void block_mult(const float* tbl, int64_t r, int lane,
                                           float (&m)[8]) {
    constexpr int N = 1 << D;
    constexpr int V = N / 64;
    constexpr int LB = D - kLaneBits;  // bits inside a lane
    constexpr int K = DIR == 0 ? KK : D - 1 - KK;
    const float* pass = tbl + (r * D + KK) * N;
    if constexpr (K < LB) {
        if constexpr (V >= 2) load_floats<V>(pass + V * lane, m);
    } else {
        constexpr int b = K - LB;
        const int lr = ((lane >> (b + 1)) << b) | (lane & ((1 << b) - 1));
        load_floats<2 * V>(pass + 2 * V * lr, m);
    }
}

__device__ __forceinline__ void lift_pair(float& a, float& b, float p, float q) {
    a = fmaf(p, b, a);
    b = fmaf(q, a, b);
    a = fmaf(p, b, a);
}

template <int D, int DIR>
__device__ __forceinline__ void request_block(const ReqTable& tb, const float* __restrict__ x,
                                              float* __restrict__ y,
                                              const int32_t* __restrict__ cls, int64_t nblocks,
                                              int64_t lw, int wv, int lane, int32_t* status) {
    constexpr int N = 1 << D;
    constexpr int V = N / 64;
    constexpr int LB = D - kLaneBits;
    const int64_t blk = lw * 4 + wv;
    if (blk >= nblocks) return;  // no barrier on this path
    int c = cls != nullptr ? __builtin_amdgcn_readfirstlane(cls[blk]) : 0;
    const bool bad = c < 0 || c >= tb.nclasses;
    if (bad) {
        // the ring is in host memory: a system-scope store, which no cache
        // between the device and that memory holds back
        if (lane == 0)
            __hip_atomic_store(status, static_cast<int32_t>(HYGT_ECLASS), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        c = 0;
    }
    const size_t table = static_cast<size_t>(DIR) * tb.nclasses + c;
    const float* tbl = tb.coef + table * static_cast<size_t>(tb.rounds) * D * N;
    float v[V];
    {
        float in[8];
        if constexpr (V == 1)
            in[0] = x[blk * N + lane];
        else
            load_floats<V>(x + blk * N + V * lane, in);
        StaticFor<0, V>::run([&](auto ii) { v[decltype(ii)::value] = in[decltype(ii)::value]; });
    }
    float m[8];
    block_mult<D, DIR, 0>(tbl, 0, lane, m);
    for (int r = 0; r < tb.rounds; ++r) {
        StaticFor<0, D>::run([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            constexpr int K = DIR == 0 ? k : D - 1 - k;
            float a[8];
            StaticFor<0, 8>::run([&](auto ii) { a[decltype(ii)::value] = m[decltype(ii)::value]; });
            // the next pass's multipliers (after the last pass: pass 0 of
            // the next round, or of this one again)
            if constexpr (k + 1 < D)
                block_mult<D, DIR, k + 1>(tbl, r, lane, m);
            else
                block_mult<D, DIR, 0>(tbl, r + 1 < tb.rounds ? r + 1 : r, lane, m);
            if constexpr (K < LB) {
                // pair t: values i and i + 2^K, i with bit K clear
                StaticFor<0, V / 2>::run([&](auto tt) {
                    constexpr int t = decltype(tt)::value;
                    constexpr int i = ins0(t, K);
                    lift_pair(v[i], v[i + (1 << K)], a[2 * t], a[2 * t + 1]);
                });
            } else {
                constexpr int mask = 1 << (K - LB);
                const bool hi = (lane & mask) != 0;
                float w[V];
                StaticFor<0, V>::run([&](auto ii) {
                    constexpr int i = decltype(ii)::value;
                    w[i] = __shfl_xor(v[i], mask, 64);
                });
                StaticFor<0, V>::run([&](auto ii) {
                    constexpr int i = decltype(ii)::value;
                    const float p = a[2 * i], q = a[2 * i + 1];
                    if constexpr (K < kLaneBits) {
                        float lo_v = hi ? w[i] : v[i];
                        float hi_v = hi ? v[i] : w[i];
                        lift_pair(lo_v, hi_v, p, q);
                        v[i] = hi ? hi_v : lo_v;
                    } else {
                        // (cos, sin): y_m = c x_m + s x_n, y_n = c x_n - s x_m
                        const float sg = hi ? -q : q;
                        v[i] = fmaf(sg, w[i], p * v[i]);
                    }
                });
            }
        });
    }
    if (tb.modes[table]) {
        const float* sg = tb.signs + table * N + V * lane;
        StaticFor<0, V>::run([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            v[i] *= sg[i];
        });
    }
    if (bad) StaticFor<0, V>::run([&](auto ii) { v[decltype(ii)::value] = 0.0f; });
    float* out = y + blk * N + V * lane;
    if constexpr (V == 4) {
        store_nt(out, make_float4(v[0], v[1], v[2], v[3]));
    } else if constexpr (V == 2) {
        typedef float vf2 __attribute__((ext_vector_type(2)));
        const vf2 o = {v[0], v[1]};
        __builtin_nontemporal_store(o, reinterpret_cast<vf2*>(out));
    } else {
        __builtin_nontemporal_store(v[0], out);
    }
}

// Requests of N <= 32: a wavefront takes G = 64 / N consecutive blocks, lane
// l element l mod N of block l / N, each group of N lanes with its block's
// own class (so the multipliers are per-lane 8-byte loads, coalesced within
// a group's table row). Every pass pairs lane l with lane l ^ 2^K inside its
// group; both run the pair's lifting and keep their own output, as above.
template <int D, int DIR>
__device__ __forceinline__ void request_small(const ReqTable& tb, const float* __restrict__ x,
                                              float* __restrict__ y,
                                              const int32_t* __restrict__ cls, int64_t nblocks,
                                              int64_t lw, int wv, int lane, int32_t* status) {
    constexpr int N = 1 << D;
    constexpr int G = 64 / N;
    const int64_t blk0 = (lw * 4 + wv) * G;
    if (blk0 >= nblocks) return;  // no barrier on this path
    const int e = lane & (N - 1);
    const int64_t blk = blk0 + (lane >> D);
    const bool valid = blk < nblocks;
    int c = 0;
    if (valid && cls != nullptr) c = cls[blk];
    const bool bad = valid && (c < 0 || c >= tb.nclasses);
    if (bad) {
        // the ring is in host memory: a system-scope store, which no cache
        // between the device and that memory holds back
        __hip_atomic_store(status, static_cast<int32_t>(HYGT_ECLASS), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
        c = 0;
    }
    const size_t table = static_cast<size_t>(DIR) * tb.nclasses + c;
    const float* tbl = tb.coef + table * static_cast<size_t>(tb.rounds) * D * N;
    float v = valid ? x[blk * N + e] : 0.0f;
    // multipliers of pass KK of round r: pair e without bit K
    auto mult = [&](int64_t r, auto kkc) -> float2 {
        constexpr int KK = decltype(kkc)::value;
        constexpr int K = DIR == 0 ? KK : D - 1 - KK;
        const int j = ((e >> (K + 1)) << K) | (e & ((1 << K) - 1));
        return reinterpret_cast<const float2*>(tbl + (r * D + KK) * N)[j];
    };
    float2 m = mult(0, std::integral_constant<int, 0>{});
    for (int r = 0; r < tb.rounds; ++r) {
        StaticFor<0, D>::run([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            constexpr int K = DIR == 0 ? k : D - 1 - k;
            const float2 a = m;
            if constexpr (k + 1 < D)
                m = mult(r, std::integral_constant<int, k + 1>{});
            else
                m = mult(r + 1 < tb.rounds ? r + 1 : r, std::integral_constant<int, 0>{});
            const bool hi = (e >> K) & 1;
            const float w = __shfl_xor(v, 1 << K, 64);
            float lo_v = hi ? w : v;
            float hi_v = hi ? v : w;
            lift_pair(lo_v, hi_v, a.x, a.y);
            v = hi ? hi_v : lo_v;
        });
    }
    if (tb.modes[table]) v *= tb.signs[table * N + e];
    if (bad) v = 0.0f;
    if (valid) __builtin_nontemporal_store(v, y + blk * N + e);
}

// The address u, of global memory, as a pointer that the compiler knows to
// be global (made from the integer as a global pointer, then converted), so
// that every access derived from it is a global rather than a generic
// (flat) load or store.
template <typename T>
__device__ __forceinline__ T* global_ptr(uint64_t u) {
    typedef __attribute__((address_space(1))) T* G;
    return (T*)reinterpret_cast<G>(u);
}

// Workgroup w belongs to the last of the launch's requests whose first
// workgroup is <= w (first_wg is non-decreasing along the launch, and a
// request without blocks shares its first workgroup with the next one),
// found by a binary search over the descriptors in the kernel's argument
// segment (wave-uniform scalar loads).
struct ReqWork {
    ReqTable tb;
    const float* x;
    float* y;
    const int32_t* cls;
    int64_t nblocks;
    int64_t lw;        // workgroup of the request
    int32_t* status;   // the request's ring entry's status
};

__device__ __forceinline__ ReqWork locate_request(const RequestArgs& a, int w) {
    typedef const __attribute__((address_space(4))) RequestArgs* ArgPtr;
    const ArgPtr pa = (ArgPtr)__builtin_amdgcn_kernarg_segment_ptr();
    int lo = 0, hi = a.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pa->req[mid].first_wg <= w) lo = mid;
        else hi = mid - 1;
    }
    const int r = lo;
    ReqWork o;
    const uint64_t ec = reinterpret_cast<uint64_t>(pa->req[r].cls);
    o.x = global_ptr<const float>(reinterpret_cast<uint64_t>(pa->req[r].x));
    o.y = global_ptr<float>(reinterpret_cast<uint64_t>(pa->req[r].y));
    o.cls = ec ? global_ptr<const int32_t>(ec) : nullptr;
    o.nblocks = pa->req[r].nblocks;
    o.lw = w - pa->req[r].first_wg;
    int64_t idx = a.first + pa->req[r].entry;
    if (idx >= a.capacity) idx -= a.capacity;
    o.status = a.status + 12 * idx;
    const int ti = pa->req[r].table;
    o.tb.modes = global_ptr<const int32_t>(reinterpret_cast<uint64_t>(pa->tab[ti].modes));
    o.tb.coef = global_ptr<const float>(reinterpret_cast<uint64_t>(pa->tab[ti].coef));
    o.tb.signs = global_ptr<const float>(reinterpret_cast<uint64_t>(pa->tab[ti].signs));
    o.tb.log2n = pa->tab[ti].log2n;
    o.tb.rounds = pa->tab[ti].rounds;
    o.tb.nclasses = pa->tab[ti].nclasses;
    o.tb.pad = 0;
    return o;
}

// A request batch: every size, a wavefront per block (N >= 64) or per
// 64 / N blocks (N <= 32).
template <int DIR>
__global__ __launch_bounds__(256) void request_kernel(RequestArgs a) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const ReqWork o = locate_request(a, blockIdx.x);
    switch (o.tb.log2n) {
        case 2: request_small<2, DIR>(o.tb, o.x, o.y, o.cls, o.nblocks, o.lw, wv, lane, o.status); break;
        case 3: request_small<3, DIR>(o.tb, o.x, o.y, o.cls, o.nblocks, o.lw, wv, lane, o.status); break;
        case 4: request_small<4, DIR>(o.tb, o.x, o.y, o.cls, o.nblocks, o.lw, wv, lane, o.status); break;
        case 5: request_small<5, DIR>(o.tb, o.x, o.y, o.cls, o.nblocks, o.lw, wv, lane, o.status); break;
        case 6: request_block<6, DIR>(o.tb, o.x, o.y, o.cls, o.nblocks, o.lw, wv, lane, o.status); break;
        case 7: request_block<7, DIR>(o.tb, o.x, o.y, o.cls, o.nblocks, o.lw, wv, lane, o.status); break;
        case 8: request_block<8, DIR>(o.tb, o.x, o.y, o.cls, o.nblocks, o.lw, wv, lane, o.status); break;
        default: break;
    }
}

}  // namespace

hipError_t launch_requests(const RequestArgs& a, int64_t workgroups, int direction,
                           hipStream_t stream) {
    if (workgroups <= 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>(workgroups));
    if (direction == 0)
        hipLaunchKernelGGL((request_kernel<0>), grid, dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL((request_kernel<1>), grid, dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace hygt

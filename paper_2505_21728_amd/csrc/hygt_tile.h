// Device helpers shared by the per-tile kernels (rotation, backward): tile
// geometry, compile-time loops, the direct row loads and the LDS-staged,
// non-temporal row stores, and the XCD-aware tile mapping. Every function is
// inline; the header is included by one or more translation units.
#pragma once

#include "hygt_internal.h"

namespace hygt {
namespace tile {

// Wavefronts (tiles) per workgroup of the single-size rotation kernels for
// N <= 64: one, so that every tile is dispatched on its own and a compute
// unit's wavefronts start and finish independently.
constexpr int kWaves = 1;
// Accelerator complex dies (XCDs) that workgroups are dispatched over.
constexpr int kXcds = 8;
// Register budget of the rotation kernels: resident wavefronts per SIMD (a
// lane holds at most 64 values).
#ifndef HYGT_WAVES_PER_SIMD
#define HYGT_WAVES_PER_SIMD 5
#endif
constexpr int kWavesPerSimd = HYGT_WAVES_PER_SIMD;
// The same for the tiles of N >= 128, whose multiplier stream holds chunks
// in VGPRs (VTableStream below).
constexpr int kSplitWavesPerSimd = 4;

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

// Read-only tables (multipliers, signs, modes) seen through the constant
// address space: loads from it are known not to be clobbered by the
// kernel's stores, so wave-uniform ones become scalar loads through the
// scalar cache even where the compiler cannot prove it from the pointers
// alone (as in a kernel that takes them from a struct of arguments).
typedef __attribute__((address_space(3))) void* lds_ptr;
typedef const __attribute__((address_space(4))) float* ctab_f;
typedef const __attribute__((address_space(4))) int32_t* ctab_i;
__device__ __forceinline__ ctab_f as_ctab(const float* p) { return (ctab_f)p; }
__device__ __forceinline__ ctab_i as_ctab(const int32_t* p) { return (ctab_i)p; }

__device__ __forceinline__ int valid_block(int b, int64_t nblocks) {
    return (b >= 0 && b < nblocks) ? b : -1;  // never touch memory outside x / y
}

// A tile goes out from registers through LDS in PARTS parts of CHP 16-byte chunks per
// block (CHP = min(N/4, kChunksPerPart)); a wavefront's LDS image of one part
// is 64 * CHP * 16 bytes.
#ifndef HYGT_CHUNKS_PER_PART
#define HYGT_CHUNKS_PER_PART 8
#endif
constexpr int kChunksPerPart = HYGT_CHUNKS_PER_PART;
template <int D>
struct TileGeo {
    static constexpr int N = 1 << D;
    static constexpr bool SPLIT = D > kLaneBits;     // several wavefronts per tile
    static constexpr int SHARE = SPLIT ? 1 << (D - kLaneBits) : 1;  // wavefronts per tile
    static constexpr int V = N / SHARE;              // values per lane
    static constexpr int LD = SPLIT ? kLaneBits : D; // log2(V)
    static constexpr int CH = V / 4;                 // 16-byte chunks per lane's row
    static constexpr int CHP = CH < 1 ? 1 : CH < kChunksPerPart ? CH : kChunksPerPart;  // per part
    static constexpr int PARTS = CH / CHP;
    static constexpr int BPI = 64 / CHP;             // blocks per memory instruction
    static constexpr int WAVES = SPLIT ? SHARE : kWaves;  // wavefronts per workgroup
    static constexpr int TILES = SPLIT ? 1 : kWaves;      // tiles per workgroup
    static constexpr int OCC = SPLIT ? kSplitWavesPerSimd : kWavesPerSimd;
};

// Block id handled by memory instruction i of every part: block
// b = i*BPI + lane/CHP of the tile.
template <int D>
__device__ __forceinline__ void instr_blocks(int* bb, int blk, int lane) {
    using G = TileGeo<D>;
    StaticFor<0, G::CHP>::run([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        bb[i] = __builtin_amdgcn_ds_bpermute((i * G::BPI + lane / G::CHP) << 2, blk);
    });
}

// Outputs are written with non-temporal stores: they are not read again by
// this launch, and keeping them out of the caches leaves room for the inputs.
__device__ __forceinline__ void store_nt(float* p, float4 f) {
    typedef float vf4 __attribute__((ext_vector_type(4)));
    const vf4 w = {f.x, f.y, f.z, f.w};
    __builtin_nontemporal_store(w, reinterpret_cast<vf4*>(p));
}

template <int D>
__device__ __forceinline__ void scatter_part(float* __restrict__ y, const float4* L,
                                             const int* bb, int lane, int part) {
    using G = TileGeo<D>;
    StaticFor<0, G::CHP>::run([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        const int b = i * G::BPI + lane / G::CHP;
        const int ch = part * G::CHP + ((lane % G::CHP) ^ swz<G::CHP>(b));
        const float4 f = L[i * 64 + lane];
        if (bb[i] >= 0) store_nt(y + static_cast<int64_t>(bb[i]) * G::N + ch * 4, f);
    });
}

// Brings a lane's row (its block, or for N = 256 its half of the block)
// into registers: V / 4 loads of 16 bytes, all in flight at once, so the
// first passes can start on the chunks that arrive first.
template <int D>
__device__ __forceinline__ void load_row(const float* __restrict__ x, int blk, float* v) {
    using G = TileGeo<D>;
    if (blk < 0) return;
    const float4* src = reinterpret_cast<const float4*>(x + static_cast<int64_t>(blk) * G::N);
    StaticFor<0, G::V / 4>::run([&](auto qq) {
        constexpr int q = decltype(qq)::value;
        const float4 f = src[q];
        v[4 * q + 0] = f.x;
        v[4 * q + 1] = f.y;
        v[4 * q + 2] = f.z;
        v[4 * q + 3] = f.w;
    });
}

// Brings a whole tile of N <= 64 into registers, a lane's block into the
// lane's row, in one round trip. The first min(N/4, 8) 16-byte chunks of
// every block come through LDS by DMA (global_load_lds_dwordx4): each
// instruction reads 64/CD whole blocks' chunks (CD chunks each) and the
// chunks land at slot b*CD + (q ^ swz(b)), from where each lane reads its
// own row without bank conflicts. For N = 64 the other 8 chunks are read by
// the lanes themselves, issued right after the DMA, so that both halves are
// in flight at once. Measured on MI355X (2^20 8x8 blocks), this beat
// per-lane loads of the whole row by 3 to 4 us per launch: coalesced
// instructions touch 8 cache lines instead of 64. Lanes without a block
// (blk < 0) read block 0, which exists whenever a launch has blocks, and
// drop it: every load is issued, so the wait below counts exactly. L: the
// wavefront's LDS area of at least 64 * min(N/4, 8) float4.
//
// With PRIO the loads are issued at the highest wavefront priority, so that
// other wavefronts' arithmetic does not hold them back. For N = 64 the
// inverse transform starts with the pass along bit 5, which pairs values
// from both halves of a block and so can start only once the whole tile is
// in; measured on MI355X (2^20 8x8 blocks, R = 4), this took its launch from
// 113.4 to 110.3 us, while the forward, which starts on the DMA half, lost
// about 1 us and issues its loads at normal priority. For N <= 32 (one DMA
// round trip in either direction) the inverse gained 1 us at N = 16 but lost
// 4 us at N = 8 (2^21 blocks), so only the inverse of N = 64 uses it.
template <int D, bool PRIO = false>
__device__ __forceinline__ void load_tile(const float* __restrict__ x, int blk, float* v,
                                          float4* L, int lane) {
    using G = TileGeo<D>;
    static_assert(!G::SPLIT && D >= 2, "one lane per block, N >= 4");
    constexpr int N = G::N;
    constexpr int CH = G::CH;                 // chunks per block
    constexpr int CD = CH < 8 ? CH : 8;       // chunks through LDS
    constexpr int BPI = 64 / CD;              // blocks per DMA instruction
    const int src = blk < 0 ? 0 : blk;
    int bb[CD];
    StaticFor<0, CD>::run([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        bb[i] = __builtin_amdgcn_ds_bpermute((i * BPI + lane / CD) << 2, src);
    });
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(3);
#if defined(__HIP_DEVICE_COMPILE__)  // the LDS-DMA builtin exists only in the device pass
    StaticFor<0, CD>::run([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        const int b = i * BPI + lane / CD;
        const int q = (lane % CD) ^ swz<CD>(b);
        __builtin_amdgcn_global_load_lds(x + static_cast<int64_t>(bb[i]) * N + q * 4,
                                         (lds_ptr)(L + i * 64), 16, 0, 0);
    });
#endif
    // Pins the issue order: the row loads below must follow the DMA loads,
    // or the wait for "all but the last CH - CD" would not cover the DMA.
    asm volatile("" ::: "memory");
    if constexpr (CH > CD) {
        const float4* row = reinterpret_cast<const float4*>(x + static_cast<int64_t>(src) * N);
        StaticFor<CD, CH>::run([&](auto qq) {
            constexpr int q = decltype(qq)::value;
            const float4 f = row[q];
            v[4 * q + 0] = f.x;
            v[4 * q + 1] = f.y;
            v[4 * q + 2] = f.z;
            v[4 * q + 3] = f.w;
        });
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
        // the DMA loads are older than the CH - CD row loads
        static_assert(CH - CD == 8, "N = 64");
        asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
    } else {
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    StaticFor<0, CD>::run([&](auto qq) {
        constexpr int q = decltype(qq)::value;
        const float4 f = L[lane * CD + (q ^ swz<CD>(lane))];
        v[4 * q + 0] = f.x;
        v[4 * q + 1] = f.y;
        v[4 * q + 2] = f.z;
        v[4 * q + 3] = f.w;
    });
    // the area is written again (staging) only after these reads
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Writes part P of a tile back: each lane writes its block's CHP chunks of
// the part into L, then the transposed slots go out as whole blocks.
template <int D, int P>
__device__ __forceinline__ void store_part(float* __restrict__ y, float4* L, const int* bb,
                                           const float* v, int lane, int sw) {
    using G = TileGeo<D>;
    constexpr int CHP = G::CHP;
    StaticFor<0, CHP>::run([&](auto qq) {
        constexpr int q = decltype(qq)::value;
        constexpr int e = 4 * (P * CHP + q);
        L[lane * CHP + (q ^ sw)] = make_float4(v[e], v[e + 1], v[e + 2], v[e + 3]);
    });
    // LDS executes one wavefront's operations in order; only the compiler's
    // ordering of the transposed reads after the row writes needs pinning.
    asm volatile("" ::: "memory");
    scatter_part<D>(y, L, bb, lane, P);
    // Later row writes into L must not overtake the transposed reads.
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Class tables (multipliers) read through the scalar cache one chunk ahead.
//
// A chunk is F consecutive floats of a table (F = 2, 4, 8, 16 or 32: the
// multipliers of up to 16 pairs), held in one or two SGPR vectors. Left to
// itself the compiler issues each chunk's scalar loads right before the
// arithmetic that needs them and waits for them there, so every chunk costs a
// full scalar-cache (or L2) round trip that only other wavefronts can hide.
// The stream below requests chunk e + 1 while chunk e is used. next() first
// passes the current chunk to an empty asm statement that also rewrites the
// table pointer: the compiler must wait for that chunk there (when it is the
// only scalar load in flight), and the loads of the following chunk, addressed
// from the rewritten pointer, cannot be issued any earlier.
template <int F>
struct Chunk {
    static_assert(F == 2 || F == 4 || F == 8 || F == 16 || F == 32, "chunk size");
    static constexpr int NV = F > 16 ? F / 16 : 1;  // SGPR vectors
    static constexpr int W = F > 16 ? 16 : F;       // floats per vector
    typedef float vec __attribute__((ext_vector_type(W), aligned(4)));
    vec a[NV];
    template <int I>
    __device__ __forceinline__ float get() const {
        return a[I / W][I % W];
    }
};

template <int F>
struct TableStream {
    uint64_t base;  // table address, rewritten (unchanged) by every next()
    Chunk<F> cur;   // the chunk requested last
    __device__ __forceinline__ void load(int64_t off) {  // off: floats from the table start
        typedef const __attribute__((address_space(4))) typename Chunk<F>::vec* P;
        const P p = reinterpret_cast<P>(base + static_cast<uint64_t>(off) * sizeof(float));
        StaticFor<0, Chunk<F>::NV>::run([&](auto k) { cur.a[decltype(k)::value] = p[decltype(k)::value]; });
    }
    __device__ __forceinline__ void begin(ctab_f table, int64_t off) {
        base = reinterpret_cast<uint64_t>(table);
        load(off);
    }
    // Returns the chunk requested by the previous call and requests the one at
    // `off` (any chunk inside the table; the last call may repeat one).
    __device__ __forceinline__ Chunk<F> next(int64_t off) {
        if constexpr (Chunk<F>::NV == 1)
            asm volatile("" : "+s"(base) : "s"(cur.a[0]));
        else
            asm volatile("" : "+s"(base) : "s"(cur.a[0]), "s"(cur.a[1]));
        const Chunk<F> got = cur;
        load(off);
        return got;
    }
};


// Class tables streamed into vector registers, for the tiles of N >= 128.
//
// Their wavefronts are few (a tile takes 2 or 4, and small batches leave one
// or two per SIMD) and meet at the exchange barriers, so the one-chunk-ahead
// scalar stream above cannot hide an L2 round trip behind other wavefronts'
// arithmetic. Here a chunk of 16 pairs takes two VGPRs: lane l holds the
// multipliers of pair l mod 16 of the chunk (one 8-byte load per lane, 128
// distinct bytes per wavefront), and an operation that needs pair j's
// multiplier reads it from lane j of its row of 16 lanes through DPP
// (row_newbcast), as a modifier of the operation itself. Vector loads return
// in order, so the stream keeps Q chunks in flight and waits only for the
// oldest. Measured on MI355X (2^15 16x16 blocks, R = 4): 46 -> 38 us; the
// same stream for N <= 64, where the VALU work dominates, was slower
// (126 -> 137 us at 2^20 8x8 blocks), so those tiles keep the scalar stream.

// a + m[lane J of this lane's row] * b, one v_fmac_f32 with a DPP source.
// The compiler cannot fuse a DPP move into a multiply-accumulate by itself
// (it does for multiplies and adds); the two wait states that a DPP read
// needs after a VALU write of its operands are checked on the built code.
template <int J>
__device__ __forceinline__ float fmac_bcast(float m, float b, float a) {
    static_assert(J >= 0 && J < 16, "lane of a row");
    asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
        : "+v"(a)
        : "v"(m), "v"(b), "i"(J));
    return a;
}

// x ^ bits for a DPP source: the two wait states before any DPP read of the
// result are part of the same statement.
__device__ __forceinline__ float xor_for_dpp(float x, unsigned bits) {
    float out;
    asm("v_xor_b32 %0, %1, %2\n\ts_nop 1" : "=v"(out) : "s"(bits), "v"(x));
    return out;
}

struct VChunk {
    float x, y;  // lane l: the two floats of pair l mod 16 of the chunk
    // float I of the chunk (2j: first multiplier of pair j, 2j + 1: second)
    // in every lane, through a DPP move that the compiler fuses into the
    // multiply or add that uses it
    template <int I>
    __device__ __forceinline__ float get() const {
        constexpr int j = I / 2;
        static_assert(j < 16, "pairs per chunk");
        const float f = (I & 1) ? y : x;
        return __int_as_float(
            __builtin_amdgcn_mov_dpp(__float_as_int(f), 0x150 + j, 0xf, 0xf, true));
    }
};

template <int Q>
struct VTableStream {
    typedef float vf2 __attribute__((ext_vector_type(2)));
    typedef const __attribute__((address_space(1))) vf2* GP;
    uint64_t base;   // table address, rewritten (unchanged) by every next()
    uint32_t pair;   // lane mod 16
    float bx[Q], by[Q];  // chunks in flight, oldest first
    __device__ __forceinline__ void init(uint64_t table, int lane) {
        base = table;
        pair = static_cast<uint32_t>(lane) & 15;
    }
    // Requests the 32 floats at `off` (floats from the table start) behind
    // those in flight.
    __device__ __forceinline__ void push(int64_t off) {
        StaticFor<0, Q - 1>::run([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            bx[i] = bx[i + 1];
            by[i] = by[i + 1];
        });
        const GP p = reinterpret_cast<GP>(base + static_cast<uint64_t>(off) * sizeof(float));
        const vf2 f = p[pair];
        bx[Q - 1] = f.x;
        by[Q - 1] = f.y;
    }
    // Returns the oldest chunk and requests the one at `off`. The empty asm
    // statement makes the compiler wait for that chunk here, and the next
    // load, addressed from the rewritten pointer, cannot be issued earlier.
    __device__ __forceinline__ VChunk next(int64_t off) {
        asm volatile("" : "+s"(base) : "v"(bx[0]), "v"(by[0]));
        const VChunk got{bx[0], by[0]};
        push(off);
        return got;
    }
};

}  // namespace tile
}  // namespace hygt

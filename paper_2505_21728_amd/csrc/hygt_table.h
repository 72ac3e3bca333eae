// Per-class multiplier tables of the lifting form, built on the device by
// one workgroup per (direction, class): by the plan for the rotation kernels
// and by the backward's preparation launch for the reverse walk.
//
// Sec. IV and Fig. 6 store the transform parameters in a compact form and
// expand them into wider multipliers at use. Here every angle is converted,
// in FP64, into the two multipliers of a lifting (three-shear) form of its
// Givens rotation, rounded once to FP32:
//
//   a += p*b;  b += q*a;  a += p*b      p = tan(phi/2), q = -sin(phi)
//
// which applies y_m = cos(phi) a + sin(phi) b, y_n = -sin(phi) a + cos(phi) b
// (the Sec. IV element definition) in place, with three FMAs and no
// temporary. The angle is first reduced to |phi| <= pi/2, using
// G(theta) = -G(theta -/+ pi), so that |p|, |q| <= 1 and every step is well
// conditioned. The resulting sign flips are tracked per element through the
// passes: an element stored with sign s holds s times its true value, a pair
// whose two signs differ is rotated by -phi instead (G(phi) diag(1,-1) =
// diag(1,-1) G(-phi)), and the signs left at the end are applied to the
// outputs. Both the reduction and the sign bookkeeping depend only on the
// angles, so every block of a class follows the same arithmetic.
//
// For N >= 128 the passes along bits 6 and 7 pair values held by different
// wavefronts, which exchange them through LDS, and each side computes its
// own output from both inputs: those passes store (cos theta, sin theta)
// rather than lifting multipliers, with the sine's sign adjusted for the
// stored signs of the pair (the signs themselves are left unchanged by such
// a pass).

#pragma once

#include <cstdint>

#include "hygt_internal.h"

namespace hygt {
namespace table {

__device__ __forceinline__ int insert_zero_bit(int j, int k) {
    // pair j of pass k: lower index m is j with a 0 inserted at bit k (Fig. 5)
    return ((j >> k) << (k + 1)) | (j & ((1 << k) - 1));
}

// Angles converted per parallel sweep of a table builder.
constexpr int kAngleBatch = 2048;
// Angles each thread of a table builder loads at once.
constexpr int kLoadsPerThread = 8;

// LDS of a table builder.
struct TableShared {
    float tanh_phi[kAngleBatch];    // tan(phi/2) of the batch's angles (cos for bits >= 6)
    float sin_phi[kAngleBatch];     // sin(phi) (sin theta for bits >= 6)
    signed char flip[kAngleBatch];  // -1 where |theta| > pi/2
};

// Sign bits of up to 256 elements (bit i of word i / 64: element i is stored
// negated), the same in every lane of the wavefront. Four named words rather
// than an array, so that the compiler keeps them in registers.
struct SignBits {
    uint64_t w0, w1, w2, w3;
    __device__ __forceinline__ int bit(int i) const {
        // the word by masks rather than by selects, which the compiler would
        // turn back into an indexed (scratch) load of the four words
        const int q = i >> 6;
        const uint64_t word = (w0 & (0 - static_cast<uint64_t>(q == 0))) |
                              (w1 & (0 - static_cast<uint64_t>(q == 1))) |
                              (w2 & (0 - static_cast<uint64_t>(q == 2))) |
                              (w3 & (0 - static_cast<uint64_t>(q == 3)));
        return static_cast<int>((word >> (i & 63)) & 1u);
    }
};

// Angle of 8-bit parameter code q (Fig. 6 keeps one byte per parameter and
// a shared table of multipliers): q steps of 2 pi / 256 from -pi, so that
// q = 128 is the zero angle. Exact in FP64.
__device__ __forceinline__ double code_angle(uint8_t q) {
    return (static_cast<double>(q) - 128.0) * (3.141592653589793238462643383279502884 / 128.0);
}

// Multiplier table of class c in direction dir (0 forward, 1 inverse), from
// FP32 angles or 8-bit codes (exactly one of the two non-NULL), run by a
// whole workgroup:
//   cbase [R*d][N]  the pairs' two multipliers per pass, application order;
//   sbase [N]       the final sign (+1 / -1) of each output;
//   *mode           1 when some final sign is -1;
//   pair_flip [R*d] (optional, N <= 64) bit j set where pair j's two stored
//                   signs differ at the start of the pass, i.e. where the
//                   stored values' rotation sense is reversed.
// The FP64 conversion of a batch of angles runs in parallel; only the sign
// walk through the passes is sequential.
__device__ __forceinline__ void build_table(TableShared& sh, int dir, int c,
                                            const float* __restrict__ angles,
                                            const uint8_t* __restrict__ codes, int log2n,
                                            int rounds, float* __restrict__ cbase,
                                            float* __restrict__ sbase, int32_t* __restrict__ mode,
                                            uint32_t* __restrict__ pair_flip) {
    const int tid = threadIdx.x;
    const int n = 1 << log2n;
    const int half = n >> 1;
    const int passes = rounds * log2n;
    const int batch_passes = kAngleBatch / half;
    SignBits S = {0, 0, 0, 0};
    for (int p0 = 0; p0 < passes; p0 += batch_passes) {
        const int p1 = min(passes, p0 + batch_passes);
        __syncthreads();
        // Every angle of the batch is loaded before the first conversion, so
        // that the loads share one memory round trip.
        const int count = (p1 - p0) * half;
        for (int e0 = 0; e0 < count; e0 += kLoadsPerThread * static_cast<int>(blockDim.x)) {
            // Pass p in application order: the inverse runs the rounds and the
            // passes backwards with negated angles (eq. (6), eq. (9)).
            size_t ai[kLoadsPerThread];
#pragma unroll
            for (int u = 0; u < kLoadsPerThread; ++u) {
                const int e = e0 + tid + u * static_cast<int>(blockDim.x);
                const int p = p0 + e / half;
                const int j = e % half;
                const int kk = p % log2n, rr = p / log2n;
                const int k = dir ? log2n - 1 - kk : kk;
                const int r = dir ? rounds - 1 - rr : rr;
                // past the batch: the class's first angle, loaded and unused
                ai[u] = e < count
                            ? ((static_cast<size_t>(c) * rounds + r) * log2n + k) * half + j
                            : static_cast<size_t>(c) * rounds * log2n * half;
            }
            double th[kLoadsPerThread];
            if (codes != nullptr) {
#pragma unroll
                for (int u = 0; u < kLoadsPerThread; ++u) th[u] = code_angle(codes[ai[u]]);
            } else {
#pragma unroll
                for (int u = 0; u < kLoadsPerThread; ++u) th[u] = static_cast<double>(angles[ai[u]]);
            }
            // The LDS table is reached through a generic reference, which the
            // compiler may not separate from the loads: without this, it waits
            // for each load before the next.
#pragma unroll
            for (int u = 0; u < kLoadsPerThread; ++u) asm volatile("" ::"v"(th[u]));
#pragma unroll
            for (int u = 0; u < kLoadsPerThread; ++u) {
                const int e = e0 + tid + u * static_cast<int>(blockDim.x);
                if (e >= count) continue;
                const int p = p0 + e / half;
                const int kk = p % log2n;
                const int k = dir ? log2n - 1 - kk : kk;
                const double t = dir ? -th[u] : th[u];
                double sn, cs;
                if (k >= kLaneBits) {  // (cos, sin) form, no reduction
                    sincos(t, &sn, &cs);
                    sh.tanh_phi[e] = static_cast<float>(cs);
                    sh.sin_phi[e] = static_cast<float>(sn);
                    sh.flip[e] = 1;
                    continue;
                }
                // G(t) = f * G(phi) with |phi| <= pi/2
                const double pi = 3.141592653589793238462643383279502884;
                double phi = t;
                signed char f = 1;
                if (phi > pi / 2) { phi -= pi; f = -1; }
                else if (phi < -pi / 2) { phi += pi; f = -1; }
                // tan(phi / 2) = sin(phi) / (1 + cos(phi)), with 1 + cos(phi) >= 1
                sincos(phi, &sn, &cs);
                sh.tanh_phi[e] = static_cast<float>(sn / (1.0 + cs));
                sh.sin_phi[e] = static_cast<float>(sn);
                sh.flip[e] = f;
            }
        }
        __syncthreads();
        // The sign walk is sequential over the passes: one wavefront takes
        // it, with the stored signs of all elements as bit masks held by
        // every lane. A pair (m, n) rotated with flip f = -1 (G(theta) =
        // -G(phi)) negates both of its stored values, and a pair whose two
        // stored signs differ is rotated by -phi; a lane per pair (two for
        // N = 256) writes the multipliers, and ballots gather the new masks.
        if (tid < 64 && n <= 64) {
            // one sign word, lane j = pair j; no cross-wavefront passes
            const int lane = tid;
            const bool own = lane < half;
            uint64_t S0 = S.w0;
            for (int p = p0; p < p1; ++p) {
                const int kk = p % log2n;
                const int k = dir ? log2n - 1 - kk : kk;
                const int e = (p - p0) * half + (own ? lane : 0);
                const int f = sh.flip[e];
                const float tp = sh.tanh_phi[e];
                const float sp = sh.sin_phi[e];
                const uint64_t F = __ballot(own && f < 0);
                const int m = insert_zero_bit(lane, k) & 63;
                const int nn = (m + (1 << k)) & 63;
                const bool differ = own && (((S0 >> m) ^ (S0 >> nn)) & 1u);
                // a pair whose stored signs differ is rotated by -phi
                const float g = differ ? -1.0f : 1.0f;
                if (own) {
                    float* cp = cbase + static_cast<size_t>(p) * n;
                    *reinterpret_cast<float2*>(cp + 2 * lane) = make_float2(g * tp, -g * sp);
                }
                if (pair_flip != nullptr) {
                    const uint64_t bits = __ballot(differ);
                    if (lane == 0) pair_flip[p] = static_cast<uint32_t>(bits);
                }
                // element l takes the flip of its pair, l with bit k removed
                const int jl = ((lane >> (k + 1)) << k) | (lane & ((1 << k) - 1));
                S0 ^= __ballot(lane < n && ((F >> jl) & 1u));
            }
            S.w0 = S0;
        } else if (tid < 64) {
            // N = 128, 256: up to four sign words and two pairs per lane (j
            // and j + 64), all in named registers (no arrays indexed at run
            // time, which would go to scratch memory)
            const int lane = tid;
            for (int p = p0; p < p1; ++p) {
                const int kk = p % log2n;
                const int k = dir ? log2n - 1 - kk : kk;
                float* cp = cbase + static_cast<size_t>(p) * n;
                const int j0 = lane, j1 = lane + 64;
                const bool own1 = j1 < half;
                const int e0 = (p - p0) * half + j0;
                const int e1 = (p - p0) * half + (own1 ? j1 : j0);
                const int f0 = sh.flip[e0], f1 = sh.flip[e1];
                const float tp0 = sh.tanh_phi[e0], tp1 = sh.tanh_phi[e1];
                const float sp0 = sh.sin_phi[e0], sp1 = sh.sin_phi[e1];
                const uint64_t F0 = __ballot(f0 < 0);
                const uint64_t F1 = __ballot(own1 && f1 < 0);
                // a pair whose stored signs differ is rotated by -phi; in the
                // (cos, sin) form (k >= 6) the sine is multiplied by sm * sq
                // and the signs stay
                auto multipliers = [&](int j, float tp, float sp) {
                    const int m = insert_zero_bit(j, k);
                    const int nn = m + (1 << k);
                    const float g = S.bit(m) != S.bit(nn) ? -1.0f : 1.0f;
                    *reinterpret_cast<float2*>(cp + 2 * j) =
                        k >= kLaneBits ? make_float2(tp, g * sp) : make_float2(g * tp, -g * sp);
                };
                multipliers(j0, tp0, sp0);
                if (own1) multipliers(j1, tp1, sp1);
                if (k < kLaneBits) {
                    // element l takes the flip of its pair, l with bit k removed
                    auto flipped = [&](int l) {
                        const int j = ((l >> (k + 1)) << k) | (l & ((1 << k) - 1));
                        const uint64_t fw = (j >> 6) ? F1 : F0;
                        return l < n && ((fw >> (j & 63)) & 1u);
                    };
                    const uint64_t E0 = __ballot(flipped(lane));
                    const uint64_t E1 = __ballot(flipped(lane + 64));
                    const uint64_t E2 = __ballot(flipped(lane + 128));
                    const uint64_t E3 = __ballot(flipped(lane + 192));
                    S.w0 ^= E0;
                    S.w1 ^= E1;
                    S.w2 ^= E2;
                    S.w3 ^= E3;
                }
            }
        }
    }
    // The final signs; the masks are the same in every lane of wavefront 0.
    if (tid < 64) {
        for (int i = tid; i < n; i += 64) sbase[i] = S.bit(i) ? -1.0f : 1.0f;
        if (tid == 0) *mode = (S.w0 | S.w1 | S.w2 | S.w3) != 0 ? 1 : 0;
    }
}

}  // namespace table
}  // namespace hygt

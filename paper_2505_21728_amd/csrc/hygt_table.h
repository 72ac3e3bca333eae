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

// Passes of one batch of a table builder, at most (R <= 64 and d <= 8 give at
// most 512 passes; N <= 64 keeps one mask word per pass, N > 64 four, with at
// most 32 passes per batch).
constexpr int kMaskWords = 512;

// LDS of a table builder.
struct TableShared {
    float tanh_phi[kAngleBatch];    // tan(phi/2) of the batch's angles (cos for bits >= 6)
    float sin_phi[kAngleBatch];     // sin(phi) (sin theta for bits >= 6)
    uint64_t emask[kMaskWords];     // elements negated by each pass of the batch
    uint64_t smask[kMaskWords];     // stored signs before each pass of the batch
    uint64_t send[4];               // stored signs after the batch
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

// 1 / n!, exact to rounding (n! itself is exact in FP64 for n <= 18).
constexpr double inv_factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return 1.0 / f;
}

// sin h and cos h for |h| <= pi/4, in FP64, from their Taylor series
// sin h = h + h z (-1/3! + z/5! - ... - z^8/19!) and
// cos h = 1 + z (-1/2! + z/4! - ... - z^8/18!), z = h^2, by Horner's rule in
// z (the first dropped terms, h^21/21! and h^20/20!, are below 1e-20 on this
// range). The library's double sincos reduces arguments of any size and took
// about 1 us per angle and wavefront here; these angles never exceed pi/4.
__device__ __forceinline__ void sincos_quarter(double h, double* s, double* c) {
    const double z = h * h;
    double ps = -inv_factorial(19);
    double pc = -inv_factorial(18);
    ps = fma(z, ps, inv_factorial(17));
    pc = fma(z, pc, inv_factorial(16));
    ps = fma(z, ps, -inv_factorial(15));
    pc = fma(z, pc, -inv_factorial(14));
    ps = fma(z, ps, inv_factorial(13));
    pc = fma(z, pc, inv_factorial(12));
    ps = fma(z, ps, -inv_factorial(11));
    pc = fma(z, pc, -inv_factorial(10));
    ps = fma(z, ps, inv_factorial(9));
    pc = fma(z, pc, inv_factorial(8));
    ps = fma(z, ps, -inv_factorial(7));
    pc = fma(z, pc, -inv_factorial(6));
    ps = fma(z, ps, inv_factorial(5));
    pc = fma(z, pc, inv_factorial(4));
    ps = fma(z, ps, -inv_factorial(3));
    pc = fma(z, pc, -inv_factorial(2));
    *s = fma(h * z, ps, h);
    *c = fma(z, pc, 1.0);
}

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
                // G(t) = f * G(phi) with |phi| <= pi/2
                const double pi = 3.141592653589793238462643383279502884;
                double phi = t;
                signed char f = 1;
                if (phi > pi / 2) { phi -= pi; f = -1; }
                else if (phi < -pi / 2) { phi += pi; f = -1; }
                double sh2, ch2;
                sincos_quarter(0.5 * phi, &sh2, &ch2);
                const double sn = 2.0 * sh2 * ch2;           // sin(phi)
                if (k >= kLaneBits) {  // (cos, sin) form of t itself: no reduction
                    const double cs = (ch2 - sh2) * (ch2 + sh2);  // cos(phi)
                    sh.tanh_phi[e] = static_cast<float>(f * cs);
                    sh.sin_phi[e] = static_cast<float>(f * sn);
                    sh.flip[e] = 1;
                    continue;
                }
                sh.tanh_phi[e] = static_cast<float>(sh2 / ch2);  // tan(phi / 2)
                sh.sin_phi[e] = static_cast<float>(sn);
                sh.flip[e] = f;
            }
        }
        __syncthreads();
        // Signs. Stored signs change only where a pair is rotated with flip
        // f = -1 (G(theta) = -G(phi)), which negates both of its values, and
        // which pairs those are depends on the angles alone. So the masks of
        // elements negated by each pass (E_p) are found for all passes in
        // parallel, the stored signs before each pass (S_p, the running XOR
        // of the E's) follow in one short sequential sweep, and the
        // multipliers of all passes are again written in parallel: a pair
        // whose two stored signs differ is rotated by -phi. A wavefront takes
        // every fourth pass; a lane takes pair j (and j + 64 for N = 256),
        // the masks held as bit masks over the elements.
        const int wave = tid >> 6;
        const int lane = tid & 63;
        const int nwaves = static_cast<int>(blockDim.x) >> 6;
        constexpr int NW = 4;  // mask words per pass (256 elements)
        const int words = n > 64 ? NW : 1;
        // E_p of the batch's passes
        for (int p = p0 + wave; p < p1; p += nwaves) {
            const int kk = p % log2n;
            const int k = dir ? log2n - 1 - kk : kk;
            const int base = (p - p0) * half;
            if (k >= kLaneBits) {  // (cos, sin) form: no flips
                if (lane < words) sh.emask[(p - p0) * words + lane] = 0;
                continue;
            }
            // F: the pairs rotated with flip -1, a bit per pair (two words for N = 256)
            const bool own0 = lane < half;
            const bool own1 = lane + 64 < half;
            const uint64_t F0 = __ballot(own0 && sh.flip[base + (own0 ? lane : 0)] < 0);
            const uint64_t F1 = __ballot(own1 && sh.flip[base + (own1 ? lane + 64 : 0)] < 0);
            // element l takes the flip of its pair, l with bit k removed
            auto flipped = [&](int l) {
                const int j = ((l >> (k + 1)) << k) | (l & ((1 << k) - 1));
                const uint64_t fw = (j >> 6) ? F1 : F0;
                return l < n && ((fw >> (j & 63)) & 1u);
            };
            const uint64_t E0 = __ballot(flipped(lane));
            if (words == 1) {
                if (lane == 0) sh.emask[p - p0] = E0;
            } else {
                const uint64_t E1 = __ballot(flipped(lane + 64));
                const uint64_t E2 = __ballot(flipped(lane + 128));
                const uint64_t E3 = __ballot(flipped(lane + 192));
                if (lane == 0) {
                    uint64_t* e = sh.emask + (p - p0) * NW;
                    e[0] = E0;
                    e[1] = E1;
                    e[2] = E2;
                    e[3] = E3;
                }
            }
        }
        __syncthreads();
        // S_p for the batch's passes: lane w of wavefront 0 sweeps word w
        if (tid < words) {
            uint64_t sw = tid == 0 ? S.w0 : tid == 1 ? S.w1 : tid == 2 ? S.w2 : S.w3;
            for (int q = 0; q < p1 - p0; ++q) {
                sh.smask[q * words + tid] = sw;
                sw ^= sh.emask[q * words + tid];
            }
            sh.send[tid] = sw;
        }
        __syncthreads();
        // multipliers of the batch's passes
        for (int p = p0 + wave; p < p1; p += nwaves) {
            const int kk = p % log2n;
            const int k = dir ? log2n - 1 - kk : kk;
            const int base = (p - p0) * half;
            SignBits Sp = {sh.smask[(p - p0) * words], 0, 0, 0};
            if (words > 1) {
                Sp.w1 = sh.smask[(p - p0) * words + 1];
                Sp.w2 = sh.smask[(p - p0) * words + 2];
                Sp.w3 = sh.smask[(p - p0) * words + 3];
            }
            float* cp = cbase + static_cast<size_t>(p) * n;
            uint64_t differ_bits = 0;
            auto multipliers = [&](int j) {
                const int m = insert_zero_bit(j, k);
                const int nn = m + (1 << k);
                const bool differ = Sp.bit(m) != Sp.bit(nn);
                const float g = differ ? -1.0f : 1.0f;
                const float tp = sh.tanh_phi[base + j];
                const float sp = sh.sin_phi[base + j];
                // (cos, sin) form (k >= 6): the sine times the pair's signs,
                // which the pass leaves unchanged
                *reinterpret_cast<float2*>(cp + 2 * j) =
                    k >= kLaneBits ? make_float2(tp, g * sp) : make_float2(g * tp, -g * sp);
                return differ;
            };
            const bool d0 = lane < half && multipliers(lane);
            if (lane + 64 < half) multipliers(lane + 64);
            differ_bits = __ballot(d0);
            if (pair_flip != nullptr && lane == 0) pair_flip[p] = static_cast<uint32_t>(differ_bits);
        }
        // the signs after the batch (read by every thread), and the LDS of
        // this batch free for the next
        __syncthreads();
        S.w0 = sh.send[0];
        if (words > 1) {
            S.w1 = sh.send[1];
            S.w2 = sh.send[2];
            S.w3 = sh.send[3];
        }
    }
    // The final signs (the same masks in every thread).
    for (int i = tid; i < n; i += blockDim.x) sbase[i] = S.bit(i) ? -1.0f : 1.0f;
    if (tid == 0) *mode = (S.w0 | S.w1 | S.w2 | S.w3) != 0 ? 1 : 0;
}

}  // namespace table
}  // namespace hygt

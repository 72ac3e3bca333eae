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

// LDS of a table builder.
struct TableShared {
    int sign[256];
    float tanh_phi[kAngleBatch];    // tan(phi/2) of the batch's angles (cos for bits >= 6)
    float sin_phi[kAngleBatch];     // sin(phi) (sin theta for bits >= 6)
    signed char flip[kAngleBatch];  // -1 where |theta| > pi/2
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
__device__ inline void build_table(TableShared& sh, int dir, int c,
                                   const float* __restrict__ angles,
                                   const uint8_t* __restrict__ codes, int log2n, int rounds,
                                   float* __restrict__ cbase, float* __restrict__ sbase,
                                   int32_t* __restrict__ mode, uint32_t* __restrict__ pair_flip) {
    const int tid = threadIdx.x;
    const int n = 1 << log2n;
    const int half = n >> 1;
    const int passes = rounds * log2n;
    const int batch_passes = kAngleBatch / half;
    for (int i = tid; i < n; i += blockDim.x) sh.sign[i] = 1;
    for (int p0 = 0; p0 < passes; p0 += batch_passes) {
        const int p1 = min(passes, p0 + batch_passes);
        __syncthreads();
        for (int e = tid; e < (p1 - p0) * half; e += blockDim.x) {
            // Pass p in application order: the inverse runs the rounds and
            // the passes backwards with negated angles (eq. (6), eq. (9)).
            const int p = p0 + e / half;
            const int j = e % half;
            const int kk = p % log2n, rr = p / log2n;
            const int k = dir ? log2n - 1 - kk : kk;
            const int r = dir ? rounds - 1 - rr : rr;
            const size_t ai = ((static_cast<size_t>(c) * rounds + r) * log2n + k) * half + j;
            double th = codes != nullptr ? code_angle(codes[ai]) : static_cast<double>(angles[ai]);
            if (dir) th = -th;
            if (k >= kLaneBits) {  // (cos, sin) form, no reduction
                sh.tanh_phi[e] = static_cast<float>(cos(th));
                sh.sin_phi[e] = static_cast<float>(sin(th));
                sh.flip[e] = 1;
                continue;
            }
            // G(th) = f * G(phi) with |phi| <= pi/2
            const double pi = 3.141592653589793238462643383279502884;
            double phi = th;
            signed char f = 1;
            if (phi > pi / 2) { phi -= pi; f = -1; }
            else if (phi < -pi / 2) { phi += pi; f = -1; }
            sh.tanh_phi[e] = static_cast<float>(tan(0.5 * phi));
            sh.sin_phi[e] = static_cast<float>(sin(phi));
            sh.flip[e] = f;
        }
        __syncthreads();
        for (int p = p0; p < p1; ++p) {
            const int kk = p % log2n;
            const int k = dir ? log2n - 1 - kk : kk;
            bool differ = false;
            if (tid < half) {
                const int e = (p - p0) * half + tid;
                const int m = insert_zero_bit(tid, k);
                const int nn = m + (1 << k);
                const int sm = sh.sign[m];
                const int sq = sh.sign[nn];
                const int f = sh.flip[e];
                differ = sm != sq;
                // a pair whose stored signs differ is rotated by -phi
                const float g = differ ? -1.0f : 1.0f;
                float* cp = cbase + static_cast<size_t>(p) * n;
                if (k >= kLaneBits) {
                    // stored (sm a, sq b) -> (sm a', sq b'): the sine is
                    // multiplied by sm * sq, the signs stay
                    cp[2 * tid + 0] = sh.tanh_phi[e];
                    cp[2 * tid + 1] = g * sh.sin_phi[e];
                } else {
                    cp[2 * tid + 0] = g * sh.tanh_phi[e];
                    cp[2 * tid + 1] = -g * sh.sin_phi[e];
                    sh.sign[m] = f * sm;
                    sh.sign[nn] = sm == sq ? f * sm : -f * sm;
                }
            }
            if (pair_flip != nullptr && tid < 64) {
                // half <= 32 pairs: all in the first wavefront
                const uint64_t bits = __ballot(differ);
                if (tid == 0) pair_flip[p] = static_cast<uint32_t>(bits);
            }
            __syncthreads();
        }
    }
    int neg = 0;
    for (int i = tid; i < n; i += blockDim.x) {
        sbase[i] = static_cast<float>(sh.sign[i]);
        neg |= sh.sign[i] < 0;
    }
    neg = __syncthreads_or(neg);
    if (tid == 0) *mode = neg ? 1 : 0;
}

}  // namespace table
}  // namespace hygt

// The QR shortening of a pivot block-pair (Section 4.2, eq. (2.8)): the
// triangular factor R of [G_p G_q] without forming Q, as an alternative to
// the Cholesky factor of the Gram matrix.  [G_p G_q] is read in chunks of
// BW rows; each chunk is factored by BW - 1 Householder reflections, which
// are applied and dropped, and its triangular factor R_1 is folded into the
// running factor R_0 by the "peel-off" procedure: BW stages of independent
// Givens rotations, stage k rotating row x of R_0 with row x - k of R_1 to
// annihilate R_1(x - k, x), so that the k-th superdiagonal of R_1 goes in
// stage k.  Here the rows of a pair are split over several workgroups (each
// folds its chunks into a factor of its own) and the inner kernel folds
// those factors together by the same procedure.
//
// Matrices live in LDS, column-major with leading dimension LD; NT threads
// (a multiple of 64) take part, a half wave (32 lanes) per column or per row
// pair.
#pragma once

#include "jsvd_blocked.h"

namespace jsvd {

namespace {

// Householder QR of the BW x BW matrix A in place: on return the upper
// triangle holds R and the rest is zero.  Step k computes the reflector
// H_k = I - tau v v^T (v_k = 1) of column k in every half wave (LAPACK's
// convention: beta = -sign(alpha) ||A(k:, k)||, tau = (beta - alpha) / beta,
// v = A(k+1:, k) / (alpha - beta)) and applies it to the columns right of k,
// one column per half wave at a time; one barrier per step.
template <int BW, int NT>
__device__ __forceinline__ void chunk_qr(double *A, int LD) {
    constexpr int RR = BW / 32;      // rows per lane
    constexpr int NHW = NT / 32;     // half waves
    const int x = threadIdx.x & 31, hw = threadIdx.x >> 5;
    for (int k = 0; k < BW - 1; ++k) {
        double vk[RR];
        double xn2 = 0.0;
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int i = x + 32 * r;
            vk[r] = i > k ? A[k * LD + i] : 0.0;
            xn2 = fma(vk[r], vk[r], xn2);
        }
        xn2 = hw_sum(xn2);
        const double alpha = A[k * LD + k];
        double tau = 0.0, beta = alpha;
        if (xn2 > 0.0) {
            beta = -copysign(sqrt(fma(alpha, alpha, xn2)), alpha);
            tau = (beta - alpha) / beta;
            const double scal = 1.0 / (alpha - beta);
#pragma unroll
            for (int r = 0; r < RR; ++r) vk[r] *= scal;
        }
        if (tau != 0.0) {
            for (int j = k + 1 + hw; j < BW; j += NHW) {
                double aj[RR];
                double d = x == 0 ? A[j * LD + k] : 0.0;  // v_k = 1 times A(k, j)
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    aj[r] = A[j * LD + x + 32 * r];
                    d = fma(vk[r], aj[r], d);   // vk is zero at and above row k
                }
                const double z = tau * hw_sum(d);
#pragma unroll
                for (int r = 0; r < RR; ++r)
                    if (x + 32 * r > k) A[j * LD + x + 32 * r] = fma(-z, vk[r], aj[r]);
                if (x == 0) A[j * LD + k] -= z;
            }
        }
        __syncthreads();
        // column k of R: beta on the diagonal, zeros below (no half wave
        // reads column k again)
        if (hw == 0) {
#pragma unroll
            for (int r = 0; r < RR; ++r) {
                const int i = x + 32 * r;
                if (i > k) A[k * LD + i] = 0.0;
            }
            if (x == 0) A[k * LD + k] = beta;
        }
    }
    __syncthreads();
}

// R0 <- the triangular factor of [R0; R1] (both BW x BW upper triangular),
// R1 <- 0, by the peel-off procedure; one barrier per stage.  A rotation
// with R1(x - k, x) = 0 is the identity.
template <int BW, int NT>
__device__ __forceinline__ void peel_off(double *R0, double *R1, int LD) {
    constexpr int NHW = NT / 32;
    const int lane = threadIdx.x & 31, hw = threadIdx.x >> 5;
    for (int k = 0; k < BW; ++k) {
        for (int x0 = k + hw; x0 < BW; x0 += NHW) {
            const int y0 = x0 - k;  // the row of R1
            const double a = R0[x0 * LD + x0], b = R1[x0 * LD + y0];
            if (b != 0.0) {
                const double r = sqrt(fma(a, a, b * b));
                const double c = a / r, s = b / r;
                for (int col = x0 + 1 + lane; col < BW; col += 32) {
                    const double u = R0[col * LD + x0], v = R1[col * LD + y0];
                    R0[col * LD + x0] = fma(c, u, s * v);
                    R1[col * LD + y0] = fma(c, v, -(s * u));
                }
                if (lane == 0) {
                    R0[x0 * LD + x0] = r;
                    R1[x0 * LD + y0] = 0.0;
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace

}  // namespace jsvd

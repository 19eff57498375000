// FP64 MFMA matrix products for the QR preprocessing and the SVD adjoint.
//
// gemm_f64_kernel is the general batched product.  Two shapes of the
// blocked Householder QR (eq. (2.1); a panel of 32 reflectors V with its
// 32 x 32 factor T) get kernels of their own, as the general tiling leaves
// them far below the HBM roofline:
//   * Y = V^T C over all rows (split over row slices): 32 output rows, a
//     contraction over thousands of rows -- laid out as the Gram kernel
//     is, each lane reading consecutive rows of one column of both
//     operands, so that the contraction runs along the rows;
//   * C <- alpha V Y + beta C with 32 reflectors: a rank-32 update of a
//     tall C, computed as (V Y)^T = Y^T V^T so that each lane's results are
//     consecutive rows of one column of C (coalesced reads and writes),
//     the 16 x 32 slice of V of a wave held in registers and the block's
//     slice of Y in LDS across the column tiles.
#include "jsvd_device.h"

namespace jsvd {

namespace {

// C = alpha op(A) op(B) + beta C [+ E diag(d)] for a batch of column-major
// matrices, or (split-K) one product whose K range is cut into slices, slice
// b summed into the b-th C of the batch.
// op(A) is M x K, op(B) is K x N.  Workgroup tile 64 x 64 (four waves of
// 32 x 32, each 2 x 2 MFMA tiles of 16 x 16), K step 16 staged in LDS.
// MFMA lane layout: lane l supplies A[l%16][l/16] and B[l/16][l%16]; the
// result holds D[l/16 + 4v][l%16] in element v.
__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmArgs g) {
    __shared__ double As[16][64 + 1];  // As[k][i] = op(A)[i0 + i][k0 + k]
    __shared__ double Bs[16][64 + 1];  // Bs[k][j] = op(B)[k0 + k][j0 + j]
    const int b = blockIdx.z;
    const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
    const double *A = g.A + (g.ksplit ? 0 : (size_t)b * g.sa);
    const double *B = g.B + (g.ksplit ? 0 : (size_t)b * g.sb);
    double *C = g.C + (size_t)b * g.sc;
    // K range of this product (split-K: one slice per batch index)
    const int kbeg = g.ksplit ? (int)min((int64_t)g.K, (int64_t)b * g.ksplit) : 0;
    const int kend = g.ksplit ? (int)min((int64_t)g.K, (int64_t)(b + 1) * g.ksplit) : g.K;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = (wave & 1) * 32, wj = (wave >> 1) * 32;
    const int l16 = lane & 15, lg = lane >> 4;
    d4 acc[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};

    for (int k0 = kbeg; k0 < kend; k0 += 16) {
        // stage op(A)[i0 .. i0+63][k0 .. k0+15] and op(B)[k0 .. k0+15][j0 .. j0+63]
        for (int e = tid; e < 64 * 16; e += 256) {
            int i, k;
            if (g.ta) {  // op(A) = A^T: element (i, k) at A[k + i * lda]; read along k
                k = e % 16;
                i = e / 16;
            } else {     // element (i, k) at A[i + k * lda]; read along i
                i = e % 64;
                k = e / 64;
            }
            const int gi = i0 + i, gk = k0 + k;
            double v = 0.0;
            if (gi < g.M && gk < kend) v = g.ta ? A[gk + (size_t)gi * g.lda] : A[gi + (size_t)gk * g.lda];
            As[k][i] = v;
        }
        for (int e = tid; e < 16 * 64; e += 256) {
            int k, j;
            if (g.tb) {  // op(B) = B^T: element (k, j) at B[j + k * ldb]; read along j
                j = e % 64;
                k = e / 64;
            } else {     // element (k, j) at B[k + j * ldb]; read along k
                k = e % 16;
                j = e / 16;
            }
            const int gk = k0 + k, gj = j0 + j;
            double v = 0.0;
            if (gk < kend && gj < g.N) v = g.tb ? B[gj + (size_t)gk * g.ldb] : B[gk + (size_t)gj * g.ldb];
            Bs[k][j] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) av[x] = As[kk + lg][wi + 16 * x + l16];
#pragma unroll
            for (int y = 0; y < 2; ++y) bv[y] = Bs[kk + lg][wj + 16 * y + l16];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) acc[x][y] = mfma16(av[x], bv[y], acc[x][y]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = i0 + wi + 16 * x + lg + 4 * v;
                const int gj = j0 + wj + 16 * y + l16;
                if (gi < g.M && gj < g.N) {
                    double r = g.alpha == 1.0 ? acc[x][y][v] : g.alpha * acc[x][y][v];
                    if (g.beta != 0.0) r = fma(g.beta, C[gi + (size_t)gj * g.ldc], r);
                    if (g.E) r += g.E[(size_t)b * g.se + gi + (size_t)gj * g.lde] * g.d[(size_t)b * g.sd + gj];
                    C[gi + (size_t)gj * g.ldc] = r;
                }
            }
}

// out_b (M x N, ld M) = A[rows of slice b]^T B[rows of slice b], slices of
// ksplit rows; M <= 16 MT.  Grid (column blocks of 64, slices), 256
// threads: the four waves take 8-row steps of the slice (each lane 2
// consecutive rows of one column of A and of B: the same rows are the
// contraction index of both MFMA operands), and their accumulators are
// summed in a fixed order at the end.
// two doubles loaded as one 16-byte access (8-byte alignment suffices)
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));

template <int MT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void gemm_tn_rows_kernel(const double *A, int64_t lda,
                                                           const double *B, int64_t ldb, int M,
                                                           int N, int64_t K, int64_t ksplit,
                                                           double *out, int64_t so) {
    constexpr int NTL = 4;  // column tiles of 16 of B per workgroup
    constexpr int S = 2;    // consecutive rows per lane
    __shared__ d4 red[MT * NTL * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, grp = lane >> 4;
    const int b = blockIdx.y;
    const int j0 = blockIdx.x * 64;
    const int64_t r0 = (int64_t)b * ksplit, r1 = min(K, r0 + ksplit);
    const double *ca[MT];
    const double *cb[NTL];
    bool va[MT], vb[NTL];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        const int c = 16 * t + i16;
        va[t] = c < M;
        ca[t] = A + (va[t] ? c : 0) * lda;
    }
#pragma unroll
    for (int t = 0; t < NTL; ++t) {
        const int c = j0 + 16 * t + i16;
        vb[t] = c < N;
        cb[t] = B + (vb[t] ? c : 0) * ldb;
    }
    d4 acc[MT][NTL];
#pragma unroll
    for (int x = 0; x < MT; ++x)
#pragma unroll
        for (int y = 0; y < NTL; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    // every column of both operands present: the S = 2 consecutive rows of a
    // lane as one 16-byte load, without selects
    const bool allv = M == 16 * MT && j0 + 64 <= N;
    for (int64_t base = r0 + wave * 4 * S; base < r1; base += 16 * S) {
        const int64_t rb = base + grp * S;
        double xa[MT][S], xb[NTL][S];
        if (allv && rb + S <= r1) {
            static_assert(S == 2, "one 16-byte load per lane and column");
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                const d2u v = *reinterpret_cast<const d2u *>(ca[t] + rb);
                xa[t][0] = v.x;
                xa[t][1] = v.y;
            }
#pragma unroll
            for (int t = 0; t < NTL; ++t) {
                const d2u v = *reinterpret_cast<const d2u *>(cb[t] + rb);
                xb[t][0] = v.x;
                xb[t][1] = v.y;
            }
        } else {
#pragma unroll
            for (int t = 0; t < MT; ++t)
#pragma unroll
                for (int s = 0; s < S; ++s) xa[t][s] = (va[t] && rb + s < r1) ? ca[t][rb + s] : 0.0;
#pragma unroll
            for (int t = 0; t < NTL; ++t)
#pragma unroll
                for (int s = 0; s < S; ++s) xb[t][s] = (vb[t] && rb + s < r1) ? cb[t][rb + s] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int x = 0; x < MT; ++x)
#pragma unroll
                for (int y = 0; y < NTL; ++y) acc[x][y] = mfma16(xa[x][s], xb[y][s], acc[x][y]);
    }
    // fixed-order sum over the four waves: ((w0 + w1) + w2) + w3
    for (int wv = 0; wv < 4; ++wv) {
        if (wave == wv) {
#pragma unroll
            for (int x = 0; x < MT; ++x)
#pragma unroll
                for (int y = 0; y < NTL; ++y) {
                    d4 &r = red[(x * NTL + y) * 64 + lane];
                    r = wv == 0 ? acc[x][y] : r + acc[x][y];
                }
        }
        __syncthreads();
    }
    double *o = out + (int64_t)b * so;
    for (int e = threadIdx.x; e < MT * NTL * 256; e += 256) {
        const int k = e >> 8, rem = e & 255, v = rem >> 6, l = rem & 63;
        const int x = k / NTL, y = k % NTL;
        const int row = 16 * x + (l >> 4) + 4 * v, col = j0 + 16 * y + (l & 15);
        if (row < M && col < N) o[row + (int64_t)col * M] = red[k * 64 + l][v];
    }
}

// C (rows x N, ld ldc) = alpha A Y + beta C with A rows x K (ld lda), Y K x N
// (ld ldy), K <= 32.  Grid (row blocks of 64, column blocks of 64), 256
// threads: the block's K x 64 slice of Y is staged in LDS once (each lane
// of a tile would otherwise fetch 16 strided columns of Y per MFMA step);
// wave w owns rows [16 w, 16 w + 16) of the block, keeps its 16 x K slice of
// A in registers (lane l: row l % 16, columns l / 16 + 4 k) and walks the
// column tiles of 16: per tile C's 16 x 16 tile is read first (beta != 0),
// then the K / 4 MFMAs of Y^T A^T, and the tile is written back as 16
// consecutive rows per column.
__global__ __launch_bounds__(256) void gemm_rank_kernel(const double *A, int64_t lda,
                                                        const double *Y, int64_t ldy,
                                                        double *C, int64_t ldc, int rows, int N,
                                                        int K, double alpha, double beta) {
    constexpr int KS = 8;       // MFMA steps of 4 along K (K <= 32)
    constexpr int CB = 64;      // columns per workgroup
    constexpr int YLD = 36;     // LDS leading dimension of the Y slice (two lanes per bank pair)
    __shared__ double ys[CB * YLD];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, grp = lane >> 4;
    const int jbeg = blockIdx.y * CB, jend = min(N, jbeg + CB);
    for (int e = threadIdx.x; e < CB * 32; e += 256) {
        const int c = e / 32, k = e % 32;
        ys[c * YLD + k] = (jbeg + c < N && k < K) ? Y[k + (int64_t)(jbeg + c) * ldy] : 0.0;
    }
    const int64_t row = (int64_t)blockIdx.x * 64 + wave * 16 + i16;
    const bool rv = row < rows;
    double av[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int kk = 4 * k + grp;
        av[k] = (rv && kk < K) ? A[row + (int64_t)kk * lda] : 0.0;
    }
    __syncthreads();
    for (int j0 = jbeg; j0 < jend; j0 += 16) {
        double cv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int col = j0 + grp + 4 * v;
            cv[v] = (beta != 0.0 && rv && col < N) ? C[row + (int64_t)col * ldc] : 0.0;
        }
        const double *yc = ys + (j0 - jbeg + i16) * YLD;  // the column of Y this lane supplies
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < KS; ++k) acc = mfma16(yc[4 * k + grp], av[k], acc);
        // acc[v] = (Y^T A^T)(j0 + grp + 4 v, row) = (A Y)(row, j0 + grp + 4 v)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int col = j0 + grp + 4 * v;
            if (rv && col < N) {
                double r = alpha == 1.0 ? acc[v] : alpha * acc[v];
                if (beta != 0.0) r = fma(beta, cv[v], r);
                C[row + (int64_t)col * ldc] = r;
            }
        }
    }
}

}  // namespace

hipError_t launch_gemm(const GemmArgs &g, hipStream_t s) {
    if (g.ta && !g.tb && g.ksplit > 0 && g.M <= 32 && g.alpha == 1.0 && g.beta == 0.0 && !g.E) {
        dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)g.batch);
        if (g.M <= 16)
            hipLaunchKernelGGL(gemm_tn_rows_kernel<1>, grid, dim3(256), 0, s, g.A, g.lda, g.B,
                               g.ldb, g.M, g.N, (int64_t)g.K, g.ksplit, g.C, g.sc);
        else
            hipLaunchKernelGGL(gemm_tn_rows_kernel<2>, grid, dim3(256), 0, s, g.A, g.lda, g.B,
                               g.ldb, g.M, g.N, (int64_t)g.K, g.ksplit, g.C, g.sc);
        return hipGetLastError();
    }
    if (!g.ta && !g.tb && g.batch == 1 && !g.ksplit && g.K <= 32 && !g.E) {
        dim3 grid((unsigned)((g.M + 63) / 64), (unsigned)((g.N + 63) / 64));
        hipLaunchKernelGGL(gemm_rank_kernel, grid, dim3(256), 0, s, g.A, g.lda, g.B, g.ldb, g.C,
                           g.ldc, g.M, g.N, g.K, g.alpha, g.beta);
        return hipGetLastError();
    }
    dim3 grid((unsigned)((g.M + 63) / 64), (unsigned)((g.N + 63) / 64), (unsigned)g.batch);
    hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

}  // namespace jsvd

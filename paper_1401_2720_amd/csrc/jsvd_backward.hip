// Reverse-mode derivative (adjoint) of the SVD, A = U diag(s) V^T with
// A m x n, m >= n, U m x n, V n x n, distinct singular values.  Given the
// adjoints dU, ds, dV of a scalar loss:
//
//   J = U^T dU,  K = V^T dV,  F_ij = 1 / (s_j^2 - s_i^2) (i != j), F_ii = 0,
//   M = diag(ds) + (F o (J - J^T)) diag(s) + diag(s) (F o (K - K^T)),
//   dA = U M V^T + (I - U U^T) dU diag(s)^{-1} V^T
//      = (U (M - J diag(s)^{-1}) + dU diag(s)^{-1}) V^T,
//
// the published SVD adjoint (the last form folds the projector into one
// product).  The paper has no backward; this is the form used by the
// autograd function of the package.  Products run on a batched FP64 MFMA
// GEMM; the elementwise middle step on a small kernel.
#include "jsvd_internal.h"

namespace jsvd {

namespace {

typedef double d4b __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4b mfma16b(double a, double b, d4b c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

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
    d4b acc[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = d4b{0.0, 0.0, 0.0, 0.0};

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
                for (int y = 0; y < 2; ++y) acc[x][y] = mfma16b(av[x], bv[y], acc[x][y]);
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

// M' = diag(ds) + F o (J - J^T) diag(s) + diag(s) F o (K - K^T) - J diag(1/s),
// one thread per entry; J, K may be null (zero).  Equal singular values set
// *degenerate.
__global__ void adjoint_middle_kernel(int64_t batch, int n, const double *s, int64_t ss,
                                      const double *ds, const double *J, const double *K,
                                      double *Mp, double *inv_s, int *degenerate) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nn = (int64_t)n * n;
    if (e >= batch * nn) return;
    const int64_t b = e / nn;
    const int r = (int)(e % nn);
    const int i = r % n, j = r / n;  // column-major (i, j)
    const double si = s[b * ss + i], sj = s[b * ss + j];
    const double *Jb = J ? J + b * nn : nullptr, *Kb = K ? K + b * nn : nullptr;
    const double jij = Jb ? Jb[i + (size_t)j * n] : 0.0, jji = Jb ? Jb[j + (size_t)i * n] : 0.0;
    const double kij = Kb ? Kb[i + (size_t)j * n] : 0.0, kji = Kb ? Kb[j + (size_t)i * n] : 0.0;
    double v;
    if (i == j) {
        v = (ds ? ds[b * ss + i] : 0.0) - jij / sj;
        inv_s[b * n + i] = 1.0 / si;
    } else {
        const double den = sj * sj - si * si;
        if (den == 0.0) *degenerate = 1;
        const double f = 1.0 / den;
        v = f * (jij - jji) * sj + si * (f * (kij - kji)) - jij / sj;
    }
    Mp[b * nn + r] = v;
}

__global__ void zero_int_kernel(int *p) {
    if (threadIdx.x == 0) *p = 0;
}

}  // namespace

hipError_t launch_gemm(const GemmArgs &g, hipStream_t s) {
    dim3 grid((unsigned)((g.M + 63) / 64), (unsigned)((g.N + 63) / 64), (unsigned)g.batch);
    hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_adjoint_middle(int64_t batch, int n, const double *s, int64_t ss,
                                 const double *ds, const double *J, const double *K, double *Mp,
                                 double *inv_s, int *degenerate, hipStream_t st) {
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, st, degenerate);
    const int64_t total = batch * (int64_t)n * n;
    hipLaunchKernelGGL(adjoint_middle_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       st, batch, n, s, ss, ds, J, K, Mp, inv_s, degenerate);
    return hipGetLastError();
}

}  // namespace jsvd

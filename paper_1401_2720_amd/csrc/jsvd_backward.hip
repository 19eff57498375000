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
// autograd function of the package.  Products run on the batched FP64 MFMA
// GEMM of jsvd_gemm.hip; the elementwise middle step on a small kernel.
#include "jsvd_internal.h"

namespace jsvd {

namespace {

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

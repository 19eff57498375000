// Small kernels around the sweeps: counter reset, V = I, column norms
// (the singular values, Section 4), the final ordering and the gathers.
#include "jsvd_rdssq.h"

namespace jsvd {

namespace {

// ------------------------------------------------------------ small kernels
__global__ void reset_counters_kernel(unsigned long long *c) {
    if (threadIdx.x < C_COUNT) c[threadIdx.x] = 0ull;
}

__global__ void init_identity_kernel(double *V, int64_t ldv, int64_t n) {
    const int64_t j = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        V[i + j * ldv] = (i == j) ? 1.0 : 0.0;
}

// sigma_j = ||g_j||_2 (the Sigma kernel of Section 4): fma accumulation
// per thread, then a fixed-shape tree in LDS.
__global__ __launch_bounds__(256) void colnorm_kernel(const double *G, int64_t ldg, int64_t m,
                                                      double *s_out) {
    __shared__ double part[256];
    const int64_t j = blockIdx.x;
    const double *g = G + j * ldg;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += 256) s = fma(g[i], g[i], s);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) s_out[j] = sqrt(part[0]);
}

// Column norms without overflow or underflow (the concern of Section 4.2),
// by DRDSSQ (Appendix A; one workgroup per column): the pair (j, s) with
// ||g_j||^2 = 2^j s.  Writes, when asked, the norm 2^(j/2) sqrt(s) and the
// exponent e_j of ||g_j|| (||g_j|| in [2^e_j, 2^(e_j+1)): j/2, less one when
// s < 1; 0 for a zero or non-finite column), and folds the exponents of the
// nonzero finite columns into range[0] (min) and range[1] (max).
__global__ __launch_bounds__(256) void colexp_kernel(const double *G, int64_t ldg, int64_t m,
                                                     double t_hi, double *s_out, int *ex,
                                                     int *range) {
    __shared__ double red[3 * 256];
    const int64_t c = blockIdx.x;
    int j;
    double s;
    wg_rdssq<256>(G + c * ldg, m, t_hi, red, j, s);
    if (threadIdx.x == 0) {
        const bool fin = s > 0.0 && s < 2.0;  // non-zero, no NaN met
        if (s_out) s_out[c] = rdssq_norm(j, s);
        if (ex) {
            const int e = fin ? j / 2 - (s < 1.0 ? 1 : 0) : 0;
            ex[c] = e;
            if (fin && range) {
                atomicMin(&range[0], e);
                atomicMax(&range[1], e);
            }
        }
    }
}

// DRDSSQ of every column (the boundary's column-norm call): the pair
// (j, s) and the norm, each output optional.
__global__ __launch_bounds__(256) void rdssq_cols_kernel(const double *A, int64_t lda, int64_t m,
                                                         double t_hi, int32_t *exps, double *ssq,
                                                         double *norms) {
    __shared__ double red[3 * 256];
    const int64_t c = blockIdx.x;
    int j;
    double s;
    wg_rdssq<256>(A + c * lda, m, t_hi, red, j, s);
    if (threadIdx.x == 0) {
        if (exps) exps[c] = j;
        if (ssq) ssq[c] = s;
        if (norms) norms[c] = rdssq_norm(j, s);
    }
}

// Output order: positions [0, n_plus) by non-increasing sigma, [n_plus, n)
// by non-decreasing sigma, ties by column index; NaN sorts as -infinity so
// that the ranks always form a permutation.
// The keys are staged through LDS in chunks shared by the workgroup (every
// thread compares its key with all keys of its part).
constexpr int kRankChunk = 2048;

__global__ __launch_bounds__(256) void rank_kernel(const double *s, int64_t n, int64_t n_plus,
                                                   int *perm) {
    __shared__ double ks[kRankChunk];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = j < n;
    const bool pos = valid && j < n_plus;
    const int64_t lo = pos ? 0 : n_plus, hi = pos ? n_plus : n;
    const double kj = valid ? ((s[j] != s[j]) ? -INFINITY : s[j]) : 0.0;
    int64_t r = lo;
    for (int64_t base = 0; base < n; base += kRankChunk) {
        __syncthreads();
        for (int t = threadIdx.x; t < kRankChunk; t += blockDim.x) {
            const double v = base + t < n ? s[base + t] : 0.0;
            ks[t] = (v != v) ? -INFINITY : v;
        }
        __syncthreads();
        if (valid) {
            const int64_t i0 = lo > base ? lo : base;
            const int64_t i1 = hi < base + kRankChunk ? hi : base + kRankChunk;
            for (int64_t i = i0; i < i1; ++i) {
                const double ki = ks[i - base];
                const bool before = pos ? (ki > kj) : (ki < kj);
                if (before || (ki == kj && i < j)) ++r;
            }
        }
    }
    if (valid) perm[r] = (int)j;
}

// dst[:, k] = src[:, perm[k]] (perm may be null: identity), divided by
// scale[perm[k]] when scale is given (u = g / sigma, 0 when sigma = 0);
// s_out[k] = scale[perm[k]].
__global__ void gather_cols_kernel(const double *src, int64_t lds, double *dst, int64_t ldd,
                                   int64_t rows, const int *perm, const double *scale,
                                   double *s_out) {
    const int64_t k = blockIdx.y;
    const int64_t c = perm ? perm[k] : k;
    const double sc = scale ? scale[c] : 1.0;
    if (s_out && blockIdx.x == 0 && threadIdx.x == 0) s_out[k] = sc;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = src[i + c * lds];
        dst[i + k * ldd] = scale ? (sc > 0.0 ? v / sc : 0.0) : v;
    }
}

// dst[row_of[i], :] = src[i, :]
__global__ void scatter_rows_kernel(const double *src, int64_t lds, double *dst, int64_t ldd,
                                    int64_t rows, const int *row_of) {
    const int64_t k = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[row_of[i] + k * ldd] = src[i + k * lds];
}

__global__ void diag_fp64_kernel(int64_t count, const double *a, const double *b, double *q,
                                 double *r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        q[i] = a[i] / b[i];
        r[i] = sqrt(a[i]);
    }
}

// The refined operations of the rotation formulas and the Cholesky pivots,
// through the same device functions the kernels call, for a rounding check.
__global__ void diag_refined_kernel(int64_t count, const double *a, const double *b,
                                    double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        const double x = a[i], y = b[i];
        out[i] = nrcp(y);
        out[count + i] = ndiv(x, y);
        out[2 * count + i] = nsqrt(x);
        double rs, d;
        rsqrt_sqrt(x, rs, d);
        out[3 * count + i] = rs;
        out[4 * count + i] = d;
    }
}

}  // namespace

hipError_t launch_reset_counters(unsigned long long *c, hipStream_t s) {
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_init_identity(double *V, int64_t ldv, int64_t n, hipStream_t s) {
    const int64_t bx = std::min<int64_t>((n + 255) / 256, 64);
    hipLaunchKernelGGL(init_identity_kernel, dim3((unsigned)bx, (unsigned)n), dim3(256), 0, s, V,
                       ldv, n);
    return hipGetLastError();
}

hipError_t launch_colnorms(const double *G, int64_t ldg, int64_t m, int64_t n, double *s_out,
                           hipStream_t s) {
    hipLaunchKernelGGL(colnorm_kernel, dim3((unsigned)n), dim3(256), 0, s, G, ldg, m, s_out);
    return hipGetLastError();
}

// B (rows x cols, ld ldb) = columns first .. first + cols - 1 of the
// identity of order rows.
__global__ void identity_cols_kernel(double *B, int64_t ldb, int64_t rows, int64_t first) {
    const int64_t c = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x)
        B[i + c * ldb] = (i == first + c) ? 1.0 : 0.0;
}

// out[0] = the number of entries of S (n of them) that are > 0.
__global__ void count_positive_kernel(const double *S, int64_t n, int *out) {
    __shared__ int part[256];
    int c = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) c += S[i] > 0.0 ? 1 : 0;
    part[threadIdx.x] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0];
}

__global__ void range_init_kernel(int *range) {
    if (threadIdx.x == 0) {
        range[0] = 0x7fffffff;
        range[1] = -0x7fffffff - 1;
    }
}

hipError_t launch_identity_cols(double *B, int64_t ldb, int64_t rows, int64_t cols, int64_t first,
                                hipStream_t s) {
    if (cols <= 0) return hipSuccess;
    const int64_t bx = std::min<int64_t>((rows + 255) / 256, 64);
    hipLaunchKernelGGL(identity_cols_kernel, dim3((unsigned)bx, (unsigned)cols), dim3(256), 0, s, B,
                       ldb, rows, first);
    return hipGetLastError();
}

hipError_t launch_count_positive(const double *S, int64_t n, int *out, hipStream_t s) {
    hipLaunchKernelGGL(count_positive_kernel, dim3(1), dim3(256), 0, s, S, n, out);
    return hipGetLastError();
}

hipError_t launch_range_init(int *range, hipStream_t s) {
    hipLaunchKernelGGL(range_init_kernel, dim3(1), dim3(64), 0, s, range);
    return hipGetLastError();
}

hipError_t launch_colexp(const double *G, int64_t ldg, int64_t m, int64_t n, double *s_out,
                         int *ex, int *range, hipStream_t s) {
    const int lg = m <= 1 ? 0 : 64 - __builtin_clzll((unsigned long long)(m - 1));
    hipLaunchKernelGGL(colexp_kernel, dim3((unsigned)n), dim3(256), 0, s, G, ldg, m,
                       rdssq_t_hi(lg), s_out, ex, range);
    return hipGetLastError();
}

hipError_t launch_rdssq_cols(const double *A, int64_t lda, int64_t m, int64_t n, int32_t *exps,
                             double *ssq, double *norms, hipStream_t s) {
    const int lg = m <= 1 ? 0 : 64 - __builtin_clzll((unsigned long long)(m - 1));
    hipLaunchKernelGGL(rdssq_cols_kernel, dim3((unsigned)n), dim3(256), 0, s, A, lda, m,
                       rdssq_t_hi(lg), exps, ssq, norms);
    return hipGetLastError();
}

hipError_t launch_rank(const double *s, int64_t n, int64_t n_plus, int *perm, hipStream_t st) {
    hipLaunchKernelGGL(rank_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, n,
                       n_plus, perm);
    return hipGetLastError();
}

hipError_t launch_gather_cols(const double *src, int64_t lds, double *dst, int64_t ldd,
                              int64_t rows, int64_t cols, const int *perm, const double *scale,
                              double *s_out, hipStream_t s) {
    const int64_t bx = std::max<int64_t>(1, std::min<int64_t>((rows + 255) / 256, 32));
    hipLaunchKernelGGL(gather_cols_kernel, dim3((unsigned)bx, (unsigned)cols), dim3(256), 0, s,
                       src, lds, dst, ldd, rows, perm, scale, s_out);
    return hipGetLastError();
}

hipError_t launch_scatter_rows(const double *src, int64_t lds, double *dst, int64_t ldd,
                               int64_t rows, int64_t cols, const int *row_of, hipStream_t s) {
    const int64_t bx = std::max<int64_t>(1, std::min<int64_t>((rows + 255) / 256, 32));
    hipLaunchKernelGGL(scatter_rows_kernel, dim3((unsigned)bx, (unsigned)cols), dim3(256), 0, s,
                       src, lds, dst, ldd, rows, row_of);
    return hipGetLastError();
}

hipError_t launch_diag_fp64(int64_t count, const double *a, const double *b, double *q,
                            double *r, hipStream_t s) {
    hipLaunchKernelGGL(diag_fp64_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                       count, a, b, q, r);
    return hipGetLastError();
}

hipError_t launch_diag_refined(int64_t count, const double *a, const double *b, double *out,
                               hipStream_t s) {
    hipLaunchKernelGGL(diag_refined_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                       s, count, a, b, out);
    return hipGetLastError();
}

}  // namespace jsvd

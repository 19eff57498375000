// QR preprocessing of a tall G (Section 2, eq. (2.1)): G P = Q [R; 0] by
// Householder reflections in panels of 32 columns (compact WY form, Q =
// H_1 ... H_n, H_k = I - tau_k v_k v_k^T with v_k(k) = 1), the columns P
// presorted by non-increasing norm.  The Jacobi method then runs on the
// n x n factor.
//
//   qr_panel_kernel   one panel, all workgroups resident: every workgroup holds a
//                     slice of the panel's rows in registers; each column
//                     is one grid-wide reduction (the norm below the
//                     diagonal and the dot products with the panel's
//                     remaining columns), summed in workgroup order, then
//                     every workgroup applies the reflection to its rows;
//   qr_t_kernel       the panel's triangular T (Q_panel = I - V T V^T) from
//                     V^T V and tau, by the column recurrence of the
//                     compact WY form;
//   the trailing update C <- C - V T^T (V^T C) and the application of Q run
//   on the FP64 MFMA GEMM (split-K for the tall V^T C products).
//
// All arithmetic is FP64, reductions have a fixed order, so results are
// bitwise reproducible run to run.
#include "jsvd_device.h"

namespace jsvd {

namespace {

constexpr int kNb = kQrPanel;      // panel width
constexpr int kQT = 256;           // threads per workgroup of the panel kernel
constexpr int kRpt = 2;            // panel rows per thread, at most

// Grid-wide barrier among resident workgroups: monotonic arrival counter,
// bounded spin (a barrier that does not complete within the bound sets the
// abort flag and lets every workgroup leave).  The workgroup barrier first
// completes the stores of all its threads; thread 0's release increment
// then publishes them at device scope (one write-back of the XCD's L2), its
// spin reads the counter without ordering, and one device-scope acquire
// after the spin (one invalidation) makes the other workgroups' stores
// visible to the whole workgroup past the second workgroup barrier.
__device__ __forceinline__ bool grid_sync(unsigned *bar, unsigned target, int *abort_flag) {
    __syncthreads();
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        unsigned spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1u << 24)) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Sums of the kNb values v[] over the workgroup's 256 threads, in a fixed
// order: red[c][t] <- v[c] of thread t; 8 segments of 32 threads summed
// sequentially, then the 8 segment sums.  Result in out[c] for c < nv.
// Thread t sums segment t / 32 of column t mod 32, so that the 16 lanes of
// a wave that read LDS together read 16 columns (distinct banks), and seg
// is padded to 9 for the same reason.
__device__ __forceinline__ void wg_sum(const double (&v)[kNb], int nv, double (*red)[kQT + 1], double (*seg)[9],
                       double *out) {
    static_assert(kNb == 32 && kQT == 256, "32 columns, 8 segments of 32 threads");
    const int t = threadIdx.x;
#pragma unroll
    for (int c = 0; c < kNb; ++c)
        if (c < nv) red[c][t] = v[c];
    __syncthreads();
    {
        const int c = t & 31, sg = t >> 5;
        if (c < nv) {
            double s = 0.0;
            for (int i = 0; i < 32; ++i) s += red[c][sg * 32 + i];
            seg[c][sg] = s;
        }
    }
    __syncthreads();
    if (t < nv) {
        double s = 0.0;
        for (int i = 0; i < 8; ++i) s += seg[t][i];
        out[t] = s;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kQT, 1) void qr_panel_kernel(QrPanelArgs a) {
    __shared__ double red[kNb][kQT + 1];
    __shared__ double seg[kNb][9];
    __shared__ double wsum[kNb];
    __shared__ double gsum[kNb];
    __shared__ double s_prow[kNb];
    __shared__ double s_w[kNb];   // v^T a_c of the current column's reflector
    const int wg = blockIdx.x, t = threadIdx.x;
    const int64_t rows = a.m - a.j;                       // panel rows j .. m-1
    const int64_t chunk = (rows + a.nwg - 1) / a.nwg;     // rows per workgroup
    const int64_t r_beg = a.j + wg * chunk;
    const int64_t r_end = min(a.m, r_beg + chunk);
    const int nb = a.nb;
    double *W = a.W;
    const int64_t ldw = a.ldw;

    double x[kRpt][kNb];
    int64_t rr[kRpt];
#pragma unroll
    for (int q = 0; q < kRpt; ++q) {
        rr[q] = r_beg + t + (int64_t)q * kQT;
        const bool in = rr[q] < r_end;
#pragma unroll
        for (int c = 0; c < kNb; ++c) x[q][c] = (in && c < nb) ? W[rr[q] + (a.j + c) * ldw] : 0.0;
    }

    // Column k of the panel is picked out of the register arrays by
    // selection over the (unrolled) column index, so that the arrays stay in
    // registers while k runs over the panel.
    for (int k = 0; k < nb; ++k) {
        const int64_t pr = a.j + k;  // pivot row
        const int par = k & 1;
        double xk[kRpt];
#pragma unroll
        for (int q = 0; q < kRpt; ++q) {
            xk[q] = 0.0;
#pragma unroll
            for (int c = 0; c < kNb; ++c) xk[q] = (c == k) ? x[q][c] : xk[q];
        }
        // partial sums over own rows below the pivot: column k with columns k .. nb-1
        // (also formed, and not used, for the columns left of k)
        double ps[kNb];
#pragma unroll
        for (int c = 0; c < kNb; ++c) ps[c] = 0.0;
#pragma unroll
        for (int q = 0; q < kRpt; ++q) {
            if (rr[q] > pr && rr[q] < r_end) {
#pragma unroll
                for (int c = 0; c < kNb; ++c) ps[c] = fma(xk[q], x[q][c], ps[c]);
            }
            if (rr[q] == pr && rr[q] < r_end) {
#pragma unroll
                for (int c = 0; c < kNb; ++c)
                    if (c >= k) a.prow[par * kNb + c] = x[q][c];
            }
        }
        wg_sum(ps, nb, red, seg, wsum);
        if (t < nb) a.partials[((size_t)par * a.nwg + wg) * kNb + t] = wsum[t];
        if (!grid_sync(a.bar, (unsigned)(a.nwg * (k + 1)), a.abort_flag)) return;
        // all workgroups: totals in workgroup order, the pivot row, the
        // reflector.  The nwg x nb partial sums (nwg <= 64) and the pivot row
        // are loaded by all threads at once into LDS (one memory round trip),
        // then each column's partials are added in workgroup order.
        {
            const int c = t & 31;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int w = (t >> 5) + 8 * i;
                if (c < nb && w < a.nwg) red[c][w] = a.partials[((size_t)par * a.nwg + w) * kNb + c];
            }
            if (t < nb) s_prow[t] = a.prow[par * kNb + t];
        }
        __syncthreads();
        if (t < nb) {
            double sum = 0.0;
            for (int w = 0; w < a.nwg; ++w) sum += red[t][w];
            gsum[t] = sum;
        }
        __syncthreads();
        const double alpha = s_prow[k];
        const double xn2 = gsum[k];  // squared norm below the pivot
        double tau = 0.0, beta = alpha, scal = 0.0;
        if (xn2 > 0.0) {
            beta = -copysign(sqrt(fma(alpha, alpha, xn2)), alpha);
            tau = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        // v^T a_c for the columns the reflection changes, zero for the others
        if (t < kNb) s_w[t] = (t > k && t < nb && tau != 0.0) ? fma(scal, gsum[t], s_prow[t]) : 0.0;
        __syncthreads();
        if (wg == 0 && t == 0) a.tau[a.j + k] = tau;
        // rows: v = e_pivot + scal * x(below); a_c -= tau v (v^T a_c), c > k
        // (without a branch: the other columns get tau v times zero added)
#pragma unroll
        for (int q = 0; q < kRpt; ++q) {
            if (rr[q] >= pr && rr[q] < r_end) {
                const bool piv = rr[q] == pr;
                const double v = piv ? 1.0 : xk[q] * scal;
                const double mtv = -tau * v;
#pragma unroll
                for (int c = 0; c < kNb; ++c) {
                    x[q][c] = fma(mtv, s_w[c], x[q][c]);
                    if (c == k) x[q][c] = piv ? beta : v;
                }
            }
        }
        __syncthreads();  // gsum, s_prow and s_w are rewritten by the next column
    }
    // write back: R above and on the diagonal, v below; explicit V of the panel
#pragma unroll
    for (int q = 0; q < kRpt; ++q) {
        if (rr[q] >= r_end) continue;
        const int64_t li = rr[q] - a.j;  // row within the panel
#pragma unroll
        for (int c = 0; c < kNb; ++c) {
            if (c < nb) W[rr[q] + (a.j + c) * ldw] = x[q][c];
            a.Vp[li + (int64_t)c * a.ldvp] = (c >= nb) ? 0.0 : (li > c ? x[q][c] : (li == c ? 1.0 : 0.0));
        }
    }
}

// T (nb x nb, upper triangular, column-major, ld kNb) with I - V T V^T =
// H_1 ... H_nb from Y = V^T V (ld kNb) and tau: T(c, c) = tau_c,
// T(0:c, c) = -tau_c T(0:c, 0:c) Y(0:c, c).
// Y and tau are staged in LDS first, so that the nb steps of the recurrence
// wait for no memory access.
__global__ void qr_t_kernel(const double *Y, const double *tau, int nb, double *T) {
    __shared__ double Ts[kNb][kNb + 1];
    __shared__ double Ys[kNb][kNb + 1];
    __shared__ double ts[kNb];
    const int t = threadIdx.x;
    for (int e = t; e < kNb * kNb; e += blockDim.x) {
        Ts[e % kNb][e / kNb] = 0.0;
        Ys[e % kNb][e / kNb] = Y[e];
    }
    if (t < nb) ts[t] = tau[t];
    __syncthreads();
    for (int c = 0; c < nb; ++c) {
        const double tc = ts[c];
        if (t < c) {
            double s = 0.0;
            for (int i = t; i < c; ++i) s = fma(Ts[t][i], Ys[i][c], s);
            Ts[t][c] = -tc * s;
        }
        if (t == 0) Ts[c][c] = tc;
        __syncthreads();
    }
    for (int e = t; e < kNb * kNb; e += blockDim.x) T[e] = Ts[e % kNb][e / kNb];
}

// out = sum of parts[0 .. np) (each count doubles, stride count) in a fixed
// order: the slices cut into 8 consecutive groups, each group summed in
// order by its own thread, then the 8 group sums in order.  256 threads per
// workgroup, 32 elements per workgroup.
__global__ __launch_bounds__(256) void sum_parts_kernel(const double *parts, int np,
                                                        int64_t count, double *out) {
    __shared__ double gs[8][33];
    const int t = threadIdx.x, l = t & 31, g = t >> 5;
    const int64_t e = (int64_t)blockIdx.x * 32 + l;
    const int per = (np + 7) / 8;
    const int p0 = min(np, g * per), p1 = min(np, p0 + per);
    double s = 0.0;
    if (e < count)
        for (int p = p0; p < p1; ++p) s += parts[(size_t)p * count + e];
    gs[g][l] = s;
    __syncthreads();
    if (g == 0 && e < count) {
        double r = gs[0][l];
#pragma unroll
        for (int k = 1; k < 8; ++k) r += gs[k][l];
        out[e] = r;
    }
}

// X (n x n, ld ldx) = R^T, R the upper triangle of W's first n rows.
__global__ void r_transpose_kernel(const double *W, int64_t ldw, int64_t n, double *X,
                                   int64_t ldx, const double *colscale) {
    const int64_t c = blockIdx.y;  // column of X = row of R
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = (i >= c) ? W[c + i * ldw] : 0.0;
        X[i + c * ldx] = colscale ? v * colscale[i] : v;
    }
}

// out[c] = 2^ex[c] (exact)
__global__ void pow2_kernel(const int *ex, int64_t n, double *out) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x)
        out[c] = ldexp(1.0, ex[c]);
}

// Explicit V of the panel at column j (rows j .. m-1 of W; unit diagonal).
__global__ void qr_extract_v_kernel(const double *W, int64_t ldw, int64_t m, int64_t j, int nb,
                                    double *Vp, int64_t ldvp) {
    const int c = blockIdx.y;
    for (int64_t li = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; li < m - j;
         li += (int64_t)gridDim.x * blockDim.x)
        Vp[li + c * ldvp] = (c >= nb) ? 0.0 : (li > c ? W[j + li + (j + c) * ldw] : (li == c ? 1.0 : 0.0));
}

// B (rows x cols, ld ldb): rows < n copied from X (ld ldx), the others zero.
__global__ void embed_kernel(const double *X, int64_t ldx, int64_t n, double *B, int64_t ldb,
                             int64_t rows) {
    const int64_t c = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x)
        B[i + c * ldb] = i < n ? X[i + c * ldx] : 0.0;
}

// out[0] = min |W(i, i)|, out[1] = max |W(i, i)| over i < n (one workgroup;
// a NaN diagonal gives out[0] = NaN).
__global__ void diag_range_kernel(const double *W, int64_t ldw, int64_t n, double *out) {
    __shared__ double lo[256], hi[256];
    double a = INFINITY, b = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double d = fabs(W[i + i * ldw]);
        a = (d != d || a != a) ? NAN : fmin(a, d);
        b = fmax(b, d);
    }
    lo[threadIdx.x] = a;
    hi[threadIdx.x] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 1; t < 256; ++t) {
            a = (lo[t] != lo[t] || a != a) ? NAN : fmin(a, lo[t]);
            b = fmax(b, hi[t]);
        }
        out[0] = a;
        out[1] = b;
    }
}

// ------------------------------------------------ QR with column pivoting
// W (rows x ncols, ld ldw) in place by Householder reflections with column
// pivoting (the P_c of eq. (2.1)), on a grid of nwg resident workgroups that
// meet at grid barriers.  Physical column c belongs to workgroup c % nwg
// and never moves; step j takes the free column of largest partial norm
// (ties: smallest index) as pivot, its owner forms the reflector from rows
// j .. rows-1 (LAPACK's convention: beta at row j, v below it with v(j) = 1
// implicit), and every owner applies it to its free columns and downdates
// their partial norms (recomputed when the downdate loses accuracy, as in
// LAPACK's xLAQP2).  The factorization stops at the first step at which
// every free column has kept at most tol of its original norm outside the
// span of the pivots so far (partial norm <= tol times the column's norm;
// a zero column counts as spent), or at min(rows, ncols): that step count is
// the numerical rank k.  The test is invariant under column scaling, so a
// column that is small but independent (a graded G) keeps its place.  jpvt[j] is
// the physical column at position j (positions >= k: the remaining columns
// in increasing order).  All reductions have a fixed order.
struct QrcpShared {
    double red[kQT];
    int redi[kQT];
};

// Sum over the workgroup of v (one value per thread), fixed order; every
// thread gets the result.
__device__ __forceinline__ double wg_total(double v, QrcpShared &sh) {
    const int t = threadIdx.x;
    sh.red[t] = v;
    __syncthreads();
    for (int off = kQT / 2; off > 0; off >>= 1) {
        if (t < off) sh.red[t] += sh.red[t + off];
        __syncthreads();
    }
    const double r = sh.red[0];
    __syncthreads();
    return r;
}

// Largest (value, smallest index) over the workgroup; every thread gets it.
__device__ __forceinline__ void wg_argmax(double v, int i, QrcpShared &sh, double &bv, int &bi) {
    const int t = threadIdx.x;
    sh.red[t] = v;
    sh.redi[t] = i;
    __syncthreads();
    for (int off = kQT / 2; off > 0; off >>= 1) {
        if (t < off) {
            const double a = sh.red[t], b = sh.red[t + off];
            const int ia = sh.redi[t], ib = sh.redi[t + off];
            if (b > a || (b == a && ib < ia)) {
                sh.red[t] = b;
                sh.redi[t] = ib;
            }
        }
        __syncthreads();
    }
    bv = sh.red[0];
    bi = sh.redi[0];
    __syncthreads();
}

__global__ __launch_bounds__(kQT) void qrcp_kernel(QrcpArgs a) {
    __shared__ QrcpShared sh;
    const int wg = blockIdx.x, t = threadIdx.x;
    const int64_t rows = a.rows;
    const int nwg = a.nwg;
    const int kmax = (int)min(rows, a.ncols);
    unsigned epoch = 0;
    // partial norms of the owned columns, and their original norms
    for (int64_t c = wg; c < a.ncols; c += nwg) {
        const double *col = a.W + c * a.ldw;
        double s = 0.0;
        for (int64_t i = t; i < rows; i += kQT) s = fma(col[i], col[i], s);
        const double nrm = sqrt(wg_total(s, sh));
        if (t == 0) {
            a.vn1[c] = nrm;
            a.vn2[c] = nrm;
            a.vn0[c] = nrm;
        }
    }
    __syncthreads();
    int k = kmax;
    for (int j = 0; j < kmax; ++j) {
        const int par = j & 1;
        // the workgroup's candidate: largest partial norm of a free column,
        // and the largest fraction of its norm that a free column has kept
        double bv = -1.0, br = 0.0;
        int bi = 0x7fffffff;
        for (int64_t c = wg + (int64_t)t * nwg; c < a.ncols; c += (int64_t)kQT * nwg) {
            const double v = a.vn1[c], v0 = a.vn0[c];
            if (v > bv || (v == bv && c < bi)) {
                bv = v;
                bi = (int)c;
            }
            if (v >= 0.0 && v0 > 0.0) br = fmax(br, v / v0);
        }
        wg_argmax(bv, bi, sh, bv, bi);
        int unused;
        wg_argmax(br, 0, sh, br, unused);
        if (t == 0) {
            a.cand_v[par * nwg + wg] = bv;
            a.cand_i[par * nwg + wg] = bi;
            a.cand_r[par * nwg + wg] = br;
        }
        if (!grid_sync(a.bar, ++epoch * (unsigned)nwg, a.abort_flag)) return;
        // the pivot: the same choice in every workgroup
        double pv = -1.0, pr = 0.0;
        int pc = 0x7fffffff;
        if (t < nwg) {
            pv = a.cand_v[par * nwg + t];
            pc = a.cand_i[par * nwg + t];
            pr = a.cand_r[par * nwg + t];
        }
        wg_argmax(pv, pc, sh, pv, pc);
        wg_argmax(pr, 0, sh, pr, unused);
        if (!(pv > 0.0) || pr <= a.tol) {
            k = j;
            break;
        }
        if (wg == 0 && t == 0) a.jpvt[j] = pc;
        if (pc % nwg == wg) {
            double *col = a.W + (int64_t)pc * a.ldw;
            double s = 0.0;
            for (int64_t i = j + 1 + t; i < rows; i += kQT) s = fma(col[i], col[i], s);
            const double xn2 = wg_total(s, sh);
            const double alpha = col[j];
            double tau = 0.0, beta = alpha, scal = 0.0;
            if (xn2 > 0.0) {
                beta = -copysign(sqrt(fma(alpha, alpha, xn2)), alpha);
                tau = (beta - alpha) / beta;
                scal = 1.0 / (alpha - beta);
            }
            for (int64_t i = j + 1 + t; i < rows; i += kQT) col[i] *= scal;
            if (t == 0) {
                col[j] = beta;
                a.tau[j] = tau;
                a.vn1[pc] = -1.0;  // used
            }
        }
        if (!grid_sync(a.bar, ++epoch * (unsigned)nwg, a.abort_flag)) return;
        const double tauj = a.tau[j];
        const double *v = a.W + (int64_t)pc * a.ldw;
        for (int64_t c = wg; c < a.ncols; c += nwg) {
            // used columns are skipped (vn1 < 0, written before the last
            // grid barrier: the same value in every thread)
            if (!(a.vn1[c] >= 0.0)) continue;
            double *col = a.W + c * a.ldw;
            if (tauj != 0.0) {
                double s = (t == 0) ? col[j] : 0.0;
                for (int64_t i = j + 1 + t; i < rows; i += kQT) s = fma(v[i], col[i], s);
                const double z = tauj * wg_total(s, sh);
                if (t == 0) col[j] -= z;
                for (int64_t i = j + 1 + t; i < rows; i += kQT) col[i] = fma(-z, v[i], col[i]);
            }
            __syncthreads();
            // partial norm of rows j+1 .. : downdate, or recompute when the
            // downdate has cancelled most of it
            const double n1 = a.vn1[c], n2 = a.vn2[c];
            __syncthreads();  // every thread has read them before thread 0 writes
            bool recompute = false;
            double nn1 = n1;
            if (n1 != 0.0) {
                const double q = fabs(col[j]) / n1;
                const double tmp = fmax(0.0, (1.0 - q) * (1.0 + q));
                const double r = n1 / n2;
                if (tmp * r * r <= 1.4901161193847656e-08)  // sqrt(2^-52)
                    recompute = true;
                else
                    nn1 = n1 * sqrt(tmp);
            }
            if (recompute) {
                double s = 0.0;
                for (int64_t i = j + 1 + t; i < rows; i += kQT) s = fma(col[i], col[i], s);
                nn1 = sqrt(wg_total(s, sh));
            }
            if (t == 0) {
                a.vn1[c] = nn1;
                if (recompute) a.vn2[c] = nn1;
            }
            __syncthreads();
        }
    }
    if (wg == 0 && t == 0) {
        // positions k .. ncols-1: the free columns, in increasing order
        int pos = k;
        for (int64_t c = 0; c < a.ncols; ++c)
            if (a.vn1[c] >= 0.0) a.jpvt[pos++] = (int)c;
        *a.rank = k;
    }
}

// X (ncols x k, ld ldx) = the transpose of the first k rows of W's upper
// trapezoid (zero below the diagonal): X(j, i) = (i <= j) ? W(i, j) : 0.
__global__ void trap_transpose_kernel(const double *W, int64_t ldw, int64_t k, int64_t ncols,
                                      double *X, int64_t ldx) {
    const int64_t i = blockIdx.y;  // column of X = row of W
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < ncols;
         j += (int64_t)gridDim.x * blockDim.x)
        X[j + i * ldx] = (i <= j) ? W[i + j * ldw] : 0.0;
}

// out[j] = a[b[j]]
__global__ void compose_kernel(const int *a, const int *b, int64_t n, int *out) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        out[j] = a[b[j]];
}

__global__ void fill_kernel(double *x, int64_t n, double v) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        x[j] = v;
}

// B (rows x cols, ld ldb) = v
__global__ void fill2d_kernel(double *B, int64_t ldb, int64_t rows, double v) {
    const int64_t c = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x)
        B[i + c * ldb] = v;
}

// the strictly lower triangle of the n x n W (ld ldw) := 0
__global__ void zero_lower_kernel(double *W, int64_t ldw, int64_t n) {
    const int64_t c = blockIdx.y;
    for (int64_t i = c + 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        W[i + c * ldw] = 0.0;
}

__global__ void qr_reset_kernel(unsigned *bar, int *abort_flag) {
    if (threadIdx.x == 0) {
        if (bar) *bar = 0u;
        if (abort_flag) *abort_flag = 0;
    }
}

}  // namespace

int qrcp_resident(int cu_count) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(&qrcp_kernel), kQT, 0) != hipSuccess)
        return 0;
    return per_cu * cu_count;
}

// The abort flag is reset with the barrier; a barrier that cannot complete
// (some of the nwg workgroups could not start beside other work on the
// device) sets it after its spin bound and every workgroup leaves.
hipError_t launch_qrcp(const QrcpArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(qr_reset_kernel, dim3(1), dim3(64), 0, s, a.bar, a.abort_flag);
    hipLaunchKernelGGL(qrcp_kernel, dim3((unsigned)a.nwg), dim3(kQT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_trap_transpose(const double *W, int64_t ldw, int64_t k, int64_t ncols, double *X,
                                 int64_t ldx, hipStream_t s) {
    if (k <= 0) return hipSuccess;
    const int64_t bx = std::max<int64_t>(1, std::min<int64_t>((ncols + 255) / 256, 16));
    hipLaunchKernelGGL(trap_transpose_kernel, dim3((unsigned)bx, (unsigned)k), dim3(256), 0, s, W,
                       ldw, k, ncols, X, ldx);
    return hipGetLastError();
}

hipError_t launch_compose(const int *a, const int *b, int64_t n, int *out, hipStream_t s) {
    hipLaunchKernelGGL(compose_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 64)),
                       dim3(256), 0, s, a, b, n, out);
    return hipGetLastError();
}

hipError_t launch_fill2d(double *B, int64_t ldb, int64_t rows, int64_t cols, double v,
                         hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const int64_t bx = std::max<int64_t>(1, std::min<int64_t>((rows + 255) / 256, 16));
    hipLaunchKernelGGL(fill2d_kernel, dim3((unsigned)bx, (unsigned)cols), dim3(256), 0, s, B, ldb,
                       rows, v);
    return hipGetLastError();
}

hipError_t launch_zero_lower(double *W, int64_t ldw, int64_t n, hipStream_t s) {
    const int64_t bx = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16));
    hipLaunchKernelGGL(zero_lower_kernel, dim3((unsigned)bx, (unsigned)n), dim3(256), 0, s, W, ldw,
                       n);
    return hipGetLastError();
}

hipError_t launch_fill(double *x, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 64)),
                       dim3(256), 0, s, x, n, v);
    return hipGetLastError();
}

int qr_panel_groups(int64_t rows) {
    const int64_t per = (int64_t)kQT * kRpt;
    return (int)((rows + per - 1) / per);
}

int qr_panel_resident(int cu_count) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(&qr_panel_kernel), kQT, 0) != hipSuccess)
        return 0;
    return per_cu * cu_count;
}

hipError_t launch_diag_range(const double *W, int64_t ldw, int64_t n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(diag_range_kernel, dim3(1), dim3(256), 0, s, W, ldw, n, out);
    return hipGetLastError();
}

hipError_t launch_qr_reset(unsigned *bar, int *abort_flag, hipStream_t s) {
    hipLaunchKernelGGL(qr_reset_kernel, dim3(1), dim3(64), 0, s, bar, abort_flag);
    return hipGetLastError();
}

// The abort flag is left as it is: once a barrier has failed, the later
// panels fall through at their first barrier and the caller falls back to
// the direct method.  An ordinary launch in stream order: the caller checks
// that the nwg <= 64 workgroups of 68 kB LDS can all be resident
// (qr_panel_resident); work of other streams or processes on the device can
// still keep some from starting, and then a barrier ends at its spin bound
// (2^24 polls of the counter) instead of hanging.
hipError_t launch_qr_panel(const QrPanelArgs &a, hipStream_t s) {
    // the kernel gathers at most 64 workgroups' partial sums per column
    // (m <= 32768 on every path that factors a panel)
    if (a.nwg < 1 || a.nwg > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(qr_reset_kernel, dim3(1), dim3(64), 0, s, a.bar, (int *)nullptr);
    hipLaunchKernelGGL(qr_panel_kernel, dim3((unsigned)a.nwg), dim3(kQT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_qr_t(const double *Y, const double *tau, int nb, double *T, hipStream_t s) {
    hipLaunchKernelGGL(qr_t_kernel, dim3(1), dim3(64), 0, s, Y, tau, nb, T);
    return hipGetLastError();
}

hipError_t launch_sum_parts(const double *parts, int np, int64_t count, double *out,
                            hipStream_t s) {
    hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)((count + 31) / 32)), dim3(256), 0, s,
                       parts, np, count, out);
    return hipGetLastError();
}

hipError_t launch_r_transpose(const double *W, int64_t ldw, int64_t n, double *X, int64_t ldx,
                              hipStream_t s, const double *colscale) {
    const int64_t bx = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16));
    hipLaunchKernelGGL(r_transpose_kernel, dim3((unsigned)bx, (unsigned)n), dim3(256), 0, s, W,
                       ldw, n, X, ldx, colscale);
    return hipGetLastError();
}

hipError_t launch_pow2(const int *ex, int64_t n, double *out, hipStream_t s) {
    const int64_t bx = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024));
    hipLaunchKernelGGL(pow2_kernel, dim3((unsigned)bx), dim3(256), 0, s, ex, n, out);
    return hipGetLastError();
}

hipError_t launch_qr_extract_v(const double *W, int64_t ldw, int64_t m, int64_t j, int nb,
                               double *Vp, int64_t ldvp, hipStream_t s) {
    const int64_t bx = std::max<int64_t>(1, std::min<int64_t>((m - j + 255) / 256, 64));
    hipLaunchKernelGGL(qr_extract_v_kernel, dim3((unsigned)bx, (unsigned)kNb), dim3(256), 0, s,
                       W, ldw, m, j, nb, Vp, ldvp);
    return hipGetLastError();
}

hipError_t launch_embed(const double *X, int64_t ldx, int64_t n, double *B, int64_t ldb,
                        int64_t rows, int64_t cols, hipStream_t s) {
    const int64_t bx = std::max<int64_t>(1, std::min<int64_t>((rows + 255) / 256, 64));
    hipLaunchKernelGGL(embed_kernel, dim3((unsigned)bx, (unsigned)cols), dim3(256), 0, s, X, ldx,
                       n, B, ldb, rows);
    return hipGetLastError();
}

}  // namespace jsvd

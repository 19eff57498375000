// Many independent small SVDs of uneven sizes in one persistent launch.
//
// The method is the same one-sided Jacobi as the dense path (Section 2,
// eqs. (2.3)-(2.5); rotations (4.1), (4.3)-(4.6)), applied pointwise: a
// problem with n <= a few hundred columns is orthogonalised pair of columns
// by pair of columns, in the p-steps of the closest parallel strategy of
// order n (rounded up to a supported order; pairs with a padding index are
// skipped), sweep after sweep until a sweep performs no proper rotation
// (cs != 1; the stopping heuristic of Section 4.5: a sweep whose rotations
// are all numerically the identity up to the tangent term ends the
// iteration, those rotations having been applied).
//
// Work distribution: a persistent grid of workgroups pulls problem indices
// from a device queue, largest n first (the order comes from a counting
// sort on the device).  A workgroup (16 waves) owns its problem: every half
// wave takes one pivot pair of the current p-step, lane x owning rows x,
// x + 32, ... of the pair's columns (kept in registers between the dot
// products and the update); the three dot products are half-wave sums.  G
// is worked on in LDS when it fits (one workgroup per CU, up to ~150 kB),
// else in its global buffer; V is updated in global memory.  A workgroup
// barrier separates p-steps.  At the end of a problem the column
// norms give sigma, the workgroup ranks them (non-increasing, ties by
// index) and gathers U = G Sigma^{-1} and V in that order through a
// per-workgroup scratch area.
#include "jsvd_internal.h"

namespace jsvd {

namespace {

constexpr double kEpsB = 1.1102230246251565e-16;      // 2^-53
constexpr double kSqrtEpsB = 1.0536712127723509e-08;  // sqrt(2^-53)
constexpr double kSqrt2OverEpsB = 134217728.0;        // 2^27

__device__ __forceinline__ double hw_sum(double v) {
    v += __builtin_amdgcn_update_dpp(0.0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x140, 0xF, 0xF, false);  // row_mirror
    const long long x = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_ds_swizzle((int)x, 0x401F);         // lane ^ 16
    const int hi = __builtin_amdgcn_ds_swizzle((int)(x >> 32), 0x401F);
    return v + __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Trigonometric rotation parameters, eqs. (4.3)-(4.6) with t = +1, cs_2.
__device__ __forceinline__ void trig_rotation(double hpp, double hqq, double hpq, double &tn,
                                              double &cs) {
    const double ct2 = (hqq - hpp) / (2.0 * hpq);
    const double sgn = ct2 < 0.0 ? -1.0 : 1.0;
    const double a = fabs(ct2);
    double act;
    if (a < kSqrtEpsB)
        act = a + 1.0;
    else if (a >= kSqrt2OverEpsB)
        act = 2.0 * a;
    else
        act = a + sqrt(fma(a, a, 1.0));
    tn = sgn * (1.0 / act);
    cs = (act >= kSqrt2OverEpsB) ? 1.0 : act / sqrt(fma(act, act, 1.0));
}

constexpr int kBatchThreads = 1024;  // 16 waves, 32 half-wave pair groups
constexpr int kGroups = kBatchThreads / 32;

// One sweep-loop of the pointwise method on a problem whose working copy of
// G is Gw (LDS or global; column-major, ld = m) and whose V is in global
// memory.  R > 0: every lane keeps its R rows of the pair's columns in
// registers between the dot products and the update (m <= 32 R); R = 0:
// any m, two passes over the columns.  Returns the sweeps performed; sets
// *converged when a sweep performed no proper rotation.
template <int R>
__device__ int pointwise_sweeps(double *Gw, double *V, int m, int n, int N,
                                const unsigned char *tbl, int max_sweeps, double tol,
                                int *s_rot, bool *converged) {
    const int tid = threadIdx.x, x = tid & 31, group = tid >> 5;
    const int half = N >> 1;
    int sweeps = 0;
    *converged = false;
    while (sweeps < max_sweeps) {
        if (tid == 0) *s_rot = 0;
        int rot = 0;  // this half wave's proper rotations in the sweep
        for (int st = 0; st < N - 1; ++st) {
            const unsigned char *ps = tbl + (size_t)st * N;
            for (int slot = group; slot < half; slot += kGroups) {
                const int p = ps[2 * slot], q = ps[2 * slot + 1];
                if (q >= n) continue;  // padding index: uniform in the half wave
                double *gp = Gw + (size_t)p * m, *gq = Gw + (size_t)q * m;
                double *vp = V ? V + (size_t)p * n : nullptr, *vq = V ? V + (size_t)q * n : nullptr;
                double hpp = 0.0, hqq = 0.0, hpq = 0.0;
                if constexpr (R > 0) {
                    double a[R], b[R], c[R], d[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int i = x + 32 * r;
                        a[r] = i < m ? gp[i] : 0.0;
                        b[r] = i < m ? gq[i] : 0.0;
                        c[r] = (V && i < n) ? vp[i] : 0.0;
                        d[r] = (V && i < n) ? vq[i] : 0.0;
                    }
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        hpp = fma(a[r], a[r], hpp);
                        hqq = fma(b[r], b[r], hqq);
                        hpq = fma(a[r], b[r], hpq);
                    }
                    hpp = hw_sum(hpp);
                    hqq = hw_sum(hqq);
                    hpq = hw_sum(hpq);
                    if (fabs(hpq) <= tol * sqrt(hpp) * sqrt(hqq)) continue;  // subphase 2
                    double tn, cs;
                    trig_rotation(hpp, hqq, hpq, tn, cs);
                    rot += cs != 1.0 ? 1 : 0;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int i = x + 32 * r;
                        const double np_ = cs == 1.0 ? fma(-tn, b[r], a[r]) : cs * fma(-tn, b[r], a[r]);
                        const double nq_ = cs == 1.0 ? fma(tn, a[r], b[r]) : cs * fma(tn, a[r], b[r]);
                        if (i < m) {
                            gp[i] = np_;
                            gq[i] = nq_;
                        }
                        if (V && i < n) {
                            vp[i] = cs == 1.0 ? fma(-tn, d[r], c[r]) : cs * fma(-tn, d[r], c[r]);
                            vq[i] = cs == 1.0 ? fma(tn, c[r], d[r]) : cs * fma(tn, c[r], d[r]);
                        }
                    }
                } else {
                    for (int i = x; i < m; i += 32) {
                        const double a0 = gp[i], b0 = gq[i];
                        hpp = fma(a0, a0, hpp);
                        hqq = fma(b0, b0, hqq);
                        hpq = fma(a0, b0, hpq);
                    }
                    hpp = hw_sum(hpp);
                    hqq = hw_sum(hqq);
                    hpq = hw_sum(hpq);
                    if (fabs(hpq) <= tol * sqrt(hpp) * sqrt(hqq)) continue;  // subphase 2
                    double tn, cs;
                    trig_rotation(hpp, hqq, hpq, tn, cs);
                    rot += cs != 1.0 ? 1 : 0;
                    for (int i = x; i < m; i += 32) {
                        const double a0 = gp[i], b0 = gq[i];
                        gp[i] = cs == 1.0 ? fma(-tn, b0, a0) : cs * fma(-tn, b0, a0);
                        gq[i] = cs == 1.0 ? fma(tn, a0, b0) : cs * fma(tn, a0, b0);
                    }
                    if (V)
                        for (int i = x; i < n; i += 32) {
                            const double a0 = vp[i], b0 = vq[i];
                            vp[i] = cs == 1.0 ? fma(-tn, b0, a0) : cs * fma(-tn, b0, a0);
                            vq[i] = cs == 1.0 ? fma(tn, a0, b0) : cs * fma(tn, a0, b0);
                        }
                }
            }
            __syncthreads();
        }
        if (x == 0 && rot) atomicAdd(s_rot, rot);
        __syncthreads();
        const int all = *s_rot;
        ++sweeps;
        __syncthreads();
        if (all == 0) {
            *converged = true;
            break;
        }
    }
    return sweeps;
}

__global__ __launch_bounds__(kBatchThreads) void batched_kernel(BatchArgs b) {
    extern __shared__ double lds_g[];  // working copy of G when it fits
    __shared__ int s_item;
    __shared__ int s_rot;
    __shared__ double s_sig[kBatchMaxN];
    __shared__ int s_perm[kBatchMaxN];
    const int tid = threadIdx.x, x = tid & 31;
    const int group = tid >> 5;  // half wave
    double *scratch = b.scratch + (size_t)blockIdx.x * b.scratch_per_wg;

    for (;;) {
        if (tid == 0) s_item = atomicAdd(b.queue, 1);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= b.count) break;  // every workgroup leaves once the queue is drained
        const int id = b.order[item];
        const int m = b.m[id], n = b.n[id];
        double *G = b.A + b.a_off[id];
        double *V = b.V ? b.V + b.v_off[id] : nullptr;
        const int N = b.tbl_order[n];
        const unsigned char *tbl = b.tbls + b.tbl_off[N >> 1];
        const double tol = kEpsB * sqrt((double)m);  // c(eps) = eps sqrt(m)
        const bool in_lds = (int64_t)m * n <= b.lds_doubles;
        double *Gw = in_lds ? lds_g : G;

        if (in_lds)
            for (int e = tid; e < m * n; e += kBatchThreads) lds_g[e] = G[e];
        if (V)
            for (int e = tid; e < n * n; e += kBatchThreads) V[e] = (e % n == e / n) ? 1.0 : 0.0;
        __syncthreads();

        bool converged = false;
        int sweeps;
        if (m <= 32)
            sweeps = pointwise_sweeps<1>(Gw, V, m, n, N, tbl, b.max_sweeps, tol, &s_rot, &converged);
        else if (m <= 64)
            sweeps = pointwise_sweeps<2>(Gw, V, m, n, N, tbl, b.max_sweeps, tol, &s_rot, &converged);
        else if (m <= 128)
            sweeps = pointwise_sweeps<4>(Gw, V, m, n, N, tbl, b.max_sweeps, tol, &s_rot, &converged);
        else if (m <= 192)
            sweeps = pointwise_sweeps<6>(Gw, V, m, n, N, tbl, b.max_sweeps, tol, &s_rot, &converged);
        else
            sweeps = pointwise_sweeps<0>(Gw, V, m, n, N, tbl, b.max_sweeps, tol, &s_rot, &converged);

        // sigma_j = ||g_j||, output order, U = G Sigma^{-1}, V permuted
        for (int j = group; j < n; j += kGroups) {
            const double *g = Gw + (size_t)j * m;
            double sacc = 0.0;
            for (int i = x; i < m; i += 32) sacc = fma(g[i], g[i], sacc);
            sacc = hw_sum(sacc);
            if (x == 0) s_sig[j] = sqrt(sacc);
        }
        __syncthreads();
        for (int j = tid; j < n; j += kBatchThreads) {
            const double kj = s_sig[j] != s_sig[j] ? -INFINITY : s_sig[j];
            int r = 0;
            for (int i = 0; i < n; ++i) {
                const double ki = s_sig[i] != s_sig[i] ? -INFINITY : s_sig[i];
                r += (ki > kj || (ki == kj && i < j)) ? 1 : 0;
            }
            s_perm[r] = j;
        }
        const double *src = Gw;
        if (!in_lds) {
            for (int e = tid; e < m * n; e += kBatchThreads) scratch[e] = G[e];
            src = scratch;
        }
        if (V)
            for (int e = tid; e < n * n; e += kBatchThreads) scratch[(size_t)m * n + e] = V[e];
        __syncthreads();
        double *S = b.S + b.s_off[id];
        for (int e = tid; e < m * n; e += kBatchThreads) {
            const int k = e / m, i = e % m, c = s_perm[k];
            const double sg = s_sig[c];
            G[e] = sg > 0.0 ? src[(size_t)c * m + i] / sg : 0.0;
        }
        if (V)
            for (int e = tid; e < n * n; e += kBatchThreads) {
                const int k = e / n, i = e % n;
                V[e] = scratch[(size_t)m * n + (size_t)s_perm[k] * n + i];
            }
        for (int k = tid; k < n; k += kBatchThreads) S[k] = s_sig[s_perm[k]];
        if (tid == 0) {
            if (b.status) b.status[id] = converged ? 0 : JSVD_NOT_CONVERGED;
            if (b.sweeps) b.sweeps[id] = sweeps;
        }
        __syncthreads();
    }
}

// Work order: problem indices by non-increasing n (counting sort).
__global__ void batch_count_kernel(const int32_t *n, int64_t count, int *hist) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) atomicAdd(&hist[n[i]], 1);
}

__global__ void batch_scan_kernel(int *hist, int max_n, int *queue) {
    // one thread: bucket start positions, largest n first
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int pos = 0;
        for (int v = max_n; v >= 0; --v) {
            const int c = hist[v];
            hist[v] = pos;
            pos += c;
        }
        *queue = 0;
    }
}

__global__ void batch_place_kernel(const int32_t *n, int64_t count, int *hist, int32_t *order) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) order[atomicAdd(&hist[n[i]], 1)] = (int32_t)i;
}

__global__ void batch_zero_kernel(int *p, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0;
}

}  // namespace

hipError_t batched_set_lds(int bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&batched_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t launch_batched(const BatchArgs &b, int grid, int max_n, int *hist, int32_t *order,
                          hipStream_t s) {
    hipLaunchKernelGGL(batch_zero_kernel, dim3(1), dim3(256), 0, s, hist, max_n + 1);
    const unsigned blocks = (unsigned)((b.count + 255) / 256);
    hipLaunchKernelGGL(batch_count_kernel, dim3(blocks), dim3(256), 0, s, b.n, b.count, hist);
    hipLaunchKernelGGL(batch_scan_kernel, dim3(1), dim3(64), 0, s, hist, max_n, b.queue);
    hipLaunchKernelGGL(batch_place_kernel, dim3(blocks), dim3(256), 0, s, b.n, b.count, hist,
                       order);
    hipLaunchKernelGGL(batched_kernel, dim3(grid), dim3(kBatchThreads),
                       (unsigned)(b.lds_doubles * sizeof(double)), s, b);
    return hipGetLastError();
}

}  // namespace jsvd

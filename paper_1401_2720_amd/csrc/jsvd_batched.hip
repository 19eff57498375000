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
// sort on the device).  A workgroup (16 waves) owns its problem.  With V
// wanted, the first g_groups half waves (16 unless tuned) rotate G and the
// others apply the previous p-step's rotations to V (published in LDS), so V
// is off the path of the rotations; without V all 32 half waves rotate G.  A half wave takes one
// pivot pair at a time, lane x owning rows x, x + 32, ... of the pair's
// columns (kept in registers between the dot products and the update); the
// three dot products are half-wave sums.  G is worked on in LDS when it fits
// (one workgroup per CU, ~148 kB), V too when there is room left, else in
// their global buffers.  A workgroup barrier separates p-steps.  At the end
// of a problem the column norms give sigma, the workgroup ranks them
// (non-increasing, ties by index) and gathers U = G Sigma^{-1} and V in that
// order (what is in global memory is permuted in place through LDS).
//
// Badly scaled problems (opts.scaled = 2): every pair is a DDRJAC pair
// (Section 4.3.1): the column norms by DRDSSQ (Appendix A), the cosine of
// the pair's angle from the columns scaled by the powers of two of their
// norms, and ct 2phi from the norm ratio, so that no square or sum leaves
// the normal range; sigma and U at the end come from DRDSSQ too.  Such
// problems all take the pointwise kernel, and stop at a sweep with no
// rotation (the pointwise rule of Section 4.5).
#include "jsvd_rdssq.h"

namespace jsvd {

namespace {

constexpr int kBatchThreads = 1024;  // 16 waves, 32 half-wave pair groups
constexpr int kGroups = kBatchThreads / 32;

// One sweep-loop of the pointwise method on a problem whose working copy of
// G is Gw and of V is Vw (each in LDS or global memory, column-major, ld = m
// and n; Vw may be null).  R > 0: every lane keeps its R rows of the pair's
// columns in registers between the dot products and the update (m <= 32 R),
// and a half wave takes K of its pivot pairs at once, so that their
// dependent chains (sums, square roots, divisions) overlap; R = 0: any m,
// one pair at a time, two passes over the columns.  Rotations go from the G
// half waves to the V half waves through (tn, cs) slots in LDS,
// double-buffered by p-step; cs = 0 marks a pair that did not rotate.
// Returns the sweeps performed; sets *converged when a sweep performed no
// proper rotation.
// DD: DDRJAC pairs (t_hi: the DRDSSQ bound for columns of length m; a NaN
// or infinite column sets *s_bad), and the stopping rule of the pointwise
// method (Section 4.5): a sweep with no rotation at all.  Between columns
// whose norms differ by many orders of magnitude a rotation with cs = 1
// still moves the smaller column by tan phi times the larger one, so the
// relaxed rule (no proper rotation) would stop too early on graded input.
template <int R, int K, bool DD>
__device__ int pointwise_sweeps(double *Gw, double *Vw, int m, int n, int N,
                                const unsigned char *tbl, int max_sweeps, double tol, int g_groups,
                                int *s_rot, double (*s_tn)[kBatchMaxN / 2],
                                double (*s_cs)[kBatchMaxN / 2], bool *converged, double t_hi,
                                int *s_bad) {
    static_assert(!DD || K == 1, "DDRJAC pairs one at a time");
    const int tid = threadIdx.x, x = tid & 31, group = tid >> 5;
    const int half = N >> 1;
    const int ng = Vw ? g_groups : kGroups;      // half waves on G
    const bool on_g = group < ng;
    const int gi = on_g ? group : group - ng;
    const int gstride = on_g ? ng : kGroups - ng;
    const int nsteps = N - 1 + (Vw ? 1 : 0);    // V trails G by one p-step
    int sweeps = 0;
    *converged = false;
    while (sweeps < max_sweeps) {
        if (tid == 0) *s_rot = 0;
        int rot = 0;  // this half wave's proper rotations in the sweep
        for (int st = 0; st < nsteps; ++st) {
            if (on_g && st < N - 1) {
                const unsigned char *ps = tbl + (size_t)st * N;
                if constexpr (R > 0) {
                    for (int s0 = gi; s0 < half; s0 += K * gstride) {
                        int pk[K], qk[K];
                        bool use[K];
                        double a[K][R], b[K][R], hpp[K], hqq[K], hpq[K];
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            const int slot = s0 + k * gstride;
                            pk[k] = slot < half ? ps[2 * slot] : 0;
                            qk[k] = slot < half ? ps[2 * slot + 1] : n;
                            use[k] = qk[k] < n;  // padding index or no slot: uniform in the half wave
#pragma unroll
                            for (int r = 0; r < R; ++r) {
                                const int i = x + 32 * r;
                                a[k][r] = (use[k] && i < m) ? Gw[(size_t)pk[k] * m + i] : 0.0;
                                b[k][r] = (use[k] && i < m) ? Gw[(size_t)qk[k] * m + i] : 0.0;
                            }
                        }
                        double tn[K], cs[K];
                        bool rk[K];
                        if constexpr (DD) {
                            int ja, jb;
                            double sa, sb;
                            hw_rdssq<R>(a[0], t_hi, ja, sa);
                            hw_rdssq<R>(b[0], t_hi, jb, sb);
                            double d = 0.0;
#pragma unroll
                            for (int r = 0; r < R; ++r)
                                d = fma(ldexp(a[0][r], -ja / 2), ldexp(b[0][r], -jb / 2), d);
                            d = hw_sum(d);
                            bool clamped;
                            tn[0] = 0.0;
                            cs[0] = 0.0;
                            rk[0] = use[0] && ddrjac_pair(ja, sa, jb, sb, d, tol, 1, tn[0], cs[0],
                                                          clamped);
                            if (!rk[0]) cs[0] = 0.0;
                            if (use[0] && x == 0 && !(sa == sa && sb == sb)) *s_bad = 1;
                        } else {
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            hpp[k] = hqq[k] = hpq[k] = 0.0;
#pragma unroll
                            for (int r = 0; r < R; ++r) {
                                hpp[k] = fma(a[k][r], a[k][r], hpp[k]);
                                hqq[k] = fma(b[k][r], b[k][r], hqq[k]);
                                hpq[k] = fma(a[k][r], b[k][r], hpq[k]);
                            }
                        }
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            hpp[k] = hw_sum(hpp[k]);
                            hqq[k] = hw_sum(hqq[k]);
                            hpq[k] = hw_sum(hpq[k]);
                        }
                        // subphases 2-5, branch-free while every operand lies in
                        // the range of the refined arithmetic (the usual case)
                        bool fast = true;
#pragma unroll
                        for (int k = 0; k < K; ++k)
                            fast = fast && (!use[k] || (in_fast_range(hpp[k]) && in_fast_range(hqq[k]) &&
                                                        (hpq[k] == 0.0 || in_fast_range(fabs(hpq[k])))));
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            if (K == 1) {  // one pair: skip the rotation when the test says so
                                tn[k] = 0.0;
                                cs[k] = 0.0;
                                rk[k] = use[k] && trig_pair(hpp[k], hqq[k], hpq[k], tol, tn[k], cs[k]);
                            } else if (fast) {
                                bool clamped;
                                rk[k] = use[k] && hpq[k] != 0.0 &&
                                        !(fabs(hpq[k]) <= tol * nsqrt(hpp[k]) * nsqrt(hqq[k]));
                                rotation_fast(hpp[k], hqq[k], hpq[k] != 0.0 ? hpq[k] : 1.0, 1, tn[k],
                                              cs[k], clamped);
                            } else {
                                tn[k] = 0.0;
                                cs[k] = 0.0;
                                rk[k] = use[k] && trig_pair(hpp[k], hqq[k], hpq[k], tol, tn[k], cs[k]);
                            }
                            if (!rk[k]) cs[k] = 0.0;
                        }
                        }  // DD
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            if (rk[k]) {
                                rot += (DD || cs[k] != 1.0) ? 1 : 0;
                                // (4.1); cs == 1 multiplies exactly
#pragma unroll
                                for (int r = 0; r < R; ++r) {
                                    const int i = x + 32 * r;
                                    const double np_ = cs[k] * fma(-tn[k], b[k][r], a[k][r]);
                                    const double nq_ = cs[k] * fma(tn[k], a[k][r], b[k][r]);
                                    if (i < m) {
                                        Gw[(size_t)pk[k] * m + i] = np_;
                                        Gw[(size_t)qk[k] * m + i] = nq_;
                                    }
                                }
                            }
                            if (Vw && x == 0 && use[k]) {
                                const int slot = s0 + k * gstride;
                                s_tn[st & 1][slot] = tn[k];
                                s_cs[st & 1][slot] = cs[k];
                            }
                        }
                    }
                } else {
                    for (int slot = gi; slot < half; slot += gstride) {
                        const int p = ps[2 * slot], q = ps[2 * slot + 1];
                        if (q >= n) continue;  // padding index: uniform in the half wave
                        double *gp = Gw + (size_t)p * m, *gq = Gw + (size_t)q * m;
                        double tn = 0.0, cs = 0.0;
                        bool rot_pair;
                        if constexpr (DD) {
                            int ja, jb;
                            double sa, sb;
                            hw_rdssq_mem(gp, m, t_hi, ja, sa);
                            hw_rdssq_mem(gq, m, t_hi, jb, sb);
                            double d = 0.0;
                            for (int i = x; i < m; i += 32)
                                d = fma(ldexp(gp[i], -ja / 2), ldexp(gq[i], -jb / 2), d);
                            d = hw_sum(d);
                            bool clamped;
                            rot_pair = ddrjac_pair(ja, sa, jb, sb, d, tol, 1, tn, cs, clamped);
                            if (x == 0 && !(sa == sa && sb == sb)) *s_bad = 1;
                        } else {
                            double hpp = 0.0, hqq = 0.0, hpq = 0.0;
                            for (int i = x; i < m; i += 32) {
                                const double a0 = gp[i], b0 = gq[i];
                                hpp = fma(a0, a0, hpp);
                                hqq = fma(b0, b0, hqq);
                                hpq = fma(a0, b0, hpq);
                            }
                            hpp = hw_sum(hpp);
                            hqq = hw_sum(hqq);
                            hpq = hw_sum(hpq);
                            rot_pair = trig_pair(hpp, hqq, hpq, tol, tn, cs);
                        }
                        if (rot_pair) {
                            rot += (DD || cs != 1.0) ? 1 : 0;
                            for (int i = x; i < m; i += 32) {
                                const double a0 = gp[i], b0 = gq[i];
                                gp[i] = cs * fma(-tn, b0, a0);
                                gq[i] = cs * fma(tn, a0, b0);
                            }
                        } else {
                            cs = 0.0;
                        }
                        if (Vw && x == 0) {
                            s_tn[st & 1][slot] = tn;
                            s_cs[st & 1][slot] = cs;
                        }
                    }
                }
            } else if (!on_g && st >= 1) {
                const int s1 = st - 1;
                const unsigned char *ps = tbl + (size_t)s1 * N;
                for (int slot = gi; slot < half; slot += gstride) {
                    const int p = ps[2 * slot], q = ps[2 * slot + 1];
                    if (q >= n) continue;
                    const double cs = s_cs[s1 & 1][slot];
                    if (cs == 0.0) continue;
                    const double tn = s_tn[s1 & 1][slot];
                    double *vp = Vw + (size_t)p * n, *vq = Vw + (size_t)q * n;
                    for (int i = x; i < n; i += 32) {
                        const double a0 = vp[i], b0 = vq[i];
                        vp[i] = cs * fma(-tn, b0, a0);
                        vq[i] = cs * fma(tn, a0, b0);
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


// The end of a problem: sigma_j = ||g_j||, the output order (non-increasing,
// ties by index, NaN last), U = G Sigma^{-1} and V in that order, status
// and sweeps.  Gw / Vw are the working copies (LDS or the global buffers;
// in_lds / v_lds say which), G / V the global buffers.  A working copy in
// global memory is permuted in place through LDS (lds, lds_cap doubles,
// free at this point except for LDS working copies), a band of rows of all
// columns at a time.
template <int NT>
__device__ __forceinline__ void permute_columns(double *X, int rows, int n, const int *perm,
                                                const double *sig, const int *ex,
                                                double *lds, int64_t lds_cap) {
    const int tid = threadIdx.x;
    const int band = (int)min<int64_t>(rows, lds_cap / n);
    for (int i0 = 0; i0 < rows; i0 += band) {
        const int nr = min(band, rows - i0);
        for (int e = tid; e < nr * n; e += NT) {
            const int k = e / nr, i = e % nr;
            lds[e] = X[(size_t)k * rows + i0 + i];
        }
        __syncthreads();
        for (int e = tid; e < nr * n; e += NT) {
            const int k = e / nr, i = e % nr, c = perm[k];
            const double v = lds[(size_t)c * nr + i];
            if (sig && ex) {  // DRDSSQ pairs: sig holds sqrt(s), ex the j of 2^j s
                const double sg = sig[c];
                X[(size_t)k * rows + i0 + i] = sg > 0.0 ? ldexp(v, -ex[c] / 2) / sg : 0.0;
            } else if (sig) {
                const double sg = sig[c];
                X[(size_t)k * rows + i0 + i] = sg > 0.0 ? v / sg : 0.0;
            } else {
                X[(size_t)k * rows + i0 + i] = v;
            }
        }
        __syncthreads();
    }
}

//
// With DRDSSQ pairs (s_ex non-null, t_hi the bound for length m): the pair
// (j, s) of each column gives sigma = 2^(j/2) sqrt(s) (infinite if it
// overflows), the order compares the pairs (j, sqrt(s)) lexicographically
// (a zero column last but NaN), and u = (2^(-j/2) g) / sqrt(s); s_rt
// receives sqrt(s).
template <int NT>
__device__ __forceinline__ void finish_problem(const BatchArgs &b, int id, int m, int n, double *G,
                                               double *V, const double *Gw, const double *Vw,
                                               bool in_lds, bool v_lds, double *lds,
                                               int64_t lds_cap, int sweeps, int status,
                                               double *s_sig, int *s_perm, int *s_ex = nullptr,
                                               double *s_rt = nullptr, double t_hi = 0.0) {
    const int tid = threadIdx.x, x = tid & 31, group = tid >> 5;
    for (int j = group; j < n; j += NT / 32) {
        const double *g = Gw + (size_t)j * m;
        if (s_ex) {
            int e;
            double sq;
            hw_rdssq_mem(g, m, t_hi, e, sq);
            if (x == 0) {
                s_ex[j] = sq > 0.0 ? e : -0x7fffffff;
                s_rt[j] = sqrt(sq);
                s_sig[j] = rdssq_norm(e, sq);
            }
        } else {
            double sacc = 0.0;
            for (int i = x; i < m; i += 32) sacc = fma(g[i], g[i], sacc);
            sacc = hw_sum(sacc);
            if (x == 0) s_sig[j] = sqrt(sacc);
        }
    }
    __syncthreads();
    for (int j = tid; j < n; j += NT) {
        int r = 0;
        if (s_ex) {
            const bool nj = s_rt[j] != s_rt[j];
            for (int i = 0; i < n; ++i) {
                const bool ni = s_rt[i] != s_rt[i];
                const bool gt = ni || nj ? (!ni && nj)
                                         : (s_ex[i] > s_ex[j] ||
                                            (s_ex[i] == s_ex[j] && s_rt[i] > s_rt[j]));
                const bool eq = ni || nj ? (ni && nj)
                                         : (s_ex[i] == s_ex[j] && s_rt[i] == s_rt[j]);
                r += (gt || (eq && i < j)) ? 1 : 0;
            }
        } else {
            const double kj = s_sig[j] != s_sig[j] ? -INFINITY : s_sig[j];
            for (int i = 0; i < n; ++i) {
                const double ki = s_sig[i] != s_sig[i] ? -INFINITY : s_sig[i];
                r += (ki > kj || (ki == kj && i < j)) ? 1 : 0;
            }
        }
        s_perm[r] = j;
    }
    __syncthreads();
    // working copies in LDS are written out directly; the LDS is then free
    if (in_lds)
        for (int e = tid; e < m * n; e += NT) {
            const int k = e / m, i = e % m, c = s_perm[k];
            const double v = Gw[(size_t)c * m + i];
            if (s_ex) {
                const double rt = s_rt[c];
                G[e] = rt > 0.0 ? ldexp(v, -s_ex[c] / 2) / rt : 0.0;
            } else {
                const double sg = s_sig[c];
                G[e] = sg > 0.0 ? v / sg : 0.0;
            }
        }
    if (V && v_lds)
        for (int e = tid; e < n * n; e += NT) {
            const int k = e / n, i = e % n;
            V[e] = Vw[(size_t)s_perm[k] * n + i];
        }
    __syncthreads();
    if (!in_lds)
        permute_columns<NT>(G, m, n, s_perm, s_ex ? s_rt : s_sig, s_ex, lds, lds_cap);
    if (V && !v_lds) permute_columns<NT>(V, n, n, s_perm, nullptr, nullptr, lds, lds_cap);
    double *S = b.S + b.s_off[id];
    for (int k = tid; k < n; k += NT) S[k] = s_sig[s_perm[k]];
    if (tid == 0) {
        if (b.status) b.status[id] = status;
        if (b.sweeps) b.sweeps[id] = sweeps;
    }
    __syncthreads();
}

// Problems at positions [queue[2], count) of the work order: the pointwise
// method, G in LDS when it fits, V in what LDS is left.  DD: DDRJAC pairs
// and DRDSSQ norms.
template <bool DD>
__global__ __launch_bounds__(kBatchThreads) void batched_kernel(BatchArgs b) {
    extern __shared__ double lds_g[];  // working copy of G when it fits
    __shared__ int s_item;
    __shared__ int s_rot;
    __shared__ int s_bad;
    __shared__ double s_sig[kBatchMaxN];
    __shared__ int s_perm[kBatchMaxN];
    __shared__ double s_tn[2][kBatchMaxN / 2];  // published rotations, by p-step parity
    __shared__ double s_cs[2][kBatchMaxN / 2];
    __shared__ int s_ex[DD ? kBatchMaxN : 1];       // DRDSSQ pairs of the final columns
    __shared__ double s_rt[DD ? kBatchMaxN : 1];
    const int tid = threadIdx.x;

    for (;;) {
        if (tid == 0) s_item = atomicAdd(&b.queue[1], 1);
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
        const double tol = kEps * sqrt((double)m);  // c(eps) = eps sqrt(m)
        const double t_hi = DD ? b.t_hi[ceil_lg(m)] : 0.0;
        const bool in_lds = (int64_t)m * n <= b.lds_doubles;
        const int64_t v_at = in_lds ? (int64_t)m * n : 0;
        const bool v_lds = V && v_at + (int64_t)n * n <= b.lds_doubles;
        double *Gw = in_lds ? lds_g : G;
        double *Vw = v_lds ? lds_g + v_at : V;

        if (in_lds)
            for (int e = tid; e < m * n; e += kBatchThreads) lds_g[e] = G[e];
        if (V)
            for (int e = tid; e < n * n; e += kBatchThreads) Vw[e] = (e % n == e / n) ? 1.0 : 0.0;
        if (tid == 0) s_bad = 0;
        __syncthreads();

        bool converged = false;
        int sweeps;
        if (m <= 32)
            sweeps = pointwise_sweeps<1, 1, DD>(Gw, Vw, m, n, N, tbl, b.max_sweeps, tol, b.g_groups, &s_rot, s_tn, s_cs, &converged, t_hi, &s_bad);
        else if (m <= 64)
            sweeps = pointwise_sweeps<2, 1, DD>(Gw, Vw, m, n, N, tbl, b.max_sweeps, tol, b.g_groups, &s_rot, s_tn, s_cs, &converged, t_hi, &s_bad);
        else if (m <= 128)
            sweeps = pointwise_sweeps<4, 1, DD>(Gw, Vw, m, n, N, tbl, b.max_sweeps, tol, b.g_groups, &s_rot, s_tn, s_cs, &converged, t_hi, &s_bad);
        else if (m <= 192)
            sweeps = pointwise_sweeps<6, 1, DD>(Gw, Vw, m, n, N, tbl, b.max_sweeps, tol, b.g_groups, &s_rot, s_tn, s_cs, &converged, t_hi, &s_bad);
        else
            sweeps = pointwise_sweeps<0, 1, DD>(Gw, Vw, m, n, N, tbl, b.max_sweeps, tol, b.g_groups, &s_rot, s_tn, s_cs, &converged, t_hi, &s_bad);
        const int status = (DD && s_bad) ? JSVD_NONFINITE
                           : converged ? 0 : JSVD_NOT_CONVERGED;
        finish_problem<kBatchThreads>(b, id, m, n, G, V, Gw, Vw, in_lds, v_lds, lds_g,
                                      b.lds_doubles, sweeps, status, s_sig, s_perm,
                                      DD ? s_ex : nullptr, DD ? s_rt : nullptr, t_hi);
    }
}

// Problems at positions [0, queue[2]) of the work order (the largest, n >=
// blk_min_n): the blocked method, G and V in their global buffers.  A
// kernel of its own so that its registers are allocated apart from the
// pointwise method's.
__global__ __launch_bounds__(kBlkThreads) __attribute__((amdgpu_waves_per_eu(4)))
void batched_blocked_kernel(BatchArgs b) {
    extern __shared__ double lds_g[];  // R, V' and the Gram reduction of the pivot pairs
    __shared__ int s_item;
    __shared__ double s_sig[kBatchMaxN];
    __shared__ int s_perm[kBatchMaxN];
    const int tid = threadIdx.x;
    const int nblk = b.queue[2];

    for (;;) {
        if (tid == 0) s_item = atomicAdd(&b.queue[0], 1);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= nblk) break;
        const int id = b.order[item];
        const int m = b.m[id], n = b.n[id];
        double *G = b.A + b.a_off[id];
        double *V = b.V ? b.V + b.v_off[id] : nullptr;
        if (V)
            for (int e = tid; e < n * n; e += kBlkThreads) V[e] = (e % n == e / n) ? 1.0 : 0.0;
        __syncthreads();
        const int r = blocked_sweeps(G, V, m, n, min(b.max_sweeps, 0xffff), b.tbl_order,
                                     b.tbl_off, b.tbls, lds_g);
        const int status = (r & kBlkNonfinite) ? JSVD_NONFINITE
                           : (r & kBlkConverged) ? 0 : JSVD_NOT_CONVERGED;
        finish_problem<kBlkThreads>(b, id, m, n, G, V, G, V, false, false, lds_g, kBlkLdsDoubles,
                                    r & 0xffff, status, s_sig, s_perm);
    }
}

// Work order: problem indices by non-increasing n (counting sort).
__global__ void batch_count_kernel(const int32_t *n, int64_t count, int *hist) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) atomicAdd(&hist[n[i]], 1);
}

__global__ void batch_scan_kernel(int *hist, int max_n, int blk_min_n, int *queue) {
    // one thread: bucket start positions, largest n first; the problems with
    // n >= blk_min_n (blk_min_n > 0) come first and go to the blocked kernel
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int pos = 0, nblk = 0;
        for (int v = max_n; v >= 0; --v) {
            const int c = hist[v];
            hist[v] = pos;
            pos += c;
            if (blk_min_n > 0 && v >= blk_min_n) nblk = pos;
        }
        queue[0] = 0;     // next blocked problem
        queue[1] = nblk;  // next pointwise problem
        queue[2] = nblk;  // number of blocked problems
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
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&batched_kernel<false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&batched_kernel<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess && bytes >= kBlkLdsDoubles * (int)sizeof(double))
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&batched_blocked_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                kBlkLdsDoubles * (int)sizeof(double));
    return e;
}

hipError_t launch_batched(const BatchArgs &b, int grid, int bgrid, int max_n, int *hist,
                          int32_t *order, hipStream_t s) {
    hipLaunchKernelGGL(batch_zero_kernel, dim3(1), dim3(256), 0, s, hist, max_n + 1);
    const unsigned blocks = (unsigned)((b.count + 255) / 256);
    hipLaunchKernelGGL(batch_count_kernel, dim3(blocks), dim3(256), 0, s, b.n, b.count, hist);
    hipLaunchKernelGGL(batch_scan_kernel, dim3(1), dim3(64), 0, s, hist, max_n, b.blk_min_n,
                       b.queue);
    hipLaunchKernelGGL(batch_place_kernel, dim3(blocks), dim3(256), 0, s, b.n, b.count, hist,
                       order);
    if (b.blk_min_n > 0 && max_n >= b.blk_min_n)
        hipLaunchKernelGGL(batched_blocked_kernel, dim3(bgrid), dim3(kBlkThreads),
                           (unsigned)(kBlkLdsDoubles * sizeof(double)), s, b);
    if (b.ddrjac)
        hipLaunchKernelGGL(batched_kernel<true>, dim3(grid), dim3(kBatchThreads),
                           (unsigned)(b.lds_doubles * sizeof(double)), s, b);
    else
        hipLaunchKernelGGL(batched_kernel<false>, dim3(grid), dim3(kBatchThreads),
                           (unsigned)(b.lds_doubles * sizeof(double)), s, b);
    return hipGetLastError();
}

}  // namespace jsvd

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
#include "jsvd_device.h"

namespace jsvd {

namespace {

__device__ __forceinline__ double hw_sum(double v) {
    v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);  // row_half_mirror
    v += dpp_mov<0x140>(v);  // row_mirror
    const long long x = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_ds_swizzle((int)x, 0x401F);         // lane ^ 16
    const int hi = __builtin_amdgcn_ds_swizzle((int)(x >> 32), 0x401F);
    return v + __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Order the LDS accesses of one wave around this point: what the wave
// wrote before is what its lanes read after (the wave's LDS operations
// complete in order).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Relative orthogonality test (subphase 2, reading: <= skips) and the
// trigonometric rotation, eqs. (4.3)-(4.6) with t = +1 and cs_2: refined
// reciprocal and square roots inside [2^-900, 2^900], IEEE outside.
__device__ __forceinline__ bool trig_pair(double hpp, double hqq, double hpq, double tol,
                                          double &tn, double &cs) {
    bool clamped;
    if (in_fast_range(hpp) && in_fast_range(hqq) && in_fast_range(fabs(hpq))) {
        if (fabs(hpq) <= tol * nsqrt(hpp) * nsqrt(hqq)) return false;
        rotation_fast(hpp, hqq, hpq, 1, tn, cs, clamped);
    } else {
        if (!(hpq != 0.0) || fabs(hpq) <= tol * sqrt(hpp) * sqrt(hqq)) return false;
        rotation(hpp, hqq, hpq, 1, tn, cs, clamped);
    }
    return true;
}

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
template <int R, int K>
__device__ int pointwise_sweeps(double *Gw, double *Vw, int m, int n, int N,
                                const unsigned char *tbl, int max_sweeps, double tol, int g_groups,
                                int *s_rot, double (*s_tn)[kBatchMaxN / 2],
                                double (*s_cs)[kBatchMaxN / 2], bool *converged) {
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
                        double tn[K], cs[K];
                        bool rk[K];
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
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            if (rk[k]) {
                                rot += cs[k] != 1.0 ? 1 : 0;
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
                        double hpp = 0.0, hqq = 0.0, hpq = 0.0, tn = 0.0, cs = 0.0;
                        for (int i = x; i < m; i += 32) {
                            const double a0 = gp[i], b0 = gq[i];
                            hpp = fma(a0, a0, hpp);
                            hqq = fma(b0, b0, hqq);
                            hpq = fma(a0, b0, hpq);
                        }
                        hpp = hw_sum(hpp);
                        hqq = hw_sum(hqq);
                        hpq = hw_sum(hpq);
                        if (trig_pair(hpp, hqq, hpq, tol, tn, cs)) {
                            rot += cs != 1.0 ? 1 : 0;
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


// ---------------------------------------------------------------- blocked
// Problems with many columns take the two-level method of the dense path
// inside their workgroup: block-columns of kBlkW columns, the closest
// parallel strategy of order nb on the blocks, and for every pivot
// block-pair the Gram matrix (2.7), its Cholesky factor R (Section 4.1),
// one sweep of the pointwise method on R accumulating V' (Section 4.3,
// block-oriented) and [G_p G_q] V', [V_p V_q] V' (2.9), skipped when the
// pair did not rotate (Section 4.4).  A pair whose Gram matrix already
// passes the relative orthogonality test everywhere is left alone.  Up to
// kBlkPairs pivot pairs are in flight: two waves per pair form the Gram
// matrix (rows split, FP64 MFMA) and apply V' (FP64 MFMA), one wave per pair
// factors it, and 8 lanes per pivot pair of R run the inner sweep.  G and V
// stay in their global buffers; R and V' live in LDS, small enough for two
// workgroups (two problems) per CU, which hide each other's latencies.
constexpr int kBlkW = 16, kBlkBW = 2 * kBlkW, kBlkLD = kBlkBW + 1, kBlkPairs = 4;
constexpr int kBlkThreads = 512;  // 8 waves: two per pivot pair in the Gram and update phases
constexpr int kBlkMat = kBlkBW * kBlkLD;  // doubles of one R or V'

// X[0:rows, cols of pq] <- X[0:rows, cols of pq] V' for the rows of one
// wave (16-row slices from row 16 sub, stride 16 nsub), V' row-major in LDS
// with leading dimension kBlkLD.  All loads of a slice precede its stores.
__device__ __forceinline__ void blk_rows_update(double *X, int ldx, int rows, int2 pq, int n,
                                                const double *vs, int sub, int nsub) {
    constexpr int KS = kBlkBW / 4;
    const int lane = threadIdx.x & 63, i16 = lane & 15, grp = lane >> 4;
    for (int base = 16 * sub; base < rows; base += 16 * nsub) {
        // V' is re-read from LDS in every slice rather than held in registers
        asm volatile("" ::: "memory");
        const int row = base + i16;
        const bool rv = row < rows;
        double bx[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int gc = (int)pair_col(4 * ks + grp, kBlkW, pq);
            bx[ks] = (rv && gc < n) ? X[gc * ldx + row] : 0.0;
        }
#pragma unroll
        for (int jt = 0; jt < kBlkBW / 16; ++jt) {
            d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                acc = mfma16(vs[(4 * ks + grp) * kBlkLD + jt * 16 + i16], bx[ks], acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gc = (int)pair_col(jt * 16 + grp + 4 * v, kBlkW, pq);
                if (rv && gc < n) X[gc * ldx + row] = acc[v];
            }
        }
    }
}

// The sweep loop of the blocked method on one problem (G: m x n, ld m; V:
// n x n, ld n, identity on entry, or null).  lds holds kBlkLdsDoubles.
// Returns the sweeps performed (max_sweeps <= 0xffff), plus kBlkConverged
// when a sweep performed no proper rotation and kBlkNonfinite when a
// Cholesky pivot was NaN or infinite.
constexpr int kBlkLdsDoubles = 2 * kBlkPairs * kBlkMat;  // R, V' (the Gram sums use V' space)
static_assert(kBlkPairs * 3 * 4 * 64 <= kBlkPairs * kBlkMat, "Gram partial sums fit in V' space");
static_assert(kBlkLdsDoubles == kBatchBlockLds, "host LDS bound of the blocked method");

constexpr int kBlkConverged = 1 << 16, kBlkNonfinite = 1 << 17;

__device__ __forceinline__ int blocked_sweeps(double *G, double *V, int m, int n, int max_sweeps,
                                              const int *tbl_order, const int64_t *tbl_off,
                                              const unsigned char *tbls, double *lds) {
    __shared__ int2 s_pq[kBlkPairs];
    __shared__ int s_need[kBlkPairs], s_rotk[kBlkPairs], s_prop, s_bad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i16 = lane & 15, grp = lane >> 4;
    const int nb = (n + kBlkW - 1) / kBlkW;
    const int NB = tbl_order[nb];
    const unsigned char *btbl = tbls + tbl_off[NB >> 1];
    const unsigned char *itbl = tbls + tbl_off[kBlkBW >> 1];
    const double tol = kEps * sqrt((double)kBlkBW);  // c(eps) at the inner level, n^ = 2w
    double *Rm = lds, *Vm = lds + kBlkPairs * kBlkMat, *red = Vm;  // red: before V' is set
    const int wk = wave >> 1, sub = wave & 1;  // pair and half of a wave's Gram / update work

    int sweeps = 0, result = 0;
    if (tid == 0) s_bad = 0;
    while (sweeps < max_sweeps) {
        if (tid == 0) s_prop = 0;
        int prop = 0;  // proper rotations of this lane's pivot pairs (lanes x == 0)
        for (int st = 0; st < NB - 1; ++st) {
            const unsigned char *row = btbl + (size_t)st * NB;
            int slot = 0;
            for (;;) {
                // the next pivot pairs of the step with a block inside the
                // problem (the same walk in every thread)
                __syncthreads();  // the previous group is done with s_pq, s_rotk
                int npg = 0;
                while (slot < NB / 2 && npg < kBlkPairs) {
                    const int p = row[2 * slot], q = row[2 * slot + 1];
                    ++slot;
                    if (p < nb || q < nb) {
                        if (tid == 0) s_pq[npg] = make_int2(p, q);
                        ++npg;
                    }
                }
                if (npg == 0) break;
                if (tid < kBlkPairs) s_need[tid] = s_rotk[tid] = 0;
                __syncthreads();

                // (1) Gram matrices: each wave sums its 16-row slices; the two
                // partial sums of a pair are added in wave order.
                d4 acc[3];
#pragma unroll
                for (int t = 0; t < 3; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
                int2 pq = make_int2(0, 0);
                bool valid[2] = {false, false};
                if (wk < npg) {
                    pq = s_pq[wk];
                    const double *col[2];
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const int64_t gc = pair_col(16 * t + i16, kBlkW, pq);
                        valid[t] = gc < n;
                        col[t] = G + (valid[t] ? gc : 0) * m;
                    }
                    for (int base = 16 * sub; base < m; base += 32) {
                        const int rb = base + 4 * grp;
                        double x[2][4];
#pragma unroll
                        for (int t = 0; t < 2; ++t)
#pragma unroll
                            for (int s2 = 0; s2 < 4; ++s2)
                                x[t][s2] = (valid[t] && rb + s2 < m) ? col[t][rb + s2] : 0.0;
#pragma unroll
                        for (int s2 = 0; s2 < 4; ++s2) {
                            acc[0] = mfma16(x[0][s2], x[0][s2], acc[0]);
                            acc[1] = mfma16(x[0][s2], x[1][s2], acc[1]);
                            acc[2] = mfma16(x[1][s2], x[1][s2], acc[2]);
                        }
                    }
                }
                for (int wv = 0; wv < 2; ++wv) {
                    if (wk < npg && sub == wv) {
                        double *Rk = Rm + wk * kBlkMat;
#pragma unroll
                        for (int t = 0; t < 3; ++t)
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                double *r = red + ((wk * 3 + t) * 4 + v) * 64 + lane;
                                const double h = (wv == 0) ? acc[t][v] : *r + acc[t][v];
                                if (wv < 1) {
                                    *r = h;
                                } else {
                                    // tile t: (0,0), (0,1), (1,1); entry (i, j) of H, both
                                    // triangles; padding columns become unit vectors
                                    const int i = (t == 2 ? 16 : 0) + grp + 4 * v;
                                    const int j = (t == 0 ? 0 : 16) + i16;
                                    const bool ok = pair_col(i, kBlkW, pq) < n && pair_col(j, kBlkW, pq) < n;
                                    const double hv = ok ? h : (i == j ? 1.0 : 0.0);
                                    Rk[j * kBlkLD + i] = hv;
                                    Rk[i * kBlkLD + j] = hv;
                                }
                            }
                    }
                    __syncthreads();
                }

                // (2) which pairs need the inner sweep: some (i, j) fails the
                // relative orthogonality test on H (reading: <= passes)
#pragma unroll
                for (int u = 0; u < kBlkPairs; ++u) {
                    bool need = false;
                    if (u < npg) {
                        const double *Rk = Rm + u * kBlkMat;
                        for (int e = tid; e < kBlkBW * kBlkBW; e += kBlkThreads) {
                            const int i = e & 31, j = e >> 5;
                            if (i < j) {
                                const double hij = Rk[j * kBlkLD + i];
                                const double hii = Rk[i * kBlkLD + i], hjj = Rk[j * kBlkLD + j];
                                need = need || (hij != 0.0 &&
                                                !(fabs(hij) <= tol * sqrt(hii) * sqrt(hjj)));
                            }
                        }
                    }
                    if (__ballot(need) != 0ull && lane == 0) atomicOr(&s_need[u], 1);
                }
                __syncthreads();
                int any = 0;
#pragma unroll
                for (int u = 0; u < kBlkPairs; ++u) any |= (u < npg) ? s_need[u] : 0;
                if (!any) continue;

                // (3) Cholesky H = R^T R (right-looking, unpivoted; Section 4.1),
                // one wave per pair in two panels of 16 rows: lane j holds rows
                // 16 kb .. 16 kb + 15 of column j in registers and the pivots and
                // multipliers are broadcast with readlane (no barrier); between the
                // panels each lane subtracts the first panel's rows from its column
                // of the trailing block, reading them from LDS.  Row k of R is H's
                // row k (as updated) times 1/sqrt(h_kk); a pivot that is not
                // positive makes row k zero, a NaN or infinite one ends the problem.
                if (wave < npg && s_need[wave]) {
                    double *Rk = Rm + wave * kBlkMat;
                    const int j = lane & 31;
                    int bad_met = 0;
#pragma unroll
                    for (int kb = 0; kb < 2; ++kb) {
                        if (kb == 1 && j >= 16) {
                            // H[16 + i][j] -= sum_k R[k][16 + i] R[k][j], k < 16, in k order
                            for (int i = 0; i <= j - 16; ++i) {
                                double hv = Rk[j * kBlkLD + 16 + i];
#pragma unroll
                                for (int k = 0; k < 16; ++k)
                                    hv = fma(-Rk[(16 + i) * kBlkLD + k], Rk[j * kBlkLD + k], hv);
                                Rk[j * kBlkLD + 16 + i] = hv;
                            }
                        }
                        wave_lds_sync();
                        double hb[16];
#pragma unroll
                        for (int i = 0; i < 16; ++i) hb[i] = Rk[j * kBlkLD + 16 * kb + i];
#pragma unroll
                        for (int k = 0; k < 16; ++k) {
                            const int kk = 16 * kb + k;
                            const double hkk = lane_value(hb[k], kk);
                            const bool bad = !(fabs(hkk) <= 0x1.fffffffffffffp+1023);
                            const bool pos = !bad && hkk > 0.0;
                            bad_met |= bad ? 1 : 0;
                            double rs, d;
                            rsqrt_sqrt(pos ? hkk : 1.0, rs, d);
                            double r = (j == kk) ? d : hb[k] * rs;
                            r = (pos && j >= kk) ? r : 0.0;
                            hb[k] = r;
#pragma unroll
                            for (int i = k + 1; i < 16; ++i)
                                hb[i] = fma(-lane_value(r, 16 * kb + i), r, hb[i]);
                        }
                        if (lane < kBlkBW) {
#pragma unroll
                            for (int i = 0; i < 16; ++i)
                                Rk[j * kBlkLD + 16 * kb + i] = (j >= 16 * kb + i) ? hb[i] : 0.0;
                        }
                        wave_lds_sync();
                    }
                    if (lane == 0 && bad_met) s_bad = 1;
                }
                for (int e = tid; e < kBlkPairs * kBlkBW * kBlkBW; e += kBlkThreads) {
                    const int k = e / (kBlkBW * kBlkBW), r = e % kBlkBW, c = (e / kBlkBW) % kBlkBW;
                    Vm[k * kBlkMat + r * kBlkLD + c] = (r == c) ? 1.0 : 0.0;
                }
                __syncthreads();

                // (4) one inner sweep on R, 8 lanes per pivot pair (rows x + 8r) on
                // waves 0-7, V' row-major.  Subphase 2 on squares where they cannot
                // leave the normal range (h_pq != 0 implies h_pp, h_qq > 0), else
                // in IEEE operations.
                {
                    constexpr int RL = kBlkBW / 8;  // rows per lane
                    const int gid = tid >> 3, k = gid >> 4, slot2 = gid & 15, x = tid & 7;
                    const bool act = k < npg && s_need[k];
                    const double tol2 = kEps * kEps * kBlkBW;  // tol^2, exact
                    double *Rk = Rm + k * kBlkMat, *Vk = Vm + k * kBlkMat;
                    for (int st2 = 0; st2 < kBlkBW - 1; ++st2) {
                        if (act) {
                            const int p = itbl[st2 * kBlkBW + 2 * slot2];
                            const int q = itbl[st2 * kBlkBW + 2 * slot2 + 1];
                            double *rp = Rk + p * kBlkLD, *rq = Rk + q * kBlkLD;
                            double a[RL], bq[RL];
#pragma unroll
                            for (int r = 0; r < RL; ++r) {
                                a[r] = rp[x + 8 * r];
                                bq[r] = rq[x + 8 * r];
                            }
                            double hpp = a[0] * a[0], hqq = bq[0] * bq[0], hpq = a[0] * bq[0];
#pragma unroll
                            for (int r = 1; r < RL; ++r) {
                                hpp = fma(a[r], a[r], hpp);
                                hqq = fma(bq[r], bq[r], hqq);
                                hpq = fma(a[r], bq[r], hpq);
                            }
                            hpp = half_row_sum(hpp);
                            hqq = half_row_sum(hqq);
                            hpq = half_row_sum(hpq);
                            double tn = 0.0, cs = 0.0;
                            bool rot;
                            if (in_trig_range(hpp, hqq)) {
                                rot = !(hpq * hpq <= tol2 * hpp * hqq);
                                bool clamped;
                                if (rot) rotation_fast(hpp, hqq, hpq, 1, tn, cs, clamped);
                            } else {
                                rot = trig_pair(hpp, hqq, hpq, tol, tn, cs);
                            }
                            if (rot) {
#pragma unroll
                                for (int r = 0; r < RL; ++r) {
                                    rp[x + 8 * r] = cs * fma(-tn, bq[r], a[r]);
                                    rq[x + 8 * r] = cs * fma(tn, a[r], bq[r]);
                                }
#pragma unroll
                                for (int r = 0; r < RL; ++r) {
                                    double *vr = Vk + (x + 8 * r) * kBlkLD;
                                    const double c0 = vr[p], d0 = vr[q];
                                    vr[p] = cs * fma(-tn, d0, c0);
                                    vr[q] = cs * fma(tn, c0, d0);
                                }
                                if (x == 0) {
                                    atomicAdd(&s_rotk[k], 1);
                                    prop += cs != 1.0 ? 1 : 0;
                                }
                            }
                        }
                        __syncthreads();
                    }
                }

                // (5) [G_p G_q] V' and [V_p V_q] V' for the pairs that rotated
                if (wk < npg && s_rotk[wk] > 0) {
                    const double *vs = Vm + wk * kBlkMat;
                    blk_rows_update(G, m, m, pq, n, vs, sub, 2);
                    if (V) blk_rows_update(V, n, n, pq, n, vs, sub, 2);
                }
            }
        }
        if (prop) atomicAdd(&s_prop, prop);
        __syncthreads();
        const int all = s_prop, bad = s_bad;
        ++sweeps;
        __syncthreads();
        if (bad) {
            result = kBlkNonfinite;
            break;
        }
        if (all == 0) {
            result = kBlkConverged;
            break;
        }
    }
    return sweeps | result;
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
                                                const double *sig, double *lds, int64_t lds_cap) {
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
            if (sig) {
                const double sg = sig[c];
                X[(size_t)k * rows + i0 + i] = sg > 0.0 ? v / sg : 0.0;
            } else {
                X[(size_t)k * rows + i0 + i] = v;
            }
        }
        __syncthreads();
    }
}

template <int NT>
__device__ __forceinline__ void finish_problem(const BatchArgs &b, int id, int m, int n, double *G,
                                               double *V, const double *Gw, const double *Vw,
                                               bool in_lds, bool v_lds, double *lds,
                                               int64_t lds_cap, int sweeps, int status,
                                               double *s_sig, int *s_perm) {
    const int tid = threadIdx.x, x = tid & 31, group = tid >> 5;
    for (int j = group; j < n; j += NT / 32) {
        const double *g = Gw + (size_t)j * m;
        double sacc = 0.0;
        for (int i = x; i < m; i += 32) sacc = fma(g[i], g[i], sacc);
        sacc = hw_sum(sacc);
        if (x == 0) s_sig[j] = sqrt(sacc);
    }
    __syncthreads();
    for (int j = tid; j < n; j += NT) {
        const double kj = s_sig[j] != s_sig[j] ? -INFINITY : s_sig[j];
        int r = 0;
        for (int i = 0; i < n; ++i) {
            const double ki = s_sig[i] != s_sig[i] ? -INFINITY : s_sig[i];
            r += (ki > kj || (ki == kj && i < j)) ? 1 : 0;
        }
        s_perm[r] = j;
    }
    __syncthreads();
    // working copies in LDS are written out directly; the LDS is then free
    if (in_lds)
        for (int e = tid; e < m * n; e += NT) {
            const int k = e / m, i = e % m, c = s_perm[k];
            const double sg = s_sig[c];
            G[e] = sg > 0.0 ? Gw[(size_t)c * m + i] / sg : 0.0;
        }
    if (V && v_lds)
        for (int e = tid; e < n * n; e += NT) {
            const int k = e / n, i = e % n;
            V[e] = Vw[(size_t)s_perm[k] * n + i];
        }
    __syncthreads();
    if (!in_lds) permute_columns<NT>(G, m, n, s_perm, s_sig, lds, lds_cap);
    if (V && !v_lds) permute_columns<NT>(V, n, n, s_perm, nullptr, lds, lds_cap);
    double *S = b.S + b.s_off[id];
    for (int k = tid; k < n; k += NT) S[k] = s_sig[s_perm[k]];
    if (tid == 0) {
        if (b.status) b.status[id] = status;
        if (b.sweeps) b.sweeps[id] = sweeps;
    }
    __syncthreads();
}

// Problems at positions [queue[2], count) of the work order: the pointwise
// method, G in LDS when it fits, V in what LDS is left.
__global__ __launch_bounds__(kBatchThreads) void batched_kernel(BatchArgs b) {
    extern __shared__ double lds_g[];  // working copy of G when it fits
    __shared__ int s_item;
    __shared__ int s_rot;
    __shared__ double s_sig[kBatchMaxN];
    __shared__ int s_perm[kBatchMaxN];
    __shared__ double s_tn[2][kBatchMaxN / 2];  // published rotations, by p-step parity
    __shared__ double s_cs[2][kBatchMaxN / 2];
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
        const bool in_lds = (int64_t)m * n <= b.lds_doubles;
        const int64_t v_at = in_lds ? (int64_t)m * n : 0;
        const bool v_lds = V && v_at + (int64_t)n * n <= b.lds_doubles;
        double *Gw = in_lds ? lds_g : G;
        double *Vw = v_lds ? lds_g + v_at : V;

        if (in_lds)
            for (int e = tid; e < m * n; e += kBatchThreads) lds_g[e] = G[e];
        if (V)
            for (int e = tid; e < n * n; e += kBatchThreads) Vw[e] = (e % n == e / n) ? 1.0 : 0.0;
        __syncthreads();

        bool converged = false;
        int sweeps;
        if (m <= 32)
            sweeps = pointwise_sweeps<1, 1>(Gw, Vw, m, n, N, tbl, b.max_sweeps, tol, b.g_groups, &s_rot, s_tn, s_cs, &converged);
        else if (m <= 64)
            sweeps = pointwise_sweeps<2, 1>(Gw, Vw, m, n, N, tbl, b.max_sweeps, tol, b.g_groups, &s_rot, s_tn, s_cs, &converged);
        else if (m <= 128)
            sweeps = pointwise_sweeps<4, 1>(Gw, Vw, m, n, N, tbl, b.max_sweeps, tol, b.g_groups, &s_rot, s_tn, s_cs, &converged);
        else if (m <= 192)
            sweeps = pointwise_sweeps<6, 1>(Gw, Vw, m, n, N, tbl, b.max_sweeps, tol, b.g_groups, &s_rot, s_tn, s_cs, &converged);
        else
            sweeps = pointwise_sweeps<0, 1>(Gw, Vw, m, n, N, tbl, b.max_sweeps, tol, b.g_groups, &s_rot, s_tn, s_cs, &converged);
        finish_problem<kBatchThreads>(b, id, m, n, G, V, Gw, Vw, in_lds, v_lds, lds_g,
                                      b.lds_doubles, sweeps, converged ? 0 : JSVD_NOT_CONVERGED,
                                      s_sig, s_perm);
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
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&batched_kernel),
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
    hipLaunchKernelGGL(batched_kernel, dim3(grid), dim3(kBatchThreads),
                       (unsigned)(b.lds_doubles * sizeof(double)), s, b);
    return hipGetLastError();
}

}  // namespace jsvd

// The one-sided Jacobi method on a matrix that one workgroup owns: the
// helpers and the two-level (blocked) sweep loop shared by the batched path
// (a whole small problem per workgroup) and by the inner level of the dense
// path's widest blocks (the third blocking level: a block Jacobi with
// 16-column sub-blocks on the Cholesky factor of a 128-column pivot block).
#pragma once

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
// Cholesky pivot was NaN or infinite.  stats (LDS, three ints the caller
// zeroes, or null) accumulates the rotations, the proper rotations and the
// pivot pairs whose V' was applied.
constexpr int kBlkLdsDoubles = 2 * kBlkPairs * kBlkMat;  // R, V' (the Gram sums use V' space)
static_assert(kBlkPairs * 3 * 4 * 64 <= kBlkPairs * kBlkMat, "Gram partial sums fit in V' space");
static_assert(kBlkLdsDoubles == kBatchBlockLds, "host LDS bound of the blocked method");
static_assert(kBlkBW == kBatchInnerOrder, "the host orders this table's pairs for the LDS banks");

constexpr int kBlkConverged = 1 << 16, kBlkNonfinite = 1 << 17;

__device__ __forceinline__ int blocked_sweeps(double *G, double *V, int m, int n, int max_sweeps,
                                              const int *tbl_order, const int64_t *tbl_off,
                                              const unsigned char *tbls, double *lds,
                                              int *stats = nullptr) {
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
                if (stats && tid < npg && s_rotk[tid] > 0) {
                    atomicAdd(&stats[0], s_rotk[tid]);
                    atomicAdd(&stats[2], 1);
                }
            }
        }
        if (prop) atomicAdd(&s_prop, prop);
        __syncthreads();
        const int all = s_prop, bad = s_bad;
        if (stats && tid == 0) stats[1] += all;
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

}  // namespace

}  // namespace jsvd

// gfx950 kernels of the two single-GPU levels of the blocked one-sided
// Jacobi (H)SVD.  One p-step of a block sweep is three launches:
//
//   gram_kernel    H_pq = [G_p G_q]^T [G_p G_q], eq. (2.7), on FP64 MFMA,
//                  split over the rows into deterministic partial sums;
//   inner_kernel   sum of the partials, Cholesky H_pq = R^T R (Section 4.1),
//                  and the inner pointwise Jacobi on R with V'_pq
//                  accumulated (Section 4.3), all in LDS, one workgroup per
//                  pivot block-pair;
//   update_kernel  [G_p G_q] V'_pq and [V_p V_q] V'_pq, eq. (2.9), on FP64
//                  MFMA, in place, skipped when the pair did not rotate
//                  (Section 4.4).
//
// All arithmetic is FP64.  The file is compiled without floating-point
// contraction: every fused multiply-add is an explicit fma() where the
// paper writes one.  No floating-point atomics are used, so results are
// bitwise reproducible run to run.
#include "jsvd_internal.h"

namespace jsvd {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4_f64.  Operand layout (wave64): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; the 16x16 result D holds
// D[l / 16 + 4 v][l % 16] in element v of lane l (measured on gfx950).
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Unit roundoff 2^-53 (Appendix A) and the thresholds of Section 4.3.1.
constexpr double kEps = 1.1102230246251565e-16;       // 2^-53
constexpr double kSqrtEps = 1.0536712127723509e-08;   // sqrt(2^-53)
constexpr double kSqrt2OverEps = 134217728.0;         // sqrt(2 / 2^-53) = 2^27

// Global column of local column c of the pivot block-pair (P, Q).
__device__ __forceinline__ int64_t pair_col(int c, int w, int2 pq) {
    return c < w ? (int64_t)pq.x * w + c : (int64_t)pq.y * w + (c - w);
}

// ----------------------------------------------------------------- Gram
// Grid (splits, npairs), 256 threads.  Each wave takes 32-row slices; lane
// l holds rows 8*(l/16) .. +7 of local column 16*t + l%16 for every column
// tile t, loaded as 16-byte vectors.  The contraction index of the MFMA
// runs over those rows, which is free to choose because both operands are
// the same slice.  Only the tiles on and above the diagonal of the
// symmetric H are formed.
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));

template <int BW>
__global__ __launch_bounds__(256) void gram_kernel(StepArgs a) {
    constexpr int T = BW / 16;
    constexpr int NT = T * (T + 1) / 2;
    constexpr int S = 8;
    constexpr int SLICE = 4 * S;  // rows per wave and iteration
    __shared__ d4 red[NT * 64];

    const int pair = blockIdx.y, split = blockIdx.x;
    const int2 pq = a.pairs[pair];
    if ((int64_t)pq.x * a.w >= a.n) return;  // both block-columns are padding
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, grp = lane >> 4;

    const double *col[T];
    bool valid[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int64_t gc = pair_col(t * 16 + i16, a.w, pq);
        valid[t] = gc < a.n;
        col[t] = a.G + (valid[t] ? gc : 0) * a.ldg;
    }

    d4 acc[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) acc[k] = d4{0.0, 0.0, 0.0, 0.0};

    const int64_t r0 = (int64_t)split * a.rows_per_split;
    const int64_t r1 = min(a.m, r0 + (int64_t)a.rows_per_split);
    for (int64_t base = r0 + wave * SLICE; base < r1; base += 4 * SLICE) {
        double x[T][S];
        const int64_t rb = base + grp * S;
        if (base + SLICE <= r1) {
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int s2 = 0; s2 < S / 2; ++s2) {
                    const d2u v = valid[t] ? *reinterpret_cast<const d2u *>(col[t] + rb + 2 * s2)
                                           : d2u{0.0, 0.0};
                    x[t][2 * s2] = v.x;
                    x[t][2 * s2 + 1] = v.y;
                }
        } else {
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int s = 0; s < S; ++s)
                    x[t][s] = (valid[t] && rb + s < r1) ? col[t][rb + s] : 0.0;
        }
        int k = 0;
#pragma unroll
        for (int ta = 0; ta < T; ++ta)
#pragma unroll
            for (int tb = ta; tb < T; ++tb, ++k)
#pragma unroll
                for (int s = 0; s < S; ++s) acc[k] = mfma16(x[ta][s], x[tb][s], acc[k]);
    }

    // Fixed-order sum over the four waves: ((w0 + w1) + w2) + w3.
    for (int wv = 0; wv < 4; ++wv) {
        if (wave == wv) {
#pragma unroll
            for (int k = 0; k < NT; ++k)
                red[k * 64 + lane] = (wv == 0) ? acc[k] : red[k * 64 + lane] + acc[k];
        }
        __syncthreads();
    }

    double *out = a.hpart + ((size_t)pair * a.splits + split) * BW * BW;
    for (int e = threadIdx.x; e < NT * 256; e += 256) {
        const int k = e >> 8, rem = e & 255, v = rem >> 6, l = rem & 63;
        int ta = 0, tb = 0, kk = 0;
        for (int x0 = 0; x0 < T; ++x0)
            for (int y0 = x0; y0 < T; ++y0, ++kk)
                if (kk == k) {
                    ta = x0;
                    tb = y0;
                }
        const int row = ta * 16 + (l >> 4) + 4 * v, colh = tb * 16 + (l & 15);
        out[row * BW + colh] = red[k * 64 + l][v];
    }
}

// ----------------------------------------------------- rotations (4.3)-(4.6)
// Trigonometric (t = +1) or hyperbolic (t = -1) rotation parameters from the
// pivot Gram entries, cs_2 cosine, with the short cuts at sqrt(eps) and
// sqrt(2/eps) and |coth 2phi| <= 1 replaced by 5/4.
__device__ __forceinline__ void rotation(double hpp, double hqq, double hpq, int t, double &tn,
                                         double &cs, bool &clamped) {
    const double tt = (double)t;
    const double h = hqq - tt * hpp;
    const double ct2 = tt * (h / (2.0 * hpq));
    const double sgn = ct2 < 0.0 ? -1.0 : 1.0;
    double a = fabs(ct2);
    clamped = false;
    if (t < 0 && a <= 1.0) {
        a = 1.25;
        clamped = true;
    }
    double act;
    if (t > 0 && a < kSqrtEps)
        act = a + 1.0;
    else if (a >= kSqrt2OverEps)
        act = 2.0 * a;
    else
        act = a + sqrt(fma(a, a, tt));
    tn = sgn * (1.0 / act);
    cs = (act >= kSqrt2OverEps) ? 1.0 : act / sqrt(fma(act, act, tt));
}

// Sum over the 16 lanes of a DPP row, identical in every lane: each level
// adds the value of a partner lane whose own partial sum is the mirror image
// (lane l <-> l^1, l^2, 7-l, 15-l within the row), so both lanes add the
// same two numbers.  The 16 lanes of the row must be active.
__device__ __forceinline__ double row_sum(double v) {
    v += __builtin_amdgcn_update_dpp(0.0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x140, 0xF, 0xF, false);  // row_mirror
    return v;
}

// ---------------------------------------------------------------- inner
// One workgroup per pivot block-pair.  BW = 2w.  R and V' live in LDS,
// column-major with a padded leading dimension.  A p-step of the inner
// strategy has BW/2 pivot pairs; every pair is handled by one DPP row of 16
// lanes, lane x owning rows x, x + 16, ... (BW/16 rows) of the pair's two
// columns of R and of V'.  The three dot products of subphase 1 are row
// sums; every row then decides and computes its rotation (subphases 2-5)
// and applies it (subphase 6); one barrier separates the p-steps.  With
// four pairs per wave the FP64 division and square-root chains of four
// rotations share one instruction stream.
template <int BW>
struct InnerCfg {
    static constexpr int kThreads = BW / 2 * 16;  // one 16-lane row per pivot pair
    static constexpr int kRows = BW / 16;         // rows per lane in the Jacobi steps
    static constexpr int kRowsPerSlot = kThreads / BW;   // Cholesky rows per slot
    static constexpr int kOwn = BW / kRowsPerSlot;       // Cholesky entries per thread
    static constexpr int kMaxSplits = 16;         // Gram partial sums per pair, at most
};

template <int BW>
__global__ __launch_bounds__(InnerCfg<BW>::kThreads) void inner_kernel(StepArgs a) {
    using Cfg = InnerCfg<BW>;
    constexpr int LD = BW + 1;
    constexpr int NTHR = Cfg::kThreads;
    constexpr int ROWS = Cfg::kRows;
    constexpr int OWN = Cfg::kOwn;
    constexpr int RPS = Cfg::kRowsPerSlot;
    constexpr int NWAVES = NTHR / 64;
    __shared__ double R[BW * LD];
    __shared__ double Vp[BW * LD];
    __shared__ double hdiag[BW];
    __shared__ int flags[2];  // [0] NaN met, [1] zero pivots
    __shared__ int cnt[NWAVES][4];

    const int pair = blockIdx.x;
    const int2 pq = a.pairs[pair];
    const int tid = threadIdx.x;
    if ((int64_t)pq.x * a.w >= a.n) {
        if (tid == 0) a.pair_rot[pair] = 0;
        return;
    }

    // ---- H_pq.  Thread t owns the upper-triangle entries (i, j), i <= j,
    // with j = t % BW and i = RPS o + t / BW for o = 0 .. OWN - 1, so that
    // each row of the Cholesky factor is produced by one group of BW lanes.
    // The partial Gram values of an entry are summed in split order.
    const int jcol = tid % BW, ibase = tid / BW;
    double h[OWN], di[OWN];
    const double *hp = a.hpart + (size_t)pair * a.splits * BW * BW;
#pragma unroll
    for (int o = 0; o < OWN; ++o) {
        const int i = RPS * o + ibase;
        double s = 0.0;
        if (i <= jcol) {
            double part[Cfg::kMaxSplits];
            const double *src = hp + i * BW + jcol;
#pragma unroll
            for (int sp = 0; sp < Cfg::kMaxSplits; ++sp)
                part[sp] = sp < a.splits ? src[(size_t)sp * BW * BW] : 0.0;
#pragma unroll
            for (int sp = 0; sp < Cfg::kMaxSplits; ++sp)
                if (sp < a.splits) s += part[sp];
            // padding columns become unit vectors orthogonal to everything
            if (pair_col(i, a.w, pq) >= a.n || pair_col(jcol, a.w, pq) >= a.n)
                s = (i == jcol) ? 1.0 : 0.0;
            if (i == jcol) hdiag[i] = s;
        }
        h[o] = s;
    }
    for (int e = tid; e < BW * BW; e += NTHR) {
        const int i = e % BW, j = e / BW;
        if (i > j) R[j * LD + i] = 0.0;
        Vp[j * LD + i] = (i == j) ? 1.0 : 0.0;
    }
    if (tid < 2) flags[tid] = 0;
    __syncthreads();
#pragma unroll
    for (int o = 0; o < OWN; ++o) di[o] = hdiag[RPS * o + ibase];

    // ---- Cholesky H = R^T R, row k of R at step k (Section 4.1).  Every
    // owner of an entry of row i keeps its own copy of the current H(i,i)
    // (updated by the same fma as the owner of that diagonal entry), so one
    // barrier per step suffices.  A pivot that is not positive (H only
    // semidefinite: dependent columns) makes row k of R zero.
    int zero_pivots = 0;
    for (int k = 0; k < BW; ++k) {
        const int ok = k / RPS;
        if ((k % RPS) == ibase && jcol >= k) {
#pragma unroll
            for (int o = 0; o < OWN; ++o) {
                if (o == ok) {
                    const double hkk = di[o];
                    double r = 0.0;
                    if (hkk > 0.0) {
                        const double d = sqrt(hkk);
                        r = (jcol == k) ? d : h[o] / d;
                    } else if (hkk != hkk) {
                        flags[0] = 1;
                    } else if (jcol == k) {
                        ++zero_pivots;
                    }
                    R[jcol * LD + k] = r;
                }
            }
        }
        __syncthreads();
        const double rkj = R[jcol * LD + k];
#pragma unroll
        for (int o = 0; o < OWN; ++o) {
            const int i = RPS * o + ibase;
            if (i > k && i <= jcol) {
                const double rki = R[i * LD + k];
                h[o] = fma(-rki, rkj, h[o]);
                di[o] = fma(-rki, rki, di[o]);
            }
        }
    }
    if (zero_pivots) atomicAdd(&flags[1], zero_pivots);
    __syncthreads();
    if (flags[0]) {
        if (tid == 0) {
            a.pair_rot[pair] = 0;
            atomicAdd(&a.counters[C_NONFINITE], 1ull);
        }
        return;
    }
    if (tid == 0 && flags[1]) atomicAdd(&a.counters[C_BREAKDOWN], (unsigned long long)flags[1]);

    // ---- inner Jacobi (Section 4.3)
    const int lane = tid & 63, wave = tid >> 6;
    const int x = lane & 15;      // first row owned by this lane
    const int slot = tid >> 4;    // pivot pair of this 16-lane row
    const double tol = kEps * sqrt((double)BW);  // c(eps) = eps sqrt(nhat), nhat = 2w
    int rot_total = 0, proper_total = 0, clamp_total = 0, sweeps = 0;

    for (int sw = 0; sw < a.max_inner_sweeps; ++sw) {
        int rot_sweep = 0;
        for (int st = 0; st < BW - 1; ++st) {
            const unsigned char *tbl = a.inner_tbl + (size_t)st * BW;  // BW/2 pairs x 2
            const int p = tbl[2 * slot], q = tbl[2 * slot + 1];
            double rp[ROWS], rq[ROWS], vp[ROWS], vq[ROWS];
            double hpp = 0.0, hqq = 0.0, hpq = 0.0;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                rp[r] = R[p * LD + x + 16 * r];
                rq[r] = R[q * LD + x + 16 * r];
                vp[r] = Vp[p * LD + x + 16 * r];
                vq[r] = Vp[q * LD + x + 16 * r];
                hpp = fma(rp[r], rp[r], hpp);
                hqq = fma(rq[r], rq[r], hqq);
                hpq = fma(rp[r], rq[r], hpq);
            }
            hpp = row_sum(hpp);
            hqq = row_sum(hqq);
            hpq = row_sum(hpq);

            const int64_t kp = pair_col(p, a.w, pq), kq = pair_col(q, a.w, pq);
            const bool pad = kq >= a.n || kp >= a.n;
            // subphase 2: relative orthogonality (reading: <= skips)
            const bool rotate = !(fabs(hpq) <= tol * sqrt(hpp) * sqrt(hqq));
            // subphase 4: hyperbolic iff kp < n+ <= kq.  The parameters are
            // computed whether or not the pair rotates (with a harmless
            // denominator when h_pq = 0), so that the test and the rotation
            // chains overlap; the test then selects.
            const int t = (kp < a.n_plus && kq >= a.n_plus) ? -1 : 1;
            double tn, cs;
            bool clamped;
            rotation(hpp, hqq, hpq == 0.0 ? 1.0 : hpq, t, tn, cs, clamped);
            if (!rotate) {
                tn = 0.0;
                cs = 1.0;
                clamped = false;
            }
            // subphase 5: keep j*sigma^2 non-increasing for trigonometric
            // pairs (h_pp' = h_pp - tn h_pq, h_qq' = h_qq + tn h_pq)
            bool swap = false;
            if (t > 0 && !pad) {
                const double npp = fma(-tn, hpq, hpp);
                const double nqq = fma(tn, hpq, hqq);
                if (kq < a.n_plus)
                    swap = npp < nqq;
                else if (kp >= a.n_plus)
                    swap = npp > nqq;
            }
            if (rotate || swap) {
                const double mtn = (t > 0) ? -tn : tn;  // (4.1) / (4.2)
                const int cp = swap ? q : p, cq = swap ? p : q;
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    double np = rp[r], nq = rq[r], nvp = vp[r], nvq = vq[r];
                    if (rotate) {
                        if (cs == 1.0) {  // the multiplication is omitted
                            np = fma(mtn, rq[r], rp[r]);
                            nq = fma(tn, rp[r], rq[r]);
                            nvp = fma(mtn, vq[r], vp[r]);
                            nvq = fma(tn, vp[r], vq[r]);
                        } else {
                            np = cs * fma(mtn, rq[r], rp[r]);
                            nq = cs * fma(tn, rp[r], rq[r]);
                            nvp = cs * fma(mtn, vq[r], vp[r]);
                            nvq = cs * fma(tn, vp[r], vq[r]);
                        }
                    }
                    R[cp * LD + x + 16 * r] = np;
                    R[cq * LD + x + 16 * r] = nq;
                    Vp[cp * LD + x + 16 * r] = nvp;
                    Vp[cq * LD + x + 16 * r] = nvq;
                }
            }
            // counts: one per pair (the 16 lanes of a row agree)
            const int r1 = rotate ? 1 : 0, p1 = (rotate && cs != 1.0) ? 1 : 0, c1 = clamped ? 1 : 0;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                rot_sweep += __builtin_amdgcn_readlane(r1, 16 * g);
                proper_total += __builtin_amdgcn_readlane(p1, 16 * g);
                clamp_total += __builtin_amdgcn_readlane(c1, 16 * g);
            }
            __syncthreads();
        }
        ++sweeps;
        rot_total += rot_sweep;
        if (lane == 0) cnt[wave][0] = rot_sweep;
        __syncthreads();
        int all = 0;
#pragma unroll
        for (int wv = 0; wv < NWAVES; ++wv) all += cnt[wv][0];
        __syncthreads();
        if (all == 0) break;  // no rotation in the inner sweep
    }

    // ---- write V'_pq and the counts
    double *vout = a.vprime + (size_t)pair * BW * BW;
    for (int e = tid; e < BW * BW; e += NTHR) {
        const int i = e % BW, j = e / BW;
        vout[j * BW + i] = Vp[j * LD + i];
    }
    if (lane == 0) {
        cnt[wave][0] = rot_total;
        cnt[wave][1] = proper_total;
        cnt[wave][2] = clamp_total;
    }
    __syncthreads();
    if (tid == 0) {
        long long r = 0, pr = 0, cl = 0;
        for (int wv = 0; wv < NWAVES; ++wv) {
            r += cnt[wv][0];
            pr += cnt[wv][1];
            cl += cnt[wv][2];
        }
        a.pair_rot[pair] = (int)r;
        atomicAdd(&a.counters[C_ROT], (unsigned long long)r);
        atomicAdd(&a.counters[C_PROPER], (unsigned long long)pr);
        atomicAdd(&a.counters[C_CLAMP], (unsigned long long)cl);
        atomicAdd(&a.counters[C_INNER_SW], (unsigned long long)sweeps);
        if (r) atomicAdd(&a.counters[C_UPDATES], 1ull);
    }
}

// --------------------------------------------------------------- update
// Grid (chunks of G rows + chunks of V rows, npairs), 256 threads.  Each
// wave takes 16-row slices and computes (X V')^T = V'^T X^T tile by tile:
// V' (staged in LDS) supplies the A operand, a slice of X the B operand
// (lane l reads row l%16 of local column 4*ks + l/16), and each result
// column is written back as 16 consecutive rows.  All loads of a slice
// precede its stores, so the update is in place.
template <int BW>
__global__ __launch_bounds__(256) void update_kernel(StepArgs a) {
    constexpr int KS = BW / 4, JT = BW / 16;
    __shared__ double vs[BW * BW];  // V'_pq transposed: vs[k * BW + j] = V'(k, j)
    const int pair = blockIdx.y;
    if (a.pair_rot[pair] == 0) return;
    const int2 pq = a.pairs[pair];
    int chunk = blockIdx.x;
    const bool isV = chunk >= a.upd_chunks_g;
    if (isV) chunk -= a.upd_chunks_g;
    double *X = isV ? a.V : a.G;
    const int64_t ldx = isV ? a.ldv : a.ldg;
    const int64_t rows = isV ? a.n : a.m;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, grp = lane >> 4;

    const double *vpr = a.vprime + (size_t)pair * BW * BW;
    for (int e = threadIdx.x; e < BW * BW; e += 256) vs[(e % BW) * BW + e / BW] = vpr[e];

    int64_t ldoff[KS];  // column offsets of the B loads (-1: padding)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int64_t gc = pair_col(4 * ks + grp, a.w, pq);
        ldoff[ks] = gc < a.n ? gc * ldx : -1;
    }
    __syncthreads();

    const int64_t r0 = (int64_t)chunk * a.upd_rows;
    const int64_t r1 = min(rows, r0 + (int64_t)a.upd_rows);
    for (int64_t base = r0 + wave * 16; base < r1; base += 64) {
        // re-read V' from LDS in every slice instead of pinning it in 2w^2/64
        // registers per lane (keeps the occupancy of this streaming kernel up)
        asm volatile("" ::: "memory");
        const int64_t row = base + i16;
        const bool rv = row < r1;
        double b[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) b[ks] = (rv && ldoff[ks] >= 0) ? X[ldoff[ks] + row] : 0.0;
        d4 acc[JT];
#pragma unroll
        for (int jt = 0; jt < JT; ++jt) acc[jt] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int jt = 0; jt < JT; ++jt)
                acc[jt] = mfma16(vs[(4 * ks + grp) * BW + jt * 16 + i16], b[ks], acc[jt]);
#pragma unroll
        for (int jt = 0; jt < JT; ++jt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t gc = pair_col(jt * 16 + grp + 4 * v, a.w, pq);
                if (rv && gc < a.n) X[gc * ldx + row] = acc[jt][v];
            }
    }
}

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

// Output order: positions [0, n_plus) by non-increasing sigma, [n_plus, n)
// by non-decreasing sigma, ties by column index; NaN sorts as -infinity so
// that the ranks always form a permutation.
__global__ void rank_kernel(const double *s, int64_t n, int64_t n_plus, int *perm) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const bool pos = j < n_plus;
    const int64_t lo = pos ? 0 : n_plus, hi = pos ? n_plus : n;
    const double kj = (s[j] != s[j]) ? -INFINITY : s[j];
    int64_t r = lo;
    for (int64_t i = lo; i < hi; ++i) {
        const double ki = (s[i] != s[i]) ? -INFINITY : s[i];
        const bool before = pos ? (ki > kj) : (ki < kj);
        if (before || (ki == kj && i < j)) ++r;
    }
    perm[r] = (int)j;
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

}  // namespace

hipError_t launch_gram(int bw, const StepArgs &a, hipStream_t s) {
    dim3 grid(a.splits, a.npairs);
    if (bw == 32)
        hipLaunchKernelGGL(gram_kernel<32>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(gram_kernel<64>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_inner(int bw, const StepArgs &a, hipStream_t s) {
    if (bw == 32)
        hipLaunchKernelGGL(inner_kernel<32>, dim3(a.npairs), dim3(InnerCfg<32>::kThreads), 0, s, a);
    else
        hipLaunchKernelGGL(inner_kernel<64>, dim3(a.npairs), dim3(InnerCfg<64>::kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_update(int bw, const StepArgs &a, hipStream_t s) {
    dim3 grid(a.upd_chunks_g + a.upd_chunks_v, a.npairs);
    if (bw == 32)
        hipLaunchKernelGGL(update_kernel<32>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(update_kernel<64>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

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

}  // namespace jsvd

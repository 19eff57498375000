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
// Grid (splits, npairs), 256 threads.  Each wave takes 16-row slices; lane
// l holds rows 4*(l/16) .. +3 of local column 16*t + l%16 for every column
// tile t.  The contraction index of the MFMA runs over those rows, which
// is free to choose because both operands are the same slice, so every
// lane loads 4 consecutive doubles of one column.  Only the tiles on and
// above the diagonal of the symmetric H are formed.
template <int BW>
__global__ __launch_bounds__(256) void gram_kernel(StepArgs a) {
    constexpr int T = BW / 16;
    constexpr int NT = T * (T + 1) / 2;
    constexpr int S = 4;
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
    for (int64_t base = r0 + wave * 16; base < r1; base += 64) {
        double x[T][S];
        const int64_t rb = base + grp * S;
        if (base + 16 <= r1) {
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int s = 0; s < S; ++s) x[t][s] = valid[t] ? col[t][rb + s] : 0.0;
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

template <int WIDTH>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int mask = 1; mask < WIDTH; mask <<= 1) v += __shfl_xor(v, mask, 64);
    return v;
}

// ---------------------------------------------------------------- inner
// One workgroup per pivot block-pair.  BW = 2w.  R and V' live in LDS,
// column-major with a padded leading dimension.  A p-step of the inner
// strategy has BW/2 pivot pairs; every pair is handled by a group of BW
// lanes (a half wave for BW = 32, a whole wave for BW = 64), lane x owning
// row x of the pair's two columns of R and of V'.  The three dot products
// of subphase 1 are butterfly sums over the group, identical in every lane.
template <int BW>
struct InnerCfg;
template <>
struct InnerCfg<32> {
    static constexpr int kThreads = 512;  // 8 waves x 2 half-wave groups
    static constexpr int kPairsPerLane = 1;
};
template <>
struct InnerCfg<64> {
    static constexpr int kThreads = 1024;  // 16 waves x 2 pairs each
    static constexpr int kPairsPerLane = 2;
};

template <int BW>
__global__ __launch_bounds__(InnerCfg<BW>::kThreads) void inner_kernel(StepArgs a) {
    constexpr int LD = BW + 1;
    constexpr int NTHR = InnerCfg<BW>::kThreads;
    constexpr int PPL = InnerCfg<BW>::kPairsPerLane;
    constexpr int NWAVES = NTHR / 64;
    __shared__ double R[BW * LD];
    __shared__ double Vp[BW * LD];
    __shared__ int cnt[NWAVES][4];

    const int pair = blockIdx.x;
    const int2 pq = a.pairs[pair];
    const int tid = threadIdx.x;
    if ((int64_t)pq.x * a.w >= a.n) {
        if (tid == 0) a.pair_rot[pair] = 0;
        return;
    }

    // ---- sum of the partial Gram matrices, in split order
    const double *hp = a.hpart + (size_t)pair * a.splits * BW * BW;
    for (int e = tid; e < BW * BW; e += NTHR) {
        const int i = e / BW, j = e % BW;
        if ((i >> 4) <= (j >> 4)) {
            double s = 0.0;
            for (int sp = 0; sp < a.splits; ++sp) s += hp[(size_t)sp * BW * BW + e];
            // padding columns become unit vectors orthogonal to everything
            if (pair_col(i, a.w, pq) >= a.n || pair_col(j, a.w, pq) >= a.n) s = (i == j) ? 1.0 : 0.0;
            R[j * LD + i] = s;
        }
    }
    __syncthreads();

    // ---- Cholesky H = R^T R on the upper triangle (Section 4.1, by rows of
    // R).  A pivot that is not positive (H only semidefinite: a block with
    // dependent columns) makes row k of R zero, which keeps R^T R = H for
    // the positive semidefinite case; NaN aborts the pair.
    int zero_pivots = 0;
    bool nonfinite = false;
    for (int k = 0; k < BW; ++k) {
        const double hkk = R[k * LD + k];  // uniform: every thread reads the same value
        if (hkk != hkk) {
            nonfinite = true;
            break;
        }
        if (hkk > 0.0) {
            const double d = sqrt(hkk);
            for (int j = k + tid; j < BW; j += NTHR) R[j * LD + k] = (j == k) ? d : R[j * LD + k] / d;
        } else {
            ++zero_pivots;
            for (int j = k + tid; j < BW; j += NTHR) R[j * LD + k] = 0.0;
        }
        __syncthreads();
        for (int e = tid; e < BW * BW; e += NTHR) {
            const int i = e % BW, j = e / BW;
            if (i > k && i <= j) R[j * LD + i] = fma(-R[i * LD + k], R[j * LD + k], R[j * LD + i]);
        }
        __syncthreads();
    }
    if (nonfinite) {
        if (tid == 0) {
            a.pair_rot[pair] = 0;
            atomicAdd(&a.counters[C_NONFINITE], 1ull);
        }
        return;
    }
    if (tid == 0 && zero_pivots) atomicAdd(&a.counters[C_BREAKDOWN], (unsigned long long)zero_pivots);
    for (int e = tid; e < BW * BW; e += NTHR) {
        const int i = e % BW, j = e / BW;
        if (i > j) R[j * LD + i] = 0.0;
        Vp[j * LD + i] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();

    // ---- inner Jacobi (Section 4.3)
    const int lane = tid & 63, wave = tid >> 6;
    const int x = (BW == 32) ? (lane & 31) : lane;  // row owned by this lane
    const double tol = kEps * sqrt((double)BW);     // c(eps) = eps sqrt(nhat), nhat = 2w
    int rot_total = 0, proper_total = 0, clamp_total = 0, sweeps = 0;

    for (int sw = 0; sw < a.max_inner_sweeps; ++sw) {
        int rot_sweep = 0;
        for (int st = 0; st < BW - 1; ++st) {
            const unsigned char *tbl = a.inner_tbl + (size_t)st * BW;  // BW/2 pairs x 2
            int p[PPL], q[PPL];
            double rp[PPL], rq[PPL], vp[PPL], vq[PPL];
            double hpp[PPL], hqq[PPL], hpq[PPL];
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                const int slot = (BW == 32) ? wave * 2 + (lane >> 5) : wave * 2 + k;
                p[k] = tbl[2 * slot];
                q[k] = tbl[2 * slot + 1];
                rp[k] = R[p[k] * LD + x];
                rq[k] = R[q[k] * LD + x];
                vp[k] = Vp[p[k] * LD + x];
                vq[k] = Vp[q[k] * LD + x];
                hpp[k] = rp[k] * rp[k];
                hqq[k] = rq[k] * rq[k];
                hpq[k] = rp[k] * rq[k];
            }
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                hpp[k] = group_sum<BW == 32 ? 32 : 64>(hpp[k]);
                hqq[k] = group_sum<BW == 32 ? 32 : 64>(hqq[k]);
                hpq[k] = group_sum<BW == 32 ? 32 : 64>(hpq[k]);
            }
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                const int64_t kp = pair_col(p[k], a.w, pq), kq = pair_col(q[k], a.w, pq);
                const bool pad = kq >= a.n || kp >= a.n;
                // subphase 2: relative orthogonality (reading: <= skips)
                const bool rotate = !(fabs(hpq[k]) <= tol * sqrt(hpp[k]) * sqrt(hqq[k]));
                // subphase 4: hyperbolic iff kp < n+ <= kq
                const int t = (kp < a.n_plus && kq >= a.n_plus) ? -1 : 1;
                double np = rp[k], nq = rq[k], nvp = vp[k], nvq = vq[k];
                double tn = 0.0, cs = 1.0;
                bool clamped = false;
                if (rotate) {
                    rotation(hpp[k], hqq[k], hpq[k], t, tn, cs, clamped);
                    const double mtn = (t > 0) ? -tn : tn;  // (4.1) / (4.2)
                    if (cs == 1.0) {
                        np = fma(mtn, rq[k], rp[k]);
                        nq = fma(tn, rp[k], rq[k]);
                        nvp = fma(mtn, vq[k], vp[k]);
                        nvq = fma(tn, vp[k], vq[k]);
                    } else {
                        np = cs * fma(mtn, rq[k], rp[k]);
                        nq = cs * fma(tn, rp[k], rq[k]);
                        nvp = cs * fma(mtn, vq[k], vp[k]);
                        nvq = cs * fma(tn, vp[k], vq[k]);
                    }
                }
                // subphase 5: keep j*sigma^2 non-increasing for trigonometric
                // pairs (h_pp' = h_pp - tn h_pq, h_qq' = h_qq + tn h_pq)
                bool swap = false;
                if (t > 0 && !pad) {
                    const double npp = rotate ? fma(-tn, hpq[k], hpp[k]) : hpp[k];
                    const double nqq = rotate ? fma(tn, hpq[k], hqq[k]) : hqq[k];
                    if (kq < a.n_plus)
                        swap = npp < nqq;
                    else if (kp >= a.n_plus)
                        swap = npp > nqq;
                }
                R[(swap ? q[k] : p[k]) * LD + x] = np;
                R[(swap ? p[k] : q[k]) * LD + x] = nq;
                Vp[(swap ? q[k] : p[k]) * LD + x] = nvp;
                Vp[(swap ? p[k] : q[k]) * LD + x] = nvq;
                // counts: one per pair (the lanes of a group agree)
                int r = rotate ? 1 : 0, pr = (rotate && cs != 1.0) ? 1 : 0, cl = clamped ? 1 : 0;
                if (BW == 32) {
                    r = __builtin_amdgcn_readlane(r, 0) + __builtin_amdgcn_readlane(r, 32);
                    pr = __builtin_amdgcn_readlane(pr, 0) + __builtin_amdgcn_readlane(pr, 32);
                    cl = __builtin_amdgcn_readlane(cl, 0) + __builtin_amdgcn_readlane(cl, 32);
                }
                rot_sweep += r;
                proper_total += pr;
                clamp_total += cl;
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
// V' supplies the A operand from registers, a slice of X the B operand
// (lane l reads row l%16 of local column 4*ks + l/16), and each result
// column is written back as 16 consecutive rows.  All loads of a slice
// precede its stores, so the update is in place.
template <int BW>
__global__ __launch_bounds__(256) void update_kernel(StepArgs a) {
    constexpr int KS = BW / 4, JT = BW / 16;
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
    double va[JT][KS];
#pragma unroll
    for (int jt = 0; jt < JT; ++jt)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) va[jt][ks] = vpr[(jt * 16 + i16) * BW + 4 * ks + grp];

    int64_t ldoff[KS];  // column offsets of the B loads (-1: padding)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int64_t gc = pair_col(4 * ks + grp, a.w, pq);
        ldoff[ks] = gc < a.n ? gc * ldx : -1;
    }
    int64_t stoff[JT][4];
#pragma unroll
    for (int jt = 0; jt < JT; ++jt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t gc = pair_col(jt * 16 + grp + 4 * v, a.w, pq);
            stoff[jt][v] = gc < a.n ? gc * ldx : -1;
        }

    const int64_t r0 = (int64_t)chunk * a.upd_rows;
    const int64_t r1 = min(rows, r0 + (int64_t)a.upd_rows);
    for (int64_t base = r0 + wave * 16; base < r1; base += 64) {
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
            for (int jt = 0; jt < JT; ++jt) acc[jt] = mfma16(va[jt][ks], b[ks], acc[jt]);
#pragma unroll
        for (int jt = 0; jt < JT; ++jt)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (rv && stoff[jt][v] >= 0) X[stoff[jt][v] + row] = acc[jt][v];
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

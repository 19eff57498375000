// p-step kernel 2 of 3: sum of the partial Gram matrices, Cholesky
// H_pq = R^T R (Section 4.1) and the inner pointwise Jacobi on R with V'_pq
// accumulated (Section 4.3), all in LDS, one workgroup per pivot block-pair.
// Further workgroups of the same launch apply the previous p-step's V'_pq
// to V (eq. (2.9)): V lies off the path from one p-step's Gram matrices to
// the next, and these workgroups stream it through HBM on the CUs that the
// pivot pairs leave idle.
#include "jsvd_qrpair.h"
#include "jsvd_rows.h"

namespace jsvd {

namespace {

// ---------------------------------------------------------------- inner
// One workgroup of 16 * BW threads per pivot block-pair (BW = 2w).  R and V'
// live in LDS, column-major with a padded leading dimension.
//
// Cholesky (Section 4.1) by block rows of 16: wave 0 factors a block row
// with lane j holding column j, pivots and multipliers broadcast by
// readlane; then the block row's contribution is subtracted from the
// trailing part of H on FP64 MFMA, one wave per 16 x 16 tile.
//
// Inner Jacobi (Section 4.3): a p-step of the inner strategy has BW/2 pivot
// pairs.  Threads [0, 4 BW) handle R: every pair is one DPP half row of 8
// lanes, lane x owning rows x, x + 8, ... of the pair's two columns; the
// three dot products (subphase 1) are half-row sums, each half row decides
// and computes its rotation (subphases 2-5), applies it to its columns of R
// (subphase 6) and publishes it.  Threads [4 BW, 8 BW) apply the previous
// p-step's rotations to V' at the same time, so V' never lies on the path of
// the rotations; the remaining waves only keep the barriers.  One barrier
// per p-step.  The rotation formulas are computed once per pair and wave
// lane group, so fewer lanes per pair (more rows per lane) means fewer
// waves repeating them: with 8 lanes the R side is one wave per SIMD.
template <int BW>
struct InnerCfg {
    static constexpr int kThreads = BW * 16;
    static constexpr int kLanes = 8;             // lanes per pivot pair
    static constexpr int kRows = BW / kLanes;    // rows per lane and column
    static constexpr int kPairs = BW / 2;        // pivot pairs per p-step
    static constexpr int kHalf = kPairs * kLanes;  // threads on R (and on V')
    static constexpr int kSteps = BW - 1;        // p-steps per inner sweep
    static constexpr int kLD = BW + 1;
};

// HYP: the problem has columns of both signs (J != I); without it every
// pair is trigonometric and the hyperbolic branches are compiled out.
// SC: scaled mode (badly scaled input).  The partial sums are of
// H~ = D^-1 H D^-1, D = diag(2^e_c); R~ = R D^-1 is kept with the column
// exponents e_c in LDS.  A pair's dot products on R~ are those of R times
// 2^-(e_p+e_q) after the factors 2^(e_p-e_q), 2^(e_q-e_p) on h_pp, h_qq, so
// the orthogonality test (scale free) and the rotation formulas see the same
// values as on R up to one exact power of two; the rotation is applied to R~
// with tan phi scaled by 2^(e_q-e_p) (into column p) and 2^(e_p-e_q) (into
// column q), to V' unscaled, and a swap also swaps the two exponents.  At
// the end the exponents of the transformed columns go back to global memory.
template <int BW, bool HYP, bool SC>
__global__ __launch_bounds__(InnerCfg<BW>::kThreads) void inner_kernel(StepArgs a) {
    using Cfg = InnerCfg<BW>;
    constexpr int NT = Cfg::kThreads;
    constexpr int HALF = Cfg::kHalf;
    constexpr int NWAVES = NT / 64;
    constexpr int LD = Cfg::kLD;
    constexpr int ROWS = Cfg::kRows;
    constexpr int NP = Cfg::kPairs;
    constexpr int NS = Cfg::kSteps;
    constexpr int EPT = BW * BW / NT;   // Gram entries summed per thread
    __shared__ double R[BW * LD];
    __shared__ double Vp[BW * LD];
    __shared__ unsigned char tb[NS * BW];   // inner strategy, (p, q) per pair and step
    __shared__ unsigned char sfl[NS * NP];  // pair flags per step, see below
    __shared__ d4 prm[2][NP];               // published rotations: mtn, tn, cs, flags
    __shared__ int flags[2];                // [0] NaN met, [1] zero pivots
    __shared__ int cnt[NWAVES][4];
    __shared__ int ex[BW];                  // scaled mode: column exponents

    if (blockIdx.x >= a.npairs) {
        // V <- V V'_pq of the previous p-step on one chunk of rows; these
        // workgroups come after the pivot pairs' in the grid, so the pairs
        // are dispatched first
        // start about 7 us late (2 x 127 x 64 cycles): the pair workgroups'
        // partial Gram loads then do not queue behind this V stream
        __builtin_amdgcn_s_sleep(127);
        __builtin_amdgcn_s_sleep(127);
        const int idx = blockIdx.x - a.npairs;
        const int vpair = idx / a.prev_chunks, chunk = idx % a.prev_chunks;
        if (a.prev_pair_rot[vpair] == 0) return;
        const int64_t r0 = (int64_t)chunk * a.prev_rows;
        const int64_t r1 = min(a.n, r0 + (int64_t)a.prev_rows);
        update_rows<BW, NWAVES, 1, true>(a.V, a.ldv, r0, r1, a.prev_pairs[vpair], a.w, a.n,
                                a.prev_vprime + (size_t)vpair * BW * BW, R);
        return;
    }
    const int pair = blockIdx.x;
    const int2 pq = a.pairs[pair];
    const int tid = threadIdx.x;
    if ((int64_t)pq.x * a.w >= a.n) {
        if (tid == 0) a.pair_rot[pair] = 0;
        return;
    }
    const int lane = tid & 63, wave = tid >> 6;

    // ---- H_pq: the partial Gram matrices summed in split order (upper
    // triangle, all loads of a batch of 8 splits issued together); padding
    // columns become unit vectors orthogonal to everything.  The strategy
    // table's loads go first, then the first batch, so that the table setup
    // below waits for its own loads only.
    constexpr int TE = (NS * NP + NT - 1) / NT;   // table entries per thread
    unsigned short tpq[TE];
#pragma unroll
    for (int u = 0; u < TE; ++u) {
        const int e = tid + u * NT;
        tpq[u] = e < NS * NP ? reinterpret_cast<const unsigned short *>(a.inner_tbl)[e] : 0;
    }
    const double *hp = a.hpart + (size_t)pair * a.splits * BW * BW;
    double hv[8][EPT];
    auto load_batch = [&](int s0) {
#pragma unroll
        for (int sp = 0; sp < 8; ++sp)
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const int e = tid + u * NT;
                hv[sp][u] = (s0 + sp < a.splits && e / BW <= e % BW)
                                ? hp[(size_t)(s0 + sp) * BW * BW + e] : 0.0;
            }
    };
    if (!a.qrf) load_batch(0);

    // ---- strategy table and pair flags: 1 hyperbolic (kp < n+ <= kq),
    // 2 a padding column, 4 both columns in the + part, 8 both in the - part
#pragma unroll
    for (int u = 0; u < TE; ++u) {
        const int e = tid + u * NT;
        if (e < NS * NP) {
            const int p = tpq[u] & 0xff, q = tpq[u] >> 8;
            tb[2 * e] = (unsigned char)p;
            tb[2 * e + 1] = (unsigned char)q;
            const int64_t kp = pair_col(p, a.w, pq), kq = pair_col(q, a.w, pq);
            int f = (kp < a.n_plus && kq >= a.n_plus) ? 1 : 0;
            f |= (kq >= a.n || kp >= a.n) ? 2 : 0;
            f |= (kq < a.n_plus) ? 4 : ((kp >= a.n_plus) ? 8 : 0);
            sfl[e] = (unsigned char)f;
        }
    }

    if (a.qrf) {
        // QR shortening (Section 4.2): the splits' triangular factors folded
        // into R by the peel-off procedure, V' (still free) holding the next
        // factor; then V' = I
        auto load_factor = [&](double *X, int sp) {
            for (int e = tid; e < BW * BW; e += NT) {
                const int i = e / BW, j = e % BW;
                X[j * LD + i] = i <= j ? hp[(size_t)sp * BW * BW + e] : 0.0;
            }
        };
        load_factor(R, 0);
        for (int sp = 1; sp < a.splits; ++sp) {
            load_factor(Vp, sp);
            __syncthreads();
            peel_off<BW, NT>(R, Vp, LD);
        }
        for (int e = tid; e < BW * BW; e += NT) {
            const int i = e % BW, j = e / BW;
            Vp[j * LD + i] = (i == j) ? 1.0 : 0.0;
        }
    } else {
        double s[EPT];
#pragma unroll
        for (int u = 0; u < EPT; ++u) s[u] = 0.0;
        for (int s0 = 0; s0 < a.splits; s0 += 8) {
            if (s0) load_batch(s0);
#pragma unroll
            for (int sp = 0; sp < 8; ++sp)
#pragma unroll
                for (int u = 0; u < EPT; ++u)
                    if (s0 + sp < a.splits) s[u] += hv[sp][u];
        }
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + u * NT, i = e / BW, j = e % BW;
            double h = (i <= j) ? s[u] : 0.0;
            if (i <= j && (pair_col(i, a.w, pq) >= a.n || pair_col(j, a.w, pq) >= a.n))
                h = (i == j) ? 1.0 : 0.0;
            R[j * LD + i] = h;
            Vp[j * LD + i] = (i == j) ? 1.0 : 0.0;
        }
    }
    if (tid < 2) flags[tid] = 0;
    if constexpr (SC) {
        for (int c = tid; c < BW; c += NT) {
            const int64_t gc = pair_col(c, a.w, pq);
            ex[c] = gc < a.n ? a.colexp[gc] : 0;
        }
    }
    __syncthreads();


    // ---- QR shortening: R is there; a NaN or infinity on its diagonal
    // stops the pair as a non-finite Cholesky pivot does
    if (a.qrf) {
        for (int c = tid; c < BW; c += NT)
            if (!(fabs(R[c * LD + c]) <= 0x1.fffffffffffffp+1023)) flags[0] = 1;
        __syncthreads();
    }

    // ---- nothing to do: when every pair (i, j) of the block pair already
    // passes the relative orthogonality test on H itself, no rotation can
    // happen in the inner sweep (no column of R would change, so its dot
    // products stay those of H up to the rounding of the Cholesky factor),
    // and the pair is left alone as if the sweep had rotated nothing.
    if (!a.qrf) {
        const double tol = kEps * sqrt((double)BW);
        bool need = false;
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + u * NT, i = e / BW, j = e % BW;
            if (i < j) {
                const double hij = R[j * LD + i], hii = R[i * LD + i], hjj = R[j * LD + j];
                need = need || (hij != 0.0 && !(fabs(hij) <= tol * sqrt(hii) * sqrt(hjj)));
            }
        }
        if (!__syncthreads_or(need ? 1 : 0)) {
            if (tid == 0) a.pair_rot[pair] = 0;
            return;
        }
    }

    // ---- Cholesky H = R^T R (Section 4.1).  A pivot that is not positive
    // (H only semidefinite: dependent columns) makes its row of R zero; a
    // pivot that is NaN or infinite stops the pair.  The panel has no branch,
    // so the updates of one pivot overlap the square root of the next; row k
    // of R is H's row k times 1/sqrt(h_kk).
    if (!a.qrf) {
#pragma unroll
    for (int kb = 0; kb < BW / 16; ++kb) {
        if (wave == 0) {
            const int j = lane;
            double hb[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) hb[i] = (j < BW) ? R[j * LD + 16 * kb + i] : 0.0;
            int zero_pivots = 0, nan_met = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int kk = 16 * kb + k;
                const double hkk = lane_value(hb[k], kk);
                const bool bad = !(fabs(hkk) <= 0x1.fffffffffffffp+1023);  // NaN or infinite
                const bool pos = !bad && hkk > 0.0;
                nan_met |= bad ? 1 : 0;
                zero_pivots += (!bad && !pos) ? 1 : 0;
                double rs, d;
                rsqrt_sqrt(pos ? hkk : 1.0, rs, d);
                double r = (j == kk) ? d : hb[k] * rs;
                r = (pos && j >= kk) ? r : 0.0;
                hb[k] = r;
#pragma unroll
                for (int i = k + 1; i < 16; ++i) hb[i] = fma(-lane_value(r, 16 * kb + i), r, hb[i]);
            }
            if (j < BW) {
#pragma unroll
                for (int i = 0; i < 16; ++i) R[j * LD + 16 * kb + i] = (j >= 16 * kb + i) ? hb[i] : 0.0;
            }
            if (lane == 0) {
                flags[0] |= nan_met;
                flags[1] += zero_pivots;
            }
        }
        __syncthreads();
        if (kb + 1 < BW / 16) {
            // H(i, j) -= sum_k R(16 kb + k, i) R(16 kb + k, j) on the 16 x 16
            // tiles (ti, tj), kb < ti <= tj, one wave and 4 FP64 MFMAs per tile
            constexpr int TB = BW / 16;
            int idx = wave, ti = -1, tj = -1;
#pragma unroll
            for (int t0 = kb + 1; t0 < TB; ++t0) {
                if (ti < 0 && idx < TB - t0) {
                    ti = t0;
                    tj = t0 + idx;
                } else if (ti < 0) {
                    idx -= TB - t0;
                }
            }
            if (ti >= 0) {
                const int l16 = lane & 15, l4 = lane >> 4;
                d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int k = 16 * kb + 4 * c + l4;
                    acc = mfma16(R[(16 * ti + l16) * LD + k], R[(16 * tj + l16) * LD + k], acc);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 16 * ti + l4 + 4 * v, j = 16 * tj + l16;
                    if (i <= j) R[j * LD + i] -= acc[v];
                }
            }
            __syncthreads();
        }
    }
    }  // !a.qrf
    if (flags[0]) {
        if (tid == 0) {
            a.pair_rot[pair] = 0;
            atomicAdd(&a.counters[C_NONFINITE], 1ull);
        }
        return;
    }
    if (tid == 0 && flags[1]) atomicAdd(&a.counters[C_BREAKDOWN], (unsigned long long)flags[1]);

    // ---- inner Jacobi (Section 4.3)
    constexpr int LN = Cfg::kLanes;
    const bool on_r = tid < HALF;
    const bool on_v = !on_r && tid < 2 * HALF;
    const int gt = on_r ? tid : (on_v ? tid - HALF : 0);
    const int x = gt % LN;      // first row owned by this lane
    const int slot = gt / LN;   // pivot pair of this lane group
    const double tol = kEps * sqrt((double)BW);  // c(eps) = eps sqrt(nhat), nhat = 2w
    const double tol2 = kEps * kEps * BW;        // tol^2, exact
    int rot_total = 0, proper_total = 0, clamp_total = 0, sweeps = 0;

    for (int sw = 0; sw < a.max_inner_sweeps; ++sw) {
        int rot_sweep = 0;
        int p = tb[2 * slot], q = tb[2 * slot + 1], f = sfl[slot];
        for (int st = 0; st < NS + 1; ++st) {
            if (on_r) {
                if (st < NS) {
                    double rp[ROWS], rq[ROWS];
#pragma unroll
                    for (int r = 0; r < ROWS; ++r) {
                        rp[r] = R[p * LD + x + LN * r];
                        rq[r] = R[q * LD + x + LN * r];
                    }
                    double hpp = 0.0, hqq = 0.0, hpq = 0.0;
#pragma unroll
                    for (int r = 0; r < ROWS; ++r) {
                        hpp = fma(rp[r], rp[r], hpp);
                        hqq = fma(rq[r], rq[r], hqq);
                        hpq = fma(rp[r], rq[r], hpq);
                    }
                    hpp = group_sum<LN>(hpp);
                    hqq = group_sum<LN>(hqq);
                    hpq = group_sum<LN>(hpq);
                    // subphase 2: relative orthogonality (reading: <= skips),
                    // on squares where they cannot leave the normal range.
                    // h_pq != 0 implies h_pp, h_qq > 0.
                    const bool mid = in_trig_range(hpp, hqq);
                    bool rotate;
                    if (mid)
                        rotate = !(hpq * hpq <= tol2 * hpp * hqq);
                    else
                        rotate = hpq != 0.0 && !(fabs(hpq) <= tol * sqrt(hpp) * sqrt(hqq));
                    // subphase 4: hyperbolic iff kp < n+ <= kq
                    const int t = (HYP && (f & 1)) ? -1 : 1;
                    // scaled mode: the pair's h in one common scale
                    int dl = 0, ep = 0, eq = 0;
                    double sp = hpp, sq = hqq;
                    if constexpr (SC) {
                        ep = ex[p];
                        eq = ex[q];
                        dl = eq - ep;
                        sp = ldexp(hpp, -dl);
                        sq = ldexp(hqq, dl);
                    }
                    double tn = 0.0, cs = 1.0;
                    bool clamped = false;
                    if (rotate) {
                        if ((!SC && mid) ||
                            (in_fast_range(sp) && in_fast_range(sq) && in_fast_range(fabs(hpq))))
                            rotation_fast(sp, sq, hpq, t, tn, cs, clamped);
                        else
                            rotation(sp, sq, hpq, t, tn, cs, clamped);
                    }
                    // subphase 5: keep j*sigma^2 non-increasing for trigonometric
                    // pairs (h_pp' = h_pp - tn h_pq, h_qq' = h_qq + tn h_pq)
                    bool swap = false;
                    if (!(f & 3)) {
                        const double npp = fma(-tn, hpq, sp);
                        const double nqq = fma(tn, hpq, sq);
                        swap = (!HYP || (f & 4)) ? (npp < nqq) : ((f & 8) ? (npp > nqq) : false);
                    }
                    // subphase 6, (4.1) / (4.2).  cs == 1 multiplies exactly.
                    const double mtn = (t > 0) ? -tn : tn;
                    if (rotate || swap) {
                        const int cp = swap ? q : p, cq = swap ? p : q;
                        const double mtr = SC ? ldexp(mtn, dl) : mtn;
                        const double tr = SC ? ldexp(tn, -dl) : tn;
#pragma unroll
                        for (int r = 0; r < ROWS; ++r) {
                            const double np = cs * fma(mtr, rq[r], rp[r]);
                            const double nq = cs * fma(tr, rp[r], rq[r]);
                            R[cp * LD + x + LN * r] = np;
                            R[cq * LD + x + LN * r] = nq;
                        }
                        if (SC && swap && x == 0) {
                            ex[p] = eq;
                            ex[q] = ep;
                        }
                    }
                    if (x == 0) {
                        prm[st & 1][slot] = d4{mtn, tn, cs, (double)((rotate || swap ? 1 : 0) | (swap ? 2 : 0))};
                        rot_sweep += rotate ? 1 : 0;
                        proper_total += (rotate && cs != 1.0) ? 1 : 0;
                        clamp_total += clamped ? 1 : 0;
                    }
                    if (st + 1 < NS) {
                        p = tb[(st + 1) * BW + 2 * slot];
                        q = tb[(st + 1) * BW + 2 * slot + 1];
                        f = sfl[(st + 1) * NP + slot];
                    }
                }
            } else if (on_v && st >= 1) {
                // V' <- V' (rotation of p-step st - 1)
                const int s1 = st - 1;
                const d4 pr = prm[s1 & 1][slot];
                const int fl = (int)pr[3];
                if (fl & 1) {
                    const int vp = tb[s1 * BW + 2 * slot], vq = tb[s1 * BW + 2 * slot + 1];
                    const int cp = (fl & 2) ? vq : vp, cq = (fl & 2) ? vp : vq;
                    const double mtn = pr[0], tn = pr[1], cs = pr[2];
                    double xp[ROWS], xq[ROWS];
#pragma unroll
                    for (int r = 0; r < ROWS; ++r) {
                        xp[r] = Vp[vp * LD + x + LN * r];
                        xq[r] = Vp[vq * LD + x + LN * r];
                    }
#pragma unroll
                    for (int r = 0; r < ROWS; ++r) {
                        Vp[cp * LD + x + LN * r] = cs * fma(mtn, xq[r], xp[r]);
                        Vp[cq * LD + x + LN * r] = cs * fma(tn, xp[r], xq[r]);
                    }
                }
            }
            __syncthreads();
        }
        ++sweeps;
        rot_total += rot_sweep;
        int rs = rot_sweep;
        for (int off = 32; off >= 1; off >>= 1) rs += __shfl_xor(rs, off);
        if (lane == 0) cnt[wave][0] = rs;
        __syncthreads();
        int all = 0;
#pragma unroll
        for (int wv = 0; wv < NWAVES; ++wv) all += cnt[wv][0];
        __syncthreads();
        if (all == 0) break;  // no rotation in the inner sweep
    }

    // ---- write V'_pq and the counts
    for (int off = 32; off >= 1; off >>= 1) {
        rot_total += __shfl_xor(rot_total, off);
        proper_total += __shfl_xor(proper_total, off);
        clamp_total += __shfl_xor(clamp_total, off);
    }
    double *vout = a.vprime + (size_t)pair * BW * BW;
    for (int e = tid; e < BW * BW; e += NT) {
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
    if constexpr (SC) {
        // exponents of the transformed columns (||g_c|| = ||r_c|| after the
        // update), written only when the update will run (some rotation)
        int all = 0;
#pragma unroll
        for (int wv = 0; wv < NWAVES; ++wv) all += cnt[wv][0];
        if (all != 0) {
            for (int c = tid; c < BW; c += NT) {
                const int64_t gc = pair_col(c, a.w, pq);
                double s2 = 0.0;
                for (int i = 0; i < BW; ++i) s2 = fma(R[c * LD + i], R[c * LD + i], s2);
                const double nrm = sqrt(s2);
                if (gc < a.n) a.colexp[gc] = ex[c] + (nrm > 0.0 && nrm <= 0x1p1000 ? ilogb(nrm) : 0);
            }
        }
    }
}

// ----------------------------------------------------------- inner, 2w = 128
// The third blocking level.  R and V' of a 128-column pivot pair (128 KiB
// each) do not both fit in LDS, so, as Section 2 does one level up, the
// inner problem is itself solved by the block method: the Cholesky factor
// R of H_pq is written to a global scratch (L2-resident) and a block Jacobi
// with 16-column sub-blocks runs on it (sub-block Gram matrices, their
// Cholesky factors, one pointwise sweep each and the sub-updates on FP64
// MFMA, as the batched path's blocked method: blocked_sweeps), accumulating
// V' directly in the pair's slot of the V' buffer.  max_inner_sweeps bounds
// the block sweeps of that inner method (1: block-oriented).  Ordinary SVD,
// unscaled; the sub-level strategy is the reverse row-cyclic one.
// 512 threads (kBlkThreads).  Extra workgroups after the pairs' apply the
// previous p-step's V' to V, as in inner_kernel.
constexpr int kW128Threads = kBlkThreads;

__global__ __launch_bounds__(kW128Threads) void inner128_kernel(StepArgs a) {
    constexpr int BW = 128, LD = BW + 1, NT = kW128Threads, NWAVES = NT / 64;
    constexpr int EPT = BW * BW / NT;  // Gram entries summed per thread
    __shared__ double L[BW * LD];      // H, then R; then the block method's R'' and V''
    __shared__ int sflag[2];           // [0] NaN or infinite pivot, [1] zero pivots
    __shared__ int stats[3];           // rotations, proper rotations, sub-pair updates
    static_assert(kBlkLdsDoubles <= BW * LD, "the block method's LDS fits in L");
    static_assert(BW * BW <= BW * LD, "V' of the V workgroups fits in L");

    if (blockIdx.x >= a.npairs) {
        __builtin_amdgcn_s_sleep(127);
        __builtin_amdgcn_s_sleep(127);
        const int idx = blockIdx.x - a.npairs;
        const int vpair = idx / a.prev_chunks, chunk = idx % a.prev_chunks;
        if (a.prev_pair_rot[vpair] == 0) return;
        const int64_t r0 = (int64_t)chunk * a.prev_rows;
        const int64_t r1 = min(a.n, r0 + (int64_t)a.prev_rows);
        update_rows<BW, NWAVES, 1, true>(a.V, a.ldv, r0, r1, a.prev_pairs[vpair], a.w, a.n,
                                         a.prev_vprime + (size_t)vpair * BW * BW, L);
        return;
    }
    const int pair = blockIdx.x;
    const int2 pq = a.pairs[pair];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if ((int64_t)pq.x * a.w >= a.n) {
        if (tid == 0) a.pair_rot[pair] = 0;
        return;
    }

    // ---- H_pq: the partial Gram matrices summed in split order (upper
    // triangle); padding columns become unit vectors
    {
        const double *hp = a.hpart + (size_t)pair * a.splits * BW * BW;
        double sacc[EPT];
#pragma unroll
        for (int u = 0; u < EPT; ++u) sacc[u] = 0.0;
        for (int sp = 0; sp < a.splits; ++sp)
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const int e = tid + u * NT;
                if (e / BW <= e % BW) sacc[u] += hp[(size_t)sp * BW * BW + e];
            }
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + u * NT, i = e / BW, j = e % BW;
            double h = (i <= j) ? sacc[u] : 0.0;
            if (i <= j && (pair_col(i, a.w, pq) >= a.n || pair_col(j, a.w, pq) >= a.n))
                h = (i == j) ? 1.0 : 0.0;
            L[j * LD + i] = h;
        }
    }
    if (tid < 2) sflag[tid] = 0;
    if (tid < 3) stats[tid] = 0;
    __syncthreads();

    // ---- nothing to do when every (i, j) passes the orthogonality test of
    // the sub-level (c(eps) = eps sqrt(32), the smaller of the two levels')
    {
        const double tol = kEps * sqrt((double)kBlkBW);
        bool need = false;
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + u * NT, i = e / BW, j = e % BW;
            if (i < j) {
                const double hij = L[j * LD + i], hii = L[i * LD + i], hjj = L[j * LD + j];
                need = need || (hij != 0.0 && !(fabs(hij) <= tol * sqrt(hii) * sqrt(hjj)));
            }
        }
        if (!__syncthreads_or(need ? 1 : 0)) {
            if (tid == 0) a.pair_rot[pair] = 0;
            return;
        }
    }

    // ---- Cholesky H = R^T R (Section 4.1) by block rows of 16: wave 0 factors
    // a block row, lane j holding columns j and j + 64 (readlane broadcasts the
    // pivots and multipliers), then the block row's contribution leaves the
    // trailing part of H on FP64 MFMA, 16 x 16 tiles spread over the waves.
    // Non-positive pivots make their row zero; NaN or infinite ones stop the
    // pair (as in inner_kernel).
#pragma unroll 1
    for (int kb = 0; kb < BW / 16; ++kb) {
        if (wave == 0) {
            double hb[2][16];
#pragma unroll
            for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                for (int i = 0; i < 16; ++i) hb[hh][i] = L[(lane + 64 * hh) * LD + 16 * kb + i];
            int zero_pivots = 0, nan_met = 0;
            const int ph = kb >= 4 ? 1 : 0;  // half holding the panel's own columns
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int kk = 16 * kb + k;
                const double hkk = lane_value(ph ? hb[1][k] : hb[0][k], kk - 64 * ph);
                const bool bad = !(fabs(hkk) <= 0x1.fffffffffffffp+1023);
                const bool pos = !bad && hkk > 0.0;
                nan_met |= bad ? 1 : 0;
                zero_pivots += (!bad && !pos) ? 1 : 0;
                double rs, d;
                rsqrt_sqrt(pos ? hkk : 1.0, rs, d);
                double rr[2];
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    const int j = lane + 64 * hh;
                    double r = (j == kk) ? d : hb[hh][k] * rs;
                    rr[hh] = (pos && j >= kk) ? r : 0.0;
                    hb[hh][k] = rr[hh];
                }
#pragma unroll
                for (int i = k + 1; i < 16; ++i) {
                    const double ri = lane_value(ph ? rr[1] : rr[0], 16 * kb + i - 64 * ph);
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh) hb[hh][i] = fma(-ri, rr[hh], hb[hh][i]);
                }
            }
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int j = lane + 64 * hh;
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    L[j * LD + 16 * kb + i] = (j >= 16 * kb + i) ? hb[hh][i] : 0.0;
            }
            if (lane == 0) {
                sflag[0] |= nan_met;
                sflag[1] += zero_pivots;
            }
        }
        __syncthreads();
        if (kb + 1 < BW / 16) {
            // H(i, j) -= sum_k R(16 kb + k, i) R(16 kb + k, j), tiles kb < ti <= tj
            constexpr int TB = BW / 16;
            const int rest = TB - 1 - kb, ntiles = rest * (rest + 1) / 2;
            for (int idx = wave; idx < ntiles; idx += NWAVES) {
                int ti = kb + 1, rem = idx;
                while (rem >= TB - ti) {
                    rem -= TB - ti;
                    ++ti;
                }
                const int tj = ti + rem;
                const int l16 = lane & 15, l4 = lane >> 4;
                d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int k = 16 * kb + 4 * c + l4;
                    acc = mfma16(L[(16 * ti + l16) * LD + k], L[(16 * tj + l16) * LD + k], acc);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 16 * ti + l4 + 4 * v, j = 16 * tj + l16;
                    if (i <= j) L[j * LD + i] -= acc[v];
                }
            }
            __syncthreads();
        }
    }
    if (sflag[0]) {
        if (tid == 0) {
            a.pair_rot[pair] = 0;
            atomicAdd(&a.counters[C_NONFINITE], 1ull);
        }
        return;
    }
    if (tid == 0 && sflag[1]) atomicAdd(&a.counters[C_BREAKDOWN], (unsigned long long)sflag[1]);

    // ---- R to the pair's scratch (upper triangle, zeros below), V' := I in
    // the pair's V' slot, then the block method on R
    double *Rg = a.rscratch + (size_t)pair * BW * BW;
    double *Vg = a.vprime + (size_t)pair * BW * BW;
    for (int e = tid; e < BW * BW; e += NT) {
        const int i = e % BW, j = e / BW;
        Rg[e] = (i <= j) ? L[j * LD + i] : 0.0;
        Vg[e] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int r = blocked_sweeps(Rg, Vg, BW, BW, max(1, min(a.max_inner_sweeps, 0xffff)),
                                 a.btbl_order, a.btbl_off, a.btbls, L, stats);
    __syncthreads();
    if (tid == 0) {
        if (r & kBlkNonfinite) {
            a.pair_rot[pair] = 0;
            atomicAdd(&a.counters[C_NONFINITE], 1ull);
        } else {
            const int rot = stats[0];
            a.pair_rot[pair] = rot;
            atomicAdd(&a.counters[C_ROT], (unsigned long long)rot);
            atomicAdd(&a.counters[C_PROPER], (unsigned long long)stats[1]);
            atomicAdd(&a.counters[C_INNER_SW], (unsigned long long)(r & 0xffff));
            if (rot) atomicAdd(&a.counters[C_UPDATES], 1ull);
        }
    }
}

}  // namespace

hipError_t launch_inner(int bw, const StepArgs &a, hipStream_t s) {
    if (bw == 128) {
        hipLaunchKernelGGL(inner128_kernel, dim3(a.npairs * (1 + a.prev_chunks)),
                           dim3(kW128Threads), 0, s, a);
        return hipGetLastError();
    }
    const dim3 grid(a.npairs * (1 + a.prev_chunks));
    const bool hyp = a.n_plus < a.n;
    const dim3 blk(InnerCfg<32>::kThreads), blk64(InnerCfg<64>::kThreads);
    if (a.colexp) {
        if (bw == 32) {
            if (hyp)
                hipLaunchKernelGGL((inner_kernel<32, true, true>), grid, blk, 0, s, a);
            else
                hipLaunchKernelGGL((inner_kernel<32, false, true>), grid, blk, 0, s, a);
        } else {
            if (hyp)
                hipLaunchKernelGGL((inner_kernel<64, true, true>), grid, blk64, 0, s, a);
            else
                hipLaunchKernelGGL((inner_kernel<64, false, true>), grid, blk64, 0, s, a);
        }
    } else {
        if (bw == 32) {
            if (hyp)
                hipLaunchKernelGGL((inner_kernel<32, true, false>), grid, blk, 0, s, a);
            else
                hipLaunchKernelGGL((inner_kernel<32, false, false>), grid, blk, 0, s, a);
        } else {
            if (hyp)
                hipLaunchKernelGGL((inner_kernel<64, true, false>), grid, blk64, 0, s, a);
            else
                hipLaunchKernelGGL((inner_kernel<64, false, false>), grid, blk64, 0, s, a);
        }
    }
    return hipGetLastError();
}

}  // namespace jsvd

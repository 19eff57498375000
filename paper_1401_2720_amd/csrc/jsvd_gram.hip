// p-step kernel 1 of 3: the pivot Gram matrices H_pq = [G_p G_q]^T [G_p G_q],
// eq. (2.7), on FP64 MFMA, split over the rows into deterministic partial sums.
#include "jsvd_device.h"

namespace jsvd {

namespace {

// ----------------------------------------------------------------- Gram
// Grid (splits, npairs), 256 threads.  Each wave takes 16-row slices; lane
// l holds rows 4*(l/16) .. +3 of local column 16*t + l%16 for every column
// tile t, loaded as 16-byte vectors.  The contraction index of the MFMA
// runs over those rows, which is free to choose because both operands are
// the same slice.  Only the tiles on and above the diagonal of the
// symmetric H are formed.  Four rows per lane (not eight); a pair whose
// columns all exist loads without per-column selects (measured at n = 4096:
// 40.3 -> 35.8 us per launch).  PF: the next slice is loaded while the
// current one is multiplied (two register buffers, two waves per SIMD),
// taken when the grid has at most two workgroups per CU (36.2 -> 35.0 us at
// n = 4096); otherwise one buffer and four waves per SIMD.
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));

// SC: scaled mode, column c multiplied by 2^-e_c (exact) as it is loaded.
template <int BW, bool SC, bool PF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PF ? 2 : 4))) void gram_kernel(StepArgs a) {
    constexpr int T = BW / 16;
    constexpr int NT = T * (T + 1) / 2;
    constexpr int S = 4;
    constexpr int SLICE = 4 * S;  // rows per wave and iteration
    // wave partial sums, element v of tile k's accumulator of lane l at
    // red[(4 k + v) 64 + l]: 64 consecutive doubles per access, no bank conflict
    __shared__ double red[NT * 4 * 64];

    // Workgroups go to the 8 XCDs round robin by linear index.  When the
    // pairs divide evenly, all splits of pair k run on XCD k mod 8, where
    // the inner kernel's workgroup k (linear index k) sums them from L2.
    int pair = blockIdx.y, split = blockIdx.x;
    if (a.npairs % 8 == 0) {
        const int lin = blockIdx.x + gridDim.x * blockIdx.y;
        const int xcd = lin % 8, s = lin / 8;
        pair = xcd + 8 * (s / a.splits);
        split = s % a.splits;
    }
    const int2 pq = a.pairs[pair];
    if ((int64_t)pq.x * a.w >= a.n) return;  // both block-columns are padding
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, grp = lane >> 4;

    const double *col[T];
    bool valid[T];
    int sh[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int64_t gc = pair_col(t * 16 + i16, a.w, pq);
        valid[t] = gc < a.n;
        col[t] = a.G + (valid[t] ? gc : 0) * a.ldg;
        sh[t] = (SC && valid[t]) ? -a.colexp[gc] : 0;
    }

    d4 acc[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) acc[k] = d4{0.0, 0.0, 0.0, 0.0};

    const int64_t r0 = (int64_t)split * a.rows_per_split;
    const int64_t r1 = min(a.m, r0 + (int64_t)a.rows_per_split);
    // every column of the pair present: loads without selects
    const bool allv = (int64_t)(pq.y + 1) * a.w <= a.n;
    auto load = [&](int64_t base, double (&x)[T][S]) {
        const int64_t rb = base + grp * S;
        if (allv && base + SLICE <= r1) {
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int s2 = 0; s2 < S / 2; ++s2) {
                    const d2u v = *reinterpret_cast<const d2u *>(col[t] + rb + 2 * s2);
                    x[t][2 * s2] = v.x;
                    x[t][2 * s2 + 1] = v.y;
                }
        } else if (base + SLICE <= r1) {
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
    };
    auto product = [&](double (&x)[T][S]) {
        if constexpr (SC) {
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int s = 0; s < S; ++s) x[t][s] = ldexp(x[t][s], sh[t]);
        }
        int k = 0;
#pragma unroll
        for (int ta = 0; ta < T; ++ta)
#pragma unroll
            for (int tb = ta; tb < T; ++tb, ++k)
#pragma unroll
                for (int s = 0; s < S; ++s) acc[k] = mfma16(x[ta][s], x[tb][s], acc[k]);
    };
    if constexpr (PF) {
        // software pipeline over the wave's slices: the loads of the next
        // slice are issued before the products of the current one; the
        // slices are multiplied in the same order as below, so the sums are
        // the same
        double xa[T][S], xb[T][S];
        int64_t base = r0 + wave * SLICE;
        if (base < r1) load(base, xa);
        while (base < r1) {
            int64_t nb = base + 4 * SLICE;
            if (nb < r1) load(nb, xb);
            product(xa);
            base = nb;
            if (base >= r1) break;
            nb = base + 4 * SLICE;
            if (nb < r1) load(nb, xa);
            product(xb);
            base = nb;
        }
    } else {
        for (int64_t base = r0 + wave * SLICE; base < r1; base += 4 * SLICE) {
            double x[T][S];
            load(base, x);
            product(x);
        }
    }

    // Fixed-order sum over the four waves: ((w0 + w1) + w2) + w3.
    for (int wv = 0; wv < 4; ++wv) {
        if (wave == wv) {
#pragma unroll
            for (int k = 0; k < NT; ++k)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double &r = red[(4 * k + v) * 64 + lane];
                    r = (wv == 0) ? acc[k][v] : r + acc[k][v];
                }
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
        out[row * BW + colh] = red[(4 * k + v) * 64 + l];
    }
}

// ------------------------------------------------------------- Gram, 2w = 128
// The 8 x 8 column tiles of a 128-column pivot pair give 36 tiles on and
// above the diagonal of H, too many accumulators for one wave.  Each of the
// four waves forms its own share over all rows of the split, so no partial
// sums cross waves: with super-tiles of two column tiles, wave 0 takes the
// super-tile pairs (0,0) (0,1) (1,1), wave 1 (2,2) (2,3) (3,3), wave 2
// (0,2) (0,3) and wave 3 (1,2) (1,3) -- 10, 10, 8 and 8 tiles, loading 4,
// 4, 6 and 6 column tiles of each 16-row slice (the waves read the same
// rows, so HBM sees each row once).
template <int ROLE>
struct Gram128Role;
template <>
struct Gram128Role<0> {
    static constexpr int NTL = 4, NP = 10;
    static constexpr int tl[NTL] = {0, 1, 2, 3};
    static constexpr int pa[NP] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
    static constexpr int pb[NP] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};
};
template <>
struct Gram128Role<1> {
    static constexpr int NTL = 4, NP = 10;
    static constexpr int tl[NTL] = {4, 5, 6, 7};
    static constexpr int pa[NP] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
    static constexpr int pb[NP] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};
};
template <>
struct Gram128Role<2> {
    static constexpr int NTL = 6, NP = 8;
    static constexpr int tl[NTL] = {0, 1, 4, 5, 6, 7};
    static constexpr int pa[NP] = {0, 0, 0, 0, 1, 1, 1, 1};
    static constexpr int pb[NP] = {2, 3, 4, 5, 2, 3, 4, 5};
};
template <>
struct Gram128Role<3> {
    static constexpr int NTL = 6, NP = 8;
    static constexpr int tl[NTL] = {2, 3, 4, 5, 6, 7};
    static constexpr int pa[NP] = {0, 0, 0, 0, 1, 1, 1, 1};
    static constexpr int pb[NP] = {2, 3, 4, 5, 2, 3, 4, 5};
};

template <int ROLE>
__device__ __forceinline__ void gram128_role(const StepArgs &a, int2 pq, int64_t r0, int64_t r1,
                                             double *out) {
    using Rl = Gram128Role<ROLE>;
    constexpr int NTL = Rl::NTL, NP = Rl::NP, S = 4, SLICE = 4 * S, BW = 128;
    const int lane = threadIdx.x & 63, i16 = lane & 15, grp = lane >> 4;
    const double *col[NTL];
    bool valid[NTL];
#pragma unroll
    for (int t = 0; t < NTL; ++t) {
        const int64_t gc = pair_col(Rl::tl[t] * 16 + i16, a.w, pq);
        valid[t] = gc < a.n;
        col[t] = a.G + (valid[t] ? gc : 0) * a.ldg;
    }
    d4 acc[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) acc[k] = d4{0.0, 0.0, 0.0, 0.0};
    const bool allv = (int64_t)(pq.y + 1) * a.w <= a.n;
    for (int64_t base = r0; base < r1; base += SLICE) {
        double x[NTL][S];
        const int64_t rb = base + grp * S;
        if (allv && base + SLICE <= r1) {
#pragma unroll
            for (int t = 0; t < NTL; ++t)
#pragma unroll
                for (int s2 = 0; s2 < S / 2; ++s2) {
                    const d2u v = *reinterpret_cast<const d2u *>(col[t] + rb + 2 * s2);
                    x[t][2 * s2] = v.x;
                    x[t][2 * s2 + 1] = v.y;
                }
        } else {
#pragma unroll
            for (int t = 0; t < NTL; ++t)
#pragma unroll
                for (int s2 = 0; s2 < S; ++s2)
                    x[t][s2] = (valid[t] && rb + s2 < r1) ? col[t][rb + s2] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
            for (int s2 = 0; s2 < S; ++s2)
                acc[k] = mfma16(x[Rl::pa[k]][s2], x[Rl::pb[k]][s2], acc[k]);
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int ta = Rl::tl[Rl::pa[k]], tb = Rl::tl[Rl::pb[k]];
#pragma unroll
        for (int v = 0; v < 4; ++v)
            out[(ta * 16 + grp + 4 * v) * BW + tb * 16 + i16] = acc[k][v];
    }
}

__global__ __launch_bounds__(256) void gram128_kernel(StepArgs a) {
    constexpr int BW = 128;
    int pair = blockIdx.y, split = blockIdx.x;
    if (a.npairs % 8 == 0) {
        const int lin = blockIdx.x + gridDim.x * blockIdx.y;
        const int xcd = lin % 8, s = lin / 8;
        pair = xcd + 8 * (s / a.splits);
        split = s % a.splits;
    }
    const int2 pq = a.pairs[pair];
    if ((int64_t)pq.x * a.w >= a.n) return;  // both block-columns are padding
    const int64_t r0 = (int64_t)split * a.rows_per_split;
    const int64_t r1 = min(a.m, r0 + (int64_t)a.rows_per_split);
    double *out = a.hpart + ((size_t)pair * a.splits + split) * BW * BW;
    switch (threadIdx.x >> 6) {
    case 0: gram128_role<0>(a, pq, r0, r1, out); break;
    case 1: gram128_role<1>(a, pq, r0, r1, out); break;
    case 2: gram128_role<2>(a, pq, r0, r1, out); break;
    default: gram128_role<3>(a, pq, r0, r1, out); break;
    }
}

}  // namespace

hipError_t launch_gram(int bw, const StepArgs &a, hipStream_t s) {
    if (bw == 128) {
        // the third blocking level runs unscaled only (the host checks)
        hipLaunchKernelGGL(gram128_kernel, dim3(a.splits, a.npairs), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    dim3 grid(a.splits, a.npairs);
    if (a.colexp) {
        if (bw == 32)
            hipLaunchKernelGGL((gram_kernel<32, true, false>), grid, dim3(256), 0, s, a);
        else if (a.gram_pf)
            hipLaunchKernelGGL((gram_kernel<64, true, true>), grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((gram_kernel<64, true, false>), grid, dim3(256), 0, s, a);
    } else {
        if (bw == 32)
            hipLaunchKernelGGL((gram_kernel<32, false, false>), grid, dim3(256), 0, s, a);
        else if (a.gram_pf)
            hipLaunchKernelGGL((gram_kernel<64, false, true>), grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((gram_kernel<64, false, false>), grid, dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace jsvd

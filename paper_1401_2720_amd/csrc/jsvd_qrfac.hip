// p-step kernel 1, QR variant: the triangular factor of each row split of
// [G_p G_q] by the QR shortening of Section 4.2 (eq. (2.8)), in place of
// the partial Gram matrices.  One workgroup per (pivot pair, row split):
// the split's rows are read once, in chunks of BW rows; the first chunk is
// factored into the running factor R_0, every later one into R_1 and
// folded into R_0 by the peel-off procedure (jsvd_qrpair.h).  The inner
// kernel folds the splits' factors of a pair together the same way, so
// that R^T R is the pair's Gram matrix without the Gram matrix being
// formed.  Scaled mode: column c is multiplied by 2^-e_c as it is loaded
// (exact), which gives the factor of G D^-1 that the scaled inner kernel
// works on.
#include "jsvd_qrpair.h"

namespace jsvd {

namespace {

template <int BW, bool SC>
__global__ __launch_bounds__(8 * BW) void qrfac_kernel(StepArgs a) {
    constexpr int NT = 8 * BW;
    constexpr int LD = BW + 1;
    __shared__ double R0[BW * LD];
    __shared__ double R1[BW * LD];

    // the pair and split of this workgroup, mapped to XCDs as the Gram
    // kernel maps them (all splits of pair k on XCD k mod 8)
    int pair = blockIdx.y, split = blockIdx.x;
    if (a.npairs % 8 == 0) {
        const int lin = blockIdx.x + gridDim.x * blockIdx.y;
        const int xcd = lin % 8, s = lin / 8;
        pair = xcd + 8 * (s / a.splits);
        split = s % a.splits;
    }
    const int2 pq = a.pairs[pair];
    if ((int64_t)pq.x * a.w >= a.n) return;  // both block-columns are padding
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)split * a.rows_per_split;
    const int64_t r1 = min(a.m, r0 + (int64_t)a.rows_per_split);

    // rows [base, base + BW) of the pair's columns into X; rows past the
    // split and padding columns are zero
    auto load_chunk = [&](double *X, int64_t base) {
        for (int e = tid; e < BW * BW; e += NT) {
            const int i = e % BW, j = e / BW;
            const int64_t gc = pair_col(j, a.w, pq), row = base + i;
            double v = 0.0;
            if (gc < a.n && row < r1) {
                v = a.G[gc * a.ldg + row];
                if constexpr (SC) v = ldexp(v, -a.colexp[gc]);
            }
            X[j * LD + i] = v;
        }
        __syncthreads();
    };

    load_chunk(R0, r0);
    chunk_qr<BW, NT>(R0, LD);
    for (int64_t base = r0 + BW; base < r1; base += BW) {
        load_chunk(R1, base);
        chunk_qr<BW, NT>(R1, LD);
        peel_off<BW, NT>(R0, R1, LD);
    }

    double *out = a.hpart + ((size_t)pair * a.splits + split) * BW * BW;
    for (int e = tid; e < BW * BW; e += NT) {
        const int i = e / BW, j = e % BW;
        out[e] = i <= j ? R0[j * LD + i] : 0.0;
    }
}

}  // namespace

hipError_t launch_qrfac(int bw, const StepArgs &a, hipStream_t s) {
    const dim3 grid(a.splits, a.npairs);
    if (a.colexp) {
        if (bw == 32)
            hipLaunchKernelGGL((qrfac_kernel<32, true>), grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((qrfac_kernel<64, true>), grid, dim3(512), 0, s, a);
    } else {
        if (bw == 32)
            hipLaunchKernelGGL((qrfac_kernel<32, false>), grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((qrfac_kernel<64, false>), grid, dim3(512), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace jsvd

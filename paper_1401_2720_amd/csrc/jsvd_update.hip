// p-step kernel 3 of 3: [G_p G_q] V'_pq and [V_p V_q] V'_pq, eq. (2.9), on
// FP64 MFMA, in place, skipped when the pair did not rotate (Section 4.4).
#include "jsvd_device.h"

namespace jsvd {

namespace {

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

    __syncthreads();

    // The pair's columns are w consecutive columns of block P, then w of
    // block Q; local columns past n (padding) are neither loaded nor stored.
    // Column addresses are recomputed per slice rather than kept in
    // registers, which keeps four waves per SIMD resident.
    double *XP = X + (int64_t)pq.x * a.w * ldx, *XQ = X + (int64_t)pq.y * a.w * ldx;
    const int64_t np = a.n - (int64_t)pq.x * a.w, nq = a.n - (int64_t)pq.y * a.w;
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
        for (int ks = 0; ks < KS; ++ks) {
            const int c = 4 * ks + grp;
            const bool in_p = c < a.w;
            const int lc = in_p ? c : c - a.w;
            b[ks] = (rv && lc < (in_p ? np : nq)) ? (in_p ? XP : XQ)[(int64_t)lc * ldx + row] : 0.0;
        }
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
                const int c = jt * 16 + grp + 4 * v;
                const bool in_p = c < a.w;
                const int lc = in_p ? c : c - a.w;
                if (rv && lc < (in_p ? np : nq)) (in_p ? XP : XQ)[(int64_t)lc * ldx + row] = acc[jt][v];
            }
    }
}

}  // namespace

hipError_t launch_update(int bw, const StepArgs &a, hipStream_t s) {
    dim3 grid(a.upd_chunks_g + a.upd_chunks_v, a.npairs);
    if (bw == 32)
        hipLaunchKernelGGL(update_kernel<32>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(update_kernel<64>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace jsvd

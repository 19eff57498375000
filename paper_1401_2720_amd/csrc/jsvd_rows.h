// The transformation of eq. (2.9) on a range of rows of one pivot
// block-pair: [X_p X_q] <- [X_p X_q] V'_pq, on FP64 MFMA, in place.  Used by
// the update kernel (rows of G and of V) and by the extra workgroups of the
// inner kernel's launch that update V for the previous p-step.
#pragma once

#include "jsvd_device.h"

namespace jsvd {

namespace {

// NW waves take 16-row slices of rows [r0, r1) and compute
// (X V')^T = V'^T X^T tile by tile: V' (staged by rows in LDS, vs holds at
// least BW * BW doubles: row i at vs + i BW, its column j at position
// j ^ (i mod 16), so that the staging stores of 16 consecutive rows of one
// column fall in 16 distinct banks, and the MFMA operand loads of 16
// consecutive columns of one row too) supplies the A operand, a slice of X
// the B operand (lane l reads row l%16 of local column 4*ks + l/16), and each
// result column is written back as 16 consecutive rows.  All loads of a
// slice precede its stores, so the update is in place.  The pair's columns
// are w consecutive columns of block P, then w of block Q; local columns
// past n (padding) are neither loaded nor stored.  JB of the BW/16 result
// tiles are accumulated at a time (fewer live registers for smaller JB).
// NTV: non-temporal loads and stores, for V, which is not read again before
// the next block sweep, so that it does not push G (read by the next Gram
// and update kernels) out of the caches.
// All 64 NW threads of the workgroup must call it (it contains a barrier).
template <int BW, int NW, int JB, bool NTV = false>
__device__ __forceinline__ void update_rows(double *X, int64_t ldx, int64_t r0, int64_t r1,
                                            int2 pq, int w, int64_t n, const double *vpr,
                                            double *vs) {
    constexpr int KS = BW / 4, JT = BW / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, grp = lane >> 4;
    for (int e = threadIdx.x; e < BW * BW; e += 64 * NW) {
        const int i = e % BW, j = e / BW;
        vs[i * BW + (j ^ (i & 15))] = vpr[e];
    }
    __syncthreads();

    // Column addresses are recomputed per slice rather than kept in
    // registers, which keeps four waves per SIMD resident.
    double *XP = X + (int64_t)pq.x * w * ldx, *XQ = X + (int64_t)pq.y * w * ldx;
    const int64_t np = n - (int64_t)pq.x * w, nq = n - (int64_t)pq.y * w;
    for (int64_t base = r0 + wave * 16; base < r1; base += 16 * NW) {
        // re-read V' from LDS in every slice instead of pinning it in 2w^2/64
        // registers per lane (keeps the occupancy of this streaming code up)
        asm volatile("" ::: "memory");
        const int64_t row = base + i16;
        const bool rv = row < r1;
        double b[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int c = 4 * ks + grp;
            const bool in_p = c < w;
            const int lc = in_p ? c : c - w;
            const double *src = (in_p ? XP : XQ) + (int64_t)lc * ldx + row;
            b[ks] = (rv && lc < (in_p ? np : nq))
                        ? (NTV ? __builtin_nontemporal_load(src) : *src)
                        : 0.0;
        }
#pragma unroll
        for (int j0 = 0; j0 < JT; j0 += JB) {
            d4 acc[JB];
#pragma unroll
            for (int jb = 0; jb < JB; ++jb) acc[jb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int jb = 0; jb < JB; ++jb)
                    acc[jb] = mfma16(vs[(4 * ks + grp) * BW + (j0 + jb) * 16 + (i16 ^ ((4 * ks + grp) & 15))],
                                     b[ks], acc[jb]);
#pragma unroll
            for (int jb = 0; jb < JB; ++jb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c = (j0 + jb) * 16 + grp + 4 * v;
                    const bool in_p = c < w;
                    const int lc = in_p ? c : c - w;
                    if (rv && lc < (in_p ? np : nq)) {
                        double *dst = (in_p ? XP : XQ) + (int64_t)lc * ldx + row;
                        if (NTV)
                            __builtin_nontemporal_store(acc[jb][v], dst);
                        else
                            *dst = acc[jb][v];
                    }
                }
        }
    }
}

}  // namespace

}  // namespace jsvd

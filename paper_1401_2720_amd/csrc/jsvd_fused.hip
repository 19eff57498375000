// p-step kernels 3 and 1 in one launch: the update of p-step s (eq. (2.9))
// and the partial Gram matrices of p-step s + 1 (eq. (2.7)) on the same rows.
//
// In the orderings whose consecutive steps exchange partners inside groups
// of two pairs -- (a0 a1) and (b0 b1) in step s, a pair of {a0, a1} x {b0,
// b1} and the other one in step s + 1 -- the four block-columns of such a
// group ("quad") depend on nothing outside it from one step to the next.  A
// workgroup owns one quad over a range of rows: it multiplies each 16-row
// slice by the V' of both old pairs on FP64 MFMA, stores the rotated rows,
// and feeds the very accumulator registers, which hold four consecutive
// rows of one column per lane (the layout the Gram contraction takes), into
// the two new pairs' Gram tiles.  G is read once per p-step instead of
// twice, and one launch per p-step goes.
#include "jsvd_device.h"

namespace jsvd {

namespace {

// 16-row slices of rows [r0, r1), one quad, 2w = 64, the waves of phase
// 0..3 taking rows r0 + 16 phase + 64 i.  RA / RB: old pair A / B rotated
// (else its columns pass through unchanged and are not stored).
// The wave's role is one of the two canonical new pairs, X' = [a0 b0] (role
// 0) or Y' = [a1 b1] (role 1); its four register tiles d[0..3] are the two
// 16-column tiles of its block of A, then the two of its block of B, and it
// stores only those columns.  Waves of both roles read all four blocks of a
// slice, so a barrier per slice keeps the stores of one role after the other
// role's loads of the same rows.  vsA / vsB hold V' by rows (row i at i*64,
// its column j at j ^ (i mod 16)), with the columns rotated so that a0's
// (b0's) come first, a1's (b1's) at 32.
template <bool RA, bool RB>
__device__ __forceinline__ void fused_slices(const StepArgs &a, int64_t r0, int64_t r1,
                                             const double *PA, const double *QA,
                                             const double *PB, const double *QB,
                                             double *XA, double *XB, const double *vsA,
                                             const double *vsB, d4 (&g)[10]) {
    constexpr int BW = 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, grp = lane >> 4;
    const int role = wave & 1, phase = wave >> 1;  // phase 0..3
    // XA / XB: the first rows of this role's block of A / of B

    // Addresses: a wave-uniform part (block, column offset, the slice's
    // first row) and a per-lane byte offset fixed for the kernel.  A rotated
    // pair is loaded as the MFMA A operand of X V' (lane (i16, grp) holds
    // row i16 of pair column 4k + grp, k < 8 in the first block); a pair
    // passing through as this role's two tiles (x[4u + v] = row grp + 4v of
    // column 16u + i16 of its block).  Every slice is whole: the host takes
    // this path only when m, and so every split's row count, is a multiple
    // of 64, and lda <= 2^25 (the byte offsets stay below 2^32).
    const uint32_t off_op = (uint32_t)((grp * a.ldg + i16) * 8);   // operand layout
    const uint32_t off_t = (uint32_t)((i16 * a.ldg + grp) * 8);    // tile layout
    auto at = [](const double *sb, uint32_t off) {
        return reinterpret_cast<const double *>(reinterpret_cast<const char *>(sb) + off);
    };
    auto load = [&](int64_t base, double (&x)[32]) {
        // the column bases are formed per slice on the scalar unit rather
        // than kept for the loop in scalar registers
        int64_t ldg = a.ldg;
        asm volatile("" : "+s"(ldg));
        if constexpr (RA) {
#pragma unroll
            for (int k = 0; k < 16; ++k)
                x[k] = *at((k < 8 ? PA : QA) + (int64_t)(4 * (k & 7)) * ldg + base, off_op);
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                x[k] = *at(XA + (int64_t)(16 * (k >> 2)) * ldg + base + 4 * (k & 3), off_t);
        }
        if constexpr (RB) {
#pragma unroll
            for (int k = 0; k < 16; ++k)
                x[16 + k] = *at((k < 8 ? PB : QB) + (int64_t)(4 * (k & 7)) * ldg + base, off_op);
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                x[16 + k] = *at(XB + (int64_t)(16 * (k >> 2)) * ldg + base + 4 * (k & 3), off_t);
        }
    };

    const int vcol = 32 * role;  // this role's columns in vsA / vsB
    auto slice = [&](int64_t base, const double (&x)[32]) {
        // V' is re-read from LDS for every slice rather than held in
        // 2 * 64 registers per lane
        asm volatile("" ::: "memory");
        d4 d[4];
        // ---- X V' for this role's tiles (or the loaded tiles as they are)
        if constexpr (RA) {
            d[0] = d4{0.0, 0.0, 0.0, 0.0};
            d[1] = d4{0.0, 0.0, 0.0, 0.0};
        } else {
            d[0] = d4{x[0], x[1], x[2], x[3]};
            d[1] = d4{x[4], x[5], x[6], x[7]};
        }
        if constexpr (RB) {
            d[2] = d4{0.0, 0.0, 0.0, 0.0};
            d[3] = d4{0.0, 0.0, 0.0, 0.0};
        } else {
            d[2] = d4{x[16], x[17], x[18], x[19]};
            d[3] = d4{x[20], x[21], x[22], x[23]};
        }
        if constexpr (RA || RB) {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int i = 4 * k + grp, sw = i16 ^ (i & 15);
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    if constexpr (RA)
                        d[s] = mfma16(x[k], vsA[i * BW + vcol + 16 * s + sw], d[s]);
                    if constexpr (RB)
                        d[2 + s] = mfma16(x[16 + k], vsB[i * BW + vcol + 16 * s + sw], d[2 + s]);
                }
            }
        }
        // ---- Gram tiles of this role's new pair over the slice: MFMA v
        // contracts rows grp + 4v, so the 16 rows are summed in four products
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int k = 0;
#pragma unroll
            for (int ta = 0; ta < 4; ++ta)
#pragma unroll
                for (int tb = ta; tb < 4; ++tb, ++k) g[k] = mfma16(d[ta][v], d[tb][v], g[k]);
        }
        // ---- store the rotated rows once both roles have read the slice:
        // lane holds rows grp + 4v of column i16 of each tile
        __syncthreads();
        int64_t ldg = a.ldg;
        asm volatile("" : "+s"(ldg));
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if constexpr (RA)
                    *const_cast<double *>(at(XA + (int64_t)(16 * s) * ldg + base + 4 * v, off_t)) =
                        d[s][v];
                if constexpr (RB)
                    *const_cast<double *>(at(XB + (int64_t)(16 * s) * ldg + base + 4 * v, off_t)) =
                        d[2 + s][v];
            }
    };

    // Both waves of a phase take the same slices, and every wave takes the
    // same number (the split's rows are a multiple of 64), so all pass the
    // same barriers.  One buffer: the loads of one wave's slice overlap the
    // products of the other wave on the same SIMD.
    const int64_t nsl = (r1 - r0) / 64;
    int64_t base = r0 + phase * 16;
    for (int64_t it = 0; it < nsl; ++it, base += 64) {
        double x[32];
        load(base, x);
        slice(base, x);
    }
}

// Grid (splits, quads), 512 threads (two waves per SIMD, 256 registers per
// lane each), one workgroup per CU.  quads[8 q ..]: old pair indices ia, ib in this p-step, new
// pair indices jx, jy in the next, and the blocks a0 (of pair ia) and b0 (of
// pair ib) that go to pair jx; a1, b1 are the other blocks.
template <int BW>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void fused_kernel(StepArgs a) {
    static_assert(BW == 64, "the fused launch is written for 2w = 64");
    constexpr int T = 4, NT = 10;
    __shared__ double lds[2 * BW * BW];  // V'_A, V'_B; then the wave partial sums
    double *vsA = lds, *vsB = lds + BW * BW;
    const int split = blockIdx.x, q = blockIdx.y;
    const int *qd = a.quads + 8 * q;
    const int ia = qd[0], ib = qd[1], jx = qd[2], jy = qd[3], a0 = qd[4], b0 = qd[5];
    const int2 pa = a.pairs[ia], pb = a.pairs[ib];
    const int a1 = a0 == pa.x ? pa.y : pa.x, b1 = b0 == pb.x ? pb.y : pb.x;
    const int offa = a0 == pa.x ? 0 : a.w, offb = b0 == pb.x ? 0 : a.w;
    const bool ra = a.pair_rot[ia] != 0, rb = a.pair_rot[ib] != 0;
    const int w = a.w;

    // V' of both old pairs by rows, columns rotated by offa / offb
    const double *vpa = a.vprime + (size_t)ia * BW * BW, *vpb = a.vprime + (size_t)ib * BW * BW;
    for (int e = threadIdx.x; e < BW * BW; e += 512) {
        const int i = e % BW, j = e / BW;
        const int ja = (j - offa) & (BW - 1), jb = (j - offb) & (BW - 1);
        vsA[i * BW + (ja ^ (i & 15))] = vpa[e];
        vsB[i * BW + (jb ^ (i & 15))] = vpb[e];
    }
    __syncthreads();

    const int64_t r0 = (int64_t)split * a.rows_per_split;
    const int64_t r1 = min(a.m, r0 + (int64_t)a.rows_per_split);
    const int64_t ldg = a.ldg;
    const double *PA = a.G + (int64_t)pa.x * w * ldg, *QA = a.G + (int64_t)pa.y * w * ldg;
    const double *PB = a.G + (int64_t)pb.x * w * ldg, *QB = a.G + (int64_t)pb.y * w * ldg;
    // this wave's role: new pair X' = [a0 b0] (even waves) or Y' = [a1 b1]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, role = wave & 1;
    double *XA = a.G + (int64_t)(role ? a1 : a0) * w * ldg;
    double *XB = a.G + (int64_t)(role ? b1 : b0) * w * ldg;
    d4 g[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) g[k] = d4{0.0, 0.0, 0.0, 0.0};
    if (ra && rb)
        fused_slices<true, true>(a, r0, r1, PA, QA, PB, QB, XA, XB, vsA, vsB, g);
    else if (ra)
        fused_slices<true, false>(a, r0, r1, PA, QA, PB, QB, XA, XB, vsA, vsB, g);
    else if (rb)
        fused_slices<false, true>(a, r0, r1, PA, QA, PB, QB, XA, XB, vsA, vsB, g);
    else
        fused_slices<false, false>(a, r0, r1, PA, QA, PB, QB, XA, XB, vsA, vsB, g);

    // Fixed-order sum over the four waves of each role (phases 0, 1, 2, 3),
    // in the LDS that held V': element v of tile k's accumulator of lane l
    // of X' at red[(4 k + v) 64 + l], of Y' 40 * 64 doubles further.
    __syncthreads();
    double *red = lds + role * 4 * NT * 64;
    for (int ph = 0; ph < 4; ++ph) {
        if ((wave >> 1) == ph) {
#pragma unroll
            for (int k = 0; k < NT; ++k)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double &r = red[(4 * k + v) * 64 + lane];
                    r = (ph == 0) ? g[k][v] : r + g[k][v];
                }
        }
        __syncthreads();
    }
    red = lds;

    // Write the upper tiles of each new pair in its own column order.  When
    // the pair is (b, a) rather than the canonical (a, b), its column c is
    // canonical column (c + w) mod 2w; elements that fall below the
    // canonical diagonal tiles are read transposed (H is symmetric).
    const int2 nx = a.next_pairs[jx], ny = a.next_pairs[jy];
    const bool swx = nx.x != a0, swy = ny.x != a1;
    for (int e = threadIdx.x; e < 2 * NT * 256; e += 512) {
        const int which = e / (NT * 256), rem = e % (NT * 256);
        const int kt = rem >> 8, el = rem & 255;
        int ta = 0, tb = 0;
        for (int x0 = 0, kk = 0; x0 < T; ++x0)
            for (int y0 = x0; y0 < T; ++y0, ++kk)
                if (kk == kt) {
                    ta = x0;
                    tb = y0;
                }
        const int r = ta * 16 + (el >> 4), c = tb * 16 + (el & 15);
        const bool sw = which == 0 ? swx : swy;
        int rc = sw ? (r + w) & (BW - 1) : r, cc = sw ? (c + w) & (BW - 1) : c;
        if ((rc >> 4) > (cc >> 4)) {
            const int t = rc;
            rc = cc;
            cc = t;
        }
        // canonical element (rc, cc): tile (rc/16, cc/16), v and lane of it
        const int ca = rc >> 4, cb = cc >> 4;
        const int ck = ca * T - ca * (ca - 1) / 2 + (cb - ca);
        const int v = (rc & 15) >> 2, l = (rc & 3) * 16 + (cc & 15);
        const double val = red[(which * 4 * NT + 4 * ck + v) * 64 + l];
        const int jp = which == 0 ? jx : jy;
        a.hpart[((size_t)jp * a.splits + split) * BW * BW + r * BW + c] = val;
    }
}

}  // namespace

hipError_t launch_fused(int nquads, const StepArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(fused_kernel<64>, dim3(a.splits, nquads), dim3(512), 0, s, a);
    return hipGetLastError();
}

}  // namespace jsvd

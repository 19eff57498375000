// p-step kernel 3 of 3: [G_p G_q] V'_pq and [V_p V_q] V'_pq, eq. (2.9), on
// FP64 MFMA, in place, skipped when the pair did not rotate (Section 4.4).
#include "jsvd_rows.h"

namespace jsvd {

namespace {

// --------------------------------------------------------------- update
// Grid (chunks of G rows + chunks of V rows, npairs), 256 threads.  The
// solver launches it on the rows of G only while the V update of a p-step
// rides along with the next p-step's inner kernel, and on the rows of V
// after the last p-step.
template <int BW>
__global__ __launch_bounds__(256) void update_kernel(StepArgs a) {
    __shared__ double vs[BW * BW];  // V'_pq by rows, in the layout update_rows uses
    const int pair = blockIdx.y;
    if (a.pair_rot[pair] == 0) return;
    int chunk = blockIdx.x;
    const bool isV = chunk >= a.upd_chunks_g;
    if (isV) chunk -= a.upd_chunks_g;
    const int64_t rows = isV ? a.n : a.m;
    const int64_t r0 = (int64_t)chunk * a.upd_rows;
    const int64_t r1 = min(rows, r0 + (int64_t)a.upd_rows);
    const double *vpr = a.vprime + (size_t)pair * BW * BW;
    constexpr int JB = BW == 128 ? 4 : BW / 16;  // result tiles accumulated at a time
    if (isV)
        update_rows<BW, 4, JB, true>(a.V, a.ldv, r0, r1, a.pairs[pair], a.w, a.n, vpr, vs);
    else
        update_rows<BW, 4, JB>(a.G, a.ldg, r0, r1, a.pairs[pair], a.w, a.n, vpr, vs);
}

}  // namespace

hipError_t launch_update(int bw, const StepArgs &a, hipStream_t s) {
    dim3 grid(a.upd_chunks_g + a.upd_chunks_v, a.npairs);
    if (grid.x == 0) return hipSuccess;
    if (bw == 32)
        hipLaunchKernelGGL(update_kernel<32>, grid, dim3(256), 0, s, a);
    else if (bw == 64)
        hipLaunchKernelGGL(update_kernel<64>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(update_kernel<128>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace jsvd

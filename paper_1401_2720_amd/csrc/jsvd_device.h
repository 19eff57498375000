// Device helpers shared by the p-step kernels of the blocked one-sided
// Jacobi (H)SVD: MFMA tile, constants of Section 4.3.1, FP64 building
// blocks, DPP row sums and the rotation formulas (4.3)-(4.6).
//
// All arithmetic is FP64.  The kernels are compiled without floating-point
// contraction: every fused multiply-add is an explicit fma() where the
// paper writes one.  No floating-point atomics are used, so results are
// bitwise reproducible run to run.
#pragma once

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

// ----------------------------------------------------- FP64 building blocks
// Correctly rounded division, reciprocal and square root for the inner
// rotations, built from the hardware reciprocal (v_rcp_f64) and reciprocal
// square root (v_rsq_f64) seeds: Newton steps and a residual correction with
// fused multiply-adds (Markstein's scheme) bring the result within one ulp,
// and a final exact rounding test picks between it and its neighbour.  Valid
// for positive normal operands whose results and residuals stay in the
// normal range (the kernels use them only inside [2^-900, 2^900]); the IEEE
// operations are used everywhere else.
//
// The rounding test.  Let x be within one ulp of the exact result z.  For
// the reciprocal and the quotient the residual e = 1 - b x (a - b x) is an
// integer multiple of the product grain of b and x that is smaller in
// magnitude than b ulp(x), i.e. it has at most 53 significant bits, so the
// fma computes it exactly; so does it for the neighbour x' of x on z's side,
// which lies on the other side of z or on it.  The nearer of x and x' is the
// one with the smaller |residual|, and neither z = 1/b nor z = a/b is ever
// the exact midpoint of two doubles (it would need 54 significant bits in a
// or in 1), so the choice is the correctly rounded result.

__device__ __forceinline__ double step_bits(double x, bool up) {
    return __builtin_bit_cast(double, __builtin_bit_cast(long long, x) + (up ? 1LL : -1LL));
}

// Reciprocal of a positive b within one ulp: two Newton steps from the seed.
__device__ __forceinline__ double nrcp_1ulp(double b) {
    double y = __builtin_amdgcn_rcp(b);
    double e = fma(-b, y, 1.0);
    y = fma(y, e, y);
    e = fma(-b, y, 1.0);
    return fma(y, e, y);
}
// Correctly rounded 1/b for a positive b.
__device__ __forceinline__ double nrcp(double b) {
    const double y = nrcp_1ulp(b);
    const double e = fma(-b, y, 1.0);
    const double yn = step_bits(y, e > 0.0);
    const double en = fma(-b, yn, 1.0);
    return fabs(en) < fabs(e) ? yn : y;
}
// Correctly rounded a/b (any signs): the quotient of the magnitudes by the
// reciprocal and one residual correction, the rounding test, then the sign.
__device__ __forceinline__ double ndiv(double a, double b) {
    const double aa = fabs(a), bb = fabs(b);
    const double y = nrcp_1ulp(bb);
    double q = aa * y;
    double r = fma(-bb, q, aa);
    q = fma(r, y, q);
    r = fma(-bb, q, aa);
    const double qn = step_bits(q, r > 0.0);
    const double rn = fma(-bb, qn, aa);
    q = fabs(rn) < fabs(r) ? qn : q;
    const long long sign =
        (__builtin_bit_cast(long long, a) ^ __builtin_bit_cast(long long, b)) & (1LL << 63);
    return __builtin_bit_cast(double, __builtin_bit_cast(long long, q) | sign);
}
// Correctly rounded sqrt(u) for a positive u.  The coupled iteration for the
// root s and half its reciprocal h and a residual correction give s within
// one ulp.  Rounding test: with s+ and s- the neighbours of s, sqrt(u) lies
// above the midpoint of s and s+ iff d = u - s^2 > s (s+ - s), and below the
// midpoint of s- and s iff d <= -s (s - s-) (the squared half ulps are
// below the grain of d; s (s+ - s) is exact and has fewer than 53
// significant bits of that grain, so comparing the fma-rounded d with it
// decides the same way as the exact d).
__device__ __forceinline__ double nsqrt(double u) {
    const double y = __builtin_amdgcn_rsq(u);
    double s = u * y, h = 0.5 * y;
    const double r = fma(-s, h, 0.5);
    s = fma(s, r, s);
    h = fma(h, r, h);
    double d = fma(-s, s, u);
    s = fma(d, h, s);
    const double su = step_bits(s, true), sd = step_bits(s, false);
    d = fma(-s, s, u);
    const double up = s * (su - s), dn = s * (s - sd);
    const double t = d > up ? su : s;
    return d <= -dn ? sd : t;
}

// 1/sqrt(u) and sqrt(u) for a positive finite u, normal or subnormal: u is
// scaled by an even power of two into [0.5, 2), where the reciprocal square
// root seed is refined by two coupled Newton steps (the root and half its
// reciprocal) and the root by a final residual correction; the scaling is
// undone exactly.  No branch.
__device__ __forceinline__ void rsqrt_sqrt(double u, double &rs, double &d) {
    const int e = __builtin_amdgcn_frexp_exp(u) >> 1;
    const double v = ldexp(u, -2 * e);
    const double y = __builtin_amdgcn_rsq(v);
    double s = v * y, h = 0.5 * y;
    double r = fma(-s, h, 0.5);
    s = fma(s, r, s);
    h = fma(h, r, h);
    r = fma(-s, h, 0.5);
    s = fma(s, r, s);
    h = fma(h, r, h);
    const double c = fma(-s, s, v);
    s = fma(c, h, s);
    rs = ldexp(h, 1 - e);
    d = ldexp(s, e);
}

// 64-bit DPP move within a row of 16 lanes (bound_ctrl: no old value).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(u & 0xffffffffu), CTRL, 0xF, 0xF, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum over the 16 lanes of a DPP row, identical in every lane: each level
// adds the value of a partner lane whose own partial sum is the mirror image
// (lane l <-> l^1, l^2, 7-l, 15-l within the row), so both lanes add the
// same two numbers.  The 16 lanes of the row must be active.
__device__ __forceinline__ double row_sum(double v) {
    v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);  // row_half_mirror
    v += dpp_mov<0x140>(v);  // row_mirror
    return v;
}

// The same over the 8 lanes of a half row (lane l <-> l^1, l^2, 7-l).
__device__ __forceinline__ double half_row_sum(double v) {
    v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);  // row_half_mirror
    return v;
}

template <int L>
__device__ __forceinline__ double group_sum(double v) {
    static_assert(L == 8 || L == 16, "lane groups of 8 or 16");
    return L == 16 ? row_sum(v) : half_row_sum(v);
}

// Value of v in lane l (wave-uniform l).
__device__ __forceinline__ double lane_value(double v, int l) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffu), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// ----------------------------------------------------- rotations (4.3)-(4.6)
// Trigonometric (t = +1) or hyperbolic (t = -1) rotation parameters from
// ct 2phi, eqs. (4.4)-(4.6): cs_2 cosine, short cuts at sqrt(eps) and
// sqrt(2/eps), |coth 2phi| <= 1 replaced by 5/4.  IEEE operations.
__device__ __forceinline__ void rotation_from_ct2(double ct2, int t, double &tn, double &cs,
                                                  bool &clamped) {
    const double tt = (double)t;
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

// The same from the pivot Gram entries: ct 2phi of eq. (4.3).
__device__ __forceinline__ void rotation(double hpp, double hqq, double hpq, int t, double &tn,
                                         double &cs, bool &clamped) {
    const double tt = (double)t;
    const double h = hqq - tt * hpp;
    rotation_from_ct2(tt * (h / (2.0 * hpq)), t, tn, cs, clamped);
}

// The same formulas, branch-free, with the refined reciprocal and square
// roots.  Valid when h_pp, h_qq and |h_pq| lie in [2^-900, 2^900] and the pair
// rotates (|h_pq| > tol sqrt(h_pp h_qq)): then every intermediate is a
// positive normal number or is discarded by a selection.
__device__ __forceinline__ void rotation_fast(double hpp, double hqq, double hpq, int t, double &tn,
                                              double &cs, bool &clamped) {
    const double tt = (double)t;
    const double h = hqq - tt * hpp;
    const double ct2 = tt * ndiv(h, 2.0 * hpq);
    const double sgn = ct2 < 0.0 ? -1.0 : 1.0;
    double a = fabs(ct2);
    clamped = (t < 0) && (a <= 1.0);
    a = clamped ? 1.25 : a;
    const double root = nsqrt(fma(a, a, tt));
    double act = (a >= kSqrt2OverEps) ? 2.0 * a : a + root;
    act = (t > 0 && a < kSqrtEps) ? a + 1.0 : act;
    tn = sgn * nrcp(act);
    const double c = ndiv(act, nsqrt(fma(act, act, tt)));
    cs = (act >= kSqrt2OverEps) ? 1.0 : c;
}

// h_pp and h_qq in [2^-450, 2^450]: then the relative orthogonality test
// can be taken on squares, and a rotating pair has |h_pq| in [2^-500, 2^450],
// inside the range of rotation_fast.
__device__ __forceinline__ bool in_trig_range(double hpp, double hqq) {
    return fmin(hpp, hqq) >= 0x1p-450 && fmax(hpp, hqq) <= 0x1p450;
}

__device__ __forceinline__ bool in_fast_range(double v) {
    return v >= 0x1p-900 && v <= 0x1p900;
}

}  // namespace

}  // namespace jsvd

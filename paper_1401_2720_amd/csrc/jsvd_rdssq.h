// DRDSSQ (Appendix A): the sum of squares of a vector by parallel
// reductions, safe from overflow and underflow, and the rotation
// parameters of the DDRJAC pairs (Section 4.3.1) built on it.
//
// A result is a pair (j, s) standing for 2^j s (the paper's (s^-2, sigma^2)
// with s^-2 = 2^j), always in the common form of Appendix A: j even and
// 0.5 <= s < 2, or (0, 0) for a zero vector; the norm is 2^(j/2) sqrt(s),
// and ordering pairs lexicographically orders the norms.  NaN or infinite
// elements give s = NaN.
//
// The procedure: M = max |x_i| and m = the smallest non-zero |x_i| by
// reductions; the elements inside the safe range [t_lo, t_hi] are summed
// unscaled, those above t_hi after scaling by 2^l (the largest l with
// 2^l M <= t_hi), those below t_lo after scaling by 2^k (the smallest k with
// 2^k m >= t_lo); each partial sum that the range of [m, M] calls for is
// reduced, put into the common form, and the partial sums are added
// smallest first, the smaller addend rescaled to the larger one's scale.
// t_lo = RU(sqrt(mu / (1 - eps))) = 2^-511 (1 + 2^-52) for every length;
// t_hi = RZ(sqrt(nu / delta_n)) depends on ceil(lg n) and is computed on the
// host (rdssq_t_hi).
#pragma once

#include "jsvd_blocked.h"

namespace jsvd {

namespace {

constexpr double kRdssqTlo = 0x1.0000000000001p-511;

__device__ __forceinline__ double hw_max(double v) {
    v = fmax(v, dpp_mov<0xB1>(v));
    v = fmax(v, dpp_mov<0x4E>(v));
    v = fmax(v, dpp_mov<0x141>(v));
    v = fmax(v, dpp_mov<0x140>(v));
    const long long x = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_ds_swizzle((int)x, 0x401F);
    const int hi = __builtin_amdgcn_ds_swizzle((int)(x >> 32), 0x401F);
    return fmax(v, __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double hw_min(double v) {
    v = fmin(v, dpp_mov<0xB1>(v));
    v = fmin(v, dpp_mov<0x4E>(v));
    v = fmin(v, dpp_mov<0x141>(v));
    v = fmin(v, dpp_mov<0x140>(v));
    const long long x = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_ds_swizzle((int)x, 0x401F);
    const int hi = __builtin_amdgcn_ds_swizzle((int)(x >> 32), 0x401F);
    return fmin(v, __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo));
}

// Whether any lane of this lane's half wave has flag set.
__device__ __forceinline__ bool hw_any(bool flag) {
    const unsigned long long b = __ballot(flag);
    const unsigned half = (threadIdx.x & 32) ? (unsigned)(b >> 32) : (unsigned)b;
    return half != 0u;
}

// Exponent f of v = y 2^f, 0.5 <= |y| < 1 (v non-zero, finite; subnormals too).
__device__ __forceinline__ int fexp(double v) { return __builtin_amdgcn_frexp_exp(v); }

// The largest l with 2^l f <= t, and the smallest k with 2^k f >= t (f, t
// positive, t normal): the exponents of f and t are aligned, and the
// significands decide one step.
__device__ __forceinline__ int rdssq_down(double f, double t) {
    const int l = fexp(t) - fexp(f);
    return ldexp(f, l) > t ? l - 1 : l;
}
__device__ __forceinline__ int rdssq_up(double f, double t) {
    const int k = fexp(t) - fexp(f);
    return ldexp(f, k) < t ? k + 1 : k;
}

// (j, s) into the common form: s = 2^e y with 1 <= y < 2 becomes 2^e' y
// with e' = -(e mod 2), j grows by e - e'.
__device__ __forceinline__ void common_form(int &j, double &s) {
    if (!(s > 0.0) || !(s <= 0x1.fffffffffffffp+1023)) return;
    const int e = fexp(s) - 1;
    const int ep = -(e & 1);
    j += e - ep;
    s = ldexp(s, ep - e);
}

// The sum of two pairs in common form: the lexicographically smaller one
// rescaled to the other's scale and added.
__device__ __forceinline__ void add_pairs(int ja, double a, int jb, double b, int &j, double &s) {
    const bool sw = ja > jb || (ja == jb && a > b);
    const int jl = sw ? jb : ja, jh = sw ? ja : jb;
    const double sl = sw ? b : a, sh = sw ? a : b;
    j = jh;
    s = ldexp(sl, jl - jh) + sh;
}

// What the range [mn, mx] of the non-zero magnitudes asks for: the scale
// exponents of the large (l) and small (k) parts and which parts exist.
struct RdssqPlan {
    bool p0, p1, p2;  // below t_lo, unscaled, above t_hi
    int k, l;
};

__device__ __forceinline__ RdssqPlan rdssq_plan(double mx, double mn, double t_hi) {
    RdssqPlan p;
    p.p1 = mn <= t_hi && mx >= kRdssqTlo;
    p.p2 = mx > t_hi;
    p.p0 = mn < kRdssqTlo;
    p.l = p.p2 ? rdssq_down(mx, t_hi) : 0;
    p.k = p.p0 ? rdssq_up(mn, kRdssqTlo) : 0;
    return p;
}

// Adds v^2 (scaled as the plan says) to the partial sum of its part.
__device__ __forceinline__ void rdssq_acc(double v, double t_hi, const RdssqPlan &p, double &s0,
                                          double &s1, double &s2) {
    const double a = fabs(v);
    if (a >= kRdssqTlo && a <= t_hi) {
        s1 = fma(v, v, s1);
    } else if (a > t_hi) {
        const double y = ldexp(v, p.l);
        s2 = fma(y, y, s2);
    } else if (a > 0.0) {
        const double y = ldexp(v, p.k);
        s0 = fma(y, y, s0);
    }
}

// Compare-and-swap of two (j, s) pairs into ascending lexicographic order.
__device__ __forceinline__ void order_pairs(int &ja, double &a, int &jb, double &b) {
    const bool sw = jb < ja || (jb == ja && b < a);
    const int tj = sw ? jb : ja;
    jb = sw ? ja : jb;
    ja = tj;
    const double ts = sw ? b : a;
    b = sw ? a : b;
    a = ts;
}

// The reduced partial sums (those the plan has) into one pair: each into
// the common form, then added smallest first.  Absent parts carry the
// largest j and sort last.
__device__ __forceinline__ void rdssq_combine(const RdssqPlan &p, double s0, double s1, double s2,
                                              int &j, double &s) {
    constexpr int kAbsent = 0x7fffffff;
    int j1 = p.p1 ? 0 : kAbsent, j2 = p.p2 ? -2 * p.l : kAbsent, j0 = p.p0 ? -2 * p.k : kAbsent;
    if (p.p1) common_form(j1, s1);
    if (p.p2) common_form(j2, s2);
    if (p.p0) common_form(j0, s0);
    order_pairs(j1, s1, j2, s2);
    order_pairs(j1, s1, j0, s0);
    order_pairs(j2, s2, j0, s0);
    j = j1;
    s = s1;
    if (j2 != kAbsent) {
        add_pairs(j, s, j2, s2, j, s);
        common_form(j, s);
    }
    if (j0 != kAbsent) {
        add_pairs(j, s, j0, s0, j, s);
        common_form(j, s);
    }
}

// DRDSSQ of a vector spread over the 32 lanes of a half wave: lane x holds
// elements x + 32 r in v[r], r < R (zero past the end).  Every lane gets
// the same (j, s).
template <int R>
__device__ __forceinline__ void hw_rdssq(const double (&v)[R], double t_hi, int &j, double &s) {
    double mx = 0.0, mn = INFINITY;
    bool bad = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double a = fabs(v[r]);
        bad = bad || !(a <= 0x1.fffffffffffffp+1023);
        mx = fmax(mx, a);
        mn = a > 0.0 ? fmin(mn, a) : mn;
    }
    mx = hw_max(mx);
    mn = hw_min(mn);
    j = 0;
    s = 0.0;
    if (hw_any(bad)) {
        s = __builtin_nan("");
        return;
    }
    if (mx == 0.0) return;
    const RdssqPlan p = rdssq_plan(mx, mn, t_hi);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) rdssq_acc(v[r], t_hi, p, s0, s1, s2);
    if (p.p0) s0 = hw_sum(s0);
    if (p.p1) s1 = hw_sum(s1);
    if (p.p2) s2 = hw_sum(s2);
    rdssq_combine(p, s0, s1, s2, j, s);
}

// The same for x[0 .. len) in memory, lane x taking x, x + 32, ...
__device__ __forceinline__ void hw_rdssq_mem(const double *x, int len, double t_hi, int &j,
                                             double &s) {
    const int lane = threadIdx.x & 31;
    double mx = 0.0, mn = INFINITY;
    bool bad = false;
    for (int i = lane; i < len; i += 32) {
        const double a = fabs(x[i]);
        bad = bad || !(a <= 0x1.fffffffffffffp+1023);
        mx = fmax(mx, a);
        mn = a > 0.0 ? fmin(mn, a) : mn;
    }
    mx = hw_max(mx);
    mn = hw_min(mn);
    j = 0;
    s = 0.0;
    if (hw_any(bad)) {
        s = __builtin_nan("");
        return;
    }
    if (mx == 0.0) return;
    const RdssqPlan p = rdssq_plan(mx, mn, t_hi);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int i = lane; i < len; i += 32) rdssq_acc(x[i], t_hi, p, s0, s1, s2);
    if (p.p0) s0 = hw_sum(s0);
    if (p.p1) s1 = hw_sum(s1);
    if (p.p2) s2 = hw_sum(s2);
    rdssq_combine(p, s0, s1, s2, j, s);
}

// DRDSSQ of x[0 .. len) by the NT threads of a workgroup (NT a power of
// two, all threads calling): per-thread maxima, minima and partial sums over
// the elements tid, tid + NT, ..., reduced by a fixed tree in red (3 NT
// doubles of LDS).  Every thread gets the same (j, s).
template <int NT>
__device__ __forceinline__ void wg_rdssq(const double *x, int64_t len, double t_hi, double *red,
                                         int &j, double &s) {
    const int tid = threadIdx.x;
    double mx = 0.0, mn = INFINITY, bad = 0.0;
    for (int64_t i = tid; i < len; i += NT) {
        const double a = fabs(x[i]);
        bad = (a <= 0x1.fffffffffffffp+1023) ? bad : 1.0;
        mx = fmax(mx, a);
        mn = a > 0.0 ? fmin(mn, a) : mn;
    }
    red[tid] = mx;
    red[NT + tid] = mn;
    red[2 * NT + tid] = bad;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if (tid < h) {
            red[tid] = fmax(red[tid], red[tid + h]);
            red[NT + tid] = fmin(red[NT + tid], red[NT + tid + h]);
            red[2 * NT + tid] = fmax(red[2 * NT + tid], red[2 * NT + tid + h]);
        }
        __syncthreads();
    }
    mx = red[0];
    mn = red[NT];
    bad = red[2 * NT];
    __syncthreads();
    j = 0;
    s = 0.0;
    if (bad != 0.0) {
        s = __builtin_nan("");
        return;
    }
    if (mx == 0.0) return;
    const RdssqPlan p = rdssq_plan(mx, mn, t_hi);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t i = tid; i < len; i += NT) rdssq_acc(x[i], t_hi, p, s0, s1, s2);
    red[tid] = s0;
    red[NT + tid] = s1;
    red[2 * NT + tid] = s2;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if (tid < h) {
            red[tid] += red[tid + h];
            red[NT + tid] += red[NT + tid + h];
            red[2 * NT + tid] += red[2 * NT + tid + h];
        }
        __syncthreads();
    }
    s0 = red[0];
    s1 = red[NT];
    s2 = red[2 * NT];
    __syncthreads();
    rdssq_combine(p, s0, s1, s2, j, s);
}

// ceil(lg n) for n >= 1.
__device__ __forceinline__ int ceil_lg(int64_t n) {
    return n <= 1 ? 0 : 64 - __clzll((unsigned long long)(n - 1));
}

// The norm 2^(j/2) sqrt(s) as a double (infinite or subnormal when it
// leaves the range).
__device__ __forceinline__ double rdssq_norm(int j, double s) {
    return s > 0.0 ? ldexp(sqrt(s), j / 2) : s;
}

// A DDRJAC pair (Section 4.3.1): from the DRDSSQ pairs (ja, sa), (jb, sb)
// of g_p and g_q and d = (2^(-ja/2) g_p)^T (2^(-jb/2) g_q), the cosine of
// the angle xi = d / (sqrt(sa) sqrt(sb)), the relative orthogonality test
// |xi| <= tol (the test of subphase 2 divided by the norms), and ct 2phi
// of (4.3) in the norm ratio rho = ||g_q|| / ||g_p||: t (rho - t / rho) /
// (2 xi).  Returns whether the pair rotates; tn and cs as (4.5)-(4.6).
__device__ __forceinline__ bool ddrjac_pair(int ja, double sa, int jb, double sb, double d,
                                            double tol, int t, double &tn, double &cs,
                                            bool &clamped) {
    clamped = false;
    if (!(sa > 0.0) || !(sb > 0.0)) return false;
    const double na = sqrt(sa), nb = sqrt(sb);
    const double xi = d / (na * nb);
    if (!(fabs(xi) > tol)) return false;
    const double tt = (double)t;
    const double rho = ldexp(nb / na, (jb - ja) / 2);
    const double ct2 = tt * ((rho - tt / rho) / (2.0 * xi));
    rotation_from_ct2(ct2, t, tn, cs, clamped);
    return true;
}

}  // namespace

}  // namespace jsvd

/*
 * Oracle: plain, slow, sequential CPU implementation of the one-sided
 * (Hestenes) Jacobi SVD and hyperbolic SVD.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no source with the GPU library.
 *
 * What it follows (Novakovic, "A hierarchically blocked Jacobi SVD
 * algorithm for single and multiple GPUs"):
 *   - Section 2, eqs. (2.3)-(2.5): a pivot pair of columns (g_p, g_q) is
 *     orthogonalised by a 2x2 transformation that diagonalises the 2x2 Gram
 *     matrix [h_pp h_pq; h_pq h_qq]; at convergence G V = U Sigma and the
 *     singular values are the column norms.
 *   - Section 2, eq. (2.10) and Section 4.3 subphase 4: for the hyperbolic
 *     SVD with J = diag(I_{n+}, -I), a pair with p < n+ <= q (zero-based)
 *     gets a hyperbolic rotation, every other pair a trigonometric one.
 *   - Section 4.3 subphase 2: the relative orthogonality test
 *     |h_pq| < c(eps) sqrt(h_pp) sqrt(h_qq), c(eps) = eps * sqrt(nhat).
 *     Reading used here: nhat = m (the length of the columns), eps = 2^-53
 *     (the unit roundoff stated in Appendix A), and "<=" instead of "<" so
 *     that a pair containing a zero column is skipped rather than divided
 *     by zero.
 *   - Section 4.3.1, eqs. (4.1)-(4.6): rotation parameters from the adapted
 *     Rutishauser formulas, the cs_2 cosine, the sqrt(eps) and sqrt(2/eps)
 *     short cuts, and the substitution |coth 2phi| := 5/4 when it is
 *     numerically not above 1 (reading: applied when |coth 2phi| <= 1,
 *     keeping its sign).
 *   - Pivot order: the sequential row-cyclic strategy R_n of Section 3
 *     (pairs (1,2),(1,3),...,(1,n),(2,3),...), repeated sweep after sweep
 *     until a whole sweep performs no rotation.  A second entry point visits
 *     the same pairs in round-robin (circle-method) rounds, each round's
 *     disjoint pairs in parallel with OpenMP; it is used only to time the
 *     CPU on large inputs and as a second valid ordering.
 *
 * Every dot product is accumulated in index order with fma.  Compile with
 * -ffp-contract=off so that no other contraction changes the rounding.
 * Define ORACLE_LONG_DOUBLE to get the same method in x87 extended
 * precision (symbols suffixed _ld), used as a brute-force reference.
 *
 * The end of the file adds DRDSSQ (Appendix A) and the DDRJAC pairs of
 * Section 4.3.1, in IEEE double only.
 *
 * Parity pins (see tests/test_oracle_*.py): closed-form 2x2 SVD, prescribed
 * spectra, LAPACK normwise agreement, extended-precision agreement, exact
 * rational evaluation of rotation orthogonality, and the invariants of the
 * SVD and of the hyperbolic SVD.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_LONG_DOUBLE
typedef long double real;
#define R_SQRT sqrtl
#define R_FMA fmal
#define R_FABS fabsl
#define R_LDEXP ldexpl
#define R_MANT_DIG 64
#define NAME(x) x##_ld
#else
typedef double real;
#define R_SQRT sqrt
#define R_FMA fma
#define R_FABS fabs
#define R_LDEXP ldexp
#define R_MANT_DIG 53
#define NAME(x) x
#endif

/* eps = 2^-p, the unit roundoff of round-to-nearest (Appendix A). */
static real unit_roundoff(void) { return R_LDEXP((real)1, -R_MANT_DIG); }

static real dot(int64_t m, const real *x, const real *y)
{
    real s = 0;
    for (int64_t i = 0; i < m; ++i)
        s = R_FMA(x[i], y[i], s);
    return s;
}

/*
 * Eqs. (4.4)-(4.6) from ct 2phi, with t = +1 (trigonometric) or t = -1
 * (hyperbolic): tn (tan or tanh) and cs (cos or cosh, the cs_2 formula).
 * Returns 1 when |coth 2phi| was substituted by 5/4.
 */
static int params_from_ct2(real ct2, int t, real *tn, real *cs)
{
    const real eps = unit_roundoff();
    const real sqrt_eps = R_SQRT(eps);
    const real sqrt_2_eps = R_SQRT(2 / eps);
    const real tt = (real)t;
    int flags = 0;
    real sgn = (ct2 < 0) ? -1 : 1;
    real a = R_FABS(ct2);
    if (t < 0 && a <= 1) { /* |coth 2phi| numerically 1: substitute 5/4 */
        a = (real)1.25;
        flags |= 1;
    }
    /* (4.4) with the two short cuts. */
    real act;
    if (t > 0 && a < sqrt_eps)
        act = a + 1;
    else if (a >= sqrt_2_eps)
        act = 2 * a;
    else
        act = a + R_SQRT(R_FMA(a, a, tt));
    /* (4.5): tn = sgn(ct 2phi) * rcp(|ct phi|). */
    *tn = sgn * (1 / act);
    /* (4.6), cs_2, with cs = 1 when |ct phi| >= sqrt(2/eps). */
    if (act >= sqrt_2_eps)
        *cs = 1;
    else
        *cs = act / R_SQRT(R_FMA(act, act, tt));
    return flags;
}

/*
 * Rotation parameters, eqs. (4.3)-(4.6), from the 2x2 Gram entries.
 */
int NAME(orc_rotation)(real hpp, real hqq, real hpq, int t, real *tn, real *cs)
{
    const real tt = (real)t;
    /* (4.3): h = h_qq - t h_pp;  ct 2phi = t h / (2 h_pq). */
    real h = hqq - tt * hpp;
    real ct2 = tt * (h / (2 * hpq));
    return params_from_ct2(ct2, t, tn, cs);
}

/* (4.4)-(4.6) from a given |ct 2phi| (the experiment of Appendix B). */
void NAME(orc_rot_params)(int64_t count, const real *abs_ct2, int t, real *tn, real *cs)
{
    for (int64_t i = 0; i < count; ++i)
        params_from_ct2(abs_ct2[i], t, tn + i, cs + i);
}

/*
 * Apply the pair transformation to columns x (= p) and y (= q) of length
 * len: (4.1) for t = +1, (4.2) for t = -1; the final multiplication by cs is
 * omitted when cs == 1.
 */
static void apply_pair(int64_t len, real *x, real *y, real tn, real cs, int t)
{
    const real mtn = (t > 0) ? -tn : tn; /* coefficient of y in the new x */
    if (cs == 1) {
        for (int64_t i = 0; i < len; ++i) {
            real xi = x[i], yi = y[i];
            x[i] = R_FMA(mtn, yi, xi);
            y[i] = R_FMA(tn, xi, yi);
        }
    } else {
        for (int64_t i = 0; i < len; ++i) {
            real xi = x[i], yi = y[i];
            x[i] = cs * R_FMA(mtn, yi, xi);
            y[i] = cs * R_FMA(tn, xi, yi);
        }
    }
}

/* stats layout (int64): 0 sweeps, 1 rotations, 2 proper rotations,
 * 3 coth substitutions, 4 converged (0/1). */
enum { ST_SWEEPS, ST_ROT, ST_PROPER, ST_CLAMP, ST_CONV, ST_N };

/* One pivot pair (p < q).  Returns 0 = skipped, 1 = rotated, 3 = rotated and
 * proper; bit 2 (4) = coth substituted. */
static int do_pair(int64_t m, int64_t n, real *G, int64_t ldg, real *V, int64_t ldv,
                   int64_t n_plus, real tol, int64_t p, int64_t q)
{
    real *gp = G + p * ldg, *gq = G + q * ldg;
    real hpp = dot(m, gp, gp);
    real hqq = dot(m, gq, gq);
    real hpq = dot(m, gp, gq);
    /* Section 4.3, subphase 2 (reading: <= skips). */
    if (R_FABS(hpq) <= tol * R_SQRT(hpp) * R_SQRT(hqq))
        return 0;
    /* Section 4.3, subphase 4: hyperbolic iff p < n+ <= q (zero-based). */
    int t = (p < n_plus && q >= n_plus) ? -1 : 1;
    real tn, cs;
    int fl = NAME(orc_rotation)(hpp, hqq, hpq, t, &tn, &cs);
    apply_pair(m, gp, gq, tn, cs, t);
    if (V)
        apply_pair(n, V + p * ldv, V + q * ldv, tn, cs, t);
    return 1 | ((cs != 1) ? 2 : 0) | ((fl & 1) ? 4 : 0);
}

static void init_identity(int64_t n, real *V, int64_t ldv)
{
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            V[i + j * ldv] = (i == j) ? 1 : 0;
}

/*
 * Cyclic one-sided Jacobi, row-cyclic order.  G (m x n, column-major,
 * leading dimension ldg) is overwritten by G V = U Sigma.  V (n x n, ldv)
 * receives the accumulated transformations (may be NULL).  n_plus = n gives
 * the ordinary SVD.  Returns 0 when converged, 1 otherwise.
 */
int NAME(orc_gesvj)(int64_t m, int64_t n, real *G, int64_t ldg, real *V, int64_t ldv,
                    int64_t n_plus, int32_t max_sweeps, int64_t *stats)
{
    const real tol = unit_roundoff() * R_SQRT((real)m);
    int64_t st[ST_N] = {0};
    if (V)
        init_identity(n, V, ldv);
    for (int32_t sw = 0; sw < max_sweeps; ++sw) {
        int64_t rot = 0;
        for (int64_t p = 0; p + 1 < n; ++p)
            for (int64_t q = p + 1; q < n; ++q) {
                int r = do_pair(m, n, G, ldg, V, ldv, n_plus, tol, p, q);
                if (r & 1) {
                    ++rot;
                    st[ST_PROPER] += (r >> 1) & 1;
                    st[ST_CLAMP] += (r >> 2) & 1;
                }
            }
        st[ST_SWEEPS] = sw + 1;
        st[ST_ROT] += rot;
        if (rot == 0) {
            st[ST_CONV] = 1;
            break;
        }
    }
    if (stats)
        memcpy(stats, st, sizeof st);
    return st[ST_CONV] ? 0 : 1;
}

/*
 * Same method, pairs visited in round-robin rounds (circle method on
 * ne = n rounded up to even; the padding index is a dummy and its pairs are
 * skipped).  The pairs of one round are disjoint and are processed in
 * parallel; the result does not depend on the thread count.
 * max_rounds_total > 0 stops after that many rounds in total (used to time a
 * bounded sample); 0 = no such limit.
 */
int NAME(orc_gesvj_rr)(int64_t m, int64_t n, real *G, int64_t ldg, real *V, int64_t ldv,
                       int64_t n_plus, int32_t max_sweeps, int64_t max_rounds_total,
                       int64_t *stats)
{
    const real tol = unit_roundoff() * R_SQRT((real)m);
    const int64_t ne = n + (n & 1);
    const int64_t half = ne / 2;
    int64_t st[ST_N] = {0};
    int64_t rounds_done = 0;
    if (V)
        init_identity(n, V, ldv);
    for (int32_t sw = 0; sw < max_sweeps; ++sw) {
        int64_t rot = 0, proper = 0, clamp = 0;
        for (int64_t r = 0; r + 1 < ne; ++r) {
            if (max_rounds_total > 0 && rounds_done >= max_rounds_total)
                goto out;
#pragma omp parallel for schedule(static) reduction(+ : rot, proper, clamp)
            for (int64_t k = 0; k < half; ++k) {
                int64_t a, b;
                if (k == 0) {
                    a = ne - 1;
                    b = r;
                } else {
                    a = (r + k) % (ne - 1);
                    b = (r + (ne - 1) - k) % (ne - 1);
                }
                int64_t p = a < b ? a : b, q = a < b ? b : a;
                if (q >= n)
                    continue;
                int res = do_pair(m, n, G, ldg, V, ldv, n_plus, tol, p, q);
                if (res & 1) {
                    ++rot;
                    proper += (res >> 1) & 1;
                    clamp += (res >> 2) & 1;
                }
            }
            ++rounds_done;
        }
        st[ST_SWEEPS] = sw + 1;
        st[ST_ROT] += rot;
        st[ST_PROPER] += proper;
        st[ST_CLAMP] += clamp;
        if (rot == 0) {
            st[ST_CONV] = 1;
            break;
        }
    }
out:
    if (stats)
        memcpy(stats, st, sizeof st);
    return st[ST_CONV] ? 0 : 1;
}

/*
 * Singular values as column norms, eq. (2.5): s_i = ||g_i||_2, u_i = g_i/s_i
 * (u_i = 0 when s_i = 0).  G is overwritten by U.
 */
void NAME(orc_colnorms)(int64_t m, int64_t n, real *G, int64_t ldg, real *s)
{
    for (int64_t j = 0; j < n; ++j) {
        real *g = G + j * ldg;
        real nrm = R_SQRT(dot(m, g, g));
        s[j] = nrm;
        for (int64_t i = 0; i < m; ++i)
            g[i] = (nrm > 0) ? g[i] / nrm : 0;
    }
}

/*
 * Many independent problems (packed, each column-major with lda = m_i and
 * ldv = n_i), each solved by the row-cyclic method and normalised; one
 * problem per thread, dynamic schedule.  S receives the column norms in
 * the unsorted column order.  sweeps[i] receives the sweep count,
 * status[i] 0 = converged, 1 = not.
 */
void NAME(orc_gesvj_many)(int64_t count, const int32_t *m, const int32_t *n,
                          const int64_t *a_off, const int64_t *s_off, const int64_t *v_off,
                          real *A, real *S, real *V, int32_t max_sweeps,
                          int32_t *sweeps, int32_t *status)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < count; ++i) {
        int64_t st[ST_N];
        int rc = NAME(orc_gesvj)(m[i], n[i], A + a_off[i], m[i], V ? V + v_off[i] : NULL, n[i],
                                 n[i], max_sweeps, st);
        NAME(orc_colnorms)(m[i], n[i], A + a_off[i], m[i], S + s_off[i]);
        sweeps[i] = (int32_t)st[ST_SWEEPS];
        status[i] = rc;
    }
}

/* Threads the OpenMP entry points use (for reporting timings). */
int NAME(orc_num_threads)(void) { return omp_get_max_threads(); }

#ifndef ORACLE_LONG_DOUBLE
/*
 * ------------------------------------------------------------------------
 * Appendix A: DRDSSQ, the scaled sum of squares, and the DDRJAC rotations of
 * Section 4.3.1 (the one-sided Jacobi method whose pair parameters come
 * from overflow- and underflow-safe column norms).  IEEE double only: the
 * thresholds are those of the double format.
 *
 * A result is a pair (j, s) that stands for 2^j s = the sum of squares
 * (the paper's (s^-2, sigma^2) with s^-2 = 2^j); the norm is 2^(j/2) sqrt(s).
 * Every result is returned in the common form of Appendix A: j even and
 * 0.5 <= s < 2 (s = 0, j = 0 for a zero vector).  Reading used: the paper
 * puts only partial sums into that form before adding them; normalising the
 * final pair as well is an exact rescaling that makes the representation
 * unique, and leaves the norm's value unchanged.
 *
 * t_lo and t_hi are the safe bounds of Appendix A rounded inwards to
 * doubles, t_lo = RU(sqrt(mu / gamma)) and t_hi = RZ(sqrt(nu / delta_n)),
 * computed exactly by the Python side of the oracle and passed in; t_hi
 * depends on the vector length through ceil(lg n), so the many-column entry
 * points take a table indexed by it.
 * ------------------------------------------------------------------------
 */

/* (j, s) -> the common form: s = 2^e y with 1 <= y < 2 becomes 2^e' y with
 * e' = -(e mod 2) in {-1, 0}, and j grows by e - e' (even). */
static void common_form(int *j, double *s)
{
    if (!(*s > 0))
        return;
    int f;
    double y = frexp(*s, &f); /* s = y 2^f, 0.5 <= y < 1 */
    int e = f - 1;            /* s = (2y) 2^e, 1 <= 2y < 2 */
    int ep = -(((e % 2) + 2) % 2);
    *j += e - ep;
    *s = ldexp(2 * y, ep);
}

/* Sum of two pairs in common form: the smaller one (lexicographically on
 * (j, s)) is rescaled to the scale of the larger and added to it. */
static void add_pairs(int ja, double a, int jb, double b, int *j, double *s)
{
    if (ja > jb || (ja == jb && a > b)) {
        int ti = ja;
        ja = jb;
        jb = ti;
        double td = a;
        a = b;
        b = td;
    }
    *j = jb;
    *s = ldexp(a, ja - jb) + b;
}

/* ceil(lg n) for n >= 1. */
static int ceil_lg(int64_t n)
{
    int l = 0;
    while (((int64_t)1 << l) < n)
        ++l;
    return l;
}

/* The largest l with 2^l f <= t (f, t positive; t normal). */
static int scale_down_exp(double f, double t)
{
    int l = ilogb(t) - ilogb(f);
    return (ldexp(f, l) > t) ? l - 1 : l;
}

/* The smallest k with 2^k f >= t (f, t positive; t normal). */
static int scale_up_exp(double f, double t)
{
    int k = ilogb(t) - ilogb(f);
    return (ldexp(f, k) < t) ? k + 1 : k;
}

/*
 * DRDSSQ (Appendix A) of x[0], x[inc], ..., x[(n-1) inc], no special values.
 * Steps: M = max |x_i| (zero vector: (0, 0)); m = the smallest non-zero
 * |x_i|; the elements in [t_lo, t_hi] are summed unscaled, those above t_hi
 * scaled by 2^l (the largest l with 2^l M <= t_hi), those below t_lo scaled
 * by 2^k (the smallest k with 2^k m >= t_lo); each non-zero partial sum
 * (2^-2l, .), (1, .), (2^-2k, .) is put into the common form and the
 * partial sums are added smallest first.  *parts receives a mask of the
 * partial sums formed (1: below t_lo, 2: unscaled, 4: above t_hi).  Partial
 * sums are accumulated in index order with fma.
 */
void orc_rdssq(int64_t n, const double *x, int64_t inc, double t_lo, double t_hi, int *j_out,
               double *s_out, int *parts)
{
    double M = 0, mn = 0;
    for (int64_t i = 0; i < n; ++i) {
        double a = fabs(x[i * inc]);
        if (a > M)
            M = a;
        if (a > 0 && (mn == 0 || a < mn))
            mn = a;
    }
    *j_out = 0;
    *s_out = 0;
    if (parts)
        *parts = 0;
    if (M == 0)
        return;
    int js[3], cnt = 0, mask = 0;
    double ss[3];
    if (mn <= t_hi && M >= t_lo) { /* [m, M] meets [t_lo, t_hi] */
        double s = 0;
        for (int64_t i = 0; i < n; ++i) {
            double v = x[i * inc], a = fabs(v);
            if (a >= t_lo && a <= t_hi)
                s = fma(v, v, s);
        }
        js[cnt] = 0;
        ss[cnt++] = s;
        mask |= 2;
    }
    if (M > t_hi) {
        int l = scale_down_exp(M, t_hi);
        double s = 0;
        for (int64_t i = 0; i < n; ++i) {
            double v = x[i * inc];
            if (fabs(v) > t_hi) {
                double y = ldexp(v, l);
                s = fma(y, y, s);
            }
        }
        js[cnt] = -2 * l;
        ss[cnt++] = s;
        mask |= 4;
    }
    if (mn < t_lo) {
        int k = scale_up_exp(mn, t_lo);
        double s = 0;
        for (int64_t i = 0; i < n; ++i) {
            double v = x[i * inc];
            if (v != 0 && fabs(v) < t_lo) {
                double y = ldexp(v, k);
                s = fma(y, y, s);
            }
        }
        js[cnt] = -2 * k;
        ss[cnt++] = s;
        mask |= 1;
    }
    for (int i = 0; i < cnt; ++i)
        common_form(&js[i], &ss[i]);
    /* the two smallest first: sort the (at most three) pairs ascending */
    for (int a = 0; a < cnt; ++a)
        for (int b = a + 1; b < cnt; ++b)
            if (js[b] < js[a] || (js[b] == js[a] && ss[b] < ss[a])) {
                int ti = js[a];
                js[a] = js[b];
                js[b] = ti;
                double td = ss[a];
                ss[a] = ss[b];
                ss[b] = td;
            }
    int j = js[0];
    double s = ss[0];
    for (int i = 1; i < cnt; ++i) {
        add_pairs(j, s, js[i], ss[i], &j, &s);
        common_form(&j, &s);
    }
    *j_out = j;
    *s_out = s;
    if (parts)
        *parts = mask;
}

/* The norm 2^(j/2) sqrt(s) of a DRDSSQ result, as a double (may overflow
 * to infinity or round to a subnormal). */
static double rdssq_norm(int j, double s) { return ldexp(sqrt(s), j / 2); }

/*
 * One pivot pair by DDRJAC: the norms of g_p and g_q by DRDSSQ, the cosine
 * of their angle xi = (g_p / ||g_p||)^T (g_q / ||g_q||) from the columns
 * scaled by the powers of two of their norms, the relative orthogonality
 * test |xi| <= tol (the test of Section 4.3, subphase 2, divided by the
 * norms), and ct 2phi of (4.3) written in the ratio rho = ||g_q|| / ||g_p||:
 * h_qq - t h_pp over 2 h_pq is (rho - t / rho) / (2 xi).  Then (4.4)-(4.6)
 * and (4.1)/(4.2) as in the ordinary method.
 */
static int do_pair_ddrjac(int64_t m, int64_t n, double *G, int64_t ldg, double *V, int64_t ldv,
                          int64_t n_plus, double tol, int64_t p, int64_t q, double t_lo,
                          double t_hi)
{
    double *gp = G + p * ldg, *gq = G + q * ldg;
    int ja, jb;
    double sa, sb;
    orc_rdssq(m, gp, 1, t_lo, t_hi, &ja, &sa, NULL);
    orc_rdssq(m, gq, 1, t_lo, t_hi, &jb, &sb, NULL);
    if (sa == 0 || sb == 0)
        return 0;
    double d = 0;
    for (int64_t i = 0; i < m; ++i)
        d = fma(ldexp(gp[i], -ja / 2), ldexp(gq[i], -jb / 2), d);
    double na = sqrt(sa), nb = sqrt(sb);
    double xi = d / (na * nb);
    if (fabs(xi) <= tol)
        return 0;
    int t = (p < n_plus && q >= n_plus) ? -1 : 1;
    double tt = (double)t;
    double rho = ldexp(nb / na, (jb - ja) / 2);
    double ct2 = tt * ((rho - tt / rho) / (2 * xi));
    double tn, cs;
    int fl = params_from_ct2(ct2, t, &tn, &cs);
    apply_pair(m, gp, gq, tn, cs, t);
    if (V)
        apply_pair(n, V + p * ldv, V + q * ldv, tn, cs, t);
    return 1 | ((cs != 1) ? 2 : 0) | ((fl & 1) ? 4 : 0);
}

/*
 * The row-cyclic one-sided Jacobi (H)SVD of orc_gesvj with DDRJAC pairs;
 * t_hi is the bound for vectors of length m.  Same arguments and result
 * otherwise.
 */
int orc_gesvj_ddrjac(int64_t m, int64_t n, double *G, int64_t ldg, double *V, int64_t ldv,
                     int64_t n_plus, int32_t max_sweeps, int64_t *stats, double t_lo,
                     double t_hi)
{
    const double tol = unit_roundoff() * sqrt((double)m);
    int64_t st[ST_N] = {0};
    if (V)
        init_identity(n, V, ldv);
    for (int32_t sw = 0; sw < max_sweeps; ++sw) {
        int64_t rot = 0;
        for (int64_t p = 0; p + 1 < n; ++p)
            for (int64_t q = p + 1; q < n; ++q) {
                int r = do_pair_ddrjac(m, n, G, ldg, V, ldv, n_plus, tol, p, q, t_lo, t_hi);
                if (r & 1) {
                    ++rot;
                    st[ST_PROPER] += (r >> 1) & 1;
                    st[ST_CLAMP] += (r >> 2) & 1;
                }
            }
        st[ST_SWEEPS] = sw + 1;
        st[ST_ROT] += rot;
        if (rot == 0) {
            st[ST_CONV] = 1;
            break;
        }
    }
    if (stats)
        memcpy(stats, st, sizeof st);
    return st[ST_CONV] ? 0 : 1;
}

/*
 * Singular values and U from the final columns by DRDSSQ: s_j = 2^(j/2)
 * sqrt(s), u = (2^(-j/2) g) / sqrt(s) (zero for a zero column).  exps and
 * ssq (may be NULL) receive the pairs.
 */
void orc_colnorms_rdssq(int64_t m, int64_t n, double *G, int64_t ldg, double *sig, int32_t *exps,
                        double *ssq, double t_lo, double t_hi)
{
    for (int64_t c = 0; c < n; ++c) {
        double *g = G + c * ldg;
        int j;
        double s;
        orc_rdssq(m, g, 1, t_lo, t_hi, &j, &s, NULL);
        sig[c] = (s > 0) ? rdssq_norm(j, s) : 0;
        if (exps)
            exps[c] = j;
        if (ssq)
            ssq[c] = s;
        double r = sqrt(s);
        for (int64_t i = 0; i < m; ++i)
            g[i] = (s > 0) ? ldexp(g[i], -j / 2) / r : 0;
    }
}

/* orc_gesvj_many with DDRJAC pairs and DRDSSQ norms; t_hi_by_lg[L] is the
 * upper bound for vectors with ceil(lg length) = L. */
void orc_gesvj_many_ddrjac(int64_t count, const int32_t *m, const int32_t *n,
                           const int64_t *a_off, const int64_t *s_off, const int64_t *v_off,
                           double *A, double *S, double *V, int32_t max_sweeps, int32_t *sweeps,
                           int32_t *status, double t_lo, const double *t_hi_by_lg)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < count; ++i) {
        int64_t st[ST_N];
        double t_hi = t_hi_by_lg[ceil_lg(m[i])];
        int rc = orc_gesvj_ddrjac(m[i], n[i], A + a_off[i], m[i], V ? V + v_off[i] : NULL, n[i],
                                  n[i], max_sweeps, st, t_lo, t_hi);
        orc_colnorms_rdssq(m[i], n[i], A + a_off[i], m[i], S + s_off[i], NULL, NULL, t_lo, t_hi);
        sweeps[i] = (int32_t)st[ST_SWEEPS];
        status[i] = rc;
    }
}
#endif /* !ORACLE_LONG_DOUBLE */

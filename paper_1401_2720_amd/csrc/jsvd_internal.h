// Internal declarations shared by the host driver and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <utility>
#include <vector>

#include "jsvd.h"

namespace jsvd {

// ---------------------------------------------------------------- strategies
using Pair = std::pair<int, int>;  // zero-based (p, q), p < q
using Step = std::vector<Pair>;
using Table = std::vector<Step>;

int strategy_order(int nb);
bool make_table(int order, int kind, Table &out);
// the pairs of each step reordered for conflict-free LDS access in the inner
// kernels (a permutation within each step; the steps and pairs unchanged)
void order_for_banks(Table &t);
// The step-to-step groups of a strategy table whose consecutive steps
// exchange partners inside groups of two pairs, (a0 a1), (b0 b1) -> pairs of
// {a0, a1} x {b0, b1}: per step s < order - 2 and group, 8 ints {ia, ib, jx,
// jy, a0, b0, 0, 0} (old pairs' indices in step s, new pairs' in step s + 1,
// the blocks of ia and ib that pair jx holds).  False when some step has no
// such structure.
bool make_quads(const Table &t, std::vector<int> &out);

// ------------------------------------------------------------------ counters
// Per-sweep device counters (unsigned 64-bit), reset at the start of a sweep.
enum Counter {
    C_ROT = 0,       // inner rotations
    C_PROPER = 1,    // inner rotations with cs != 1
    C_CLAMP = 2,     // |coth 2phi| substitutions
    C_BREAKDOWN = 3, // non-positive Cholesky pivots
    C_INNER_SW = 4,  // inner sweeps
    C_UPDATES = 5,   // pivot block-pairs with a transformation to apply
    C_NONFINITE = 6, // NaN met in a pivot Gram matrix
    C_COUNT = 8
};

// ------------------------------------------------------- one p-step's launch
struct StepArgs {
    double *G;
    int64_t ldg;
    int64_t m;          // rows of G
    double *V;          // may be null (no V accumulation)
    int64_t ldv;
    int64_t n;          // real columns (and rows of V)
    int w;              // block width
    int n_plus;         // columns [0, n_plus) carry +1 in J
    const int2 *pairs;  // this p-step's pivot block-pairs, zero-based
    int npairs;
    int splits;         // Gram row splits per pair
    int rows_per_split; // multiple of 64
    double *hpart;      // [npairs][splits][bw*bw] partial Gram matrices (row-major tiles)
    double *vprime;     // [npairs][bw*bw] column-major V'_pq
    int *pair_rot;      // [npairs] rotations done in the pair (0 = skip update)
    unsigned long long *counters;
    const unsigned char *inner_tbl;  // [(bw-1)][bw/2][2] zero-based inner pairs
    int max_inner_sweeps;
    int upd_rows;       // rows per update workgroup, multiple of 64
    int upd_chunks_g;   // update workgroups over the rows of G (per pair)
    int upd_chunks_v;   // update workgroups over the rows of V (per pair)
    // the V update of the previous p-step, done by prev_chunks extra
    // workgroups per pivot pair in the inner kernel's launch (0: none)
    const int2 *prev_pairs;
    const double *prev_vprime;
    const int *prev_pair_rot;
    int prev_chunks;
    int prev_rows;      // rows of V per such workgroup
    // scaled mode (badly scaled input): per column c of G an exponent e_c
    // with ||g_c|| in [2^e_c, 2^(e_c+1)); the Gram kernel forms
    // D^-1 H D^-1 (D = diag(2^e_c)), the inner kernel works on R D^-1 and
    // writes the exponents of the transformed columns.  Null: not scaled.
    int *colexp;
    // 2w = 128 (the third blocking level): per pivot pair a 128 x 128
    // scratch for the Cholesky factor R, and the strategy tables of the
    // block method inside the pair (every order up to 256, zero-based pairs)
    double *rscratch;
    // QR shortening (Section 4.2): hpart holds the splits' triangular
    // factors of [G_p G_q] (qrfac kernel) instead of partial Gram matrices,
    // and the inner kernel folds them together in place of the Cholesky
    int qrf;
    // Gram kernel with the two-buffer software pipeline (the grid has at
    // most two workgroups per CU)
    int gram_pf;
    const int *btbl_order;
    const int64_t *btbl_off;
    const unsigned char *btbls;
    // the update fused with the next p-step's Gram kernel: the quads of this
    // p-step (8 ints each: old pairs ia, ib, new pairs jx, jy, blocks a0 of
    // ia and b0 of ib that go to jx, two unused) and the next p-step's pairs
    const int *quads;
    const int2 *next_pairs;
};

hipError_t launch_gram(int bw, const StepArgs &a, hipStream_t s);
hipError_t launch_qrfac(int bw, const StepArgs &a, hipStream_t s);
hipError_t launch_inner(int bw, const StepArgs &a, hipStream_t s);
hipError_t launch_update(int bw, const StepArgs &a, hipStream_t s);
hipError_t launch_fused(int nquads, const StepArgs &a, hipStream_t s);

// ------------------------------------------------------ batched small SVDs
constexpr int kBatchMaxN = 256;  // largest n of a problem in the batched path
constexpr int kBatchBlockMinN = 65;     // built-in: batched problems with n >= this are blocked
constexpr int kBatchBlockLds = 8448;   // doubles of LDS the blocked method needs
constexpr int kBatchInnerOrder = 32;   // 2w of the blocked method's inner sweeps

struct BatchArgs {
    int64_t count;
    const int32_t *m, *n;                       // device, per problem
    const int64_t *a_off, *s_off, *v_off;       // device, element offsets
    double *A, *S, *V;                          // V may be null
    const int32_t *order;                       // device, work order (by non-increasing n)
    int *queue;                                 // device: next blocked, next pointwise, blocked count
    const int *tbl_order;                       // device [kBatchMaxN + 1]: strategy order for n
    const int64_t *tbl_off;                     // device: offset of the order-N table at [N/2]
    const unsigned char *tbls;                  // device: concatenated zero-based pair tables
    int max_sweeps;
    int32_t *status, *sweeps;                   // device, per problem (may be null)
    int64_t lds_doubles;                        // problems with m n <= this work in LDS
    int g_groups;                               // half waves rotating G when V is wanted (of 32)
    int blk_min_n;                              // problems with n >= this are blocked (0: none)
    int ddrjac;                                 // 1: DDRJAC pairs and DRDSSQ norms (no blocked problems)
    double t_hi[32];                            // DRDSSQ upper bound by ceil(lg m)
};

hipError_t batched_set_lds(int bytes);

// The upper safe bound of DRDSSQ (Appendix A) for vectors of length n with
// ceil(lg n) = lg: RZ(sqrt(nu / delta_n)), nu the largest double,
// delta_n = 2^lg (1 + 2^-53)^(1 + lg); 0 <= lg <= 63.
double rdssq_t_hi(int lg);

// grid: workgroups of the pointwise kernel; bgrid: of the blocked kernel
// (two fit on a CU).
hipError_t launch_batched(const BatchArgs &b, int grid, int bgrid, int max_n, int *hist,
                          int32_t *order, hipStream_t s);

// ------------------------------------------------------------ SVD adjoint
struct GemmArgs {
    int64_t batch;
    int M, N, K;                 // C (M x N) = op(A) (M x K) op(B) (K x N)
    bool ta, tb;                 // op = transpose
    const double *A, *B;
    int64_t lda, ldb, sa, sb;    // leading dimensions and batch strides (elements)
    double *C;
    int64_t ldc, sc;
    const double *E, *d;         // optional: C += E diag(d)
    int64_t lde, se, sd;
    double alpha = 1.0, beta = 0.0;  // C = alpha op(A) op(B) + beta C (+ E diag(d))
    int64_t ksplit = 0;          // > 0: batch b sums K indices [b ksplit, min(K, (b+1) ksplit))
                                 // of one product (A, B not strided; C strided by sc)
};

hipError_t launch_gemm(const GemmArgs &g, hipStream_t s);
hipError_t launch_adjoint_middle(int64_t batch, int n, const double *s, int64_t ss,
                                 const double *ds, const double *J, const double *K, double *Mp,
                                 double *inv_s, int *degenerate, hipStream_t st);

// ------------------------------------------------------------ QR (eq. (2.1))
constexpr int kQrPanel = 32;  // Householder panel width

struct QrPanelArgs {
    double *W;            // m x n, column-major (ld ldw), factored in place
    int64_t ldw, m, n;
    int64_t j;            // first column (and pivot row) of the panel
    int nb;               // columns in the panel, <= kQrPanel
    double *tau;          // n: reflector scalars
    double *Vp;           // out: explicit V of the panel, (m - j) x kQrPanel, ld ldvp
    int64_t ldvp;
    double *partials;     // 2 x nwg x kQrPanel
    double *prow;         // 2 x kQrPanel
    unsigned *bar;        // grid barrier counter
    int *abort_flag;      // set when a barrier does not complete
    int nwg;              // workgroups, <= 64 (all resident at once)
};

// QR with column pivoting of W (rows x ncols), in place, on nwg resident
// workgroups (see jsvd_qr.hip).
struct QrcpArgs {
    double *W;
    int64_t ldw, rows, ncols;
    double *tau;           // [ncols] reflector scalars (the first rank used)
    int *jpvt;             // [ncols] out: physical column at each position
    double *vn1, *vn2;     // [ncols] partial norms, by physical column
    double *vn0;           // [ncols] original column norms
    double *cand_v;        // [2 nwg] per-workgroup pivot candidates
    double *cand_r;        // [2 nwg] per-workgroup largest kept fraction of a norm
    int *cand_i;           // [2 nwg]
    int *rank;             // out: the numerical rank
    unsigned *bar;         // grid barrier counter
    int *abort_flag;       // set when a barrier does not complete
    int nwg;
    double tol;            // stop when every free column's partial norm <= tol * its norm
};
int qrcp_resident(int cu_count);
hipError_t launch_qrcp(const QrcpArgs &a, hipStream_t s);
hipError_t launch_trap_transpose(const double *W, int64_t ldw, int64_t k, int64_t ncols, double *X,
                                 int64_t ldx, hipStream_t s);
hipError_t launch_compose(const int *a, const int *b, int64_t n, int *out, hipStream_t s);
hipError_t launch_fill(double *x, int64_t n, double v, hipStream_t s);
hipError_t launch_fill2d(double *B, int64_t ldb, int64_t rows, int64_t cols, double v,
                         hipStream_t s);
hipError_t launch_zero_lower(double *W, int64_t ldw, int64_t n, hipStream_t s);
int qr_panel_groups(int64_t rows);
int qr_panel_resident(int cu_count);  // panel workgroups that fit on the device at once
hipError_t launch_qr_reset(unsigned *bar, int *abort_flag, hipStream_t s);
hipError_t launch_diag_range(const double *W, int64_t ldw, int64_t n, double *out, hipStream_t s);
hipError_t launch_qr_panel(const QrPanelArgs &a, hipStream_t s);
hipError_t launch_qr_t(const double *Y, const double *tau, int nb, double *T, hipStream_t s);
hipError_t launch_sum_parts(const double *parts, int np, int64_t count, double *out,
                            hipStream_t s);
// X = the transpose of W's upper triangle; colscale (may be null): column i
// of W multiplied by colscale[i] on the way (exact powers of two).
hipError_t launch_r_transpose(const double *W, int64_t ldw, int64_t n, double *X, int64_t ldx,
                              hipStream_t s, const double *colscale = nullptr);
hipError_t launch_pow2(const int *ex, int64_t n, double *out, hipStream_t s);
hipError_t launch_qr_extract_v(const double *W, int64_t ldw, int64_t m, int64_t j, int nb,
                               double *Vp, int64_t ldvp, hipStream_t s);
hipError_t launch_embed(const double *X, int64_t ldx, int64_t n, double *B, int64_t ldb,
                        int64_t rows, int64_t cols, hipStream_t s);

hipError_t launch_reset_counters(unsigned long long *c, hipStream_t s);
hipError_t launch_init_identity(double *V, int64_t ldv, int64_t n, hipStream_t s);
hipError_t launch_colnorms(const double *G, int64_t ldg, int64_t m, int64_t n, double *s_out,
                           hipStream_t s);
hipError_t launch_range_init(int *range, hipStream_t s);
hipError_t launch_colexp(const double *G, int64_t ldg, int64_t m, int64_t n, double *s_out,
                         int *ex, int *range, hipStream_t s);
hipError_t launch_rank(const double *s, int64_t n, int64_t n_plus, int *perm, hipStream_t st);
hipError_t launch_rdssq_cols(const double *A, int64_t lda, int64_t m, int64_t n, int32_t *exps,
                             double *ssq, double *norms, hipStream_t s);
hipError_t launch_identity_cols(double *B, int64_t ldb, int64_t rows, int64_t cols, int64_t first,
                                hipStream_t s);
hipError_t launch_count_positive(const double *S, int64_t n, int *out, hipStream_t s);
hipError_t launch_gather_cols(const double *src, int64_t lds, double *dst, int64_t ldd,
                              int64_t rows, int64_t cols, const int *perm, const double *scale,
                              double *s_out, hipStream_t s);
hipError_t launch_scatter_rows(const double *src, int64_t lds, double *dst, int64_t ldd,
                               int64_t rows, int64_t cols, const int *row_of, hipStream_t s);
hipError_t launch_diag_fp64(int64_t count, const double *a, const double *b, double *q,
                            double *r, hipStream_t s);
hipError_t launch_diag_refined(int64_t count, const double *a, const double *b, double *out,
                               hipStream_t s);

}  // namespace jsvd

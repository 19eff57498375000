/*
 * jsvd -- block one-sided Jacobi SVD and hyperbolic SVD on AMD Instinct
 * MI355X (gfx950), FP64.
 *
 * The method is the two single-GPU levels of the hierarchically blocked
 * one-sided Jacobi algorithm (Novakovic, "A hierarchically blocked Jacobi
 * SVD algorithm for single and multiple graphics processing units"):
 *   - block level (Section 2, eqs. (2.6)-(2.9); Section 4): the columns of
 *     G and V are split into block-columns of width w; a parallel pivot
 *     strategy (Section 3) pairs them; for each pair (p, q) the Gram matrix
 *     H_pq = [G_p G_q]^T [G_p G_q] is formed and Cholesky-factored, eq.
 *     (2.7), an inner Jacobi orthogonalises the 2w x 2w factor
 *     (Section 4.3), and the accumulated transformation V'_pq updates
 *     [G_p G_q] and [V_p V_q], eq. (2.9);
 *   - a block sweep repeats until it performs no proper rotation
 *     (Section 4.5).
 *
 * Conventions for every entry point below
 *   - Matrices are column-major (Section 4), doubles, in device memory
 *     owned by the caller; leading dimensions are in elements.
 *   - All work is enqueued on the stream given to jsvd_create /
 *     jsvd_set_stream.  A call returns after its work has finished (it
 *     synchronises the stream once per block sweep to read the one
 *     convergence counter, as the paper's host loop does).
 *   - The library owns the handle, its strategy tables and the workspaces it
 *     allocates with hipMalloc on first use for a shape and keeps until
 *     jsvd_destroy (jsvd_workspace_size and jsvd_workspace_size_batched say
 *     how much).  A handle must not be used by two threads at once.
 *   - Return codes: JSVD_OK; a negative value -i means argument i is
 *     invalid (nothing was run); a positive value is a run-time condition,
 *     after which the outputs are still written.
 */
#ifndef JSVD_H
#define JSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JSVD_OK 0
#define JSVD_NOT_CONVERGED 1   /* max_sweeps reached with proper rotations left */
/* 2 is not used: a Cholesky pivot that is not positive (Section 4.1 is silent
 * on it; the pivot block Gram matrix is then only semidefinite) is not an
 * error here -- it makes its row of R zero, the iteration goes on and
 * jsvd_info.chol_breakdowns counts it; a NaN or infinite pivot returns
 * JSVD_NONFINITE. */
#define JSVD_NONFINITE 3       /* a NaN or infinity appeared in the input or the iteration */
#define JSVD_HIP_ERROR 4       /* a HIP runtime call failed */
#define JSVD_DEGENERATE 5      /* equal singular values: the adjoint of U and V is undefined */
#define JSVD_NO_MEMORY 6       /* workspace allocation failed, or a workspace would have to
                                  grow while the stream is being captured */

/* Parallel pivot strategies of Section 3, used at both levels. */
#define JSVD_STRAT_RREV 0 /* reverse of the p-strategy closest to row-cyclic (default) */
#define JSVD_STRAT_R 1    /* p-strategy closest to row-cyclic, Definition 3.1 */
#define JSVD_STRAT_CREV 2 /* reverse of the p-strategy closest to column-cyclic */
#define JSVD_STRAT_C 3    /* p-strategy closest to column-cyclic */
#define JSVD_STRAT_RR 4   /* round-robin (tournament) ordering, one of the comparison
                             strategies of Section 6: pairs (1,2),(3,4),... first, then
                             every index but the first moves one place round the ring
                             (Brent and Luk's parallel ordering) */

typedef struct jsvd_handle_s *jsvd_handle_t;

typedef struct {
    int32_t block_w;          /* block-column width w: 0 = choose (tuning table of the handle,
                                 else by size), else 16, 32 or 64.  64 is the third blocking
                                 level: the inner problem of a 128-column pivot pair is
                                 itself solved by the block method with 16-column
                                 sub-blocks (ordinary unscaled SVD only: the hyperbolic
                                 SVD and the scaled mode take 32 instead) */
    int32_t strategy;         /* JSVD_STRAT_* (default JSVD_STRAT_RREV) */
    int32_t max_inner_sweeps; /* M_s of Section 4.3: 0 = choose (default: 1), 1 = block-oriented,
                                 > 1 = full block (the paper's setting is 30) */
    int32_t max_sweeps;       /* limit on block sweeps (default 30) */
    int32_t want_v;           /* 1 = accumulate V (default), 0 = do not touch V */
    int32_t sort;             /* 1 = order the output (default), 0 = column order as computed */
    int32_t qr;               /* QR preprocessing of a tall G, eq. (2.1), jsvd_gesvd only:
                                 0 = choose (when m >= 2n, default), 1 = never, 2 = always */
    int32_t scaled;           /* scaled mode for badly scaled G (Section 4.2): every column
                                 is scaled by a power of two (exactly) before its Gram
                                 matrices are formed, so that no square or sum leaves the
                                 normal range; 0 = when some column norm lies outside
                                 [2^-480, 2^481) (default; costs one pass over G and one
                                 stream synchronisation), 1 = never, 2 = always.  Covers
                                 norms over the whole normal range and, within one pivot
                                 block-pair, ratios of column norms up to about 2^1000
                                 (tested to 2^900).
                                 A badly scaled tall G keeps the QR preprocessing: its
                                 columns are scaled by the same powers of two before the
                                 Householder QR, and the Jacobi method runs on
                                 (R D)^T in the scaled mode. */
    int32_t factorize;        /* how a pivot block-pair is shortened to its 2w x 2w triangular
                                 factor R: 0 = Cholesky of the Gram matrix (Section 4.1,
                                 default), 1 = the QR shortening of Section 4.2 (eq. (2.8)):
                                 Householder QR of chunks of 2w rows, chunk factors folded
                                 together by the peel-off Givens procedure, the Gram matrix
                                 never formed (slower; R's accuracy does not depend on the
                                 square of the pair's condition number).  With 1, block_w 64
                                 is taken as 32. */
    int32_t fuse;             /* 1: where the ordering exchanges partners inside
                                 groups of two pivot pairs from one p-step to the next
                                 (the Mantharam-Eberlein orderings for a power-of-two
                                 number of blocks, jsvd_quad_table), 2w = 64, no padding
                                 columns, m a multiple of 64 (and lda <= 2^25), the
                                 unscaled Cholesky path: the update of a
                                 p-step (eq. (2.9)) and the next p-step's Gram matrices
                                 (eq. (2.7)) in one launch, G read once per p-step;
                                 elsewhere, and with 0 (default), three launches per
                                 p-step.  The Gram partial sums are formed in another
                                 order, so the results agree with the three-launch path
                                 to rounding.  On the MI355X the fused launch takes
                                 longer than the two it replaces (its MFMA issue, not
                                 HBM, bounds both), hence the default. */
} jsvd_opts;

typedef struct {
    int32_t sweeps;            /* block sweeps performed */
    int32_t converged;         /* 1 if the last sweep had no proper rotation */
    int64_t rotations;         /* inner rotations performed, all sweeps */
    int64_t proper_rotations;  /* of which with cos != 1 (Section 4.3, subphase 4) */
    int64_t inner_sweeps;      /* inner sweeps summed over all pivot block-pairs */
    int64_t pair_updates;      /* pivot block-pairs whose V'_pq was applied */
    int32_t chol_breakdowns;   /* non-positive Cholesky pivots met (the block Gram matrix was
                                  only semidefinite); each makes its row of R zero */
    int32_t hyp_clamps;        /* |coth 2phi| <= 1 replaced by 5/4 (Section 4.3.1) */
    int32_t block_w;           /* w actually used */
    int32_t n_blocks;          /* block-columns in the pivot strategy (with padding) */
    double seconds;            /* wall time of the call */
    int32_t preprocessed;      /* 1 if the Jacobi method ran on R^T of a QR of G (eq. (2.1));
                                  2 if G was rank deficient and it ran on the L_0 of the
                                  LQ factorization (2.2) after a QR with column pivoting */
    int32_t scaled;            /* 1 if the scaled mode ran (opts.scaled) */
    int32_t rank;              /* preprocessed == 2: the numerical rank k of G (the number
                                  of singular values computed as positive); else n */
} jsvd_info;

/*
 * Choices measured on the device by the project's autotuner
 * (python -m paper_1401_2720_amd.autotune), which a handle can hold in place
 * of its built-in size rule.
 *   count          : entries used in n_upper and block_w, 1..8 (0: no w table).
 *   n_upper[i]     : strictly increasing; a problem takes the block_w of the
 *                    first entry with n <= n_upper[i], or of the last entry.
 *   block_w[i]     : 16, 32 or 64.
 *   gram_wg[i]     : tile shape of the Gram kernel for that entry: about this
 *                    many workgroups per launch (the rows are split into
 *                    gram_wg / (pivot pairs) ranges, 1..16); 0 = built-in
 *                    (512), else 64..8192.
 *   update_wg[i]   : tile shape of the update kernel: about this many
 *                    workgroups per launch (row chunks per pivot pair =
 *                    update_wg / pairs); 0 = built-in (1024), else 64..8192.
 *   batch_g_groups : of the 32 half waves of a batched workgroup, those that
 *                    rotate G when V is wanted (the others apply the
 *                    rotations to V); 0 = built-in (16), else 4..28.
 *   batch_block_min_n : batched problems with n >= this run the blocked
 *                    method (block-columns of 16); 0 = built-in, 33..257
 *                    (257: no problem is blocked).
 */
typedef struct {
    int32_t count;
    int64_t n_upper[8];
    int32_t block_w[8];
    int32_t gram_wg[8];
    int32_t update_wg[8];
    int32_t batch_g_groups;
    int32_t batch_block_min_n;
} jsvd_tuning;

/* Install (tuning != NULL, copied) or remove (NULL) the tuned choices of a
 * handle: they decide w when opts->block_w == 0, the tile shapes of the
 * Gram and update kernels, the batched kernel's split and which batched
 * problems are blocked.  Returns JSVD_OK, -1 if h is NULL, -2 for an invalid table. */
int jsvd_set_tuning(jsvd_handle_t h, const jsvd_tuning *tuning);

/* Fill *opts with the defaults listed above.  Returns JSVD_OK, or -1 if
 * opts is NULL. */
int jsvd_default_opts(jsvd_opts *opts);

/* Create a handle bound to a HIP stream (a hipStream_t; NULL = the null
 * stream).  The current HIP device at this call is the handle's device.
 * Returns JSVD_OK, -1 if h is NULL, or JSVD_HIP_ERROR. */
int jsvd_create(jsvd_handle_t *h, void *hip_stream);

/* Rebind the handle to another stream of the same device. */
int jsvd_set_stream(jsvd_handle_t h, void *hip_stream);

/* Free the handle and its device workspace. */
int jsvd_destroy(jsvd_handle_t h);

/*
 * Ordinary SVD, G = U Sigma V^T (Section 2, eqs. (2.3)-(2.5); Section 4).
 *   m, n   : rows and columns, m >= n >= 1 (the paper transposes when m < n;
 *            here m < n is rejected).
 *   A      : device, m x n, leading dimension lda >= m.  In: G.  Out: U
 *            (economy, m x n, orthonormal columns; u_i = 0 for sigma_i = 0).
 *   S      : device, n doubles.  Out: singular values, non-increasing when
 *            opts->sort, else in computed column order.
 *   V      : device, n x n, leading dimension ldv >= n; may be NULL when
 *            opts->want_v == 0.  Out: right singular vectors.
 *   opts   : host, may be NULL for defaults.
 *   info   : host, may be NULL.  Statistics of the run.
 * With QR preprocessing (opts->qr; by default when m >= 2n) the columns of
 * G are presorted by non-increasing norm, G P = Q [R; 0] by blocked
 * Householder reflections (eq. (2.1); column presorting in place of column
 * pivoting), the Jacobi method runs on R^T (n x n) giving R^T V_x = U_x Sigma,
 * and U = Q [V_x; 0], V = P U_x.  If R is numerically singular (some
 * |r_ii| <= n 2^-53 max |r_jj|), G is rank deficient: R is factored again
 * with column pivoting, R P_2 = Q_2 [R_0; ~0] (R_0 k x n, k the numerical
 * rank: the pivoted norms fall to n 2^-53 of the first), R_0 by the LQ
 * factorization R_0 = [L_0 0] Q_3^T (eq. (2.2)), the Jacobi method runs on
 * L_0 (k x k) giving L_0 V_x = U_x Sigma_k, and U = Q [Q_2 [U_x; 0]; 0] (the
 * other n - k columns zero), V = P P_2 Q_3 [V_x 0; 0 I], Sigma = (Sigma_k, 0)
 * (info->preprocessed = 2, info->rank = k).  If a factorization's grid
 * barrier cannot complete (other work on the device keeps some of its
 * workgroups from starting), or k = 0, the call solves G directly instead.
 * The QR path needs m <= 32768.
 * Returns JSVD_OK, a negative argument index, JSVD_NOT_CONVERGED,
 * JSVD_NONFINITE, JSVD_HIP_ERROR or JSVD_NO_MEMORY.
 */
int jsvd_gesvd(jsvd_handle_t h, int64_t m, int64_t n, double *A, int64_t lda, double *S,
               double *V, int64_t ldv, const jsvd_opts *opts, jsvd_info *info);

/*
 * Full SVD, G = U [Sigma; 0] V^T with U of order m (the form of eq. (2.1)'s
 * G = Q [R_0; 0] carried through to U): jsvd_gesvd (QR preprocessing and
 * all options as there; the output is always sorted), then the last m - k
 * columns of U, k the number of positive singular values, are completed to
 * an orthonormal basis: a Householder QR of the economy U (zero columns
 * last) and Q applied to the identity's columns k .. m-1.
 *   A      : device, m x n (lda >= m).  In: G.  Out: the economy U.
 *   U      : device, m x m, leading dimension ldu >= m (argument 7).  Out:
 *            columns 0 .. k-1 equal to A's, the rest orthonormal to them.
 *   S, V, opts, info : as for jsvd_gesvd (arguments 8, 9, 10, 11, 12).
 * Needs m <= 32768 (the completion holds a QR workspace of about
 * 8 (m n + 256 m) bytes beside U).
 * Returns JSVD_OK, a negative argument index, JSVD_NOT_CONVERGED,
 * JSVD_NONFINITE, JSVD_HIP_ERROR (also when the completion's QR panel could
 * not run its workgroups together) or JSVD_NO_MEMORY.
 */
int jsvd_gesvd_full(jsvd_handle_t h, int64_t m, int64_t n, double *A, int64_t lda, double *U,
                    int64_t ldu, double *S, double *V, int64_t ldv, const jsvd_opts *opts,
                    jsvd_info *info);

/*
 * Hyperbolic SVD, G = U Sigma V^{-1} with V^T J V = J (eq. (2.10); Section
 * 4.3, subphases 4-5).  J = diag(j_1..j_n), j_i = +1 or -1, given on the host.
 * Pairs of columns with opposite signs are orthogonalised by hyperbolic
 * rotations (4.2), the others by trigonometric ones (4.1).
 *   J      : host, n entries, each +1 or -1 (argument 6).
 *   J_out  : host, n entries, may be NULL.  Out: the sign of each output
 *            column.  Internally the columns are stably permuted so that J
 *            is partitioned as diag(I, -I) (the paper keeps J partitioned);
 *            J_out is that partitioned J.
 *   V      : device, n x n.  Out: V with rows in the input column order and
 *            columns in the output order, so that G V = U Sigma and
 *            V^T J V = diag(J_out).
 *   Other arguments as for jsvd_gesvd.  With opts->sort the positive part
 *   is ordered by non-increasing sigma and the negative part by
 *   non-decreasing sigma, i.e. j_i sigma_i^2 is non-increasing.
 * The hyperbolic SVD exists when rank(G) = rank(G J G^T) (Section 2).
 */
int jsvd_hsvd(jsvd_handle_t h, int64_t m, int64_t n, double *A, int64_t lda,
              const int8_t *J, int8_t *J_out, double *S, double *V, int64_t ldv,
              const jsvd_opts *opts, jsvd_info *info);

/*
 * Many independent ordinary SVDs of uneven sizes (the same one-sided Jacobi
 * method, Section 2 eqs. (2.3)-(2.5) with the rotations (4.3)-(4.6), in the
 * p-steps of the closest parallel strategy of Section 3: pointwise for the
 * smaller problems, and for those with n >= jsvd_batched_block_min_n(h) the
 * two-level method with block-columns of 16 (Gram matrix (2.7), Cholesky,
 * one inner sweep on R, update (2.9))), in two persistent launches (the
 * blocked problems, then the others): workgroups pull problems from a device
 * queue, largest n first, and each runs its problem to its own convergence (a
 * sweep with no proper rotation, Section 4.5) or opts->max_sweeps.
 *   batch        : number of problems (0 is allowed: nothing is done).
 *   max_m, max_n : host bounds on the sizes, 1 <= max_n <= 256, max_n <= max_m;
 *                  they size the per-workgroup scratch.
 *   m, n         : device int32[batch], 1 <= n[i] <= m[i], m[i] <= max_m, n[i] <= max_n.
 *   a_off        : device int64[batch]: problem i is A + a_off[i], column-major, lda = m[i];
 *                  in: G_i, out: U_i (m[i] x n[i]).
 *   s_off        : device int64[batch]: singular values of i at S + s_off[i] (n[i], non-increasing).
 *   v_off        : device int64[batch] or NULL when opts->want_v == 0: V_i at V + v_off[i],
 *                  n[i] x n[i], ldv = n[i].
 *   status       : device int32[batch] or NULL: 0 converged, JSVD_NOT_CONVERGED when
 *                  max_sweeps ended it, JSVD_NONFINITE when a blocked problem met a
 *                  NaN or infinite Cholesky pivot, or (opts->scaled = 2) a column
 *                  held a NaN or an infinity.
 *   sweeps       : device int32[batch] or NULL: sweeps performed.
 * Only opts->max_sweeps, opts->want_v and opts->scaled are used (block_w does
 * not apply: blocked problems use 16).  opts->scaled = 2 is the mode for
 * badly scaled problems: every problem runs the pointwise method with DDRJAC
 * pairs (Section 4.3.1): the column norms by DRDSSQ (Appendix A, see
 * jsvd_colnorms), the cosine of the pair's angle from the columns scaled by
 * the powers of two of their norms, ct 2phi of (4.3) from the ratio of the
 * norms, then (4.4)-(4.6); sigma and U from DRDSSQ of the final columns
 * (sigma_i infinite if it overflows); a problem stops at a sweep with no
 * rotation at all (the pointwise rule of Section 4.5: on graded columns a
 * rotation with cos = 1 still moves the smaller column).  It covers
 * entries anywhere in the
 * double range (subnormals included) as long as, within a problem, the
 * ratio of two column norms stays below about 2^1000.  0 and 1: the
 * ordinary pairs, which need every column's squares and sums in the normal
 * range (the default; the input is not inspected).  The handle's tuned
 * batch_g_groups, if any, sets
 * how a workgroup of the pointwise kernel divides its half waves between G
 * and V, and its batch_block_min_n which problems are blocked.  The work is
 * enqueued on the handle's stream and the call returns without waiting; the
 * problems must not overlap in A, S or V.
 * Workspace: the batched call has a device workspace of its own (apart from
 * the one of jsvd_gesvd, jsvd_hsvd and jsvd_svd_backward, which therefore
 * never free it).  It grows when a call needs more, except while the stream
 * is being captured: such a call returns JSVD_NO_MEMORY (nothing enqueued);
 * to capture a call, size the workspace first with jsvd_reserve_batched or
 * an eager call of at least that size.  A workspace that a capture used is
 * never freed before jsvd_destroy (the graph holds its address): a later,
 * larger call allocates a new one, and the graph still replays correctly.
 * Returns JSVD_OK, a negative argument index, JSVD_HIP_ERROR or
 * JSVD_NO_MEMORY.
 */
int jsvd_gesvd_batched(jsvd_handle_t h, int64_t batch, int32_t max_m, int32_t max_n,
                       const int32_t *m, const int32_t *n, const int64_t *a_off,
                       const int64_t *s_off, const int64_t *v_off, double *A, double *S,
                       double *V, const jsvd_opts *opts, int32_t *status, int32_t *sweeps);

/*
 * The batched SVD of jsvd_gesvd_batched for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc): the same kernels and results, bit for bit, with
 * the work order and queue counters in a fixed device array of the library
 * instead of the handle's workspace, so that the call allocates nothing, not
 * even on its first use.  The array holds JSVD_NOALLOC_MAX_BATCH problems
 * (about 4 MiB; each device the library runs on keeps one until the process
 * ends).  Arguments, ownership and return codes as for jsvd_gesvd_batched,
 * except that batch > JSVD_NOALLOC_MAX_BATCH returns -2 (nothing enqueued)
 * and JSVD_NO_MEMORY does not occur.  All calls on one device share its
 * array, whose counters every call re-initialises with kernels on its own
 * stream: two calls whose work can overlap on the same device (other
 * streams, other handles, other threads) race; keep them on one stream.
 */
#define JSVD_NOALLOC_MAX_BATCH 1048576
int jsvd_gesvd_batched_noalloc(jsvd_handle_t h, int64_t batch, int32_t max_m, int32_t max_n,
                               const int32_t *m, const int32_t *n, const int64_t *a_off,
                               const int64_t *s_off, const int64_t *v_off, double *A, double *S,
                               double *V, const jsvd_opts *opts, int32_t *status,
                               int32_t *sweeps);

/*
 * Device workspace, in bytes, that jsvd_gesvd (or, for a J with both signs,
 * jsvd_hsvd) needs for an m x n problem with these options (NULL: defaults):
 * the pivot Gram partials, V'_pq slots and counters of the block sweeps
 * (Sections 4.1-4.5), and for the QR preprocessing of a tall G (eq. (2.1))
 * its factor and reflectors.  The library allocates it on first use and
 * keeps it in the handle; nothing is allocated by this call.
 * Returns JSVD_OK, -1 if h is NULL, -2/-3 for invalid m/n, -4 for invalid
 * options, -5 if bytes is NULL.
 */
int jsvd_workspace_size(jsvd_handle_t h, int64_t m, int64_t n, const jsvd_opts *opts,
                        size_t *bytes);

/*
 * Device workspace, in bytes, of jsvd_gesvd_batched for a batch of `batch`
 * problems within the bounds max_m, max_n (arguments as for that call;
 * opts may be NULL): the work order and the queue counters (about 4 bytes
 * per problem; the end of each problem permutes its columns in place
 * through LDS).
 * Returns JSVD_OK, -1 if h is NULL, -2..-4 as jsvd_gesvd_batched, -5 for
 * invalid options, -6 if bytes is NULL.
 */
int jsvd_workspace_size_batched(jsvd_handle_t h, int64_t batch, int32_t max_m, int32_t max_n,
                                const jsvd_opts *opts, size_t *bytes);

/*
 * Allocate now the batched workspace for such a batch (and upload the
 * batched strategy tables), so that the next jsvd_gesvd_batched within these
 * bounds allocates nothing and can be captured into a HIP graph even as the
 * first call.  Synchronises the handle's stream if the workspace grows.
 * Returns JSVD_OK, the argument errors of jsvd_workspace_size_batched (-6
 * does not occur), JSVD_HIP_ERROR or JSVD_NO_MEMORY (also when called while
 * the stream is being captured and the workspace would have to grow).
 */
int jsvd_reserve_batched(jsvd_handle_t h, int64_t batch, int32_t max_m, int32_t max_n,
                         const jsvd_opts *opts);

/*
 * Adjoint (reverse-mode derivative) of the SVD for a batch of equally sized
 * problems (not in the paper; the published SVD adjoint):
 *   J = U^T dU, K = V^T dV, F_ij = 1/(s_j^2 - s_i^2) (i != j), F_ii = 0,
 *   dA = U [diag(dS) + (F o (J - J^T)) diag(S) + diag(S) (F o (K - K^T))] V^T
 *        + (I - U U^T) dU diag(S)^{-1} V^T,
 * computed as (U (M - J diag(S)^{-1}) + dU diag(S)^{-1}) V^T with FP64 MFMA
 * products.  All arrays are device memory, batch after batch, column-major
 * and contiguous: U and dU batch x (m x n), S and dS batch x n, V and dV
 * batch x (n x n), dA batch x (m x n).  dU, dS and dV may each be NULL (a
 * zero adjoint).  Requires m >= n >= 1 and distinct, non-zero singular
 * values.  Synchronises the stream before returning.
 * Returns JSVD_OK, a negative argument index, JSVD_DEGENERATE,
 * JSVD_HIP_ERROR or JSVD_NO_MEMORY.
 */
int jsvd_svd_backward(jsvd_handle_t h, int64_t batch, int64_t m, int64_t n, const double *U,
                      const double *S, const double *V, const double *dU, const double *dS,
                      const double *dV, double *dA);

/*
 * The parallel pivot strategy table of Section 3 for an even order
 * (2 <= order <= 4096; order = 2^k * o with o in {1,3,5,7,9,11}) and kind
 * JSVD_STRAT_*: (order - 1) p-steps of order/2 pairs.  Orders that are not
 * powers of two start from Algorithm 3.1 at 2o and are expanded by
 * Algorithm 3.2; powers of two are expanded from order 2.
 *   pairs : host, (order - 1) * (order / 2) * 2 int32, written as one-based
 *           (p, q) with p < q, p-step by p-step.
 * Returns JSVD_OK, -1 for an unsupported order, -2 for an unknown kind,
 * -3 for pairs == NULL.
 */
int jsvd_strategy_table(int32_t order, int32_t kind, int32_t *pairs);

/*
 * The table the inner kernels use for a pivot block-pair of 2w = order
 * columns (order 32 or 64): jsvd_strategy_table's with the pairs of each
 * p-step reordered for conflict-free LDS access.  The pairs of a parallel
 * step are disjoint (Section 3), so their order within the step changes no
 * result; the steps and the set of pairs in each are those of
 * jsvd_strategy_table.  Same layout, arguments and return codes, and -1
 * also for an order other than 32 or 64.
 */
int jsvd_inner_table(int32_t order, int32_t kind, int32_t *pairs);

/*
 * The step-to-step groups that the fused update-and-Gram launch works on
 * (opts.fuse): for a table of jsvd_strategy_table whose consecutive p-steps
 * exchange partners inside groups of two pairs -- (a0, a1) and (b0, b1) in
 * p-step s, and in p-step s + 1 one pair of {a0, a1} x {b0, b1} and the
 * other -- per p-step s < order - 2 and group, 8 int32: the two pairs'
 * zero-based indices ia, ib within p-step s, the two new pairs' indices jx,
 * jy within p-step s + 1, the block a0 of pair ia and b0 of pair ib that
 * pair jx holds (zero-based block indices), and two zeros.
 *   quads : host, (order - 2) * (order / 4) * 8 int32.
 * Returns JSVD_OK, 1 when the table has no such structure (quads is not
 * written; the p-steps then take three launches), -1 for an unsupported
 * order, -2 for an unknown kind, -3 for quads == NULL.
 */
int jsvd_quad_table(int32_t order, int32_t kind, int32_t *quads);

/* Smallest supported strategy order >= max(nb, 2) (even, 2^k * o, o <= 11). */
int32_t jsvd_strategy_order(int32_t nb);

/* The smallest n of a problem that jsvd_gesvd_batched solves by the blocked
 * method on this handle (its tuned batch_block_min_n, else the built-in
 * value); a value above 256 means none.  Returns -1 if h is NULL. */
int32_t jsvd_batched_block_min_n(jsvd_handle_t h);

/*
 * Measurement aid: per-kernel GPU time of the block sweeps, taken with HIP
 * events recorded on the handle's stream around every launch of the
 * p-step kernels (index 0 = Gram, 1 = inner Cholesky and Jacobi, 2 =
 * update, 3 = the update fused with the next p-step's Gram kernel).  jsvd_kernel_timing(h, k) with k > 0 turns it on for every k-th
 * p-step of each sweep (k = 1: all; a larger k keeps the events' own cost
 * out of the run) and zeroes the totals; (h, 0) turns it off.
 * jsvd_kernel_times writes the totals since the last reset: ms[4] (host) in
 * milliseconds and launches[4] (host), the number of timed launches.
 * Both return JSVD_OK, -i for a NULL argument i, or -2 for k < 0.
 */
int jsvd_kernel_timing(jsvd_handle_t h, int enable);
int jsvd_kernel_times(jsvd_handle_t h, double *ms, int64_t *launches);

/* Static description of a return code. */
const char *jsvd_error_string(int code);

/*
 * Diagnostic: run IEEE FP64 division a[i]/b[i] and sqrt(a[i]) for count
 * values on the device (the paper assumes both correctly rounded, Section 4).
 * a, b, quot, root: device arrays of count doubles.  Returns JSVD_OK or
 * JSVD_HIP_ERROR.
 */
int jsvd_diag_fp64(jsvd_handle_t h, int64_t count, const double *a, const double *b,
                   double *quot, double *root);

/*
 * Diagnostic: the refined FP64 operations that the inner rotations (4.3)-(4.6)
 * and the Cholesky pivots of Section 4.1 use in place of IEEE division and
 * square root, evaluated on the device by the very functions of the kernels,
 * for count operand pairs (a[i], b[i]):
 *   out[0 count + i] = reciprocal of b[i]     (Newton-refined hardware seed)
 *   out[1 count + i] = a[i] / b[i]            (that reciprocal and one residual
 *                                              correction)
 *   out[2 count + i] = sqrt(a[i])             (coupled root / half-reciprocal
 *                                              iteration, residual correction)
 *   out[3 count + i] = 1 / sqrt(a[i])         (the Cholesky's pair, after an
 *   out[4 count + i] = sqrt(a[i])              exact power-of-two scaling)
 * a, b: device arrays of count doubles; out: device array of 5 count doubles.
 * The operands are meant for the ranges the kernels use them in (positive
 * normal numbers in [2^-900, 2^900]; for the last pair any positive finite
 * a).  Returns JSVD_OK, -1 if h is NULL, -2 for count < 0, -3 for a NULL
 * array, or JSVD_HIP_ERROR.
 */
int jsvd_diag_refined(jsvd_handle_t h, int64_t count, const double *a, const double *b,
                      double *out);

/*
 * DRDSSQ, the sum of squares of Appendix A, of every column of A: safe from
 * overflow and underflow over the whole double range, subnormals included.
 * For column c (m elements) with M = max |a_ic| and mu_c the smallest
 * non-zero |a_ic|: the elements in [t_lo, t_hi] are summed unscaled, those
 * above t_hi scaled by 2^l (the largest l with 2^l M <= t_hi), those below
 * t_lo scaled by 2^k (the smallest k with 2^k mu_c >= t_lo), each partial sum
 * by a fixed reduction tree; each is put into the common form (2^j s, j
 * even, 0.5 <= s < 2) and they are added smallest first.  The bounds are
 * those of Appendix A rounded inwards (jsvd_rdssq_bounds).
 *   A      : device, m x n column-major, leading dimension lda >= m.
 *   exps   : device int32[n] or NULL: j of the result 2^j s (even).
 *   ssq    : device double[n] or NULL: s, in [0.5, 2); 0 (with j = 0) for a
 *            zero column; NaN for a column holding a NaN or an infinity.
 *   norms  : device double[n] or NULL: ||a_c|| = 2^(j/2) sqrt(s) as a double
 *            (infinite when it overflows, rounded when it is subnormal).
 * One workgroup per column; enqueued on the handle's stream, returns without
 * waiting.  Returns JSVD_OK, -1 if h is NULL, -2 for m < 1 or m > 2^40, -3
 * for n < 0 or n >= 2^31, -4 for a NULL A (n > 0), -5 for lda < m, -6 if all
 * three outputs are NULL, or JSVD_HIP_ERROR.
 */
int jsvd_colnorms(jsvd_handle_t h, int64_t m, int64_t n, const double *A, int64_t lda,
                  int32_t *exps, double *ssq, double *norms);

/*
 * The safe bounds of DRDSSQ (Appendix A) for vectors of length n with
 * ceil(lg n) = lg (0 <= lg <= 63), rounded inwards to doubles:
 *   t_lo = RU(sqrt(mu / (1 - eps)))                       = 2^-511 (1 + 2^-52),
 *   t_hi = RZ(sqrt(nu / (2^lg (1 + eps)^(1 + lg)))),
 * mu the smallest positive normal double, nu the largest double, eps = 2^-53.
 * No element in [t_lo, t_hi] has a square that underflows, and no sum of n
 * such squares overflows.  Host only (no device call).  Returns JSVD_OK, -1
 * for lg outside [0, 63], -2 for a NULL pointer.
 */
int jsvd_rdssq_bounds(int32_t lg, double *t_lo, double *t_hi);

#ifdef __cplusplus
}
#endif

#endif /* JSVD_H */

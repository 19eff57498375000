// Host driver and C ABI.  The host only controls the iteration, as in
// Section 4 of the paper: it launches one p-step after another, reads one
// block of per-sweep counters after each block sweep, and stops when a
// sweep performed no proper rotation (Section 4.5) or the sweep limit is
// reached.  Everything else runs in the kernels of jsvd_gram.hip, jsvd_inner.hip,
// jsvd_update.hip and jsvd_aux.hip.
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>

#include "jsvd_internal.h"

using namespace jsvd;

// The upper safe bound of DRDSSQ (Appendix A), t_hi = RZ(sqrt(nu / delta_n))
// with nu = (1 - 2^-53) 2^1024 and delta_n = 2^lg (1 + eps)^(1 + lg), eps =
// 2^-53.  Written as 2^((1024 - lg) / 2) sqrt((1 - eps) / (1 + eps)^(1 + lg)),
// the root's second factor is 1 - c eps + kappa eps^2 + O(lg^3 eps^3) with
// c = (lg + 2) / 2 and kappa = lg / 4 + (lg + 2)^2 / 8 > 0.  Even lg: the
// power of two is exact and c an integer, so the value lies just above the
// double 2^(512 - lg/2) (1 - c eps), which is the result.  Odd lg: the
// power carries a factor sqrt(2), and the value is computed in long double
// (64-bit significand; powl, the division and sqrtl together stay within a
// few units of 2^-64) and rounded toward zero to double.
double jsvd::rdssq_t_hi(int lg) {
    if (lg % 2 == 0) {
        const double c = (double)((lg + 2) / 2);
        return std::ldexp(1.0 - c * 0x1p-53, 512 - lg / 2);
    }
    const long double eps = 0x1p-53L;
    const long double nu = (long double)DBL_MAX;
    const long double dn = std::ldexp(std::pow(1.0L + eps, (long double)(lg + 1)), lg);
    const long double x = std::sqrt(nu / dn);
    double d = (double)x;
    if ((long double)d > x) d = std::nextafter(d, 0.0);
    return d;
}

namespace {

struct DeviceTable {
    void *ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace

// Pinned host words of a handle: the per-sweep counters, then single
// values read back from the device (QR abort flag, R's diagonal range,
// the adjoint's degeneracy flag).
constexpr int kHostSlots = 16;
constexpr int kSlotFlag = C_COUNT;       // one int
constexpr int kSlotRange = C_COUNT + 2;  // two doubles

struct jsvd_handle_s {
    int device = 0;
    hipStream_t stream = nullptr;
    void *ws = nullptr;          // device workspace of gesvd / hsvd / backward
    size_t ws_bytes = 0;
    void *bws = nullptr;         // device workspace of the batched call
    size_t bws_bytes = 0;
    bool bws_captured = false;   // a graph capture used bws: it must not be freed
    std::vector<void *> bws_retired;  // captured workspaces replaced by larger ones,
                                      // kept for their graphs until jsvd_destroy
    unsigned long long *host_counters = nullptr;  // pinned, kHostSlots words
    std::map<std::pair<int, int>, DeviceTable> block_tables;  // (order, kind) -> int2[]
    std::map<std::pair<int, int>, DeviceTable> inner_tables;  // (bw, kind) -> uchar[]
    std::map<std::pair<int, int>, DeviceTable> quad_tables;   // (order, kind) -> int[8][]
    // batched path: strategy tables of every order up to kBatchMaxN
    void *batch_tables = nullptr;   // uchar pairs
    void *batch_meta = nullptr;     // int tbl_order[kBatchMaxN+1], int64 tbl_off[kBatchMaxN/2+1]
    int cu_count = 0;
    int batch_lds = 0;              // dynamic LDS bytes of the batched kernel
    jsvd_tuning tuning{};           // measured choices (count == 0: none)
    int *colexp = nullptr;          // scaled mode: column exponents (n) + range (2)
    int64_t colexp_cap = 0;
    void *qr_ws = nullptr;          // QR preprocessing workspace (kept apart from ws,
    size_t qr_ws_bytes = 0;         // which the Jacobi solve of R^T may reallocate)
    void *qr_ws2 = nullptr;         // rank-deficient G: the pivoted QR of R and the LQ step
    size_t qr_ws2_bytes = 0;
    int qr_resident = 0;            // QR panel workgroups that can be resident at once
    void *noalloc_scratch = nullptr;  // device address of this device's fixed scratch
    // per-kernel timing (measurement aid): 4 events per p-step
    bool timing = false;
    int timing_stride = 1;          // time every timing_stride-th p-step
    std::vector<hipEvent_t> events;
    double kernel_ms[4] = {0, 0, 0, 0};  // Gram, inner, update, fused update and Gram
    int64_t launches[4] = {0, 0, 0, 0};
};

namespace {

#define HIP_TRY(expr)                         \
    do {                                      \
        hipError_t e_ = (expr);               \
        if (e_ != hipSuccess) return JSVD_HIP_ERROR; \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// The batched call's workspace grows when a call needs more.  While the
// stream is being captured it cannot (no allocation there): such a call gets
// JSVD_NO_MEMORY.  A workspace that a capture used is never freed before
// jsvd_destroy, since the graph holds its address: growing then allocates a
// new one and keeps the old one aside.
int ensure_batch_workspace(jsvd_handle_s *h, size_t bytes, bool capturing) {
    if (bytes <= h->bws_bytes) return JSVD_OK;
    if (capturing) return JSVD_NO_MEMORY;
    if (h->bws) {
        if (h->bws_captured) {
            h->bws_retired.push_back(h->bws);
        } else {
            if (hipStreamSynchronize(h->stream) != hipSuccess) return JSVD_HIP_ERROR;
            (void)hipFree(h->bws);
        }
        h->bws = nullptr;
        h->bws_bytes = 0;
        h->bws_captured = false;
    }
    if (hipMalloc(&h->bws, bytes) != hipSuccess) {
        h->bws = nullptr;
        return JSVD_NO_MEMORY;
    }
    h->bws_bytes = bytes;
    return JSVD_OK;
}

bool stream_capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
    return cs == hipStreamCaptureStatusActive;
}

int ensure_workspace(jsvd_handle_s *h, size_t bytes) {
    if (bytes <= h->ws_bytes) return JSVD_OK;
    if (h->ws) {
        if (hipStreamSynchronize(h->stream) != hipSuccess) return JSVD_HIP_ERROR;
        (void)hipFree(h->ws);
        h->ws = nullptr;
        h->ws_bytes = 0;
    }
    if (hipMalloc(&h->ws, bytes) != hipSuccess) {
        h->ws = nullptr;
        return JSVD_NO_MEMORY;
    }
    h->ws_bytes = bytes;
    return JSVD_OK;
}

int get_block_table(jsvd_handle_s *h, int order, int kind, const int2 **out) {
    auto key = std::make_pair(order, kind);
    auto it = h->block_tables.find(key);
    if (it == h->block_tables.end()) {
        Table t;
        if (!make_table(order, kind, t)) return JSVD_HIP_ERROR;
        std::vector<int2> flat;
        for (const auto &st : t)
            for (const auto &pr : st) flat.push_back(make_int2(pr.first, pr.second));
        DeviceTable d;
        d.bytes = flat.size() * sizeof(int2);
        HIP_TRY(hipMalloc(&d.ptr, d.bytes));
        HIP_TRY(hipMemcpy(d.ptr, flat.data(), d.bytes, hipMemcpyHostToDevice));
        it = h->block_tables.emplace(key, d).first;
    }
    *out = static_cast<const int2 *>(it->second.ptr);
    return JSVD_OK;
}

// The step-to-step quads of a block table (make_quads), or null when the
// ordering has none (the p-step then takes three launches).
int get_quad_table(jsvd_handle_s *h, int order, int kind, const int **out) {
    auto key = std::make_pair(order, kind);
    auto it = h->quad_tables.find(key);
    if (it == h->quad_tables.end()) {
        Table t;
        if (!make_table(order, kind, t)) return JSVD_HIP_ERROR;
        std::vector<int> flat;
        DeviceTable d;
        if (make_quads(t, flat)) {
            d.bytes = flat.size() * sizeof(int);
            HIP_TRY(hipMalloc(&d.ptr, d.bytes));
            HIP_TRY(hipMemcpy(d.ptr, flat.data(), d.bytes, hipMemcpyHostToDevice));
        }
        it = h->quad_tables.emplace(key, d).first;
    }
    *out = static_cast<const int *>(it->second.ptr);
    return JSVD_OK;
}

int get_inner_table(jsvd_handle_s *h, int bw, int kind, const unsigned char **out) {
    auto key = std::make_pair(bw, kind);
    auto it = h->inner_tables.find(key);
    if (it == h->inner_tables.end()) {
        Table t;
        if (!make_table(bw, kind, t)) return JSVD_HIP_ERROR;
        if (bw <= 64) order_for_banks(t);  // inner_kernel's lane groups (not the 2w = 128 kernel)
        std::vector<unsigned char> flat;
        for (const auto &st : t)
            for (const auto &pr : st) {
                flat.push_back(static_cast<unsigned char>(pr.first));
                flat.push_back(static_cast<unsigned char>(pr.second));
            }
        DeviceTable d;
        d.bytes = flat.size();
        HIP_TRY(hipMalloc(&d.ptr, d.bytes));
        HIP_TRY(hipMemcpy(d.ptr, flat.data(), d.bytes, hipMemcpyHostToDevice));
        it = h->inner_tables.emplace(key, d).first;
    }
    *out = static_cast<const unsigned char *>(it->second.ptr);
    return JSVD_OK;
}

jsvd_opts defaults() {
    jsvd_opts o;
    o.block_w = 0;
    o.strategy = JSVD_STRAT_RREV;
    o.max_inner_sweeps = 0;
    o.max_sweeps = 30;
    o.want_v = 1;
    o.sort = 1;
    o.qr = 0;
    o.scaled = 0;
    o.factorize = 0;
    o.fuse = 0;
    return o;
}

// Block width and inner sweep limit when the caller leaves them to the
// library (measured on MI355X: 2w = 64 pays off once the p-steps' HBM
// traffic dominates, from n of about 3000; the block-oriented variant,
// M_s = 1, was faster than the full block one at every size measured).
int choose_w(int64_t m, int64_t n) {
    (void)m;
    return n >= 3072 ? 32 : 16;
}

int choose_inner_sweeps(int64_t m, int64_t n) {
    (void)m;
    (void)n;
    return 1;
}

// Block width and kernel tile shapes of a solve: w is the caller's, else
// the handle's tuning table, else the built-in size rule; the shapes
// (workgroups per Gram and update launch) come from the tuning entry of the
// problem's size, else the built-in 512 and 1024.
struct Shapes {
    int w, gram_wg, update_wg;
};

Shapes pick_shapes(const jsvd_handle_s *h, const jsvd_opts &o, int64_t m, int64_t n) {
    Shapes sh{o.block_w, 0, 0};
    if (h->tuning.count > 0) {
        int i = 0;
        while (i + 1 < h->tuning.count && n > h->tuning.n_upper[i]) ++i;
        if (!sh.w) sh.w = h->tuning.block_w[i];
        sh.gram_wg = h->tuning.gram_wg[i];
        sh.update_wg = h->tuning.update_wg[i];
    }
    if (!sh.w) sh.w = choose_w(m, n);
    if (!sh.gram_wg) sh.gram_wg = 512;
    if (!sh.update_wg) sh.update_wg = 1024;
    return sh;
}

int pick_w(const jsvd_handle_s *h, const jsvd_opts &o, int64_t m, int64_t n) {
    return pick_shapes(h, o, m, n).w;
}

// Gram row splits of a solve (at most 16, rows per split a multiple of 64),
// aiming at gram_wg workgroups per launch.
int gram_splits(int64_t m, int npairs, int gram_wg, int64_t *rows_per_split) {
    int splits = std::min(16, std::max(1, gram_wg / npairs));
    const int64_t rps = (int64_t)align_up((size_t)((m + splits - 1) / splits), 64);
    *rows_per_split = rps;
    return (int)((m + rps - 1) / rps);
}

// The workgroups a p-step's first launch aims at: the tuned Gram figure, or,
// for the QR shortening, the row splits whose chains are shortest.  A QR
// workgroup's chain is about 2 bw barrier stages per bw-row chunk (bw - 1
// reflections, then bw peel-off stages to fold it in) and the inner kernel's
// fold of the splits' factors bw stages per split after the first, so s
// splits of c chunks cost about 2 ceil(c / s) + s - 1 chains of bw stages;
// s is kept to grids that stay resident (two bw x (bw + 1) matrices of LDS
// per workgroup: two per CU at bw = 64, four at bw = 32).  With the update
// fused into the next p-step's Gram launch, one fused workgroup per CU
// (each owns two pairs' columns: 2 cu_count pair-splits).
int split_target(const jsvd_handle_s *h, const jsvd_opts &o, const Shapes &shp, int64_t m,
                 int npairs, int bw, bool fused) {
    if (fused) return 2 * h->cu_count;
    if (o.factorize != 1) return shp.gram_wg;
    const int64_t chunks = (m + bw - 1) / bw;
    const int64_t resident = (int64_t)(bw >= 64 ? 2 : 4) * h->cu_count;
    int best = 1;
    int64_t best_cost = 2 * chunks;
    for (int sp = 2; sp <= 16 && (int64_t)sp * npairs <= resident; ++sp) {
        const int64_t cost = 2 * ((chunks + sp - 1) / sp) + sp - 1;
        if (cost < best_cost) {
            best = sp;
            best_cost = cost;
        }
    }
    return best * npairs;
}

// Workspace carve-up for one solve.
struct Layout {
    size_t hpart, vprime, pair_rot, counters, perm, s_tmp, tmp, perm_in, rscratch, total;
};

Layout plan(int64_t m, int64_t n, int bw, int npairs, int splits, bool hsvd) {
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    L.hpart = take((size_t)npairs * splits * bw * bw * sizeof(double));
    // two slots: a p-step's V'_pq is read by the next p-step's launch
    L.vprime = take((size_t)2 * npairs * bw * bw * sizeof(double));
    L.pair_rot = take((size_t)2 * npairs * sizeof(int));
    L.counters = take(C_COUNT * sizeof(unsigned long long));
    L.perm = take((size_t)n * sizeof(int));
    L.s_tmp = take((size_t)n * sizeof(double));
    L.tmp = take((size_t)std::max(m * n, n * n) * sizeof(double));
    L.perm_in = take(hsvd ? (size_t)n * sizeof(int) : 0);
    // 2w = 128: the Cholesky factors of the pivot pairs (the inner block method)
    L.rscratch = take(bw == 128 ? (size_t)npairs * bw * bw * sizeof(double) : 0);
    L.total = off;
    return L;
}

// Column exponents of G (e_c with ||g_c|| in [2^e_c, 2^(e_c+1))) into the
// handle's buffer, and whether G is badly scaled: some column norm outside
// [2^-480, 2^481), where the squares and sums of the Gram matrices could
// leave the normal range (Section 4.2).  One pass over G and one stream
// synchronisation.
int column_exponents(jsvd_handle_s *h, int64_t m, int64_t n, const double *A, int64_t lda,
                     bool *bad) {
    if (n + 2 > h->colexp_cap) {
        if (h->colexp) {
            if (hipStreamSynchronize(h->stream) != hipSuccess) return JSVD_HIP_ERROR;
            (void)hipFree(h->colexp);
        }
        h->colexp = nullptr;
        h->colexp_cap = 0;
        if (hipMalloc(&h->colexp, (size_t)(n + 2) * sizeof(int)) != hipSuccess) {
            h->colexp = nullptr;
            return JSVD_NO_MEMORY;
        }
        h->colexp_cap = n + 2;
    }
    int *range = h->colexp + n;
    HIP_TRY(launch_range_init(range, h->stream));
    HIP_TRY(launch_colexp(A, lda, m, n, nullptr, h->colexp, range, h->stream));
    if (bad) {
        int *hr = reinterpret_cast<int *>(h->host_counters);
        HIP_TRY(hipMemcpyAsync(hr, range, 2 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        *bad = hr[0] <= hr[1] && (hr[0] < -480 || hr[1] > 480);
    }
    return JSVD_OK;
}

// The solver shared by the SVD and the hyperbolic SVD.  A holds G with J
// already partitioned (columns [0, n_plus) positive).
int solve(jsvd_handle_s *h, int64_t m, int64_t n, double *A, int64_t lda, double *S, double *V,
          int64_t ldv, int64_t n_plus, const jsvd_opts &o, jsvd_info *info, bool hsvd,
          const int *perm_in_host) {
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = h->stream;
    int rc = 0;
    // scaled mode (opts.scaled: 2 on, 1 off, 0 when G is badly scaled)
    bool scaled = o.scaled == 2;
    if (o.scaled != 1) {
        bool bad = false;
        if ((rc = column_exponents(h, m, n, A, lda, o.scaled == 0 ? &bad : nullptr))) return rc;
        scaled = scaled || bad;
    }
    const Shapes shp = pick_shapes(h, o, m, n);
    // w = 64 (the third blocking level) runs the ordinary, unscaled SVD with
    // the Cholesky factorization; the hyperbolic SVD, the scaled mode and the
    // QR shortening take w = 32 instead
    const bool qrf = o.factorize == 1;
    const int w = (shp.w == 64 && (n_plus < n || scaled || qrf)) ? 32 : shp.w;
    const int bw = 2 * w;
    const int nb_real = (int)((n + w - 1) / w);
    const int order = strategy_order(nb_real);
    const int npairs = order / 2;
    const int nsteps = order - 1;
    const bool want_v = o.want_v != 0;
    // the update fused with the next p-step's Gram kernel where the ordering
    // has step-to-step quads (make_quads): 2w = 64, no padding columns, rows
    // a multiple of 64 (whole 16-row slices for the four waves of a role),
    // lane byte offsets of up to 16 columns below 2^32, unscaled, the
    // Cholesky factorization
    const int *quads = nullptr;
    if (o.fuse && bw == 64 && !scaled && !qrf && (int64_t)order * w == n && m % 64 == 0 &&
        lda <= ((int64_t)1 << 25) &&
        (rc = get_quad_table(h, order, o.strategy, &quads)))
        return rc;
    const bool fused = quads != nullptr;
    const int nquads = npairs / 2;

    // Gram row splits (at most 16) and update row chunks: aim at a few
    // workgroups per CU.  The V update of a p-step is done by the next
    // p-step's inner launch, in about two workgroups per CU that the pivot
    // pairs leave free (a workgroup there has 16 * 2w threads).
    const int target_wg = shp.update_wg;
    int64_t rps = 0;
    const int splits = gram_splits(m, npairs, split_target(h, o, shp, m, npairs, bw, fused), &rps);
    const int per_pair = std::max(1, target_wg / npairs);
    const int64_t upd_rows_g = align_up((size_t)((m + per_pair - 1) / per_pair), 64);
    const int64_t upd_rows_v = align_up((size_t)((n + per_pair - 1) / per_pair), 64);
    const int free_cu = std::max(h->cu_count - npairs, std::max(1, h->cu_count / 4));
    const int v_per_pair = std::max(1, 2 * free_cu / npairs);
    // 16-row slices per pass of such a workgroup (16 * 2w threads; 512 at 2w = 128)
    const int inner_waves = bw == 128 ? 8 : 16 * bw / 64;
    const int64_t prev_rows =
        align_up((size_t)((n + v_per_pair - 1) / v_per_pair), (size_t)16 * inner_waves);

    Layout L = plan(m, n, bw, npairs, splits, hsvd);
    rc = ensure_workspace(h, L.total);
    if (rc) return rc;
    char *ws = static_cast<char *>(h->ws);

    const int2 *blk = nullptr;
    const unsigned char *inner = nullptr;
    if ((rc = get_block_table(h, order, o.strategy, &blk))) return rc;
    if ((rc = get_inner_table(h, bw, o.strategy, &inner))) return rc;

    StepArgs a;
    a.G = A;
    a.ldg = lda;
    a.m = m;
    a.V = want_v ? V : nullptr;
    a.ldv = ldv;
    a.n = n;
    a.w = w;
    a.n_plus = (int)n_plus;
    a.pairs = nullptr;
    a.npairs = npairs;
    a.splits = splits;
    a.rows_per_split = (int)rps;
    a.gram_pf = (int64_t)splits * npairs <= 2 * (int64_t)h->cu_count ? 1 : 0;
    a.hpart = reinterpret_cast<double *>(ws + L.hpart);
    double *const vprime0 = reinterpret_cast<double *>(ws + L.vprime);
    int *const pair_rot0 = reinterpret_cast<int *>(ws + L.pair_rot);
    a.vprime = vprime0;
    a.pair_rot = pair_rot0;
    a.counters = reinterpret_cast<unsigned long long *>(ws + L.counters);
    a.inner_tbl = inner;
    a.colexp = scaled ? h->colexp : nullptr;
    a.rscratch = bw == 128 ? reinterpret_cast<double *>(ws + L.rscratch) : nullptr;
    a.qrf = qrf ? 1 : 0;
    a.btbl_order = static_cast<const int *>(h->batch_meta);
    a.btbl_off = reinterpret_cast<const int64_t *>(
        static_cast<char *>(h->batch_meta) + align_up((kBatchMaxN + 1) * sizeof(int), 256));
    a.btbls = static_cast<const unsigned char *>(h->batch_tables);
    a.quads = nullptr;
    a.next_pairs = nullptr;
    if (bw == 128 && !h->batch_tables) return JSVD_HIP_ERROR;
    a.max_inner_sweeps = o.max_inner_sweeps > 0 ? o.max_inner_sweeps : choose_inner_sweeps(m, n);
    a.upd_rows = (int)upd_rows_g;
    a.upd_chunks_g = (int)((m + upd_rows_g - 1) / upd_rows_g);
    a.upd_chunks_v = 0;
    a.prev_pairs = nullptr;
    a.prev_vprime = nullptr;
    a.prev_pair_rot = nullptr;
    a.prev_chunks = 0;
    a.prev_rows = (int)prev_rows;
    const int v_chunks = want_v ? (int)((n + prev_rows - 1) / prev_rows) : 0;

    if (want_v) HIP_TRY(launch_init_identity(V, ldv, n, st));

    jsvd_info inf{};
    std::memset(&inf, 0, sizeof inf);
    inf.block_w = w;
    inf.scaled = scaled ? 1 : 0;
    inf.n_blocks = order;
    inf.rank = (int32_t)n;
    int status = JSVD_OK;
    bool converged = false;
    if (h->timing) {
        while (h->events.size() < (size_t)4 * nsteps) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            h->events.push_back(e);
        }
    }
    int64_t g = 0;  // p-steps launched in this solve
    for (int sweep = 0; sweep < o.max_sweeps; ++sweep) {
        HIP_TRY(launch_reset_counters(a.counters, st));
        for (int s = 0; s < nsteps; ++s, ++g) {
            // the previous p-step's V update rides along with this inner launch
            a.prev_pairs = a.pairs;
            a.prev_vprime = a.vprime;
            a.prev_pair_rot = a.pair_rot;
            a.prev_chunks = g > 0 ? v_chunks : 0;
            a.pairs = blk + (size_t)s * npairs;
            a.vprime = vprime0 + (size_t)(g % 2) * npairs * bw * bw;
            a.pair_rot = pair_rot0 + (size_t)(g % 2) * npairs;
            // events around the kernels of every timing_stride-th p-step
            const bool timed = h->timing && s % h->timing_stride == 0;
            hipEvent_t *ev = timed ? &h->events[(size_t)4 * s] : nullptr;
            if (ev) HIP_TRY(hipEventRecord(ev[0], st));
            // fused: the previous p-step's launch formed this one's Gram
            // partials, except at the first p-step of a sweep
            if (!fused || s == 0) HIP_TRY(qrf ? launch_qrfac(bw, a, st) : launch_gram(bw, a, st));
            if (ev) HIP_TRY(hipEventRecord(ev[1], st));
            HIP_TRY(launch_inner(bw, a, st));
            if (ev) HIP_TRY(hipEventRecord(ev[2], st));
            if (fused && s + 1 < nsteps) {
                StepArgs f = a;
                f.quads = quads + (size_t)s * nquads * 8;
                f.next_pairs = blk + (size_t)(s + 1) * npairs;
                HIP_TRY(launch_fused(nquads, f, st));
            } else {
                HIP_TRY(launch_update(bw, a, st));
            }
            if (ev) HIP_TRY(hipEventRecord(ev[3], st));
        }
        HIP_TRY(hipMemcpyAsync(h->host_counters, a.counters, C_COUNT * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (h->timing) {
            for (int s = 0; s < nsteps; s += h->timing_stride) {
                hipEvent_t *ev = &h->events[(size_t)4 * s];
                // interval k of a p-step and the kernel it timed: 0 Gram
                // (none when fused, past the first p-step), 1 inner, 2 update
                // or the fused update and Gram (3)
                const bool fz = fused && s + 1 < nsteps;
                const int kind[3] = {(fused && s > 0) ? -1 : 0, 1, fz ? 3 : 2};
                for (int k = 0; k < 3; ++k) {
                    if (kind[k] < 0) continue;
                    float ms = 0.f;
                    HIP_TRY(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
                    h->kernel_ms[kind[k]] += ms;
                    h->launches[kind[k]] += 1;
                }
            }
        }
        const unsigned long long *c = h->host_counters;
        inf.sweeps = sweep + 1;
        inf.rotations += (int64_t)c[C_ROT];
        inf.proper_rotations += (int64_t)c[C_PROPER];
        inf.inner_sweeps += (int64_t)c[C_INNER_SW];
        inf.pair_updates += (int64_t)c[C_UPDATES];
        inf.chol_breakdowns += (int32_t)c[C_BREAKDOWN];
        inf.hyp_clamps += (int32_t)c[C_CLAMP];
        if (c[C_NONFINITE]) {
            status = JSVD_NONFINITE;
            break;
        }
        if (c[C_PROPER] == 0) {  // Section 4.5: no proper rotation in the sweep
            converged = true;
            break;
        }
    }
    inf.converged = converged ? 1 : 0;
    if (status == JSVD_OK && !converged) status = JSVD_NOT_CONVERGED;
    if (want_v && g > 0) {  // the last p-step's V update
        StepArgs av = a;
        av.upd_rows = (int)upd_rows_v;
        av.upd_chunks_g = 0;
        av.upd_chunks_v = (int)((n + upd_rows_v - 1) / upd_rows_v);
        HIP_TRY(launch_update(bw, av, st));
    }

    // ---- singular values, U, and the output order
    double *s_tmp = reinterpret_cast<double *>(ws + L.s_tmp);
    int *perm = reinterpret_cast<int *>(ws + L.perm);
    double *tmp = reinterpret_cast<double *>(ws + L.tmp);
    if (scaled)
        HIP_TRY(launch_colexp(A, lda, m, n, s_tmp, nullptr, nullptr, st));
    else
        HIP_TRY(launch_colnorms(A, lda, m, n, s_tmp, st));
    if (o.sort) {
        HIP_TRY(launch_rank(s_tmp, n, n_plus, perm, st));
        HIP_TRY(hipMemcpy2DAsync(tmp, m * sizeof(double), A, lda * sizeof(double),
                                 m * sizeof(double), n, hipMemcpyDeviceToDevice, st));
        HIP_TRY(launch_gather_cols(tmp, m, A, lda, m, n, perm, s_tmp, S, st));
        if (want_v) {
            HIP_TRY(hipMemcpy2DAsync(tmp, n * sizeof(double), V, ldv * sizeof(double),
                                     n * sizeof(double), n, hipMemcpyDeviceToDevice, st));
            HIP_TRY(launch_gather_cols(tmp, n, V, ldv, n, n, perm, nullptr, nullptr, st));
        }
    } else {
        HIP_TRY(launch_gather_cols(A, lda, A, lda, m, n, nullptr, s_tmp, S, st));
    }
    if (want_v && hsvd && perm_in_host) {
        int *pin = reinterpret_cast<int *>(ws + L.perm_in);
        HIP_TRY(hipMemcpyAsync(pin, perm_in_host, n * sizeof(int), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpy2DAsync(tmp, n * sizeof(double), V, ldv * sizeof(double),
                                 n * sizeof(double), n, hipMemcpyDeviceToDevice, st));
        HIP_TRY(launch_scatter_rows(tmp, n, V, ldv, n, n, pin, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    const auto t1 = std::chrono::steady_clock::now();
    inf.seconds = std::chrono::duration<double>(t1 - t0).count();
    if (info) *info = inf;
    return status;
}


// ------------------------------------------------------------ QR path
// G P = Q [R; 0] (eq. (2.1), column presorting by norm in place of column
// pivoting), the Jacobi method on X = R^T, then U = Q [V_x; 0], V = P U_x.
int gemm_splitk(const double *A, int64_t lda, const double *B, int64_t ldb, int M, int N,
                int64_t K, double *parts, int64_t parts_cap, double *out, hipStream_t st) {
    // out (M x N, ld M) = A^T B with A K x M and B K x N, K cut into slices:
    // enough slices for about 1024 workgroups (four per CU) with 64 columns
    // of B each, at least 16, slices of at least 64 rows, and as many as the
    // partial buffer (parts_cap doubles) holds
    const int64_t col_blocks = (N + 63) / 64;
    int64_t np = std::max<int64_t>(16, (1024 + col_blocks - 1) / col_blocks);
    np = std::min<int64_t>({np, 256, std::max<int64_t>(1, K / 64),
                            std::max<int64_t>(1, parts_cap / ((int64_t)M * N))});
    const int64_t ks = align_up((size_t)((K + np - 1) / np), 16);
    const int used = (int)((K + ks - 1) / ks);
    GemmArgs g;
    g.batch = used;
    g.M = M; g.N = N; g.K = (int)K; g.ta = true; g.tb = false;
    g.A = A; g.lda = lda; g.sa = 0;
    g.B = B; g.ldb = ldb; g.sb = 0;
    g.C = parts; g.ldc = M; g.sc = (int64_t)M * N;
    g.E = nullptr; g.d = nullptr; g.lde = g.se = g.sd = 0;
    g.ksplit = ks;
    HIP_TRY(launch_gemm(g, st));
    HIP_TRY(launch_sum_parts(parts, used, (int64_t)M * N, out, st));
    return JSVD_OK;
}

int gemm_plain(bool ta, const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
               int64_t ldc, int M, int N, int K, double alpha, double beta, hipStream_t st) {
    GemmArgs g;
    g.batch = 1;
    g.M = M; g.N = N; g.K = K; g.ta = ta; g.tb = false;
    g.A = A; g.lda = lda; g.sa = 0;
    g.B = B; g.ldb = ldb; g.sb = 0;
    g.C = C; g.ldc = ldc; g.sc = 0;
    g.E = nullptr; g.d = nullptr; g.lde = g.se = g.sd = 0;
    g.alpha = alpha;
    g.beta = beta;
    HIP_TRY(launch_gemm(g, st));
    return JSVD_OK;
}

// Workspace carve-up of the QR preprocessing (kept apart from the solve's).
// ncols: the widest block Q is applied to (n for U = Q [V_x; 0], up to m for
// the full U).
struct QrLayout {
    size_t oW, oX, oVx, oVp, oT, oTau, oParts, oY1, oY2, oPart, oProw, oNrm, oScl, oPerm, oBar,
        total;
    int64_t parts_cap;
};

QrLayout qr_plan(int64_t m, int64_t n, int64_t ncols = 0) {
    constexpr int NB = kQrPanel;
    const int64_t npan = (n + NB - 1) / NB;
    const int64_t nc = std::max(n, ncols);
    QrLayout q;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off += align_up(bytes, 256); return at; };
    q.oW = take((size_t)m * n * 8);
    q.oX = take((size_t)n * n * 8);
    q.oVx = take((size_t)n * n * 8);
    q.oVp = take((size_t)m * NB * 8);
    q.oT = take((size_t)npan * NB * NB * 8);
    q.oTau = take((size_t)n * 8);
    q.parts_cap = (int64_t)32 * NB * nc;
    q.oParts = take((size_t)q.parts_cap * 8);
    q.oY1 = take((size_t)NB * nc * 8);
    q.oY2 = take((size_t)NB * nc * 8);
    q.oPart = take((size_t)2 * 64 * NB * 8);
    q.oProw = take((size_t)2 * NB * 8);
    q.oNrm = take((size_t)n * 8);
    q.oScl = take((size_t)2 * n * 8);
    q.oPerm = take((size_t)n * 4);
    q.oBar = take(128);
    q.total = off;
    return q;
}

// Pointers into the QR workspace of a layout.
struct QrWork {
    double *W, *X, *Vx, *Vp, *T, *tau, *parts, *Y1, *Y2, *part, *prow, *nrm, *scl, *d_range;
    int *perm, *abort_flag;
    unsigned *bar;
    int64_t parts_cap;  // doubles in parts (split-K partial products)
};

int qr_workspace(jsvd_handle_s *h, const QrLayout &q, QrWork *w) {
    if (q.total > h->qr_ws_bytes) {
        if (h->qr_ws) {
            if (hipStreamSynchronize(h->stream) != hipSuccess) return JSVD_HIP_ERROR;
            (void)hipFree(h->qr_ws);
        }
        h->qr_ws = nullptr;
        h->qr_ws_bytes = 0;
        if (hipMalloc(&h->qr_ws, q.total) != hipSuccess) {
            h->qr_ws = nullptr;
            return JSVD_NO_MEMORY;
        }
        h->qr_ws_bytes = q.total;
    }
    char *ws = static_cast<char *>(h->qr_ws);
    auto d = [&](size_t o) { return reinterpret_cast<double *>(ws + o); };
    w->W = d(q.oW); w->X = d(q.oX); w->Vx = d(q.oVx); w->Vp = d(q.oVp); w->T = d(q.oT);
    w->tau = d(q.oTau); w->parts = d(q.oParts); w->Y1 = d(q.oY1); w->Y2 = d(q.oY2);
    w->parts_cap = q.parts_cap;
    w->part = d(q.oPart); w->prow = d(q.oProw); w->nrm = d(q.oNrm); w->scl = d(q.oScl);
    w->perm = reinterpret_cast<int *>(ws + q.oPerm);
    w->bar = reinterpret_cast<unsigned *>(ws + q.oBar);
    w->abort_flag = reinterpret_cast<int *>(ws + q.oBar + 8);
    w->d_range = d(q.oBar + 64);
    return JSVD_OK;
}

// Blocked Householder QR of w.W (m x n, ld m) in place (eq. (2.1) without
// the column permutation): reflectors below the diagonal (LAPACK's
// convention, v(k) = 1 implicit), R on and above it, T of each panel's
// compact WY form in w.T.  A panel barrier that cannot complete sets
// w.abort_flag (read by the caller).
int hh_factor(jsvd_handle_s *h, const QrWork &w, int64_t m, int64_t n) {
    hipStream_t st = h->stream;
    constexpr int NB = kQrPanel;
    const int64_t npan = (n + NB - 1) / NB;
    HIP_TRY(launch_qr_reset(w.bar, w.abort_flag, st));
    for (int64_t p = 0; p < npan; ++p) {
        const int64_t j = p * NB;
        const int nb = (int)std::min<int64_t>(NB, n - j);
        const int64_t rows = m - j;
        QrPanelArgs qa;
        qa.W = w.W; qa.ldw = m; qa.m = m; qa.n = n; qa.j = j; qa.nb = nb;
        qa.tau = w.tau; qa.Vp = w.Vp; qa.ldvp = m; qa.partials = w.part; qa.prow = w.prow;
        qa.bar = w.bar; qa.abort_flag = w.abort_flag; qa.nwg = qr_panel_groups(rows);
        HIP_TRY(launch_qr_panel(qa, st));
        // T of the panel from V^T V
        int rc = gemm_splitk(w.Vp, m, w.Vp, m, NB, NB, rows, w.parts, w.parts_cap, w.Y1, st);
        if (rc) return rc;
        HIP_TRY(launch_qr_t(w.Y1, w.tau + j, nb, w.T + p * NB * NB, st));
        if (j + nb < n) {
            // trailing columns: C <- C - V T^T (V^T C)
            const int nc = (int)(n - j - nb);
            double *C = w.W + j + (j + nb) * m;
            if ((rc = gemm_splitk(w.Vp, m, C, m, NB, nc, rows, w.parts, w.parts_cap, w.Y1, st))) return rc;
            if ((rc = gemm_plain(true, w.T + p * NB * NB, NB, w.Y1, NB, w.Y2, NB, NB, nc, NB, 1.0,
                                 0.0, st)))
                return rc;
            if ((rc = gemm_plain(false, w.Vp, m, w.Y2, NB, C, m, (int)rows, nc, NB, -1.0, 1.0, st)))
                return rc;
        }
    }
    return JSVD_OK;
}

// B <- Q B for B m x ncols (ld ldb), Q the product of the reflectors that
// hh_factor left in w.W: the panels applied in reverse order.
int hh_apply_q(jsvd_handle_s *h, const QrWork &w, int64_t m, int64_t n, double *B, int64_t ldb,
               int64_t ncols) {
    hipStream_t st = h->stream;
    constexpr int NB = kQrPanel;
    const int64_t npan = (n + NB - 1) / NB;
    for (int64_t p = npan - 1; p >= 0; --p) {
        const int64_t j = p * NB;
        const int nb = (int)std::min<int64_t>(NB, n - j);
        const int64_t rows = m - j;
        HIP_TRY(launch_qr_extract_v(w.W, m, m, j, nb, w.Vp, m, st));
        double *Bj = B + j;
        int rc = gemm_splitk(w.Vp, m, Bj, ldb, NB, (int)ncols, rows, w.parts, w.parts_cap, w.Y1, st);
        if (rc) return rc;
        if ((rc = gemm_plain(false, w.T + p * NB * NB, NB, w.Y1, NB, w.Y2, NB, NB, (int)ncols, NB,
                             1.0, 0.0, st)))
            return rc;
        if ((rc = gemm_plain(false, w.Vp, m, w.Y2, NB, Bj, ldb, (int)rows, (int)ncols, NB, -1.0,
                             1.0, st)))
            return rc;
    }
    return JSVD_OK;
}

// T of each panel of reflectors that are already in w.W (m rows, ld m, n of
// them, tau in w.tau), so that hh_apply_q can apply them: the part of
// hh_factor that follows the panel factorization.
int hh_build_t(jsvd_handle_s *h, const QrWork &w, int64_t m, int64_t n) {
    hipStream_t st = h->stream;
    constexpr int NB = kQrPanel;
    const int64_t npan = (n + NB - 1) / NB;
    for (int64_t p = 0; p < npan; ++p) {
        const int64_t j = p * NB;
        const int nb = (int)std::min<int64_t>(NB, n - j);
        HIP_TRY(launch_qr_extract_v(w.W, m, m, j, nb, w.Vp, m, st));
        int rc = gemm_splitk(w.Vp, m, w.Vp, m, NB, NB, m - j, w.parts, w.parts_cap, w.Y1, st);
        if (rc) return rc;
        HIP_TRY(launch_qr_t(w.Y1, w.tau + j, nb, w.T + p * NB * NB, st));
    }
    return JSVD_OK;
}

// After hh_factor: whether a panel's grid barrier failed, whether R's
// diagonal (in w.W) holds a NaN or an infinity (G was not finite), and
// whether R is numerically singular (finite, min |r_ii| <= n 2^-53 max
// |r_jj|); one stream synchronisation, the values read through the handle's
// pinned words.
int qr_check(jsvd_handle_s *h, const QrWork &w, int64_t m, int64_t n, bool *aborted,
             bool *singular, bool *nonfinite = nullptr) {
    hipStream_t st = h->stream;
    HIP_TRY(launch_diag_range(w.W, m, n, w.d_range, st));
    int *hab = reinterpret_cast<int *>(h->host_counters + kSlotFlag);
    double *range = reinterpret_cast<double *>(h->host_counters + kSlotRange);
    HIP_TRY(hipMemcpyAsync(hab, w.abort_flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(range, w.d_range, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *aborted = *hab != 0;
    const bool fin = std::isfinite(range[0]) && std::isfinite(range[1]);
    if (nonfinite) *nonfinite = !fin;
    *singular = fin && !(range[0] > (double)n * 0x1p-53 * range[1]);
    return JSVD_OK;
}

// Rank-deficient G after G P = Q_1 [R; 0] (eqs. (2.1)-(2.2)): the pivoted
// QR of R, R P_2 = Q_2 [R_0; ~0] with R_0 k x n of full row rank k; the LQ
// factorization of R_0 as the QR of R_0^T = Q_3 [L_0^T; 0]; the Jacobi method
// on L_0 (k x k), L_0 V_x = U_x Sigma_k; then
//   U = Q_1 [Q_2 [U_x; 0]; 0] (k columns; the other n - k zero),
//   V = P P_2 Q_3 [V_x 0; 0 I_(n-k)],  Sigma = (Sigma_k, 0).
// Sets *fallback (nothing written to A, S, V) when a factorization's grid
// barrier did not complete or k = 0; the caller then solves G directly.
int gesvd_rank_deficient(jsvd_handle_s *h, const QrWork &w1, int64_t m, int64_t n, double *A,
                         int64_t lda, double *S, double *V, int64_t ldv, const jsvd_opts &o,
                         jsvd_info *info, bool *fallback,
                         std::chrono::steady_clock::time_point t0) {
    hipStream_t st = h->stream;
    constexpr int NB = kQrPanel;
    *fallback = true;
    const int64_t nn = n * n;
    const int64_t npan = (n + NB - 1) / NB;
    const int nwg = (int)std::max<int64_t>(
        1, std::min<int64_t>({n, (int64_t)std::max(1, h->cu_count), (int64_t)qrcp_resident(h->cu_count)}));
    // workspace: seven n x n matrices, the two reflector sets' T, tau, the
    // pivoted QR's norms and candidates, and the GEMM scratch of hh_*
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off += align_up(bytes, 256); return at; };
    const size_t oRn = take(nn * 8), oR2 = take(nn * 8), oX = take(nn * 8), oL0 = take(nn * 8),
                 oVx = take(nn * 8), oB1 = take(nn * 8), oC = take(nn * 8),
                 oT2 = take(npan * NB * NB * 8), oT3 = take(npan * NB * NB * 8),
                 oTau2 = take(n * 8), oTau3 = take(n * 8), oVn1 = take(n * 8), oVn2 = take(n * 8),
                 oVn0 = take(n * 8), oCr = take(2 * (size_t)nwg * 8),
                 oCv = take(2 * (size_t)nwg * 8), oCi = take(2 * (size_t)nwg * 4),
                 oJp = take(n * 4), oRow = take(n * 4), oVp = take((size_t)n * NB * 8),
                 oParts = take((size_t)32 * NB * n * 8), oY1 = take((size_t)NB * n * 8),
                 oY2 = take((size_t)NB * n * 8), oPart = take((size_t)2 * 64 * NB * 8),
                 oProw = take((size_t)2 * NB * 8), oBar = take(128);
    if (off > h->qr_ws2_bytes) {
        if (h->qr_ws2) {
            if (hipStreamSynchronize(st) != hipSuccess) return JSVD_HIP_ERROR;
            (void)hipFree(h->qr_ws2);
        }
        h->qr_ws2 = nullptr;
        h->qr_ws2_bytes = 0;
        if (hipMalloc(&h->qr_ws2, off) != hipSuccess) {
            h->qr_ws2 = nullptr;
            return JSVD_NO_MEMORY;
        }
        h->qr_ws2_bytes = off;
    }
    char *ws = static_cast<char *>(h->qr_ws2);
    auto d = [&](size_t o2) { return reinterpret_cast<double *>(ws + o2); };
    double *Rn = d(oRn), *R2 = d(oR2), *X = d(oX), *L0 = d(oL0), *Vx = d(oVx), *B1 = d(oB1),
           *C = d(oC);
    int *jpvt = reinterpret_cast<int *>(ws + oJp), *rowof = reinterpret_cast<int *>(ws + oRow);
    unsigned *bar = reinterpret_cast<unsigned *>(ws + oBar);
    int *abort_flag = reinterpret_cast<int *>(ws + oBar + 8);
    int *rank_d = reinterpret_cast<int *>(ws + oBar + 16);
    // the reflector sets of the pivoted QR (in R2) and of the LQ step (in X)
    QrWork w2{}, w3{};
    for (QrWork *q : {&w2, &w3}) {
        q->Vp = d(oVp); q->parts = d(oParts); q->Y1 = d(oY1); q->Y2 = d(oY2);
        q->parts_cap = (int64_t)32 * NB * n;
        q->part = d(oPart); q->prow = d(oProw); q->bar = bar; q->abort_flag = abort_flag;
        q->d_range = d(oBar + 64);
    }
    w2.W = R2; w2.T = d(oT2); w2.tau = d(oTau2);
    w3.W = X; w3.T = d(oT3); w3.tau = d(oTau3);

    // R P_2 = Q_2 R_2 with column pivoting, stopped at the numerical rank k
    HIP_TRY(hipMemcpy2DAsync(Rn, (size_t)n * 8, w1.W, (size_t)m * 8, (size_t)n * 8, (size_t)n,
                             hipMemcpyDeviceToDevice, st));
    HIP_TRY(launch_zero_lower(Rn, n, n, st));
    QrcpArgs qa;
    qa.W = Rn; qa.ldw = n; qa.rows = n; qa.ncols = n; qa.tau = w2.tau; qa.jpvt = jpvt;
    qa.vn1 = d(oVn1); qa.vn2 = d(oVn2); qa.vn0 = d(oVn0); qa.cand_v = d(oCv); qa.cand_r = d(oCr);
    qa.cand_i = reinterpret_cast<int *>(ws + oCi); qa.rank = rank_d; qa.bar = bar;
    qa.abort_flag = abort_flag; qa.nwg = nwg; qa.tol = (double)n * 0x1p-53;
    HIP_TRY(launch_qrcp(qa, st));
    int *hk = reinterpret_cast<int *>(h->host_counters + kSlotFlag);
    int *hab = reinterpret_cast<int *>(h->host_counters + kSlotFlag + 1);
    HIP_TRY(hipMemcpyAsync(hk, rank_d, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hab, abort_flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int64_t k = *hk;
    // fall back on a failed barrier, a zero R, or full numerical rank (R's
    // small diagonal came from a graded, not a dependent, G)
    if (*hab != 0 || k <= 0 || k >= n) return JSVD_OK;
    // R_2 in pivoted (logical) column order, then X = R_0^T (n x k)
    HIP_TRY(launch_gather_cols(Rn, n, R2, n, n, n, jpvt, nullptr, nullptr, st));
    HIP_TRY(launch_trap_transpose(R2, n, k, n, X, n, st));
    // LQ of R_0: X = Q_3 [L_0^T; 0]
    int rc = hh_factor(h, w3, n, k);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(hab, abort_flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (*hab != 0) return JSVD_OK;  // fall back
    *fallback = false;
    HIP_TRY(launch_r_transpose(X, n, k, L0, k, st));
    // the Jacobi method on L_0: L_0 V_x = U_x Sigma_k (L0 <- U_x)
    jsvd_opts oj = o;
    oj.want_v = 1;
    oj.qr = 1;
    oj.sort = 1;
    jsvd_info inf{};
    const int status = solve(h, k, k, L0, k, S, Vx, k, k, oj, &inf, false, nullptr);
    if (status != JSVD_OK && status != JSVD_NOT_CONVERGED) return status;
    HIP_TRY(launch_fill(S + k, n - k, 0.0, st));
    // U = Q_1 [Q_2 [U_x; 0]; 0]
    if ((rc = hh_build_t(h, w2, n, k))) return rc;
    HIP_TRY(launch_embed(L0, k, k, B1, n, n, k, st));
    if ((rc = hh_apply_q(h, w2, n, k, B1, n, k))) return rc;
    HIP_TRY(launch_embed(B1, n, n, A, lda, m, k, st));
    HIP_TRY(launch_fill2d(A + k * lda, lda, m, n - k, 0.0, st));
    if ((rc = hh_apply_q(h, w1, m, n, A, lda, k))) return rc;
    // V = P P_2 Q_3 [V_x 0; 0 I]
    if (o.want_v) {
        HIP_TRY(launch_embed(Vx, k, k, C, n, n, k, st));
        HIP_TRY(launch_identity_cols(C + k * n, n, n, n - k, k, st));
        if ((rc = hh_apply_q(h, w3, n, k, C, n, n))) return rc;
        HIP_TRY(launch_compose(w1.perm, jpvt, n, rowof, st));
        HIP_TRY(launch_scatter_rows(C, n, V, ldv, n, n, rowof, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    inf.preprocessed = 2;
    inf.rank = (int32_t)k;
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return status;
}

//
// scaled (a badly scaled G, §4.2): the columns are scaled by the powers of
// two of their norms before the factorization, W = G P D^-1 with D =
// diag(2^e_c), ||g_c|| in [2^e_c, 2^(e_c+1)) (exact), so that no sum of the
// Householder reflections leaves the normal range; then G P = Q (R~ D) and
// the Jacobi method runs on X = (R~ D)^T (whose columns the scaled mode of
// the Jacobi method handles).  A singular R~ sends G to the direct method.
int gesvd_qr(jsvd_handle_s *h, int64_t m, int64_t n, double *A, int64_t lda, double *S,
             double *V, int64_t ldv, const jsvd_opts &o, jsvd_info *info, bool scaled = false) {
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = h->stream;
    QrWork w;
    int rc = qr_workspace(h, qr_plan(m, n), &w);
    if (rc) return rc;

    // presort: W = G P, columns by non-increasing norm (ties by index)
    double *dscale = w.scl + n;  // scaled: W's column k is G's perm[k] over dscale[k]
    if (scaled) {
        // norms and exponents by DRDSSQ (Appendix A); h->colexp was sized by
        // the caller's scaling check
        HIP_TRY(launch_colexp(A, lda, m, n, w.nrm, h->colexp, nullptr, st));
        HIP_TRY(launch_pow2(h->colexp, n, w.scl, st));
    } else {
        HIP_TRY(launch_colnorms(A, lda, m, n, w.nrm, st));
    }
    HIP_TRY(launch_rank(w.nrm, n, n, w.perm, st));
    HIP_TRY(launch_gather_cols(A, lda, w.W, m, m, n, w.perm, scaled ? w.scl : nullptr,
                               scaled ? dscale : nullptr, st));
    if ((rc = hh_factor(h, w, m, n))) return rc;
    // A grid barrier of the panel kernel that did not complete (some panel
    // workgroups could not start beside other work on the device), or R
    // numerically singular (dependent columns): solve G directly, so that V
    // stays orthogonal and zero singular values stay exact.  G itself is
    // untouched so far (the factorization works on the copy W).
    bool aborted = false, singular = false;
    bool nonfinite = false;
    if ((rc = qr_check(h, w, m, n, &aborted, &singular, &nonfinite))) return rc;
    if (!aborted && singular && !scaled) {
        bool fallback = false;
        rc = gesvd_rank_deficient(h, w, m, n, A, lda, S, V, ldv, o, info, &fallback, t0);
        if (!fallback) return rc;
    }
    if (aborted || singular || nonfinite) {  // the direct method reports a NaN in G
        jsvd_opts od = o;
        od.qr = 1;
        return solve(h, m, n, A, lda, S, V, ldv, n, od, info, false, nullptr);
    }

    // Jacobi on X = R^T (scaled: (R~ D)^T): X V_x = U_x Sigma
    HIP_TRY(launch_r_transpose(w.W, m, n, w.X, n, st, scaled ? dscale : nullptr));
    jsvd_opts oj = o;
    oj.want_v = 1;
    oj.qr = 1;
    jsvd_info inf{};
    int status = solve(h, n, n, w.X, n, S, w.Vx, n, n, oj, &inf, false, nullptr);
    if (status != JSVD_OK && status != JSVD_NOT_CONVERGED) return status;

    // U = Q [V_x; 0]
    HIP_TRY(launch_embed(w.Vx, n, n, A, lda, m, n, st));
    if ((rc = hh_apply_q(h, w, m, n, A, lda, n))) return rc;
    // V = P U_x: row i of U_x is row perm[i] of V
    if (o.want_v) HIP_TRY(launch_scatter_rows(w.X, n, V, ldv, n, n, w.perm, st));
    HIP_TRY(hipStreamSynchronize(st));
    inf.preprocessed = 1;
    inf.rank = (int32_t)n;
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return status;
}

// Strategy tables of every supported order <= strategy_order(kBatchMaxN)
// (R-reverse) for the batched kernels, and the LDS they may take.
int ensure_batch_tables(jsvd_handle_s *h) {
    if (h->batch_tables) return JSVD_OK;
    std::vector<unsigned char> flat;
    std::vector<int> tbl_order(kBatchMaxN + 1, 2);
    const int top = strategy_order(kBatchMaxN);
    std::vector<int64_t> tbl_off(top / 2 + 1, 0);
    for (int N = 2; N <= top; N += 2) {
        if (strategy_order(N) != N) continue;
        Table t;
        if (!make_table(N, JSVD_STRAT_RREV, t)) return JSVD_HIP_ERROR;
        if (N == kBatchInnerOrder) order_for_banks(t);  // the blocked method's inner sweeps
        tbl_off[N / 2] = (int64_t)flat.size();
        for (const auto &stp : t)
            for (const auto &pr : stp) {
                flat.push_back((unsigned char)pr.first);
                flat.push_back((unsigned char)pr.second);
            }
    }
    for (int k = 1; k <= kBatchMaxN; ++k) tbl_order[k] = strategy_order(k);
    void *tables = nullptr, *meta = nullptr;
    const size_t meta_bytes =
        align_up(tbl_order.size() * sizeof(int), 256) + tbl_off.size() * sizeof(int64_t);
    if (hipMalloc(&tables, flat.size()) != hipSuccess) return JSVD_NO_MEMORY;
    if (hipMalloc(&meta, meta_bytes) != hipSuccess) {
        (void)hipFree(tables);
        return JSVD_NO_MEMORY;
    }
    h->batch_tables = tables;
    h->batch_meta = meta;
    HIP_TRY(hipMemcpy(h->batch_tables, flat.data(), flat.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(h->batch_meta, tbl_order.data(), tbl_order.size() * sizeof(int),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(static_cast<char *>(h->batch_meta) +
                          align_up(tbl_order.size() * sizeof(int), 256),
                      tbl_off.data(), tbl_off.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, h->device));
    h->cu_count = prop.multiProcessorCount;
    // LDS for the working copy of G: what the CU has, less the static part
    const size_t lds_total = prop.sharedMemPerMultiprocessor ? prop.sharedMemPerMultiprocessor
                                                             : prop.sharedMemPerBlock;
    h->batch_lds = (int)std::min<size_t>(lds_total, 160 * 1024) - 12 * 1024;
    if (h->batch_lds < 0 || batched_set_lds(h->batch_lds) != hipSuccess) h->batch_lds = 0;
    return JSVD_OK;
}

// Launch geometry and workspace carve-up of a batched call: the work order
// histogram, the order itself and the queue counters.
struct BatchPlan {
    int grid, bgrid;
    size_t off_hist, off_order, off_queue, total;
};

constexpr size_t batch_off_order() { return ((kBatchMaxN + 1) * sizeof(int) + 255) / 256 * 256; }
constexpr size_t batch_off_queue(int64_t batch) {
    return batch_off_order() + ((size_t)batch * sizeof(int32_t) + 255) / 256 * 256;
}
constexpr size_t batch_ws_bytes(int64_t batch) { return batch_off_queue(batch) + 256; }

BatchPlan batch_plan(const jsvd_handle_s *h, int64_t batch) {
    BatchPlan p;
    const int cus = std::max(1, h->cu_count);
    p.grid = (int)std::min<int64_t>(std::max<int64_t>(batch, 1), cus);
    p.bgrid = (int)std::min<int64_t>(std::max<int64_t>(batch, 1), 2 * (int64_t)cus);
    p.off_hist = 0;
    p.off_order = batch_off_order();
    p.off_queue = batch_off_queue(batch);
    p.total = batch_ws_bytes(batch);
    return p;
}

// ------------------------------------------- allocation-free batched call
// The work order and queue counters of jsvd_gesvd_batched_noalloc live in
// this fixed device array (each device the library runs on holds its own
// copy until the process ends).  In host code `scratch` only names the
// symbol: its device address comes from hipGetSymbolAddress, taken once per
// device when a handle is created there, and only that address is passed on.
constexpr size_t kNoAllocScratchBytes = batch_ws_bytes(JSVD_NOALLOC_MAX_BATCH);
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mutex;
std::map<int, void *> g_scratch_ptr;  // device -> address of its scratch

// With `device` current: the device address of its scratch (null on error).
void *device_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) return it->second;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) ptr = nullptr;
    if (ptr) g_scratch_ptr.emplace(device, ptr);
    return ptr;
}

int check_batched_sizes(jsvd_handle_t h, int64_t batch, int32_t max_m, int32_t max_n) {
    if (!h) return -1;
    if (batch < 0) return -2;
    if (max_m < 1 || max_m > (1 << 20)) return -3;
    if (max_n < 1 || max_n > kBatchMaxN || max_n > max_m) return -4;
    return JSVD_OK;
}

int check_opts(const jsvd_opts &o) {
    if (o.block_w != 0 && o.block_w != 16 && o.block_w != 32 && o.block_w != 64) return -1;
    if (o.strategy < JSVD_STRAT_RREV || o.strategy > JSVD_STRAT_RR) return -1;
    if (o.max_sweeps < 1 || o.max_inner_sweeps < 0) return -1;
    if (o.qr < 0 || o.qr > 2) return -1;
    if (o.scaled < 0 || o.scaled > 2) return -1;
    if (o.factorize < 0 || o.factorize > 1) return -1;
    if (o.fuse < 0 || o.fuse > 1) return -1;
    return JSVD_OK;
}

// Whether jsvd_gesvd takes the QR path (before the scaling check, which can
// still send a badly scaled G to the direct method).
bool wants_qr(const jsvd_handle_s *h, const jsvd_opts &o, int64_t m, int64_t n) {
    return (o.qr == 2 || (o.qr == 0 && m >= 2 * n)) && m <= 32768 && n >= 1 &&
           qr_panel_groups(m) <= h->qr_resident;
}

int check_common(jsvd_handle_t h, int64_t m, int64_t n, double *A, int64_t lda,
                 const jsvd_opts &o) {
    if (!h) return -1;
    if (m < 1 || m < n) return -2;
    if (n < 1) return -3;
    if (!A) return -4;
    if (lda < m) return -5;
    if (check_opts(o)) return -9;
    if (m > (int64_t)1 << 31 || n > (int64_t)1 << 20) return -2;
    return JSVD_OK;
}

}  // namespace

extern "C" {

int jsvd_default_opts(jsvd_opts *opts) {
    if (!opts) return -1;
    *opts = defaults();
    return JSVD_OK;
}

int jsvd_create(jsvd_handle_t *h, void *hip_stream) {
    if (!h) return -1;
    auto *p = new (std::nothrow) jsvd_handle_s();
    if (!p) return JSVD_NO_MEMORY;
    if (hipGetDevice(&p->device) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&p->host_counters),
                      kHostSlots * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
        delete p;
        return JSVD_HIP_ERROR;
    }
    std::memset(p->host_counters, 0, kHostSlots * sizeof(unsigned long long));
    p->stream = static_cast<hipStream_t>(hip_stream);
    if (hipDeviceGetAttribute(&p->cu_count, hipDeviceAttributeMultiprocessorCount, p->device) !=
        hipSuccess)
        p->cu_count = 0;
    p->qr_resident = qr_panel_resident(p->cu_count);
    // the fixed scratch of the allocation-free batched call on this device
    p->noalloc_scratch = device_scratch(p->device);
    // the batched path's strategy tables, so that its first call need not
    // allocate them
    const int rc = ensure_batch_tables(p);
    if (rc) {
        jsvd_destroy(p);
        return rc;
    }
    *h = p;
    return JSVD_OK;
}

int jsvd_set_stream(jsvd_handle_t h, void *hip_stream) {
    if (!h) return -1;
    h->stream = static_cast<hipStream_t>(hip_stream);
    return JSVD_OK;
}

int jsvd_set_tuning(jsvd_handle_t h, const jsvd_tuning *t) {
    if (!h) return -1;
    if (!t) {
        h->tuning = jsvd_tuning{};
        return JSVD_OK;
    }
    if (t->count < 0 || t->count > 8) return -2;
    for (int i = 0; i < t->count; ++i) {
        if (t->block_w[i] != 16 && t->block_w[i] != 32 && t->block_w[i] != 64) return -2;
        if (i > 0 && t->n_upper[i] <= t->n_upper[i - 1]) return -2;
        if (t->gram_wg[i] != 0 && (t->gram_wg[i] < 64 || t->gram_wg[i] > 8192)) return -2;
        if (t->update_wg[i] != 0 && (t->update_wg[i] < 64 || t->update_wg[i] > 8192)) return -2;
    }
    if (t->batch_g_groups != 0 && (t->batch_g_groups < 4 || t->batch_g_groups > 28)) return -2;
    if (t->batch_block_min_n != 0 && (t->batch_block_min_n < 33 || t->batch_block_min_n > 257))
        return -2;
    h->tuning = *t;
    return JSVD_OK;
}

int jsvd_destroy(jsvd_handle_t h) {
    if (!h) return -1;
    (void)hipStreamSynchronize(h->stream);
    if (h->ws) (void)hipFree(h->ws);
    if (h->bws) (void)hipFree(h->bws);
    for (void *p : h->bws_retired) (void)hipFree(p);
    for (auto &kv : h->block_tables) (void)hipFree(kv.second.ptr);
    for (auto &kv : h->inner_tables) (void)hipFree(kv.second.ptr);
    for (auto &kv : h->quad_tables)
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    if (h->batch_tables) (void)hipFree(h->batch_tables);
    if (h->batch_meta) (void)hipFree(h->batch_meta);
    if (h->host_counters) (void)hipHostFree(h->host_counters);
    if (h->qr_ws) (void)hipFree(h->qr_ws);
    if (h->qr_ws2) (void)hipFree(h->qr_ws2);
    if (h->colexp) (void)hipFree(h->colexp);
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    delete h;
    return JSVD_OK;
}

int jsvd_gesvd(jsvd_handle_t h, int64_t m, int64_t n, double *A, int64_t lda, double *S,
               double *V, int64_t ldv, const jsvd_opts *opts, jsvd_info *info) {
    const jsvd_opts o = opts ? *opts : defaults();
    int rc = check_common(h, m, n, A, lda, o);
    if (rc) return rc == -9 ? -9 : rc;
    if (!S) return -6;
    if (o.want_v && !V) return -7;
    if (o.want_v && ldv < n) return -8;
    if (hipSetDevice(h->device) != hipSuccess) return JSVD_HIP_ERROR;
    bool qr = wants_qr(h, o, m, n);
    bool bad = false;
    if (qr && o.scaled != 1) {
        // a badly scaled G takes the QR with its columns scaled by powers of
        // two (gesvd_qr)
        if ((rc = column_exponents(h, m, n, A, lda, o.scaled == 0 ? &bad : nullptr))) return rc;
        bad = bad || o.scaled == 2;
    }
    if (qr) return gesvd_qr(h, m, n, A, lda, S, V, ldv, o, info, bad);
    return solve(h, m, n, A, lda, S, V, ldv, n, o, info, false, nullptr);
}

int jsvd_gesvd_full(jsvd_handle_t h, int64_t m, int64_t n, double *A, int64_t lda, double *U,
                    int64_t ldu, double *S, double *V, int64_t ldv, const jsvd_opts *opts,
                    jsvd_info *info) {
    jsvd_opts o = opts ? *opts : defaults();
    int rc = check_common(h, m, n, A, lda, o);
    if (rc) return rc == -9 ? -11 : rc;
    if (m > 32768) return -2;
    if (!U) return -6;
    if (ldu < m) return -7;
    if (!S) return -8;
    if (o.want_v && !V) return -9;
    if (o.want_v && ldv < n) return -10;
    o.sort = 1;  // the completion relies on the zero singular values coming last
    if ((rc = jsvd_gesvd(h, m, n, A, lda, S, V, ldv, &o, info)) != JSVD_OK &&
        rc != JSVD_NOT_CONVERGED)
        return rc;
    const int status = rc;
    hipStream_t st = h->stream;
    // k = number of positive singular values; U's columns k .. n-1 are zero
    int *hk = reinterpret_cast<int *>(h->host_counters + kSlotFlag);
    {
        QrWork w;
        if ((rc = qr_workspace(h, qr_plan(m, n, m), &w))) return rc;
        HIP_TRY(launch_count_positive(S, n, w.perm, st));
        HIP_TRY(hipMemcpyAsync(hk, w.perm, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const int64_t k = *hk;
        // Q R = U (Householder); Q's columns k .. m-1 are orthogonal to the
        // first k columns of U, which Q spans
        HIP_TRY(hipMemcpy2DAsync(w.W, (size_t)m * sizeof(double), A, (size_t)lda * sizeof(double),
                                 (size_t)m * sizeof(double), (size_t)n, hipMemcpyDeviceToDevice,
                                 st));
        if ((rc = hh_factor(h, w, m, n))) return rc;
        bool aborted = false, singular = false;
        if ((rc = qr_check(h, w, m, n, &aborted, &singular))) return rc;
        if (aborted) return JSVD_HIP_ERROR;
        if (k > 0)
            HIP_TRY(hipMemcpy2DAsync(U, (size_t)ldu * sizeof(double), A,
                                     (size_t)lda * sizeof(double), (size_t)m * sizeof(double),
                                     (size_t)k, hipMemcpyDeviceToDevice, st));
        if (k < m) {
            double *Ck = U + k * ldu;
            HIP_TRY(launch_identity_cols(Ck, ldu, m, m - k, k, st));
            if ((rc = hh_apply_q(h, w, m, n, Ck, ldu, m - k))) return rc;
        }
        HIP_TRY(hipStreamSynchronize(st));
    }
    return status;
}

int jsvd_hsvd(jsvd_handle_t h, int64_t m, int64_t n, double *A, int64_t lda, const int8_t *J,
              int8_t *J_out, double *S, double *V, int64_t ldv, const jsvd_opts *opts,
              jsvd_info *info) {
    const jsvd_opts o = opts ? *opts : defaults();
    int rc = check_common(h, m, n, A, lda, o);
    if (rc) return rc == -9 ? -11 : rc;
    if (!J) return -6;
    if (!S) return -8;
    if (o.want_v && !V) return -9;
    if (o.want_v && ldv < n) return -10;
    std::vector<int> perm_in;  // stable partition: positives first
    for (int64_t i = 0; i < n; ++i) {
        if (J[i] != 1 && J[i] != -1) return -6;
        if (J[i] == 1) perm_in.push_back((int)i);
    }
    const int64_t n_plus = (int64_t)perm_in.size();
    for (int64_t i = 0; i < n; ++i)
        if (J[i] == -1) perm_in.push_back((int)i);
    bool identity = true;
    for (int64_t i = 0; i < n; ++i) identity = identity && perm_in[i] == i;
    if (hipSetDevice(h->device) != hipSuccess) return JSVD_HIP_ERROR;
    if (!identity) {
        // permute the columns of G so that J = diag(I, -I)
        const size_t tmp_bytes = align_up((size_t)m * n * sizeof(double), 256);
        if ((rc = ensure_workspace(h, tmp_bytes + (size_t)n * sizeof(int)))) return rc;
        double *tmp = static_cast<double *>(h->ws);
        int *pd = reinterpret_cast<int *>(static_cast<char *>(h->ws) + tmp_bytes);
        HIP_TRY(hipMemcpyAsync(pd, perm_in.data(), n * sizeof(int), hipMemcpyHostToDevice,
                               h->stream));
        HIP_TRY(hipMemcpy2DAsync(tmp, m * sizeof(double), A, lda * sizeof(double),
                                 m * sizeof(double), n, hipMemcpyDeviceToDevice, h->stream));
        HIP_TRY(launch_gather_cols(tmp, m, A, lda, m, n, pd, nullptr, nullptr, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    rc = solve(h, m, n, A, lda, S, V, ldv, n_plus, o, info, true,
               identity ? nullptr : perm_in.data());
    if (J_out)
        for (int64_t i = 0; i < n; ++i) J_out[i] = (int8_t)(i < n_plus ? 1 : -1);
    return rc;
}

int jsvd_strategy_table(int32_t order, int32_t kind, int32_t *pairs) {
    if (kind < JSVD_STRAT_RREV || kind > JSVD_STRAT_RR) return -2;
    if (!pairs) return -3;
    if (order < 2 || order % 2 || strategy_order(order) != order || order > 4096) return -1;
    Table t;
    if (!make_table(order, kind, t)) return -1;
    size_t k = 0;
    for (const auto &st : t)
        for (const auto &pr : st) {
            pairs[k++] = pr.first + 1;
            pairs[k++] = pr.second + 1;
        }
    return JSVD_OK;
}

int jsvd_inner_table(int32_t order, int32_t kind, int32_t *pairs) {
    if (kind < JSVD_STRAT_RREV || kind > JSVD_STRAT_RR) return -2;
    if (!pairs) return -3;
    if (order != 32 && order != 64) return -1;
    Table t;
    if (!make_table(order, kind, t)) return -1;
    order_for_banks(t);
    size_t k = 0;
    for (const auto &st : t)
        for (const auto &pr : st) {
            pairs[k++] = pr.first + 1;
            pairs[k++] = pr.second + 1;
        }
    return JSVD_OK;
}

int jsvd_quad_table(int32_t order, int32_t kind, int32_t *quads) {
    if (kind < JSVD_STRAT_RREV || kind > JSVD_STRAT_RR) return -2;
    if (!quads) return -3;
    Table t;
    if (!make_table(order, kind, t)) return -1;
    std::vector<int> flat;
    if (!make_quads(t, flat)) return 1;
    std::copy(flat.begin(), flat.end(), quads);
    return JSVD_OK;
}

int32_t jsvd_strategy_order(int32_t nb) { return strategy_order(nb); }

int32_t jsvd_batched_block_min_n(jsvd_handle_t h) {
    if (!h) return -1;
    return h->tuning.batch_block_min_n ? h->tuning.batch_block_min_n : kBatchBlockMinN;
}

}  // extern "C"

namespace {

// Arguments of a batched call (jsvd_gesvd_batched's numbering).
int check_batched_args(jsvd_handle_t h, int64_t batch, int32_t max_m, int32_t max_n,
                       const int32_t *m, const int32_t *n, const int64_t *a_off,
                       const int64_t *s_off, const int64_t *v_off, const double *A,
                       const double *S, const double *V, const jsvd_opts &o) {
    int rc0 = check_batched_sizes(h, batch, max_m, max_n);
    if (rc0) return rc0;
    if (!m) return -5;
    if (!n) return -6;
    if (!a_off) return -7;
    if (!s_off) return -8;
    if (o.want_v && !v_off) return -9;
    if (!A) return -10;
    if (!S) return -11;
    if (o.want_v && !V) return -12;
    if (o.max_sweeps < 1 || o.scaled < 0 || o.scaled > 2) return -13;
    return JSVD_OK;
}

// Enqueue the batched solve with its workspace at ws (batch_plan(h,
// batch).total bytes): the work-order kernels, then the two persistent
// launches.  Allocates nothing.
int launch_batched_solve(jsvd_handle_s *h, int64_t batch, int32_t max_n, const int32_t *m,
                         const int32_t *n, const int64_t *a_off, const int64_t *s_off,
                         const int64_t *v_off, double *A, double *S, double *V,
                         const jsvd_opts &o, int32_t *status, int32_t *sweeps, char *ws) {
    const BatchPlan bp = batch_plan(h, batch);
    BatchArgs b;
    b.count = batch;
    b.m = m;
    b.n = n;
    b.a_off = a_off;
    b.s_off = s_off;
    b.v_off = o.want_v ? v_off : nullptr;
    b.A = A;
    b.S = S;
    b.V = o.want_v ? V : nullptr;
    b.order = reinterpret_cast<int32_t *>(ws + bp.off_order);
    b.queue = reinterpret_cast<int *>(ws + bp.off_queue);
    b.tbl_order = static_cast<const int *>(h->batch_meta);
    b.tbl_off = reinterpret_cast<const int64_t *>(
        static_cast<char *>(h->batch_meta) + align_up((kBatchMaxN + 1) * sizeof(int), 256));
    b.tbls = static_cast<const unsigned char *>(h->batch_tables);
    b.max_sweeps = o.max_sweeps;
    b.status = status;
    b.sweeps = sweeps;
    b.lds_doubles = h->batch_lds / (int64_t)sizeof(double);
    // the end of a problem permutes its columns through LDS, a band of rows
    // of all columns at a time
    if (b.lds_doubles < kBatchMaxN) return JSVD_HIP_ERROR;
    b.g_groups = h->tuning.batch_g_groups ? h->tuning.batch_g_groups : 16;
    {
        const int mn = h->tuning.batch_block_min_n ? h->tuning.batch_block_min_n
                                                   : kBatchBlockMinN;
        const bool room = b.lds_doubles >= kBatchBlockLds;
        b.blk_min_n = (room && mn <= kBatchMaxN) ? mn : 0;
    }
    // opts.scaled = 2: DDRJAC pairs and DRDSSQ norms, every problem pointwise
    b.ddrjac = o.scaled == 2 ? 1 : 0;
    if (b.ddrjac) b.blk_min_n = 0;
    for (int lg = 0; lg < 32; ++lg) b.t_hi[lg] = b.ddrjac ? rdssq_t_hi(lg) : 0.0;
    HIP_TRY(launch_batched(b, bp.grid, bp.bgrid, max_n, reinterpret_cast<int *>(ws + bp.off_hist),
                           reinterpret_cast<int32_t *>(ws + bp.off_order), h->stream));
    return JSVD_OK;
}

}  // namespace

extern "C" {

int jsvd_gesvd_batched(jsvd_handle_t h, int64_t batch, int32_t max_m, int32_t max_n,
                       const int32_t *m, const int32_t *n, const int64_t *a_off,
                       const int64_t *s_off, const int64_t *v_off, double *A, double *S,
                       double *V, const jsvd_opts *opts, int32_t *status, int32_t *sweeps) {
    const jsvd_opts o = opts ? *opts : defaults();
    const int rc0 = check_batched_args(h, batch, max_m, max_n, m, n, a_off, s_off, v_off, A, S,
                                       V, o);
    if (rc0) return rc0;
    if (batch == 0) return JSVD_OK;
    if (hipSetDevice(h->device) != hipSuccess) return JSVD_HIP_ERROR;
    const bool capturing = stream_capturing(h->stream);
    if (!h->batch_tables) {
        if (capturing) return JSVD_NO_MEMORY;
        int rc = ensure_batch_tables(h);
        if (rc) return rc;
    }
    int rc = ensure_batch_workspace(h, batch_plan(h, batch).total, capturing);
    if (rc) return rc;
    if (capturing) h->bws_captured = true;
    return launch_batched_solve(h, batch, max_n, m, n, a_off, s_off, v_off, A, S, V, o, status,
                                sweeps, static_cast<char *>(h->bws));
}

int jsvd_gesvd_batched_noalloc(jsvd_handle_t h, int64_t batch, int32_t max_m, int32_t max_n,
                               const int32_t *m, const int32_t *n, const int64_t *a_off,
                               const int64_t *s_off, const int64_t *v_off, double *A, double *S,
                               double *V, const jsvd_opts *opts, int32_t *status,
                               int32_t *sweeps) {
    const jsvd_opts o = opts ? *opts : defaults();
    const int rc0 = check_batched_args(h, batch, max_m, max_n, m, n, a_off, s_off, v_off, A, S,
                                       V, o);
    if (rc0) return rc0;
    if (batch > JSVD_NOALLOC_MAX_BATCH) return -2;
    if (batch == 0) return JSVD_OK;
    if (!h->noalloc_scratch || !h->batch_tables) return JSVD_HIP_ERROR;
    if (batch_plan(h, batch).total > kNoAllocScratchBytes) return -2;
    if (hipSetDevice(h->device) != hipSuccess) return JSVD_HIP_ERROR;
    return launch_batched_solve(h, batch, max_n, m, n, a_off, s_off, v_off, A, S, V, o, status,
                                sweeps, static_cast<char *>(h->noalloc_scratch));
}

int jsvd_svd_backward(jsvd_handle_t h, int64_t batch, int64_t m, int64_t n, const double *U,
                      const double *S, const double *V, const double *dU, const double *dS,
                      const double *dV, double *dA) {
    if (!h) return -1;
    if (batch < 1) return -2;
    if (m < 1 || m < n || m > (1 << 24)) return -3;
    if (n < 1 || n > 32768) return -4;
    if (!U) return -5;
    if (!S) return -6;
    if (!V) return -7;
    if (!dA) return -11;
    if (hipSetDevice(h->device) != hipSuccess) return JSVD_HIP_ERROR;
    hipStream_t st = h->stream;
    const size_t nn = (size_t)n * n;
    const size_t off_J = 0;
    const size_t off_K = off_J + align_up((size_t)batch * nn * sizeof(double), 256);
    const size_t off_M = off_K + align_up((size_t)batch * nn * sizeof(double), 256);
    const size_t off_T = off_M + align_up((size_t)batch * nn * sizeof(double), 256);
    const size_t off_inv = off_T + align_up((size_t)batch * m * n * sizeof(double), 256);
    const size_t off_flag = off_inv + align_up((size_t)batch * n * sizeof(double), 256);
    int rc = ensure_workspace(h, off_flag + 256);
    if (rc) return rc;
    char *ws = static_cast<char *>(h->ws);
    double *J = dU ? reinterpret_cast<double *>(ws + off_J) : nullptr;
    double *K = dV ? reinterpret_cast<double *>(ws + off_K) : nullptr;
    double *Mp = reinterpret_cast<double *>(ws + off_M);
    double *T = reinterpret_cast<double *>(ws + off_T);
    double *inv_s = reinterpret_cast<double *>(ws + off_inv);
    int *flag = reinterpret_cast<int *>(ws + off_flag);

    GemmArgs g;
    g.batch = batch;
    g.E = nullptr;
    g.d = nullptr;
    g.lde = g.se = g.sd = 0;
    if (dU) {  // J = U^T dU  (n x n)
        g.M = (int)n; g.N = (int)n; g.K = (int)m; g.ta = true; g.tb = false;
        g.A = U; g.lda = m; g.sa = m * n;
        g.B = dU; g.ldb = m; g.sb = m * n;
        g.C = J; g.ldc = n; g.sc = (int64_t)nn;
        HIP_TRY(launch_gemm(g, st));
    }
    if (dV) {  // K = V^T dV  (n x n)
        g.M = (int)n; g.N = (int)n; g.K = (int)n; g.ta = true; g.tb = false;
        g.A = V; g.lda = n; g.sa = (int64_t)nn;
        g.B = dV; g.ldb = n; g.sb = (int64_t)nn;
        g.C = K; g.ldc = n; g.sc = (int64_t)nn;
        HIP_TRY(launch_gemm(g, st));
    }
    HIP_TRY(launch_adjoint_middle(batch, (int)n, S, n, dS, J, K, Mp, inv_s, flag, st));
    // T = U M' + dU diag(1/s)  (m x n)
    g.M = (int)m; g.N = (int)n; g.K = (int)n; g.ta = false; g.tb = false;
    g.A = U; g.lda = m; g.sa = m * n;
    g.B = Mp; g.ldb = n; g.sb = (int64_t)nn;
    g.C = T; g.ldc = m; g.sc = m * n;
    if (dU) {
        g.E = dU; g.lde = m; g.se = m * n;
        g.d = inv_s; g.sd = n;
    }
    HIP_TRY(launch_gemm(g, st));
    // dA = T V^T
    g.E = nullptr; g.d = nullptr;
    g.M = (int)m; g.N = (int)n; g.K = (int)n; g.ta = false; g.tb = true;
    g.A = T; g.lda = m; g.sa = m * n;
    g.B = V; g.ldb = n; g.sb = (int64_t)nn;
    g.C = dA; g.ldc = m; g.sc = m * n;
    HIP_TRY(launch_gemm(g, st));
    int *hflag = reinterpret_cast<int *>(h->host_counters + kSlotFlag);
    HIP_TRY(hipMemcpyAsync(hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return *hflag ? JSVD_DEGENERATE : JSVD_OK;
}

int jsvd_kernel_timing(jsvd_handle_t h, int enable) {
    if (!h) return -1;
    if (enable < 0) return -2;
    h->timing = enable != 0;
    h->timing_stride = enable > 0 ? enable : 1;
    for (int k = 0; k < 4; ++k) {
        h->kernel_ms[k] = 0.0;
        h->launches[k] = 0;
    }
    return JSVD_OK;
}

int jsvd_kernel_times(jsvd_handle_t h, double *ms, int64_t *launches) {
    if (!h) return -1;
    if (!ms) return -2;
    if (!launches) return -3;
    for (int k = 0; k < 4; ++k) {
        ms[k] = h->kernel_ms[k];
        launches[k] = h->launches[k];
    }
    return JSVD_OK;
}

const char *jsvd_error_string(int code) {
    switch (code) {
    case JSVD_OK: return "success";
    case JSVD_NOT_CONVERGED: return "not converged within the block sweep limit";
    case JSVD_NONFINITE: return "non-finite value in the input or the iteration";
    case JSVD_HIP_ERROR: return "HIP runtime error";
    case JSVD_DEGENERATE: return "equal singular values: the adjoint is undefined";
    case JSVD_NO_MEMORY:
        return "device workspace allocation failed (or a captured workspace would have to grow)";
    default: return code < 0 ? "invalid argument" : "unknown status";
    }
}

int jsvd_diag_fp64(jsvd_handle_t h, int64_t count, const double *a, const double *b,
                   double *quot, double *root) {
    if (!h) return -1;
    if (count < 0) return -2;
    if (!a || !b || !quot || !root) return -3;
    if (count == 0) return JSVD_OK;
    if (hipSetDevice(h->device) != hipSuccess) return JSVD_HIP_ERROR;
    HIP_TRY(launch_diag_fp64(count, a, b, quot, root, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return JSVD_OK;
}

int jsvd_diag_refined(jsvd_handle_t h, int64_t count, const double *a, const double *b,
                      double *out) {
    if (!h) return -1;
    if (count < 0) return -2;
    if (!a || !b || !out) return -3;
    if (count == 0) return JSVD_OK;
    if (hipSetDevice(h->device) != hipSuccess) return JSVD_HIP_ERROR;
    HIP_TRY(launch_diag_refined(count, a, b, out, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return JSVD_OK;
}

int jsvd_workspace_size(jsvd_handle_t h, int64_t m, int64_t n, const jsvd_opts *opts,
                        size_t *bytes) {
    const jsvd_opts o = opts ? *opts : defaults();
    if (!h) return -1;
    if (m < 1 || m < n || m > (int64_t)1 << 31) return -2;
    if (n < 1 || n > (int64_t)1 << 20) return -3;
    if (check_opts(o)) return -4;
    if (!bytes) return -5;
    // the Jacobi solve runs on G (m x n) or, after the QR preprocessing, on
    // R^T (n x n); the hyperbolic SVD adds the input column permutation
    auto solve_bytes = [&](int64_t mm, int64_t nn, bool hsvd) {
        const Shapes shp = pick_shapes(h, o, mm, nn);
        auto bytes_at = [&](int w) {
            const int order = strategy_order((int)((nn + w - 1) / w));
            int64_t rps = 0;
            size_t bytes = 0;
            // the fused update-and-Gram path (opts.fuse, 2w = 64) may split more
            const int fuse_max = (o.fuse && w == 32) ? 1 : 0;
            for (int fused = 0; fused <= fuse_max; ++fused) {
                const int tgt = split_target(h, o, shp, mm, order / 2, 2 * w, fused != 0);
                const int splits = gram_splits(mm, order / 2, tgt, &rps);
                bytes = std::max(bytes, plan(mm, nn, 2 * w, order / 2, splits, hsvd).total);
            }
            return bytes;
        };
        // w = 64 falls back to 32 for the hyperbolic SVD and the scaled mode
        if (shp.w == 64) return hsvd ? bytes_at(32) : std::max(bytes_at(64), bytes_at(32));
        return bytes_at(shp.w);
    };
    size_t total = std::max(solve_bytes(m, n, false), solve_bytes(m, n, true));
    if (wants_qr(h, o, m, n)) total = std::max(total, solve_bytes(n, n, false)) + qr_plan(m, n).total;
    if (o.scaled != 1) total += align_up((size_t)(n + 2) * sizeof(int), 256);
    *bytes = total;
    return JSVD_OK;
}

int jsvd_workspace_size_batched(jsvd_handle_t h, int64_t batch, int32_t max_m, int32_t max_n,
                                const jsvd_opts *opts, size_t *bytes) {
    const jsvd_opts o = opts ? *opts : defaults();
    int rc = check_batched_sizes(h, batch, max_m, max_n);
    if (rc) return rc;
    if (o.max_sweeps < 1) return -5;
    if (!bytes) return -6;
    *bytes = batch_plan(h, batch).total;
    return JSVD_OK;
}

int jsvd_reserve_batched(jsvd_handle_t h, int64_t batch, int32_t max_m, int32_t max_n,
                         const jsvd_opts *opts) {
    const jsvd_opts o = opts ? *opts : defaults();
    int rc = check_batched_sizes(h, batch, max_m, max_n);
    if (rc) return rc;
    if (o.max_sweeps < 1) return -5;
    if (hipSetDevice(h->device) != hipSuccess) return JSVD_HIP_ERROR;
    if ((rc = ensure_batch_tables(h))) return rc;
    return ensure_batch_workspace(h, batch_plan(h, batch).total,
                                  stream_capturing(h->stream));
}

int jsvd_rdssq_bounds(int32_t lg, double *t_lo, double *t_hi) {
    if (lg < 0 || lg > 63) return -1;
    if (!t_lo || !t_hi) return -2;
    *t_lo = 0x1.0000000000001p-511;
    *t_hi = rdssq_t_hi(lg);
    return JSVD_OK;
}

int jsvd_colnorms(jsvd_handle_t h, int64_t m, int64_t n, const double *A, int64_t lda,
                  int32_t *exps, double *ssq, double *norms) {
    if (!h) return -1;
    if (m < 1 || m > ((int64_t)1 << 40)) return -2;
    if (n < 0 || n > 0x7fffffff) return -3;
    if (!A && n > 0) return -4;
    if (lda < m) return -5;
    if (!exps && !ssq && !norms) return -6;
    if (n == 0) return JSVD_OK;
    if (hipSetDevice(h->device) != hipSuccess) return JSVD_HIP_ERROR;
    HIP_TRY(launch_rdssq_cols(A, lda, m, n, exps, ssq, norms, h->stream));
    return JSVD_OK;
}

}  // extern "C"

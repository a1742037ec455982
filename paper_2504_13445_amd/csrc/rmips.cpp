// librmips host side: validation, workspace layout, stage ordering and the
// bound-ordered visit loop of Alg. 2, behind the C ABI of include/rmips.h.
#include "../../include/rmips.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "common.h"
#include "kernels.h"

using namespace rmips;

namespace rmips {

// Per-launch timing: a pool of HIP events reused from call to call, the
// launches recorded since the stream was last waited for, and the totals per
// kernel name (in the order the names first appeared).
struct ProfRecorder {
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec { const char *name; size_t b, e; };
    std::vector<Rec> recs;
    std::vector<size_t> open;
    std::vector<std::pair<std::string, std::pair<int64_t, double>>> totals;

    size_t take() {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) e = nullptr;
            pool.push_back(e);
        }
        return used++;
    }
    // the stream must be idle: every recorded event has completed
    void resolve() {
        for (const Rec &r : recs) {
            float ms = 0.0f;
            if (pool[r.b] && pool[r.e] &&
                hipEventElapsedTime(&ms, pool[r.b], pool[r.e]) != hipSuccess)
                ms = 0.0f;
            auto it = std::find_if(totals.begin(), totals.end(),
                                   [&](const auto &t) { return t.first == r.name; });
            if (it == totals.end()) {
                totals.push_back({r.name, {0, 0.0}});
                it = totals.end() - 1;
            }
            it->second.first += 1;
            it->second.second += ms;
        }
        recs.clear();
        open.clear();
        used = 0;
    }
    ~ProfRecorder() {
        for (hipEvent_t e : pool)
            if (e) (void)hipEventDestroy(e);
    }
};

thread_local ProfRecorder *g_prof = nullptr;

void prof_begin(hipStream_t st, const char *name) {
    ProfRecorder *p = g_prof;
    const size_t b = p->take();
    if (p->pool[b]) (void)hipEventRecord(p->pool[b], st);
    p->recs.push_back({name, b, b});
    p->open.push_back(p->recs.size() - 1);
}

void prof_end(hipStream_t st) {
    ProfRecorder *p = g_prof;
    const size_t e = p->take();
    if (p->pool[e]) (void)hipEventRecord(p->pool[e], st);
    if (!p->open.empty()) {
        p->recs[p->open.back()].e = e;
        p->open.pop_back();
    }
}

}  // namespace rmips

struct rmips_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int32_t cap_override = 0;
    int32_t batch_first = 0, batch_max = 0;
    int32_t *bound_out = nullptr;  // device, m int32 (testing knob)
    int32_t *h_status = nullptr;  // pinned, small
    int32_t *h_vis = nullptr;     // pinned: visit-order bounds and prefixes, top-N
    int64_t h_vis_cap = 0;        // its size in int32 entries
    // input checks of the calls that return without waiting: each copies
    // its device flag into the next pinned slot h_status[1 + i]; rmips_sync
    // reads them once the stream is done
    int pending = 0;
    // per-launch timing (rmips_set_profiling)
    bool prof_on = false;
    ProfRecorder prof;
    // device address of the relaxed-score kernels' scratch array on this
    // device (rmips_soft_bwd_noalloc); NULL until taken
    void *soft_scratch = nullptr;
};

namespace {
// Points the launches of a C-ABI call at the context's recorder while the
// call enqueues (when profiling is on).
struct ProfGuard {
    explicit ProfGuard(rmips_ctx *c) { g_prof = (c && c->prof_on) ? &c->prof : nullptr; }
    ~ProfGuard() { g_prof = nullptr; }
};
}  // namespace
constexpr int PENDING_SLOTS = 63;

namespace {

// Split dimension d' of Eq. (3) (Sec. 5.1): min(d, DPRIME_MAX).  A larger
// d' than the paper's tightens the bound (fewer items are visited in stage
// (b)); the matrix-core bound pass pays for it in K only.  With d' = d the
// rotation is the identity and the bound is the inner product itself.
constexpr int DPRIME_MAX = 62;
int dprime(int d) { return std::min(d, DPRIME_MAX); }
int aug_len(int d) { return (dprime(d) + 2 + 15) & ~15; }  // ka: 16, 32, 48 or 64
constexpr int T0_TILES = 6;             // tiles of phase 1 of stage (a)
constexpr int BATCH_FIRST = 256;
constexpr int BATCH_MAX = 4096;
constexpr int RHO_LO_BIT = 8;  // ratio key bits below this are not sorted on
constexpr int GRAM_SAMPLE = 16384;

rmips_status fail(rmips_ctx *c, rmips_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

#define HIPTRY(expr)                                                              \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess)                                                     \
            return fail(ctx, RMIPS_EDEVICE, std::string(#expr) + ": " +           \
                                                hipGetErrorString(e_));           \
    } while (0)

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures.
struct Carve {
    uint8_t *base;
    size_t off = 0;
    explicit Carve(void *b) : base((uint8_t *)b) {}
    template <class T> T *take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// Screening error constants: |vh - v| <= R_u N_p + Nh_u R_p + c Nh_u Nh_p +
// c2 N_u N_p + E_ABS.  c = gamma_D bounds the matrix-core sum of D products
// with a unit roundoff of 2^-23 (twice round-to-nearest, as the order and
// rounding inside the matrix core are not specified); c2 covers v's own
// FP64 rounding (d 2^-53) and the FP32 rounding of the comparisons (8 2^-24).
struct ErrConst { float c, c2, g64; };

ErrConst err_const(int D, int d) {
    const double u = std::ldexp(1.0, -23), slack = 1.0 + std::ldexp(1.0, -16);
    const double g64 = d * std::ldexp(1.0, -53);
    ErrConst e;
    e.c = (float)(D * u / (1.0 - D * u) * slack);
    e.c2 = (float)((g64 + 8.0 * std::ldexp(1.0, -24)) * slack);
    e.g64 = (float)(g64 * slack);
    return e;
}

struct ThreshLayout {
    int prec, D, rowb, ntiles, nsplit, cap;
    int64_t mpad;
    void *Uq, *Pq;
    float *Nu, *Nhu, *Ru, *su;          // users, caller order
    float *Np, *Nhp, *Rp, *sp, *Npid;   // items, norm order (Npid: by id)
    float *tmax_nh, *tmax_r;
    unsigned int *rmax;
    uint32_t *keys;
    int32_t *perm;
    void *sort_scratch;
    float2 *cand;
    int32_t *cand_id;
    int32_t *cand_cnt, *lists, *lcnt;
    float *Luse;
    uint32_t *ukey;
    int32_t *uord, *nall;
    void *usort;
    int *bad;
};

void thresh_plan(int prec, int64_t n, int64_t m, int d, int k, int cap_override, ThreshLayout &L,
                 Carve &cv) {
    L.prec = prec;
    L.D = padded_dim(prec, d);
    L.rowb = L.D * elem_bytes(prec);
    L.ntiles = (int)((m + TILE_ITEMS - 1) / TILE_ITEMS);
    L.mpad = (int64_t)L.ntiles * TILE_ITEMS;
    // splits of the item range: about six rounds of screening workgroups
    // (256 users each, one per compute unit) over the whole chip
    int64_t utiles = (n + 255) / 256;
    int64_t ns = (1536 + utiles - 1) / utiles;
    ns = std::max<int64_t>(1, std::min<int64_t>(ns, 8));
    ns = std::min<int64_t>(ns, L.ntiles);
    L.nsplit = (int)ns;
    // candidate capacity per user (all splits together): well above the
    // candidate counts of typical users; users beyond it are screened again
    // with a tighter bound.  FP8's wider error band needs longer lists.
    if (cap_override > 0) {
        L.cap = cap_override;
    } else {
        int64_t capU = std::max<int64_t>(256, 16 * (int64_t)k);
        if (prec == RMIPS_FP8_E4M3) capU *= 4;
        L.cap = (int)(((capU + L.nsplit - 1) / L.nsplit + 7) / 8 * 8);
    }
    const int64_t npad = (n + 63) / 64 * 64;
    L.Uq = cv.take<uint8_t>((size_t)npad * L.rowb);
    L.Nu = cv.take<float>(npad);
    L.Nhu = cv.take<float>(npad);
    L.Ru = cv.take<float>(npad);
    L.su = cv.take<float>(npad);
    L.Pq = cv.take<uint8_t>((size_t)L.mpad * L.rowb);
    L.Np = cv.take<float>(L.mpad);
    L.Nhp = cv.take<float>(L.mpad);
    L.Rp = cv.take<float>(L.mpad);
    L.sp = cv.take<float>(L.mpad);
    L.tmax_nh = cv.take<float>(L.ntiles);
    L.tmax_r = cv.take<float>(L.ntiles);
    L.Npid = cv.take<float>(m);
    L.keys = cv.take<uint32_t>(m);
    L.perm = cv.take<int32_t>(m);
    L.sort_scratch = cv.take<uint8_t>(radix_sort_scratch_bytes(m));
    L.cand = cv.take<float2>((size_t)n * L.nsplit * L.cap);
    L.cand_id = cv.take<int32_t>((size_t)n * L.nsplit * L.cap);
    // counts per (user, split); refinement passes use up to 8 splits
    L.cand_cnt = cv.take<int32_t>((size_t)n * 8);
    L.lists = cv.take<int32_t>((size_t)3 * n);
    L.lcnt = cv.take<int32_t>(64);
    L.Luse = cv.take<float>(n);
    L.ukey = cv.take<uint32_t>(n);
    L.uord = cv.take<int32_t>(n);
    L.usort = cv.take<uint8_t>(radix_sort_scratch_bytes(n));
    L.nall = cv.take<int32_t>(64);
    // the input flag and the largest R/N share a block (one fill clears both)
    L.bad = cv.take<int>(64);
    L.rmax = reinterpret_cast<unsigned int *>(L.bad + 32);
}

constexpr const char *BAD_INPUT = "input holds a NaN/Inf or a vector norm above 2^60";

rmips_status sync_pending(rmips_ctx *ctx) {
    HIPTRY(hipStreamSynchronize(ctx->stream));
    ctx->prof.resolve();
    bool bad = false;
    for (int i = 0; i < ctx->pending; ++i) bad |= ctx->h_status[1 + i] != 0;
    ctx->pending = 0;
    if (bad) return fail(ctx, RMIPS_ENONFINITE, BAD_INPUT);
    return RMIPS_OK;
}

// The input check of a call that returns without waiting: the device flag
// is copied into a pinned slot in stream order and read by rmips_sync (or
// here, when every slot is taken, after waiting for the earlier ones).
rmips_status defer_check(rmips_ctx *ctx, const int *bad) {
    if (ctx->pending == PENDING_SLOTS) {
        rmips_status s = sync_pending(ctx);
        if (s != RMIPS_OK) {
            // an earlier call's inputs were bad: report it now, and keep this
            // call's check for later
            HIPTRY(hipMemcpyAsync(ctx->h_status + 1, bad, sizeof(int), hipMemcpyDeviceToHost,
                                  ctx->stream));
            ctx->pending = 1;
            return s;
        }
    }
    HIPTRY(hipMemcpyAsync(ctx->h_status + 1 + ctx->pending, bad, sizeof(int),
                          hipMemcpyDeviceToHost, ctx->stream));
    ++ctx->pending;
    return RMIPS_OK;
}

// Stage (a) into (tau, tau_id, topk); also leaves the prepared item/user
// arrays of L in the workspace for later stages.
rmips_status run_thresholds(rmips_ctx *ctx, const float *U, int64_t n, const float *P,
                            int64_t m, int d, int k, ThreshLayout &L, double *tau,
                            int32_t *tau_id, int32_t *topk,
                            unsigned long long *pairs = nullptr,
                            unsigned long long *rpairs = nullptr, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr, unsigned long long *cstats = nullptr,
                            bool clear_flags = true) {
    hipStream_t st = ctx->stream;
    // bad and rmax, 32 words apart in every layout (a caller may have
    // cleared them already)
    if (clear_flags) HIPTRY(hipMemsetAsync(L.bad, 0, 33 * sizeof(int), st));
    launch_rows_prep(P, m, d, L.D, nullptr, L.Npid, L.keys, L.perm, L.bad, st);
    HIPTRY(radix_sort_u32(L.keys, L.perm, m, L.sort_scratch, st));
    launch_quant(L.prec, P, L.perm, m, L.mpad, d, L.D, TILE_ITEMS, L.Pq, L.Np, L.Nhp, L.Rp,
                 L.sp, L.rmax, L.bad, st);
    launch_tile_max(L.Nhp, L.Rp, L.ntiles, L.tmax_nh, L.tmax_r, st);
    launch_quant(L.prec, U, nullptr, n, n, d, L.D, 1, L.Uq, L.Nu, L.Nhu, L.Ru, L.su, nullptr,
                 L.bad, st);
    HIPTRY(hipGetLastError());
    // (the caller reads L.bad later, in stream order; the kernels below stay
    // in bounds whatever the values)

    const ErrConst ec = err_const(L.D, d);
    ThreshArgs a{};
    a.prec = L.prec;
    a.Uq = L.Uq; a.Nu = L.Nu; a.Nhu = L.Nhu; a.Ru = L.Ru; a.su = L.su; a.n = n;
    a.Pq = L.Pq; a.Np = L.Np; a.Nhp = L.Nhp; a.Rp = L.Rp; a.sp = L.sp;
    a.tmax_nh = L.tmax_nh; a.tmax_r = L.tmax_r; a.rmax_bits = L.rmax;
    a.perm = L.perm; a.m = m; a.ntiles = L.ntiles;
    a.U = U; a.P = P; a.d = d;
    a.D = L.D; a.k = k; a.t0tiles = T0_TILES; a.nsplit = L.nsplit; a.cap = L.cap;
    a.c_err = ec.c; a.c2 = ec.c2; a.e_abs = E_ABS; a.g64 = ec.g64;
    a.cand = L.cand; a.cand_id = L.cand_id; a.cand_cnt = L.cand_cnt;
    a.lists = L.lists; a.lcnt = L.lcnt; a.refine = 2; a.Luse = L.Luse;
    a.ukey = L.ukey; a.uord = L.uord; a.usort = L.usort; a.nall = L.nall;
    a.tau = tau; a.tau_id = tau_id; a.topk = topk;
    a.pairs = pairs; a.rpairs = rpairs; a.ev0 = ev0; a.ev1 = ev1; a.cstats = cstats;
    if (thresh_screen_lds(L.prec, L.D) > 160 * 1024 || (size_t)final_stride(L.cap * L.nsplit) * 24 > 150 * 1024)
        return fail(ctx, RMIPS_EUNSUPPORTED, "screening tile or candidate lists exceed LDS");
    launch_thresh(a, st);
    HIPTRY(hipGetLastError());
    return RMIPS_OK;
}

rmips_status validate_common(rmips_ctx *ctx, int64_t n, int64_t m, int d, int k,
                             rmips_prec prec) {
    if (!ctx) return RMIPS_EINVAL;
    if (n < 1 || n > (int64_t)INT32_MAX) return fail(ctx, RMIPS_EINVAL, "n out of range");
    if (m < 1 || m > (int64_t)INT32_MAX / 2) return fail(ctx, RMIPS_EINVAL, "m out of range");
    if (d < 1 || d > RMIPS_D_MAX) return fail(ctx, RMIPS_EINVAL, "d out of range");
    if (k < 1 || k > RMIPS_K_MAX || k > m) return fail(ctx, RMIPS_EINVAL, "k out of range");
    if (prec != RMIPS_FP32 && prec != RMIPS_BF16 && prec != RMIPS_FP8_E4M3)
        return fail(ctx, RMIPS_EUNSUPPORTED, "unknown screening precision");
    return RMIPS_OK;
}

// An orthonormal basis of the dominant dp-dimensional eigenspace of the
// symmetric G (d x d) by block power iteration; returns W (dp x d) with
// orthonormal rows.  Any orthonormal W keeps the Eq. (3) bound valid; the
// dominant eigenspace only makes it tight.
void top_eigvecs(const std::vector<double> &G, int d, int dp, std::vector<double> &W) {
    const int b = dp;
    // Q, Z: b columns of length d, each contiguous (column j at j * d)
    std::vector<double> Q((size_t)d * b), Z((size_t)d * b);
    for (int j = 0; j < b; ++j)
        for (int i = 0; i < d; ++i)
            Q[(size_t)j * d + i] = (i == j) ? 1.0 : std::sin(1.0 + 0.7 * i + 1.3 * j) * 1e-3;
    auto dot = [d](const double *x, const double *y) {  // eight partial sums
        double p[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int i = 0;
        for (; i + 8 <= d; i += 8)
            for (int e = 0; e < 8; ++e) p[e] += x[i + e] * y[i + e];
        for (; i < d; ++i) p[0] += x[i] * y[i];
        return ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
    };
    auto orth = [&](std::vector<double> &X) {
        // modified Gram-Schmidt over columns, twice for orthogonality to FP64 precision
        for (int pass = 0; pass < 2; ++pass)
            for (int j = 0; j < b; ++j) {
                double *xj = &X[(size_t)j * d];
                for (int q = 0; q < j; ++q) {
                    const double *xq = &X[(size_t)q * d];
                    const double c = dot(xj, xq);
                    for (int i = 0; i < d; ++i) xj[i] -= c * xq[i];
                }
                const double nrm = std::sqrt(dot(xj, xj));
                const double inv = (nrm > 0) ? 1.0 / nrm : 0.0;
                for (int i = 0; i < d; ++i) xj[i] *= inv;
            }
    };
    auto gmul = [&](const std::vector<double> &X, std::vector<double> &Y) {
        for (int j = 0; j < b; ++j)
            for (int i = 0; i < d; ++i) Y[(size_t)j * d + i] = dot(&G[(size_t)i * d], &X[(size_t)j * d]);
    };
    orth(Q);
    // block power iteration; any orthonormal result keeps the bound valid,
    // and the bound depends only on the span of W's rows (a rotation within
    // it changes nothing), so no Ritz vectors are needed
    for (int it = 0; it < 6; ++it) {
        gmul(Q, Z);
        orth(Z);
        Q.swap(Z);
    }
    W.assign((size_t)dp * d, 0.0);
    for (int r = 0; r < dp; ++r)
        for (int i = 0; i < d; ++i) W[(size_t)r * d + i] = Q[(size_t)r * d + i];
}

// counters of rmips_topn (64-bit words): [0] stage (b) rechecks, [2] stage
// (c) bound pairs, [8, 8 + CSTAT_SLOTS) pairs screened by stage (a)'s main
// pass, then by its refinement passes, [CTR_CS, CTR_CS + 4 * CSTAT_SLOTS)
// stage (a) candidate statistics
constexpr int CTR_PAIRS = 8;
constexpr int CTR_RPAIRS = CTR_PAIRS + CSTAT_SLOTS;
constexpr int CTR_CS = CTR_RPAIRS + CSTAT_SLOTS;
constexpr int CTR_WORDS = CTR_CS + 4 * CSTAT_SLOTS;
// block of a batch's results: status (64 words: the running top-N's in
// [0, 2), stage (a)'s input flag in [RES_BAD], its largest R/N in
// [RES_RMAX]), the counters, the top-N list; one fill clears all but the list
constexpr size_t RES_STATUS = 0, RES_CTR = 256, RES_TOP = RES_CTR + 8 * CTR_WORDS,
                 RES_BYTES = RES_TOP + 8 * RMIPS_N_MAX;
constexpr int RES_BAD = 12, RES_RMAX = 44;

struct TopnLayout {
    ThreshLayout T;
    double *tau;
    int32_t *tau_id;
    uint32_t *ukeys;
    int32_t *uperm;
    void *usort;
    int32_t *cs;
    UserSide us;
    void *Us;
    double *G, *Gs, *W;
    uint4 *Pa, *Ua;  // augmented BF16 hi | lo rows, 4 ka bytes each
    int nsplitB;
    int32_t *partialB, *uscore, *inv;
    uint32_t *vkeys;
    int32_t *visit, *vis_us, *vis_cs, *vis_cid;
    int nsplitC_max;
    int32_t *partialC, *batch_scores;
    uint64_t *top;
    int32_t *status;
    int64_t *rechecks;
    int32_t *ulen_dev;
};

void user_side_plan(int64_t n, UserSide &us, Carve &cv) {
    us.N = cv.take<float>(n);
    us.Nh = cv.take<float>(n);
    us.R = cv.take<float>(n);
    us.sinv = cv.take<float>(n);
    us.tau_hi = cv.take<float>(n);
    us.tau_lo = cv.take<float>(n);
    us.tau = cv.take<double>(n);
    us.tau_id = cv.take<int32_t>(n);
    us.uid = cv.take<int32_t>(n);
    us.thr = cv.take<float4>(n);
}

void topn_plan(int prec, int64_t n, int64_t m, int d, int k, int cap_override, int bmax,
               TopnLayout &L, Carve &cv) {
    thresh_plan(prec, n, m, d, k, cap_override, L.T, cv);
    L.tau = cv.take<double>(n);
    L.tau_id = cv.take<int32_t>(n);
    L.ukeys = cv.take<uint32_t>(n);
    L.uperm = cv.take<int32_t>(n);
    L.usort = cv.take<uint8_t>(radix_sort_scratch_bytes(std::max(n, m)));
    L.cs = cv.take<int32_t>(L.T.mpad);
    user_side_plan(n, L.us, cv);
    L.Us = cv.take<uint8_t>((size_t)n * L.T.rowb);
    L.G = cv.take<double>((size_t)d * d);
    L.Gs = cv.take<double>(gram_scratch_bytes(d) / sizeof(double));
    L.W = cv.take<double>((size_t)DPRIME_MAX * d);
    L.Pa = cv.take<uint4>((size_t)L.T.mpad * aug_len(d) / 4);
    L.Ua = cv.take<uint4>((size_t)n * aug_len(d) / 4);
    L.nsplitB = bound_splits(m, aug_len(d));
    L.partialB = cv.take<int32_t>((size_t)L.nsplitB * m);
    L.uscore = cv.take<int32_t>(m);
    L.inv = cv.take<int32_t>(m);
    L.vkeys = cv.take<uint32_t>(m);
    L.visit = cv.take<int32_t>(m);
    L.vis_us = cv.take<int32_t>(2 * m);  // bounds, then prefixes: one copy to the host
    L.vis_cs = L.vis_us + m;
    L.vis_cid = cv.take<int32_t>(m);
    L.nsplitC_max = 256;
    L.partialC = cv.take<int32_t>((size_t)L.nsplitC_max * bmax);
    L.batch_scores = cv.take<int32_t>(bmax);
    // the results of a batch in one block, copied to the host at once:
    // status, the top-N list, the counters
    uint8_t *res = cv.take<uint8_t>(RES_BYTES);
    L.status = reinterpret_cast<int32_t *>(res + RES_STATUS);
    L.top = reinterpret_cast<uint64_t *>(res + RES_TOP);
    L.rechecks = reinterpret_cast<int64_t *>(res + RES_CTR);
    // stage (a)'s flags live in the status words (copied with every batch)
    L.T.bad = L.status + RES_BAD;
    L.T.rmax = reinterpret_cast<unsigned int *>(L.status + RES_RMAX);
    L.ulen_dev = cv.take<int32_t>(1);
}

// splits of the user range of a counting launch: about four rounds of
// counting workgroups (256 items each, one per compute unit), each split
// with at least two 64-user chunks
int count_splits(int64_t nb, int64_t ulen, int maxs) {
    int64_t iblocks = (nb + 255) / 256;
    int64_t chunks = (ulen + 63) / 64;
    int64_t s = (2048 + iblocks - 1) / iblocks;
    s = std::min<int64_t>(s, std::max<int64_t>(1, chunks / 2));
    return (int)std::max<int64_t>(1, std::min<int64_t>(s, maxs));
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

rmips_status rmips_create(rmips_ctx **out, int device, void *hip_stream) {
    if (!out) return RMIPS_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return RMIPS_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return RMIPS_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return RMIPS_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return RMIPS_EUNSUPPORTED;
    rmips_ctx *c = new rmips_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    // the scratch array's address on this device (current here); on failure
    // rmips_soft_bwd_noalloc tries again and reports the error
    if (soft_scratch_init(device, &c->soft_scratch) != hipSuccess) c->soft_scratch = nullptr;
    if (hipHostMalloc((void **)&c->h_status, 256, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return RMIPS_EDEVICE;
    }
    *out = c;
    return RMIPS_OK;
}

void rmips_destroy(rmips_ctx *ctx) {
    if (!ctx) return;
    if (ctx->h_status) (void)hipHostFree(ctx->h_status);
    if (ctx->h_vis) (void)hipHostFree(ctx->h_vis);
    delete ctx;
}

const char *rmips_last_error(const rmips_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

rmips_status rmips_set_stream(rmips_ctx *ctx, void *hip_stream) {
    if (!ctx) return RMIPS_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return RMIPS_OK;
}

rmips_status rmips_set_candidate_cap(rmips_ctx *ctx, int32_t cap) {
    if (!ctx || cap < 0 || cap > 4096) return RMIPS_EINVAL;
    ctx->cap_override = cap;
    return RMIPS_OK;
}

rmips_status rmips_set_batch(rmips_ctx *ctx, int32_t first, int32_t max) {
    if (!ctx || first < 0 || max < 0 || first > BATCH_MAX || max > BATCH_MAX ||
        (first && max && first > max))
        return RMIPS_EINVAL;
    ctx->batch_first = first;
    ctx->batch_max = max;
    return RMIPS_OK;
}

rmips_status rmips_set_bound_output(rmips_ctx *ctx, int32_t *uscore) {
    if (!ctx) return RMIPS_EINVAL;
    ctx->bound_out = uscore;
    return RMIPS_OK;
}

static bool prec_ok(rmips_prec p) {
    return p == RMIPS_FP32 || p == RMIPS_BF16 || p == RMIPS_FP8_E4M3;
}

size_t rmips_thresholds_workspace_size(int64_t n, int64_t m, int32_t d, int32_t k,
                                       rmips_prec prec) {
    if (n < 1 || m < 1 || d < 1 || d > RMIPS_D_MAX || k < 1 || k > RMIPS_K_MAX || k > m ||
        !prec_ok(prec))
        return 0;
    Carve cv(nullptr);
    ThreshLayout L;
    thresh_plan(prec, n, m, d, k, 0, L, cv);
    return cv.off + 256;
}

struct ScoresLayout {
    int D, rowb;
    void *Uq, *Qq;
    float *Nu, *Nhu, *Ru, *su, *Nq, *Nhq, *Rq, *sq;
    UserSide us;
    int32_t *partial;
    int *bad;
    int64_t *rech;
};

void scores_plan(int prec, int64_t n, int64_t nq, int d, ScoresLayout &L, Carve &cv) {
    L.D = padded_dim(prec, d);
    L.rowb = L.D * elem_bytes(prec);
    const int64_t npad = (n + 63) / 64 * 64, qpad = (nq + 63) / 64 * 64;
    L.Uq = cv.take<uint8_t>((size_t)npad * L.rowb);
    L.Nu = cv.take<float>(npad); L.Nhu = cv.take<float>(npad);
    L.Ru = cv.take<float>(npad); L.su = cv.take<float>(npad);
    L.Qq = cv.take<uint8_t>((size_t)qpad * L.rowb);
    L.Nq = cv.take<float>(qpad); L.Nhq = cv.take<float>(qpad);
    L.Rq = cv.take<float>(qpad); L.sq = cv.take<float>(qpad);
    user_side_plan(n, L.us, cv);
    L.partial = cv.take<int32_t>((size_t)256 * nq);
    L.bad = cv.take<int>(64);
    L.rech = cv.take<int64_t>(8);
}

size_t rmips_scores_workspace_size(int64_t n, int64_t nq, int32_t d, rmips_prec prec) {
    if (n < 1 || nq < 1 || d < 1 || d > RMIPS_D_MAX || !prec_ok(prec)) return 0;
    Carve cv(nullptr);
    ScoresLayout L;
    scores_plan(prec, n, nq, d, L, cv);
    return cv.off + 256;
}

size_t rmips_topn_workspace_size(int64_t n, int64_t m, int32_t d, int32_t k, int32_t N,
                                 rmips_prec prec) {
    if (rmips_thresholds_workspace_size(n, m, d, k, prec) == 0 || N < 1 ||
        N > RMIPS_N_MAX || N > m)
        return 0;
    Carve cv(nullptr);
    TopnLayout L;
    topn_plan(prec, n, m, d, k, 0, BATCH_MAX, L, cv);
    return cv.off + 256;
}

rmips_status rmips_thresholds(rmips_ctx *ctx, const float *U, int64_t n, const float *P,
                              int64_t m, int32_t d, int32_t k, rmips_prec prec, void *ws,
                              size_t ws_bytes, double *tau, int32_t *tau_id, int32_t *topk) {
    rmips_status s = validate_common(ctx, n, m, d, k, prec);
    if (s != RMIPS_OK) return s;
    if (!U || !P || !ws || !tau || !tau_id) return fail(ctx, RMIPS_EINVAL, "null pointer");
    Carve probe(nullptr);
    ThreshLayout L;
    thresh_plan(prec, n, m, d, k, ctx->cap_override, L, probe);
    if (ws_bytes < probe.off + 256) return fail(ctx, RMIPS_EWORKSPACE, "workspace too small");
    HIPTRY(hipSetDevice(ctx->device));
    ProfGuard pguard(ctx);
    Carve cv(ws);
    thresh_plan(prec, n, m, d, k, ctx->cap_override, L, cv);
    s = run_thresholds(ctx, U, n, P, m, d, k, L, tau, tau_id, topk);
    if (s != RMIPS_OK) return s;
    return defer_check(ctx, L.bad);
}

rmips_status rmips_scores(rmips_ctx *ctx, const float *U, int64_t n, const double *tau,
                          const int32_t *tau_id, const float *Q, const int32_t *q_ids,
                          int64_t nq, int32_t d, rmips_prec prec, void *ws, size_t ws_bytes,
                          int32_t *scores) {
    if (!ctx) return RMIPS_EINVAL;
    if (n < 1 || n > (int64_t)INT32_MAX || nq < 1 || nq > (int64_t)INT32_MAX / 2 || d < 1 ||
        d > RMIPS_D_MAX)
        return fail(ctx, RMIPS_EINVAL, "size out of range");
    if (!prec_ok(prec)) return fail(ctx, RMIPS_EUNSUPPORTED, "unknown screening precision");
    if (!U || !tau || !tau_id || !Q || !ws || !scores)
        return fail(ctx, RMIPS_EINVAL, "null pointer");
    if (ws_bytes < rmips_scores_workspace_size(n, nq, d, prec))
        return fail(ctx, RMIPS_EWORKSPACE, "workspace too small");
    HIPTRY(hipSetDevice(ctx->device));
    ProfGuard pguard(ctx);
    hipStream_t st = ctx->stream;
    Carve cv(ws);
    ScoresLayout L;
    scores_plan(prec, n, nq, d, L, cv);
    HIPTRY(hipMemsetAsync(L.bad, 0, sizeof(int), st));
    launch_quant(prec, U, nullptr, n, n, d, L.D, 1, L.Uq, L.Nu, L.Nhu, L.Ru, L.su, nullptr,
                 L.bad, st);
    launch_quant(prec, Q, nullptr, nq, nq, d, L.D, 1, L.Qq, L.Nq, L.Nhq, L.Rq, L.sq, nullptr,
                 L.bad, st);
    HIPTRY(hipGetLastError());
    // (the input flag is read by rmips_sync; the kernels below stay in
    // bounds whatever the values)
    const ErrConst ec = err_const(L.D, d);
    launch_user_side(tau, tau_id, L.Nu, L.Nhu, L.Ru, L.su, nullptr, n, ec.c2, L.us, st);
    CountArgs a{};
    a.prec = prec;
    a.Pq = L.Qq; a.Np = L.Nq; a.Nhp = L.Nhq; a.Rp = L.Rq; a.sp = L.sq;
    a.rows = nullptr; a.nb = nq;
    a.item_tie = q_ids; a.item_orig = nullptr; a.Porig = Q;
    a.Us = L.Uq; a.ulen = n; a.us = L.us; a.Uorig = U; a.d = d; a.D = L.D;
    a.c_err = ec.c; a.c2 = ec.c2; a.e_abs = E_ABS;
    a.nsplit = count_splits(nq, n, 256);
    a.partial = L.partial;
    a.rechecks = L.rech;
    HIPTRY(hipMemsetAsync(L.rech, 0, sizeof(int64_t), st));
    launch_count(a, st);
    launch_colsum(L.partial, a.nsplit, nq, scores, st);
    HIPTRY(hipGetLastError());
    return defer_check(ctx, L.bad);
}

rmips_status rmips_sync(rmips_ctx *ctx) {
    if (!ctx) return RMIPS_EINVAL;
    HIPTRY(hipSetDevice(ctx->device));
    return sync_pending(ctx);
}

rmips_status rmips_set_profiling(rmips_ctx *ctx, int32_t on) {
    if (!ctx) return RMIPS_EINVAL;
    HIPTRY(hipSetDevice(ctx->device));
    HIPTRY(hipStreamSynchronize(ctx->stream));
    ctx->prof.resolve();
    if (on) ctx->prof.totals.clear();
    ctx->prof_on = on != 0;
    return RMIPS_OK;
}

rmips_status rmips_profile_entry(rmips_ctx *ctx, int32_t i, char *name, int32_t name_cap,
                                 int64_t *launches, double *ms_total) {
    if (!ctx || !name || name_cap < 1 || !launches || !ms_total) return RMIPS_EINVAL;
    HIPTRY(hipSetDevice(ctx->device));
    HIPTRY(hipStreamSynchronize(ctx->stream));
    ctx->prof.resolve();
    if (i < 0 || (size_t)i >= ctx->prof.totals.size())
        return fail(ctx, RMIPS_EINVAL, "no such profile entry");
    const auto &t = ctx->prof.totals[(size_t)i];
    std::snprintf(name, (size_t)name_cap, "%s", t.first.c_str());
    *launches = t.second.first;
    *ms_total = t.second.second;
    return RMIPS_OK;
}

rmips_status rmips_topn(rmips_ctx *ctx, const float *U, int64_t n, const float *P, int64_t m,
                        int32_t d, int32_t k, int32_t N, rmips_prec prec, void *ws,
                        size_t ws_bytes, int32_t *top_ids, int32_t *top_scores,
                        rmips_stats *stats) {
    rmips_status s = validate_common(ctx, n, m, d, k, prec);
    if (s != RMIPS_OK) return s;
    if (N < 1 || N > RMIPS_N_MAX || N > m) return fail(ctx, RMIPS_EINVAL, "N out of range");
    if (!U || !P || !ws || !top_ids || !top_scores)
        return fail(ctx, RMIPS_EINVAL, "null pointer");
    const int bfirst = ctx->batch_first > 0 ? ctx->batch_first : BATCH_FIRST;
    const int bmax = ctx->batch_max > 0 ? ctx->batch_max : BATCH_MAX;
    {
        Carve probe(nullptr);
        TopnLayout L0;
        topn_plan(prec, n, m, d, k, ctx->cap_override, BATCH_MAX, L0, probe);
        if (ws_bytes < probe.off + 256)
            return fail(ctx, RMIPS_EWORKSPACE, "workspace too small");
    }
    HIPTRY(hipSetDevice(ctx->device));
    ProfGuard pguard(ctx);
    hipStream_t st = ctx->stream;
    Carve cv(ws);
    TopnLayout L;
    topn_plan(prec, n, m, d, k, ctx->cap_override, BATCH_MAX, L, cv);
    const int D = L.T.D;
    const ErrConst ec = err_const(D, d);

    constexpr int NEV = 10;
    hipEvent_t ev[NEV] = {};
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() { for (int i = 0; i < NEV; ++i) if (e[i]) (void)hipEventDestroy(e[i]); }
    } guard{ev};
    for (auto &e : ev) HIPTRY(hipEventCreate(&e));
    unsigned long long *ctr = reinterpret_cast<unsigned long long *>(L.rechecks);
    // status words (with stage (a)'s flags) and counters in one fill
    HIPTRY(hipMemsetAsync(L.status, 0, RES_TOP, st));
    HIPTRY(hipEventRecord(ev[0], st));

    // The Gram matrix of a user sample (for the rotation of Eq. (3)) does
    // not depend on tau: it goes to the host first, and the host computes
    // its eigenvectors while the GPU runs stage (a).  With d' = d any
    // orthonormal basis gives the same bound: the identity.
    const int dp = dprime(d), ka = aug_len(d);
    const bool rotate = dp < d;
    std::vector<double> G, W;
    if (rotate) {
        const int64_t ns = std::min<int64_t>(n, GRAM_SAMPLE);
        launch_gram(U, ns, n / ns, d, L.G, L.Gs, st);
        G.resize((size_t)d * d);
        HIPTRY(hipMemcpyAsync(G.data(), L.G, sizeof(double) * d * d, hipMemcpyDeviceToHost, st));
    }
    HIPTRY(hipEventRecord(ev[3], st));

    // ---- stage (a): exact thresholds (the input check is read at the
    // synchronisation before stage (b))
    s = run_thresholds(ctx, U, n, P, m, d, k, L.T, L.tau, L.tau_id, nullptr, ctr + CTR_PAIRS,
                       ctr + CTR_RPAIRS, ev[4], ev[5], ctr + CTR_CS, false);
    if (s != RMIPS_OK) return s;
    HIPTRY(hipEventRecord(ev[1], st));
    if (rotate) {
        HIPTRY(hipEventSynchronize(ev[3]));
        top_eigvecs(G, d, dp, W);
    }

    // ---- stage (c): Cauchy-Schwarz prefix and Eq. (3)/(6) bound counts
    // users by their ratio keys without the low 8 bits (3 passes instead of
    // 4): each item's prefix may take users whose ratio is up to 2^-15
    // relative above its norm, which the bound and the count then test
    launch_rho_keys(L.tau, L.T.Nu, n, L.ukeys, L.uperm, st);
    HIPTRY(radix_sort_u32(L.ukeys, L.uperm, n, L.usort, st, RHO_LO_BIT, 32));
    launch_cs_prefix(L.ukeys, n, L.T.Np, m, RHO_LO_BIT, L.cs, st);
    launch_user_side(L.tau, L.tau_id, L.T.Nu, L.T.Nhu, L.T.Ru, L.T.su, L.uperm, n, ec.c2, L.us,
                     st);
    launch_gather_padded(L.T.Uq, L.uperm, n, L.T.rowb, L.Us, st);
    if (rotate)
        HIPTRY(hipMemcpyAsync(L.W, W.data(), sizeof(double) * dp * d, hipMemcpyHostToDevice, st));
    // Relative slack s of the bound, in units of ||u|| ||p||: the BF16
    // split drops at most 3.01 * 2^-16 |a_i||b_i| per term; the matrix-core
    // sums of the 3 ka <= 192 exact BF16 products (12 chained steps) add at
    // most gamma_204 (unit 2^-23, 3.19 * 2^-16) times 1.02 sum |a_i||b_i|;
    // and sum |a_i||b_i| <= ||a|| ||b|| <= 1.415 ||p|| ||u||: 8.9 * 2^-16 in
    // all, below s = 2^-12; the FP32 rounding of W x (2^-24 relative) is far
    // below the margin.  The absolute slack covers BF16 and FP32 underflow
    // (norms are below 2^60).
    const float slack = 0x1p-12f;
    const double *Wd = rotate ? L.W : nullptr;  // nullptr: the identity
    launch_rotate_aug(P, L.T.perm, m, L.T.mpad, d, Wd, dp, ka, 1.0f, L.Pa, st);
    launch_rotate_aug(U, L.uperm, n, n, d, Wd, dp, ka, slack, L.Ua, st);
    BoundArgs ba{};
    ba.ka = ka;
    ba.Pb = L.Pa; ba.m = m; ba.mpad = L.T.mpad; ba.Ub = L.Ua; ba.tau_lo = L.us.tau_lo;
    ba.abs_slack = 0x1p-60f; ba.cs = L.cs;
    ba.nsplit = L.nsplitB; ba.partial = L.partialB; ba.pairs = ctr + 2;
    HIPTRY(hipEventRecord(ev[6], st));
    launch_bound(ba, st);
    HIPTRY(hipEventRecord(ev[7], st));
    launch_colsum(L.partialB, L.nsplitB, m, L.uscore, st);
    // visit order: (uscore desc, id asc)
    launch_invert_perm(L.T.perm, m, L.inv, st);
    if (ctx->bound_out) launch_gather_i32(L.uscore, L.inv, m, ctx->bound_out, st);
    launch_visit_keys(L.uscore, L.inv, m, L.vkeys, L.visit, L.status, st);
    // the keys are ~uscore with 0 <= uscore <= n: only the bits of n vary
    HIPTRY(radix_sort_u32(L.vkeys, L.visit, m, L.usort, st, 0, 32 - __builtin_clz((unsigned)n)));
    launch_gather3_i32(L.uscore, L.cs, L.T.perm, L.visit, m, L.vis_us, L.vis_cs, L.vis_cid, st);
    // pinned host copies (grown once per larger m): bounds and prefixes in
    // visit order, then room for a batch's result block
    const int64_t need = 2 * m + (int64_t)(RES_BYTES / sizeof(int32_t));
    if (ctx->h_vis_cap < need) {
        if (ctx->h_vis) HIPTRY(hipHostFree(ctx->h_vis));
        ctx->h_vis = nullptr;
        ctx->h_vis_cap = 0;
        HIPTRY(hipHostMalloc((void **)&ctx->h_vis, sizeof(int32_t) * need, hipHostMallocDefault));
        ctx->h_vis_cap = need;
    }
    int32_t *h_us = ctx->h_vis, *h_cs = ctx->h_vis + m;
    HIPTRY(hipMemcpyAsync(h_us, L.vis_us, sizeof(int32_t) * 2 * m, hipMemcpyDeviceToHost, st));
    HIPTRY(hipEventRecord(ev[2], st));
    // (no synchronisation here: the first batch goes out at once, and these
    // copies arrive with its results; its input check is read then, before
    // anything is returned)

    // ---- stage (b): exact scores in bound order, running top-N, stop rule
    // (every batch ends with the status, the top-N list and the statistics
    // copied to the host: the last batch's copies are the results)
    uint8_t *h_res = reinterpret_cast<uint8_t *>(ctx->h_vis + 2 * m);
    const int32_t *h_st = reinterpret_cast<const int32_t *>(h_res + RES_STATUS);
    const uint64_t *top = reinterpret_cast<const uint64_t *>(h_res + RES_TOP);
    const int64_t *h_ctr = reinterpret_cast<const int64_t *>(h_res + RES_CTR);
    int64_t r0 = 0, visited = 0, batches = 0, screened = 0, launches = 0;
    float ms_count_k = 0.0f;
    // First batch: the items with the largest bounds.  After it, the items
    // that can still enter the top-N are exactly those whose bound reaches
    // the current N-th score: a prefix of the visit order, scored next.
    int64_t bsz = std::min(bfirst, bmax);
    while (r0 < m && bsz > 0) {
        const int64_t r1 = std::min<int64_t>(m, r0 + bsz);
        const int64_t nb = r1 - r0;
        // the batch's users: the longest prefix of its items; the first
        // batch's is taken on the device (the host does not have the prefixes
        // yet), with n for the launch shape
        const bool first = batches == 0;
        int64_t ulen = 0;
        if (first) {
            launch_max_i32(L.vis_cs, nb, L.ulen_dev, st);
            ulen = n;
        } else {
            for (int64_t r = r0; r < r1; ++r) ulen = std::max<int64_t>(ulen, h_cs[r]);
        }
        CountArgs a{};
        a.prec = prec;
        a.Pq = L.T.Pq; a.Np = L.T.Np; a.Nhp = L.T.Nhp; a.Rp = L.T.Rp; a.sp = L.T.sp;
        a.rows = L.visit + r0; a.nb = nb;
        a.item_tie = L.T.perm; a.item_orig = L.T.perm; a.Porig = P;
        a.Us = L.Us; a.ulen = ulen; a.us = L.us; a.Uorig = U; a.d = d; a.D = D;
        a.ulen_dev = first ? L.ulen_dev : nullptr;
        a.c_err = ec.c; a.c2 = ec.c2; a.e_abs = E_ABS;
        a.nsplit = count_splits(nb, ulen, L.nsplitC_max);
        a.partial = L.partialC;
        a.rechecks = L.rechecks;
        if (ulen > 0) {
            HIPTRY(hipEventRecord(ev[8], st));
            launch_count(a, st);
            HIPTRY(hipEventRecord(ev[9], st));
            launch_colsum(L.partialC, a.nsplit, nb, L.batch_scores, st);
            ++launches;
        } else {
            HIPTRY(hipMemsetAsync(L.batch_scores, 0, sizeof(int32_t) * nb, st));
        }
        launch_topn_merge(L.batch_scores, nb, L.vis_cid + r0, N, L.top, L.status, st);
        HIPTRY(hipGetLastError());
        HIPTRY(hipEventRecord(ev[3], st));
        HIPTRY(hipMemcpyAsync(h_res, L.status, RES_BYTES, hipMemcpyDeviceToHost, st));
        HIPTRY(hipStreamSynchronize(st));
        if (ulen > 0) {
            float t = 0.0f;
            (void)hipEventElapsedTime(&t, ev[8], ev[9]);
            ms_count_k += t;
        }
        if (first) {
            if (h_st[RES_BAD] != 0) return fail(ctx, RMIPS_ENONFINITE, BAD_INPUT);
            ulen = 0;  // the batch's own user count, for the statistics
            for (int64_t r = r0; r < r1; ++r) ulen = std::max<int64_t>(ulen, h_cs[r]);
        }
        visited += nb;
        ++batches;
        screened += nb * ulen;
        const int tauN = h_st[0];
        r0 = r1;
        if (tauN < 0) {
            bsz = bmax;  // fewer than N items seen so far
            continue;
        }
        // items whose bound is strictly below the N-th score cannot enter
        int64_t e = r0;
        while (e < m && h_us[e] >= tauN) ++e;
        bsz = std::min<int64_t>(e - r0, bmax);
    }
    ctx->prof.resolve();  // (the stream is idle after the last batch)
    if (batches == 0) return fail(ctx, RMIPS_EDEVICE, "no item batch was scored");
    if (h_st[1] != N) return fail(ctx, RMIPS_EDEVICE, "top-N list incomplete");
    for (int i = 0; i < N; ++i) {
        top_scores[i] = (int32_t)(top[i] >> 32);
        top_ids[i] = (int32_t)(~(uint32_t)(top[i] & 0xffffffffu));
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->visited_items = visited;
        stats->batches = batches;
        const int64_t *h = h_ctr;
        int64_t tp = 0, rp = 0, cs[4] = {0, 0, 0, 0};
        for (int i = 0; i < CSTAT_SLOTS; ++i) {
            tp += h[CTR_PAIRS + i];
            rp += h[CTR_RPAIRS + i];
            for (int j = 0; j < 4; ++j) cs[j] += h[CTR_CS + 4 * i + j];
        }
        stats->cand_pairs = cs[1];
        stats->cand_listed = cs[0];
        stats->overflow_users = cs[2];
        stats->refine_users = cs[3];
        stats->recheck_pairs = h[0];
        stats->thresh_pairs = tp;
        stats->refine_pairs = rp;
        stats->bound_pairs = h[2];
        stats->count_pairs = screened;
        stats->screened_pairs = screened + tp + rp;
        stats->count_launches = launches;
        float t01 = 0, t12 = 0, t23 = 0, t03 = 0, tsc = 0, tbd = 0;
        (void)hipEventElapsedTime(&t01, ev[0], ev[1]);
        (void)hipEventElapsedTime(&t12, ev[1], ev[2]);
        (void)hipEventElapsedTime(&t23, ev[2], ev[3]);
        (void)hipEventElapsedTime(&t03, ev[0], ev[3]);
        (void)hipEventElapsedTime(&tsc, ev[4], ev[5]);
        (void)hipEventElapsedTime(&tbd, ev[6], ev[7]);
        stats->ms_thresh = t01;
        stats->ms_bound = t12;
        stats->ms_count = t23;
        stats->ms_total = t03;
        stats->ms_screen = tsc;
        stats->ms_count_kernels = ms_count_k;
        stats->ms_bound_kernel = tbd;
    }
    return RMIPS_OK;
}

static rmips_status soft_common(rmips_ctx *ctx, const float *U, int64_t n, const float *tau,
                                const float *Q, int64_t nq, int32_t d, float T, void *ws,
                                size_t ws_bytes) {
    if (!ctx) return RMIPS_EINVAL;
    if (n < 1 || nq < 1 || nq > (int64_t)INT32_MAX / 2 || d < 1 || d > RMIPS_D_MAX)
        return fail(ctx, RMIPS_EINVAL, "size out of range");
    if (!(T > 0.0f) || !std::isfinite(T)) return fail(ctx, RMIPS_EINVAL, "T must be > 0");
    if (!U || !tau || !Q || !ws) return fail(ctx, RMIPS_EINVAL, "null pointer");
    if (ws_bytes < rmips_soft_workspace_size(n, nq, d))
        return fail(ctx, RMIPS_EWORKSPACE, "workspace too small");
    HIPTRY(hipSetDevice(ctx->device));
    return RMIPS_OK;
}

rmips_status rmips_soft_fwd(rmips_ctx *ctx, const float *U, int64_t n, const float *tau,
                            const float *Q, int64_t nq, int32_t d, float T, void *ws,
                            size_t ws_bytes, float *S) {
    rmips_status s = soft_common(ctx, U, n, tau, Q, nq, d, T, ws, ws_bytes);
    if (s != RMIPS_OK) return s;
    if (!S) return fail(ctx, RMIPS_EINVAL, "null pointer");
    ProfGuard pguard(ctx);
    launch_soft(U, n, tau, Q, nq, d, T, nullptr, S, nullptr, ws, ctx->stream);
    HIPTRY(hipGetLastError());
    return RMIPS_OK;
}

rmips_status rmips_soft_bwd(rmips_ctx *ctx, const float *U, int64_t n, const float *tau,
                            const float *Q, int64_t nq, int32_t d, float T, const float *dS,
                            void *ws, size_t ws_bytes, float *dQ) {
    rmips_status s = soft_common(ctx, U, n, tau, Q, nq, d, T, ws, ws_bytes);
    if (s != RMIPS_OK) return s;
    if (!dS || !dQ) return fail(ctx, RMIPS_EINVAL, "null pointer");
    ProfGuard pguard(ctx);
    launch_soft(U, n, tau, Q, nq, d, T, dS, nullptr, dQ, ws, ctx->stream);
    HIPTRY(hipGetLastError());
    return RMIPS_OK;
}

rmips_status rmips_soft_bwd_noalloc(rmips_ctx *ctx, const float *U, int64_t n,
                                    const float *tau, const float *Q, int64_t nq, int32_t d,
                                    float T, const float *dS, float *dQ) {
    if (!ctx) return RMIPS_EINVAL;
    if (n < 1 || nq < 1 || nq > (int64_t)INT32_MAX / 2 || d < 1 || d > RMIPS_D_MAX)
        return fail(ctx, RMIPS_EINVAL, "size out of range");
    if (!soft_noalloc_fits(nq, d))
        return fail(ctx, RMIPS_EINVAL,
                    "nq * (d rounded up to 32) exceeds 65536, the size of the static scratch");
    if (!(T > 0.0f) || !std::isfinite(T)) return fail(ctx, RMIPS_EINVAL, "T must be > 0");
    if (!U || !tau || !Q || !dS || !dQ) return fail(ctx, RMIPS_EINVAL, "null pointer");
    HIPTRY(hipSetDevice(ctx->device));
    if (!ctx->soft_scratch) HIPTRY(soft_scratch_init(ctx->device, &ctx->soft_scratch));
    ProfGuard pguard(ctx);
    launch_soft(U, n, tau, Q, nq, d, T, dS, nullptr, dQ, ctx->soft_scratch, ctx->stream);
    HIPTRY(hipGetLastError());
    return RMIPS_OK;
}

size_t rmips_soft_workspace_size(int64_t n, int64_t nq, int32_t d) {
    if (n < 1 || nq < 1 || d < 1 || d > RMIPS_D_MAX) return 0;
    return soft_ws_bytes(n, nq, d);
}

}  // extern "C"

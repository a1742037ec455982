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
    int32_t dprime = 0;  // d' of the Eq. (3) bound (0: d' = d)
    int32_t prepass = -1;  // d' of rmips_topn's pre-pass (-1: automatic, 0: none)
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

// Split dimension d' of Eq. (3) (Sec. 4.2; d' = 10 in the paper's
// experiments, Sec. 5.1).  By default d' = d: the rotation is then the
// identity and the bound is the inner product itself plus the certified
// slack, so that stage (b) counts little more than the items that can reach
// the N-th score; the matrix-core bound pass pays for the larger d' in K
// only.  rmips_set_dprime selects a rotation onto the top-d' eigenvectors
// of a user sample instead (d' <= DPRIME_ROT_MAX).
constexpr int DPRIME_ROT_MAX = 62;
int dprime(const rmips_ctx *c, int d) { return (c->dprime > 0 && c->dprime < d) ? c->dprime : d; }
// Pre-pass of rmips_topn with the d' = d bound: every item's bound is first
// taken with a rotation onto DPRIME_ROT_MAX dimensions (a quarter of the
// terms at d = 200), and the d' = d bound only for the items whose pre-pass
// bound still reaches the N-th score after the first batch.  Automatic
// where the identity rows are at least twice as long as the rotated ones and
// the screening precision is FP32 or BF16: the items that the pre-pass
// leaves above the first batch's N-th score usually take a second, small
// batch, which streams every user again; with the wide bands of the 8-, 6-
// and 4-bit formats that batch costs more than the pre-pass saves.
int aug_len(int dp);
int prepass_dim(const rmips_ctx *c, int d, int dmain, int prec) {
    if (dmain < d || c->prepass == 0) return 0;
    const int dp = c->prepass > 0 ? c->prepass : DPRIME_ROT_MAX;
    if (dp >= d) return 0;
    if (c->prepass < 0 &&
        (aug_len(d) < 2 * aug_len(dp) || (prec != RMIPS_FP32 && prec != RMIPS_BF16)))
        return 0;
    return dp;
}
// augmented row length ka for d' values and two more columns: a multiple of
// 16, of 32 past 176 (the bound kernel of the longest rows takes 32 terms a
// step), at most 288 for d' <= 256; the identity's (d' = d) is the longest
int aug_len(int dp) {
    const int k16 = (dp + 2 + 15) & ~15;
    return k16 > 176 ? (dp + 2 + 31) & ~31 : k16;
}
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

// The prepared inputs: screening copies of users (caller order) and items
// (norm order), their norms and scales, the item order.  An index keeps
// them from its build to its queries.
void prep_plan(int prec, int64_t n, int64_t m, int d, ThreshLayout &L, Carve &cv) {
    L.prec = prec;
    L.D = padded_dim(prec, d);
    L.rowb = L.D * elem_bytes(prec);
    L.ntiles = (int)((m + TILE_ITEMS - 1) / TILE_ITEMS);
    L.mpad = (int64_t)L.ntiles * TILE_ITEMS;
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
    L.perm = cv.take<int32_t>(m);
}

// Stage (a)'s scratch: sort keys, candidate lists, refinement lists.
void thresh_scratch_plan(int prec, int64_t n, int64_t m, int d, int k, int cap_override,
                         ThreshLayout &L, Carve &cv) {
    // splits of the item range: about six rounds of screening workgroups
    // (256 users each, one per compute unit) over the whole chip
    int64_t utiles = (n + 255) / 256;
    int64_t ns = (1536 + utiles - 1) / utiles;
    ns = std::max<int64_t>(1, std::min<int64_t>(ns, 8));
    ns = std::min<int64_t>(ns, L.ntiles);
    L.nsplit = (int)ns;
    // candidate capacity per user (all splits together): well above the
    // candidate counts of typical users; users beyond it are screened again
    // with a tighter bound.  The wider error bands need longer lists: four
    // times for e4m3 (longer lists cost its final selection more than its
    // refinements save) and for e2m3 up to d = 128, eight for e2m3 beyond
    // (at d = 200 half of the users overflowed four times and went to the
    // exact fallback; at d = 50 and 100 the longer lists only slow the final
    // selection) and for e2m1.
    // (even: each list is written as two halves)
    if (cap_override > 0) {
        L.cap = (cap_override + 1) & ~1;
    } else {
        int64_t capU = std::max<int64_t>(256, 16 * (int64_t)k);
        if (prec == RMIPS_FP8_E4M3 || (prec == RMIPS_FP6_E2M3 && d <= 128)) capU *= 4;
        if ((prec == RMIPS_FP6_E2M3 && d > 128) || prec == RMIPS_FP4_E2M1) capU *= 8;
        L.cap = (int)(((capU + L.nsplit - 1) / L.nsplit + 7) / 8 * 8);
    }
    L.keys = cv.take<uint32_t>(m);
    L.sort_scratch = cv.take<uint8_t>(radix_sort_scratch_bytes(m));
    L.cand = cv.take<float2>((size_t)n * L.nsplit * L.cap);
    L.cand_id = cv.take<int32_t>((size_t)n * L.nsplit * L.cap);
    // counts per (user, split, half); refinement passes use up to 8 splits
    L.cand_cnt = cv.take<int32_t>((size_t)n * 16);
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

void thresh_plan(int prec, int64_t n, int64_t m, int d, int k, int cap_override, ThreshLayout &L,
                 Carve &cv) {
    prep_plan(prec, n, m, d, L, cv);
    thresh_scratch_plan(prec, n, m, d, k, cap_override, L, cv);
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
                            int32_t *tau_id, int32_t *topk, double *topv,
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
    a.tau = tau; a.tau_id = tau_id; a.topk = topk; a.topv = topk ? topv : nullptr;
    a.pairs = pairs; a.rpairs = rpairs; a.ev0 = ev0; a.ev1 = ev1; a.cstats = cstats;
    if (thresh_screen_lds(L.prec, L.D) > 160 * 1024 || (size_t)final_stride(L.cap * L.nsplit) * final_entry_bytes() > 150 * 1024)
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
    if (prec != RMIPS_FP32 && prec != RMIPS_BF16 && prec != RMIPS_FP8_E4M3 &&
        prec != RMIPS_FP6_E2M3 && prec != RMIPS_FP4_E2M1)
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
// (c) bound pairs, [3] those of the d' = d bound after a pre-pass,
// [8, 8 + CSTAT_SLOTS) pairs screened by stage (a)'s main
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

// Users in the order of their pruning ratio rho_u = tau_u / ||u|| (stage
// (c)): the order, each item's Cauchy-Schwarz prefix, the counting stage's
// per-user records and screening rows in that order.
struct PrefixLayout {
    double *tau;
    int32_t *tau_id;
    uint32_t *ukeys;
    int32_t *uperm;
    void *usort;
    int32_t *cs;
    UserSide us;
    void *Us;
};

// Eq. (3)/(6) bound counts: the Gram matrix of a user sample, the
// augmented BF16 rows (2 ka bytes each) and per-split partial counts.
struct BoundLayout {
    double *G, *Gs;
    uint4 *Pa, *Ua;
    int nsplitB;
    int32_t *partialB;
};

// Stage (b): the visit order and its bounds, prefixes and ids, the batch
// partial counts, and the block of a batch's results.
struct CountLayout {
    int32_t *inv;
    uint32_t *vkeys;
    int32_t *visit, *vis_us, *vis_cs, *vis_cid;
    int nsplitC_max;
    int32_t *partialC, *batch_scores;
    uint64_t *top;
    int32_t *status;
    int64_t *rechecks;
    int32_t *ulen_dev;
    // a re-bounded segment of the visit order (local slots): norm-order rows,
    // prefixes, caller ids, both bounds, slot orders
    int32_t *sg_row, *sg_cs, *sg_id, *sg_b0, *sg_b, *sg_v1, *sg_v2;
};

struct TopnLayout {
    ThreshLayout T;
    PrefixLayout X;
    double *W;
    BoundLayout B;
    int32_t *uscore;
    CountLayout C;
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

void prefix_plan(int64_t n, int64_t m, int64_t mpad, int rowb, PrefixLayout &X, Carve &cv) {
    X.tau = cv.take<double>(n);
    X.tau_id = cv.take<int32_t>(n);
    X.ukeys = cv.take<uint32_t>(n);
    X.uperm = cv.take<int32_t>(n);
    X.usort = cv.take<uint8_t>(radix_sort_scratch_bytes(std::max(n, m)));
    X.cs = cv.take<int32_t>(mpad);
    user_side_plan(n, X.us, cv);
    X.Us = cv.take<uint8_t>((size_t)n * rowb);
}

void bound_plan(int64_t n, int64_t m, int64_t mpad, int d, BoundLayout &B, Carve &cv) {
    B.G = cv.take<double>((size_t)d * d);
    B.Gs = cv.take<double>(gram_scratch_bytes(d) / sizeof(double));
    // ka BF16 values per row, for the longest rows (d' = d)
    B.Pa = cv.take<uint4>((size_t)mpad * aug_len(d) / 8);
    B.Ua = cv.take<uint4>((size_t)n * aug_len(d) / 8);
    B.nsplitB = bound_splits(m, aug_len(d));
    B.partialB = cv.take<int32_t>((size_t)B.nsplitB * m);
}

void count_plan(int64_t m, int bmax, CountLayout &C, Carve &cv, bool with_inv) {
    C.inv = with_inv ? cv.take<int32_t>(m) : nullptr;
    C.vkeys = cv.take<uint32_t>(m);
    C.visit = cv.take<int32_t>(m);
    C.vis_us = cv.take<int32_t>(2 * m);  // bounds, then prefixes: one copy to the host
    C.vis_cs = C.vis_us + m;
    C.vis_cid = cv.take<int32_t>(m);
    C.nsplitC_max = 256;
    C.partialC = cv.take<int32_t>((size_t)C.nsplitC_max * bmax);
    C.batch_scores = cv.take<int32_t>(bmax);
    // the results of a batch in one block, copied to the host at once:
    // status, the top-N list, the counters
    uint8_t *res = cv.take<uint8_t>(RES_BYTES);
    C.status = reinterpret_cast<int32_t *>(res + RES_STATUS);
    C.top = reinterpret_cast<uint64_t *>(res + RES_TOP);
    C.rechecks = reinterpret_cast<int64_t *>(res + RES_CTR);
    C.ulen_dev = cv.take<int32_t>(1);
    int32_t *sg = cv.take<int32_t>((size_t)7 * m);
    C.sg_row = sg; C.sg_cs = sg + m; C.sg_id = sg + 2 * m; C.sg_b0 = sg + 3 * m;
    C.sg_b = sg + 4 * m; C.sg_v1 = sg + 5 * m; C.sg_v2 = sg + 6 * m;
}

void topn_plan(int prec, int64_t n, int64_t m, int d, int k, int cap_override, int bmax,
               TopnLayout &L, Carve &cv) {
    thresh_plan(prec, n, m, d, k, cap_override, L.T, cv);
    prefix_plan(n, m, L.T.mpad, L.T.rowb, L.X, cv);
    L.W = cv.take<double>((size_t)DPRIME_ROT_MAX * d);
    bound_plan(n, m, L.T.mpad, d, L.B, cv);
    L.uscore = cv.take<int32_t>(m);
    count_plan(m, bmax, L.C, cv, true);
    // stage (a)'s flags live in the status words (copied with every batch)
    L.T.bad = L.C.status + RES_BAD;
    L.T.rmax = reinterpret_cast<unsigned int *>(L.C.status + RES_RMAX);
}

// A k_max index (Alg. 1's offline stage): the prepared inputs, each
// user's k_max largest values and their ids (the lists A_i, exact), the
// rotation W of Eq. (3), the inverse item order, the Eq. (3)/(6) bound of
// every item for every k <= k_max (k-major, norm order), and a header.
constexpr int32_t INDEX_MAGIC = 0x584d5200;  // with a version in the low byte
constexpr int INDEX_HDR_WORDS = 8;
struct IndexLayout {
    ThreshLayout T;
    double *topv;
    int32_t *topk;
    double *W;
    int32_t *inv;
    int32_t *table;
    int32_t *hdr;
};

void index_plan(int prec, int64_t n, int64_t m, int d, int kmax, IndexLayout &I, Carve &cv) {
    prep_plan(prec, n, m, d, I.T, cv);
    I.topv = cv.take<double>((size_t)n * kmax);
    I.topk = cv.take<int32_t>((size_t)n * kmax);
    I.W = cv.take<double>((size_t)DPRIME_ROT_MAX * d);
    I.inv = cv.take<int32_t>(m);
    I.table = cv.take<int32_t>((size_t)kmax * m);
    I.hdr = cv.take<int32_t>(INDEX_HDR_WORDS);
}

// header words: version, n, m, d, kmax, precision, the d' of the build's
// bound (a record only: queries accept any), 0
constexpr int INDEX_HDR_DPRIME = 6;
void index_header(int64_t n, int64_t m, int d, int kmax, int prec, int dp,
                  int32_t (&h)[INDEX_HDR_WORDS]) {
    h[0] = INDEX_MAGIC | 1;
    h[1] = (int32_t)n;
    h[2] = (int32_t)m;
    h[3] = d;
    h[4] = kmax;
    h[5] = prec;
    h[INDEX_HDR_DPRIME] = dp;
    h[7] = 0;
}

// scratch of an index build: stage (a)'s, the rho order, the bound's
void index_build_plan(int prec, int64_t n, int64_t m, int d, int kmax, int cap_override,
                      IndexLayout &I, PrefixLayout &X, BoundLayout &B, Carve &cv) {
    thresh_scratch_plan(prec, n, m, d, kmax, cap_override, I.T, cv);
    prefix_plan(n, m, I.T.mpad, I.T.rowb, X, cv);
    bound_plan(n, m, I.T.mpad, d, B, cv);
}

// scratch of an index query: the rho order and stage (b)
void index_query_plan(int64_t n, int64_t m, const IndexLayout &I, PrefixLayout &X,
                      CountLayout &C, Carve &cv) {
    prefix_plan(n, m, I.T.mpad, I.T.rowb, X, cv);
    count_plan(m, BATCH_MAX, C, cv, false);
    C.inv = I.inv;
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

// Stage (c), first part: users sorted by their ratio keys without the low
// 8 bits (3 passes instead of 4): each item's prefix may take users whose
// ratio is up to 2^-15 relative above its norm, which the bound and the
// count then test; the counting stage's per-user records and screening
// rows in that order.  X.tau / X.tau_id hold the thresholds.
void run_prefix(const ThreshLayout &T, PrefixLayout &X, int64_t n, int64_t m, float c2,
                hipStream_t st, bool with_rows = true) {
    launch_rho_keys(X.tau, T.Nu, n, X.ukeys, X.uperm, st);
    (void)radix_sort_u32(X.ukeys, X.uperm, n, X.usort, st, RHO_LO_BIT, 32);
    launch_cs_prefix(X.ukeys, n, T.Np, m, RHO_LO_BIT, X.cs, st);
    launch_user_side(X.tau, X.tau_id, T.Nu, T.Nhu, T.Ru, T.su, X.uperm, n, c2, X.us, st);
    if (with_rows) launch_gather_padded(T.Uq, X.uperm, n, T.rowb, X.Us, st);
}

// Relative slack s of the Eq. (3) bound, in units of ||u|| ||p||: each
// augmented value is stored as BF16 hi(x) = rn(x), |x - hi(x)| <= 2^-9 |x|,
// so each product hi(a) hi(b) is within (2 * 2^-9 + 2^-18) |a| |b| of a b,
// at most 1.003 * 2^-8 * 1.415 ||p|| ||u|| over a row (sum |a_i||b_i| <=
// ||a|| ||b|| <= 1.415 ||p|| ||u||); the matrix-core FP32 sums of <= 288
// exact BF16 products add gamma_288 (< 2^-15.8) of the same, and the FP32
// rounding of W x (2^-24 relative) is far below: 1.43 * 2^-8 in all.  The
// slack column hi(||p||) hi(s ||u||) gives at least s (1 - 2^-9)^2 ||p||
// ||u||: s = 2^-7 covers that with room.  The absolute slack covers BF16
// and FP32 underflow (norms are below 2^60), subnormal operands flushed by
// the matrix cores included: the flushed terms of a row sum to at most
// 2^-126 sqrt(ka) 1.42 * 2^60 < 2^-61, and products that underflow FP32 to
// far less.
constexpr float BOUND_SLACK = 0x1p-7f;
constexpr float BOUND_ABS_SLACK = 0x1p-60f;

// Stage (c), second part: the Eq. (3)/(6) bound count of every item (norm
// order) into `uscore`, over the users of its prefix (users' augmented rows
// in rho order; the items' rows must already be in B.Pa).  Wd: the rotation
// (dp x d), NULL for the identity (dp = d).
void run_bound(const float *U, const PrefixLayout &X, const BoundLayout &B, const double *Wd,
               int dp, int64_t n, int64_t m, int64_t mpad, int d, unsigned long long *pairs,
               hipEvent_t e0, hipEvent_t e1, int32_t *uscore, hipStream_t st) {
    const int ka = aug_len(dp);
    launch_rotate_aug(U, X.uperm, n, n, d, Wd, dp, ka, BOUND_SLACK, B.Ua, st);
    BoundArgs ba{};
    ba.ka = ka;
    ba.Pb = B.Pa; ba.m = m; ba.mpad = mpad; ba.Ub = B.Ua; ba.tau_lo = X.us.tau_lo;
    ba.abs_slack = BOUND_ABS_SLACK; ba.cs = X.cs;
    ba.nsplit = B.nsplitB; ba.partial = B.partialB; ba.pairs = pairs;
    if (e0) (void)hipEventRecord(e0, st);
    launch_bound(ba, st);
    if (e1) (void)hipEventRecord(e1, st);
    launch_colsum(B.partialB, B.nsplitB, m, uscore, st);
}

// The second bound of rmips_topn's pre-pass (see prepass_dim): what the
// d' = d bound of a segment of the visit order needs.
struct Refine {
    const float *U, *P;
    const ThreshLayout *T;
    const PrefixLayout *X;
    const BoundLayout *B;
    int64_t n, m;
    int d;
    int32_t *uscore;                 // norm order: tightened in place
    unsigned long long *pairs;       // stats (may be NULL)
};

// Positions [r0, r1) of the visit order hold every item whose pre-pass bound
// reaches the current N-th score and that is not yet scored.  Their d' = d
// bounds (the identity rows, items in norm order so that each block's first
// prefix is its longest), each tightened to the smaller of its two bounds,
// then the segment re-sorted in place by (bound desc, id asc), with its
// prefixes and ids.  Items past r1 keep pre-pass bounds below that score.
hipError_t refine_segment(const Refine &R, CountLayout &C, int64_t r0, int64_t r1,
                          hipStream_t st) {
    const int64_t ns = r1 - r0;
    const int ka = aug_len(R.d);
    uint32_t *key = C.vkeys;  // free once the visit order is sorted
    const int mbits = 32 - __builtin_clz((unsigned)R.m);
    hipError_t e = hipMemcpyAsync(C.sg_row, C.visit + r0, sizeof(int32_t) * ns,
                                  hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(key, C.visit + r0, sizeof(int32_t) * ns, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    e = radix_sort_u32(key, C.sg_row, ns, R.X->usort, st, 0, mbits);  // norm order
    if (e != hipSuccess) return e;
    launch_gather3_i32(R.X->cs, R.T->perm, R.uscore, C.sg_row, ns, C.sg_cs, C.sg_id, C.sg_b0,
                       st);
    launch_rotate_aug(R.P, C.sg_id, ns, ns, R.d, nullptr, R.d, ka, 1.0f, R.B->Pa, st);
    launch_rotate_aug(R.U, R.X->uperm, R.n, R.n, R.d, nullptr, R.d, ka, BOUND_SLACK, R.B->Ua,
                      st);
    BoundArgs ba{};
    ba.ka = ka;
    ba.Pb = R.B->Pa; ba.m = ns; ba.mpad = ns; ba.Ub = R.B->Ua; ba.tau_lo = R.X->us.tau_lo;
    ba.abs_slack = BOUND_ABS_SLACK; ba.cs = C.sg_cs;
    // few items: more splits of each block's users than the full pass takes,
    // within the partial counts' room
    const int64_t room = (int64_t)R.B->nsplitB * R.m / ns;
    ba.nsplit = bound_splits(ns, ka, (int)std::min<int64_t>(256, room));
    ba.partial = R.B->partialB; ba.pairs = R.pairs;
    launch_bound(ba, st, "k_bound/rebound");
    launch_colsum(R.B->partialB, ba.nsplit, ns, C.sg_b, st);
    launch_seg_bound(C.sg_b, C.sg_b0, C.sg_row, ns, R.uscore, st);
    // (bound desc, id asc): the slots by id, then stably by ~bound
    launch_seg_init(C.sg_id, ns, key, C.sg_v1, st);
    e = radix_sort_u32(key, C.sg_v1, ns, R.X->usort, st, 0, mbits);
    if (e != hipSuccess) return e;
    launch_visit_keys(C.sg_b, C.sg_v1, ns, key, C.sg_v2, nullptr, st);
    e = radix_sort_u32(key, C.sg_v2, ns, R.X->usort, st, 0,
                       32 - __builtin_clz((unsigned)R.n));
    if (e != hipSuccess) return e;
    launch_gather3_i32(C.sg_row, C.sg_b, C.sg_cs, C.sg_v2, ns, C.visit + r0, C.vis_us + r0,
                       C.vis_cs + r0, st);
    launch_gather_i32(C.sg_id, C.sg_v2, ns, C.vis_cid + r0, st);
    return hipGetLastError();
}

// Host side of stage (b): events and the counters a caller reports.
struct CountRun {
    hipEvent_t ev_vis, ev_end, ev_k0, ev_k1;  // visit order ready, last copy, kernel brackets
    int64_t visited = 0, batches = 0, screened = 0, launches = 0;
    int64_t rebound = 0;  // items of the re-bounded segment
    float ms_count_k = 0.0f;
};

rmips_status run_count_topn(rmips_ctx *ctx, const float *U, const float *P,
                            const ThreshLayout &T, const PrefixLayout &X, CountLayout &C,
                            const int32_t *uscore, int64_t n, int64_t m, int d, int N,
                            const ErrConst &ec, int bfirst, int bmax, CountRun &cr,
                            int32_t *top_ids, int32_t *top_scores, const int32_t **h_ctr_out,
                            const Refine *rf);

}  // namespace

namespace {

// Stage (b) of Alg. 2 from the bounds `uscore` (norm order): the visit order
// (uscore desc, id asc), then batches of exact scores with the running
// top-N until the next bound is below the current N-th score.  The first
// batch goes out without a host synchronisation; stage (a)'s input check
// (status word RES_BAD) is read with its results.  On success writes the
// top-N (host) and points *h_ctr_out at the host copy of the counters.
// With `rf` (bounds from a pre-pass), the items still open once an N-th
// score is known are re-bounded with d' = d (refine_segment) before the
// next batch.
rmips_status run_count_topn(rmips_ctx *ctx, const float *U, const float *P,
                            const ThreshLayout &T, const PrefixLayout &X, CountLayout &C,
                            const int32_t *uscore, int64_t n, int64_t m, int d, int N,
                            const ErrConst &ec, int bfirst, int bmax, CountRun &cr,
                            int32_t *top_ids, int32_t *top_scores, const int32_t **h_ctr_out,
                            const Refine *rf) {
    hipStream_t st = ctx->stream;
    launch_visit_keys(uscore, C.inv, m, C.vkeys, C.visit, C.status, st);
    // the keys are ~uscore with 0 <= uscore <= n: only the bits of n vary
    HIPTRY(radix_sort_u32(C.vkeys, C.visit, m, X.usort, st, 0, 32 - __builtin_clz((unsigned)n)));
    launch_gather3_i32(uscore, X.cs, T.perm, C.visit, m, C.vis_us, C.vis_cs, C.vis_cid, st);
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
    HIPTRY(hipMemcpyAsync(h_us, C.vis_us, sizeof(int32_t) * 2 * m, hipMemcpyDeviceToHost, st));
    HIPTRY(hipEventRecord(cr.ev_vis, st));
    // (no synchronisation here: the first batch goes out at once, and these
    // copies arrive with its results; the input check is read then, before
    // anything is returned)

    // every batch ends with the status, the top-N list and the statistics
    // copied to the host: the last batch's copies are the results
    uint8_t *h_res = reinterpret_cast<uint8_t *>(ctx->h_vis + 2 * m);
    const int32_t *h_st = reinterpret_cast<const int32_t *>(h_res + RES_STATUS);
    const uint64_t *top = reinterpret_cast<const uint64_t *>(h_res + RES_TOP);
    int64_t r0 = 0;
    bool refined = rf == nullptr;
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
        const bool first = cr.batches == 0;
        int64_t ulen = 0;
        if (first) {
            launch_max_i32(C.vis_cs, nb, C.ulen_dev, st);
            ulen = n;
        } else {
            for (int64_t r = r0; r < r1; ++r) ulen = std::max<int64_t>(ulen, h_cs[r]);
        }
        // the batch's slots in norm order (the host's copies of the bounds
        // and prefixes stay in visit order; the batch is a set)
        launch_batch_order(C.visit + r0, C.vis_cid + r0, nb, st);
        CountArgs a{};
        a.prec = T.prec;
        a.Pq = T.Pq; a.Np = T.Np; a.Nhp = T.Nhp; a.Rp = T.Rp; a.sp = T.sp;
        a.rows = C.visit + r0; a.nb = nb;
        a.item_tie = T.perm; a.item_orig = T.perm; a.Porig = P;
        a.Us = X.Us; a.ulen = ulen; a.us = X.us; a.Uorig = U; a.d = d; a.D = T.D;
        a.ulen_dev = first ? C.ulen_dev : nullptr;
        a.c_err = ec.c; a.c2 = ec.c2; a.e_abs = E_ABS;
        a.nsplit = count_splits(nb, ulen, C.nsplitC_max);
        a.partial = C.partialC;
        a.rechecks = C.rechecks;
        if (ulen > 0) {
            HIPTRY(hipEventRecord(cr.ev_k0, st));
            launch_count(a, st);
            HIPTRY(hipEventRecord(cr.ev_k1, st));
            launch_colsum(C.partialC, a.nsplit, nb, C.batch_scores, st);
            ++cr.launches;
        } else {
            HIPTRY(hipMemsetAsync(C.batch_scores, 0, sizeof(int32_t) * nb, st));
        }
        launch_topn_merge(C.batch_scores, nb, C.vis_cid + r0, N, C.top, C.status, st);
        HIPTRY(hipGetLastError());
        HIPTRY(hipEventRecord(cr.ev_end, st));
        HIPTRY(hipMemcpyAsync(h_res, C.status, RES_BYTES, hipMemcpyDeviceToHost, st));
        HIPTRY(hipStreamSynchronize(st));
        if (ulen > 0) {
            float t = 0.0f;
            (void)hipEventElapsedTime(&t, cr.ev_k0, cr.ev_k1);
            cr.ms_count_k += t;
        }
        if (first) {
            if (h_st[RES_BAD] != 0) return fail(ctx, RMIPS_ENONFINITE, BAD_INPUT);
            ulen = 0;  // the batch's own user count, for the statistics
            for (int64_t r = r0; r < r1; ++r) ulen = std::max<int64_t>(ulen, h_cs[r]);
        }
        cr.visited += nb;
        ++cr.batches;
        cr.screened += nb * ulen;
        const int tauN = h_st[0];
        r0 = r1;
        if (tauN < 0) {
            bsz = bmax;  // fewer than N items seen so far
            continue;
        }
        // items whose bound is strictly below the N-th score cannot enter
        int64_t e = r0;
        while (e < m && h_us[e] >= tauN) ++e;
        if (!refined && e > r0) {
            refined = true;
            cr.rebound = e - r0;
            HIPTRY(refine_segment(*rf, C, r0, e, st));
            // (the counters again, in case no batch follows)
            HIPTRY(hipMemcpyAsync(h_res + RES_CTR, C.status + RES_CTR / sizeof(int32_t),
                                  RES_TOP - RES_CTR, hipMemcpyDeviceToHost, st));
            HIPTRY(hipMemcpyAsync(h_us + r0, C.vis_us + r0, sizeof(int32_t) * (e - r0),
                                  hipMemcpyDeviceToHost, st));
            HIPTRY(hipMemcpyAsync(h_cs + r0, C.vis_cs + r0, sizeof(int32_t) * (e - r0),
                                  hipMemcpyDeviceToHost, st));
            HIPTRY(hipStreamSynchronize(st));
            e = r0;
            while (e < m && h_us[e] >= tauN) ++e;
        }
        bsz = std::min<int64_t>(e - r0, bmax);
    }
    ctx->prof.resolve();  // (the stream is idle after the last batch)
    if (cr.batches == 0) return fail(ctx, RMIPS_EDEVICE, "no item batch was scored");
    if (h_st[1] != N) return fail(ctx, RMIPS_EDEVICE, "top-N list incomplete");
    for (int i = 0; i < N; ++i) {
        top_scores[i] = (int32_t)(top[i] >> 32);
        top_ids[i] = (int32_t)(~(uint32_t)(top[i] & 0xffffffffu));
    }
    *h_ctr_out = reinterpret_cast<const int32_t *>(h_res + RES_CTR);
    return RMIPS_OK;
}


// ------------------------------------------------------- budgeted index
// Alg. 1 under an inner-product budget (Sec. 4.2) and Alg. 2 with
// Inc-RMIPS (Sec. 4.3).  Positions j = 1..m are the items in descending
// order of the FP64 sum of squares (ties by id).
constexpr int32_t BUDGET_MAGIC = 0x42554400;  // with a version in the low byte
constexpr int BUDGET_HDR_WORDS = 16;
constexpr int H_BHDR = 96;   // pinned status words that receive the header
constexpr int H_BCTR = 112;  // pinned status words for a query's counters
constexpr int BUDGET_DP = 10;  // d' of Eq. (3) in the paper's experiments (Sec. 5.1)
int budget_dp(int d) { return std::min(d, std::min(BUDGET_DP, BUDGET_DP_MAX)); }

struct BudgetLayout {
    int32_t *hdr;
    double *info;                  // the build's figures (rmips_budget_info)
    int32_t *order, *posof;        // position - 1 -> id, id -> position - 1
    double *np2s, *Pl, *nrp, *npn; // items in position order: |p|^2, Eq. (3) data
    double *nu2, *Ul, *nru, *nun;  // users: |u|^2, Eq. (3) data
    double *W;                     // the rotation's first dp rows (dp x d)
    double *Av;                    // lists A_i: values (n x kmax)
    int32_t *Aj;                   //            item ids
    int32_t *pos;                  // pos_i for users of U'', else 0
    double *lam;                   // lambda_i (Eq. 7) for users of U'', else -inf
    int32_t *key, *rank;           // j' + 1 - b1 and x_i for users of U', else 0
    int64_t *b2;                   // B_{2,i} for users of U', else 0
    int32_t *uscore;               // uscore_k(p): kmax x m, by item id
};

void budget_plan(int64_t n, int64_t m, int d, int kmax, BudgetLayout &B, Carve &cv) {
    const int dp = budget_dp(d);
    B.hdr = cv.take<int32_t>(BUDGET_HDR_WORDS);
    B.info = cv.take<double>(8);
    B.order = cv.take<int32_t>(m);
    B.posof = cv.take<int32_t>(m);
    B.np2s = cv.take<double>(m);
    B.Pl = cv.take<double>((size_t)m * dp);
    B.nrp = cv.take<double>(m);
    B.npn = cv.take<double>(m);
    B.nu2 = cv.take<double>(n);
    B.Ul = cv.take<double>((size_t)n * dp);
    B.nru = cv.take<double>(n);
    B.nun = cv.take<double>(n);
    B.W = cv.take<double>((size_t)dp * d);
    B.Av = cv.take<double>((size_t)n * kmax);
    B.Aj = cv.take<int32_t>((size_t)n * kmax);
    B.pos = cv.take<int32_t>(n);
    B.lam = cv.take<double>(n);
    B.key = cv.take<int32_t>(n);
    B.rank = cv.take<int32_t>(n);
    B.b2 = cv.take<int64_t>(n);
    B.uscore = cv.take<int32_t>((size_t)kmax * m);
}

void budget_header(int64_t n, int64_t m, int d, int kmax, int32_t (&h)[BUDGET_HDR_WORDS]) {
    std::memset(h, 0, sizeof(h));
    h[0] = BUDGET_MAGIC | 1;
    h[1] = (int32_t)n;
    h[2] = (int32_t)m;
    h[3] = d;
    h[4] = kmax;
    h[5] = budget_dp(d);
}

// Scratch of a build and of a query (one workspace serves both): stage (a)
// for up to n users with k <= kmax, gathered rows, and the query's sets.
struct BudgetScratch {
    ThreshLayout T;
    float *PgT;          // items transposed (d x m), position order
    double *np2;         // item sums of squares by id
    float *Ug;           // gathered user rows (U' at the build, rescans at a query)
    double *topv, *tau;
    int32_t *topk, *tau_id;
    int32_t *ux, *t, *u2, *lims;
    double *G, *Gs;
    int32_t *X, *X2, *R, *ctr;
    uint8_t *xflag, *visited;
    int32_t *base, *slot, *cnt, *score;
    uint32_t *vkey;
    int32_t *vval;
    void *vsort;
};

void budget_scratch_plan(int prec, int64_t n, int64_t m, int d, int kmax, int cap_override,
                         BudgetScratch &S, Carve &cv) {
    thresh_plan(prec, n, m, d, kmax, cap_override, S.T, cv);
    S.PgT = cv.take<float>((size_t)m * d);
    S.np2 = cv.take<double>(m);
    S.Ug = cv.take<float>((size_t)n * d);
    S.topv = cv.take<double>((size_t)n * kmax);
    S.topk = cv.take<int32_t>((size_t)n * kmax);
    S.tau = cv.take<double>(n);
    S.tau_id = cv.take<int32_t>(n);
    S.ux = cv.take<int32_t>(n);
    S.t = cv.take<int32_t>(n);
    S.u2 = cv.take<int32_t>(n);
    S.lims = cv.take<int32_t>(n);
    S.G = cv.take<double>((size_t)d * d);
    S.Gs = reinterpret_cast<double *>(cv.take<uint8_t>(gram_scratch_bytes(d)));
    S.X = cv.take<int32_t>(n);
    S.X2 = cv.take<int32_t>(n);
    S.R = cv.take<int32_t>(n);
    S.ctr = cv.take<int32_t>(64);
    S.xflag = cv.take<uint8_t>(n);
    S.visited = cv.take<uint8_t>(m);
    S.base = cv.take<int32_t>(m);
    S.slot = cv.take<int32_t>(m);
    S.cnt = cv.take<int32_t>(BUDGET_BATCH_BIG);
    S.score = cv.take<int32_t>(BUDGET_BATCH_BIG);
    S.vkey = cv.take<uint32_t>(m);
    S.vval = cv.take<int32_t>(m);
    S.vsort = cv.take<uint8_t>(radix_sort_scratch_bytes(m));
}

// beta of Eq. (5): alpha (exp(beta X) - 1) / beta + gamma X = B2.  The left
// side grows with beta from gamma X (beta -> -inf) without bound, so the
// root is bracketed by doubling and halved down to adjacent doubles; -inf
// when B2 <= gamma X (then f(x) = gamma).
double budget_solve_beta(double X, double B2, double alpha, double gamma) {
    const double want = B2 - gamma * X;
    if (!(want > 0.0) || !(alpha > 0.0)) return -INFINITY;
    auto g = [&](double b) { return b == 0.0 ? alpha * X : alpha * std::expm1(b * X) / b; };
    const double g0 = g(0.0);
    if (g0 == want) return 0.0;
    double lo, hi;
    if (g0 < want) {
        lo = 0.0;
        hi = 1.0 / X;
        while (g(hi) < want) hi *= 2.0;
    } else {
        hi = 0.0;
        lo = -1.0 / X;
        while (g(lo) > want) lo *= 2.0;
    }
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        (g(mid) < want ? lo : hi) = mid;
    }
    return 0.5 * (lo + hi);
}

// The budget B_{2,i} = floor(f(x)) of the user of rank x among X users of
// U' (at most 2^40): Eq. (4), or the uniform, linear and quadratic
// functions of Sec. 5.2, each with integral B2 over [0, X].
int64_t budget_items(int kind, double x, double X, double B2, double alpha, double beta,
                     double gamma) {
    double f;
    switch (kind) {
    case RMIPS_BUDGET_EXP: f = alpha * std::exp(beta * x) + gamma; break;
    case RMIPS_BUDGET_UNIFORM: f = B2 / X; break;
    case RMIPS_BUDGET_LINEAR: f = 2.0 * B2 * x / (X * X); break;
    default: f = 3.0 * B2 * x * x / (X * X * X); break;
    }
    if (!(f > 0.0)) return 0;
    if (f >= 1099511627776.0) return 1099511627776LL;
    return (int64_t)std::floor(f);
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
    if (hipHostMalloc((void **)&c->h_status, 512, hipHostMallocDefault) != hipSuccess) {
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

rmips_status rmips_set_dprime(rmips_ctx *ctx, int32_t dprime) {
    if (!ctx || dprime < 0 || dprime > DPRIME_ROT_MAX) return RMIPS_EINVAL;
    ctx->dprime = dprime;
    return RMIPS_OK;
}

rmips_status rmips_set_prepass(rmips_ctx *ctx, int32_t dprime) {
    if (!ctx || dprime < -1 || dprime > DPRIME_ROT_MAX) return RMIPS_EINVAL;
    ctx->prepass = dprime;
    return RMIPS_OK;
}

rmips_status rmips_set_bound_output(rmips_ctx *ctx, int32_t *uscore) {
    if (!ctx) return RMIPS_EINVAL;
    ctx->bound_out = uscore;
    return RMIPS_OK;
}

static bool prec_ok(rmips_prec p) {
    return p == RMIPS_FP32 || p == RMIPS_BF16 || p == RMIPS_FP8_E4M3 || p == RMIPS_FP6_E2M3 ||
           p == RMIPS_FP4_E2M1;
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
    s = run_thresholds(ctx, U, n, P, m, d, k, L, tau, tau_id, topk, nullptr);
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
    const ErrConst ec = err_const(L.T.D, d);

    constexpr int NEV = 10;
    hipEvent_t ev[NEV] = {};
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() { for (int i = 0; i < NEV; ++i) if (e[i]) (void)hipEventDestroy(e[i]); }
    } guard{ev};
    for (auto &e : ev) HIPTRY(hipEventCreate(&e));
    unsigned long long *ctr = reinterpret_cast<unsigned long long *>(L.C.rechecks);
    // status words (with stage (a)'s flags) and counters in one fill
    HIPTRY(hipMemsetAsync(L.C.status, 0, RES_TOP, st));
    HIPTRY(hipEventRecord(ev[0], st));

    // The Gram matrix of a user sample (for the rotation of Eq. (3)) does
    // not depend on tau: it goes to the host first, and the host computes
    // its eigenvectors while the GPU runs stage (a).  With d' = d any
    // orthonormal basis gives the same bound: the identity.  With a
    // pre-pass the rotated bound comes first and d' = d follows for the
    // items it leaves open.
    const int dmain = dprime(ctx, d), dpre = prepass_dim(ctx, d, dmain, prec);
    const int dp = dpre > 0 ? dpre : dmain, ka = aug_len(dp);
    const bool rotate = dp < d;
    std::vector<double> G, W;
    if (rotate) {
        const int64_t ns = std::min<int64_t>(n, GRAM_SAMPLE);
        launch_gram(U, ns, n / ns, d, L.B.G, L.B.Gs, st);
        G.resize((size_t)d * d);
        HIPTRY(hipMemcpyAsync(G.data(), L.B.G, sizeof(double) * d * d, hipMemcpyDeviceToHost,
                              st));
    }
    HIPTRY(hipEventRecord(ev[3], st));

    // ---- stage (a): exact thresholds (the input check is read at the
    // synchronisation before stage (b))
    s = run_thresholds(ctx, U, n, P, m, d, k, L.T, L.X.tau, L.X.tau_id, nullptr, nullptr,
                       ctr + CTR_PAIRS, ctr + CTR_RPAIRS, ev[4], ev[5], ctr + CTR_CS, false);
    if (s != RMIPS_OK) return s;
    HIPTRY(hipEventRecord(ev[1], st));
    if (rotate) {
        HIPTRY(hipEventSynchronize(ev[3]));
        top_eigvecs(G, d, dp, W);
    }

    // ---- stage (c): Cauchy-Schwarz prefix and Eq. (3)/(6) bound counts
    run_prefix(L.T, L.X, n, m, ec.c2, st);
    if (rotate)
        HIPTRY(hipMemcpyAsync(L.W, W.data(), sizeof(double) * dp * d, hipMemcpyHostToDevice, st));
    const double *Wd = rotate ? L.W : nullptr;  // nullptr: the identity
    launch_rotate_aug(P, L.T.perm, m, L.T.mpad, d, Wd, dp, ka, 1.0f, L.B.Pa, st);
    run_bound(U, L.X, L.B, Wd, dp, n, m, L.T.mpad, d, ctr + 2, ev[6], ev[7], L.uscore, st);
    launch_invert_perm(L.T.perm, m, L.C.inv, st);
    HIPTRY(hipGetLastError());

    // ---- stage (b): exact scores in bound order, running top-N, stop rule
    CountRun cr;
    cr.ev_vis = ev[2]; cr.ev_end = ev[3]; cr.ev_k0 = ev[8]; cr.ev_k1 = ev[9];
    const int32_t *h = nullptr;
    Refine rf{U, P, &L.T, &L.X, &L.B, n, m, d, L.uscore, ctr + 3};
    s = run_count_topn(ctx, U, P, L.T, L.X, L.C, L.uscore, n, m, d, N, ec, bfirst, bmax, cr,
                       top_ids, top_scores, &h, dpre > 0 ? &rf : nullptr);
    if (s != RMIPS_OK) return s;
    if (ctx->bound_out) {
        launch_gather_i32(L.uscore, L.C.inv, m, ctx->bound_out, st);
        HIPTRY(hipGetLastError());
        HIPTRY(hipStreamSynchronize(st));
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->visited_items = cr.visited;
        stats->batches = cr.batches;
        const int64_t *hc = reinterpret_cast<const int64_t *>(h);
        int64_t tp = 0, rp = 0, cs[4] = {0, 0, 0, 0};
        for (int i = 0; i < CSTAT_SLOTS; ++i) {
            tp += hc[CTR_PAIRS + i];
            rp += hc[CTR_RPAIRS + i];
            for (int j = 0; j < 4; ++j) cs[j] += hc[CTR_CS + 4 * i + j];
        }
        stats->cand_pairs = cs[1];
        stats->cand_listed = cs[0];
        stats->overflow_users = cs[2];
        stats->refine_users = cs[3];
        stats->recheck_pairs = hc[0];
        stats->thresh_pairs = tp;
        stats->refine_pairs = rp;
        stats->bound_pairs = hc[2];
        stats->count_pairs = cr.screened;
        stats->screened_pairs = cr.screened + tp + rp;
        stats->count_launches = cr.launches;
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
        stats->ms_count_kernels = cr.ms_count_k;
        stats->ms_bound_kernel = tbd;
        stats->rebound_items = cr.rebound;
        stats->rebound_pairs = hc[3];
        stats->prepass_dprime = dpre;
    }
    return RMIPS_OK;
}

// ---------------------------------------------------------------- k_max index
static bool index_sizes_ok(int64_t n, int64_t m, int32_t d, int32_t kmax, rmips_prec prec) {
    return n >= 1 && n <= (int64_t)INT32_MAX && m >= 1 && m <= (int64_t)INT32_MAX / 2 && d >= 1 &&
           d <= RMIPS_D_MAX && kmax >= 1 && kmax <= RMIPS_K_MAX && kmax <= m && prec_ok(prec);
}

size_t rmips_index_size(int64_t n, int64_t m, int32_t d, int32_t kmax, rmips_prec prec) {
    if (!index_sizes_ok(n, m, d, kmax, prec)) return 0;
    Carve cv(nullptr);
    IndexLayout I;
    index_plan(prec, n, m, d, kmax, I, cv);
    return cv.off + 256;
}

size_t rmips_index_workspace_size(int64_t n, int64_t m, int32_t d, int32_t kmax,
                                  rmips_prec prec) {
    if (!index_sizes_ok(n, m, d, kmax, prec)) return 0;
    Carve ci(nullptr);
    IndexLayout I;
    index_plan(prec, n, m, d, kmax, I, ci);
    Carve cb(nullptr);
    PrefixLayout X;
    BoundLayout B;
    index_build_plan(prec, n, m, d, kmax, 0, I, X, B, cb);
    Carve cq(nullptr);
    CountLayout C;
    index_query_plan(n, m, I, X, C, cq);
    return std::max(cb.off, cq.off) + 256;
}

// The index's header, read back (a synchronisation) before any launch that
// takes item or user indices from the index: an index built with other
// sizes has its arrays at other offsets, and those would not be indices.
constexpr int H_HDR = 64;  // pinned status words that receive it
static rmips_status check_index_header(rmips_ctx *ctx, const int32_t *hdr_dev, int64_t n,
                                       int64_t m, int32_t d, int32_t kmax, rmips_prec prec) {
    HIPTRY(hipMemcpyAsync(ctx->h_status + H_HDR, hdr_dev, sizeof(int32_t) * INDEX_HDR_WORDS,
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPTRY(hipStreamSynchronize(ctx->stream));
    int32_t want[INDEX_HDR_WORDS];
    const int32_t *got = ctx->h_status + H_HDR;
    index_header(n, m, d, kmax, prec, got[INDEX_HDR_DPRIME], want);
    if (std::memcmp(got, want, sizeof(want)) != 0)
        return fail(ctx, RMIPS_EINVAL,
                    "index not built by rmips_index_build with these n, m, d, kmax, precision");
    return RMIPS_OK;
}

static rmips_status index_args(rmips_ctx *ctx, int64_t n, int64_t m, int32_t d, int32_t kmax,
                               rmips_prec prec, void *index, size_t index_bytes) {
    if (!ctx) return RMIPS_EINVAL;
    if (!index_sizes_ok(n, m, d, kmax, prec))
        return fail(ctx, RMIPS_EINVAL, "sizes out of range (1 <= kmax <= min(m, 32))");
    if (!index) return fail(ctx, RMIPS_EINVAL, "null pointer");
    if (index_bytes < rmips_index_size(n, m, d, kmax, prec))
        return fail(ctx, RMIPS_EWORKSPACE, "index buffer too small");
    return RMIPS_OK;
}

rmips_status rmips_index_build(rmips_ctx *ctx, const float *U, int64_t n, const float *P,
                               int64_t m, int32_t d, int32_t kmax, rmips_prec prec,
                               void *index, size_t index_bytes, void *ws, size_t ws_bytes) {
    rmips_status s = index_args(ctx, n, m, d, kmax, prec, index, index_bytes);
    if (s != RMIPS_OK) return s;
    if (!U || !P || !ws) return fail(ctx, RMIPS_EINVAL, "null pointer");
    {
        Carve ci(nullptr);
        IndexLayout I0;
        index_plan(prec, n, m, d, kmax, I0, ci);
        Carve cb(nullptr);
        PrefixLayout X0;
        BoundLayout B0;
        index_build_plan(prec, n, m, d, kmax, ctx->cap_override, I0, X0, B0, cb);
        if (ws_bytes < cb.off + 256) return fail(ctx, RMIPS_EWORKSPACE, "workspace too small");
    }
    HIPTRY(hipSetDevice(ctx->device));
    ProfGuard pguard(ctx);
    hipStream_t st = ctx->stream;
    Carve ci(index), cw(ws);
    IndexLayout I;
    index_plan(prec, n, m, d, kmax, I, ci);
    PrefixLayout X;
    BoundLayout B;
    index_build_plan(prec, n, m, d, kmax, ctx->cap_override, I, X, B, cw);
    ThreshLayout &T = I.T;
    const ErrConst ec = err_const(T.D, d);
    const int dp = dprime(ctx, d), ka = aug_len(dp);
    const bool rotate = dp < d;
    // no valid header until the build has succeeded
    HIPTRY(hipMemsetAsync(I.hdr, 0, sizeof(int32_t) * INDEX_HDR_WORDS, st));
    hipEvent_t evg = nullptr;
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() { if (*e) (void)hipEventDestroy(*e); }
    } guard{&evg};
    HIPTRY(hipEventCreate(&evg));
    std::vector<double> G, W;
    if (rotate) {
        const int64_t ns = std::min<int64_t>(n, GRAM_SAMPLE);
        launch_gram(U, ns, n / ns, d, B.G, B.Gs, st);
        G.resize((size_t)d * d);
        HIPTRY(hipMemcpyAsync(G.data(), B.G, sizeof(double) * d * d, hipMemcpyDeviceToHost, st));
        HIPTRY(hipEventRecord(evg, st));
    }
    // stage (a) once with k = kmax: every user's kmax largest values and
    // their ids (exact, in the tie order) go to the index
    s = run_thresholds(ctx, U, n, P, m, d, kmax, T, X.tau, X.tau_id, I.topk, I.topv);
    if (s != RMIPS_OK) return s;
    if (rotate) {
        HIPTRY(hipEventSynchronize(evg));
        top_eigvecs(G, d, dp, W);
        HIPTRY(hipMemcpyAsync(I.W, W.data(), sizeof(double) * dp * d, hipMemcpyHostToDevice, st));
    }
    const double *Wd = rotate ? I.W : nullptr;
    launch_rotate_aug(P, T.perm, m, T.mpad, d, Wd, dp, ka, 1.0f, B.Pa, st);
    launch_invert_perm(T.perm, m, I.inv, st);
    // the bound of every item for each k: users in the rho order of that
    // k's thresholds, one bound pass per k (row k - 1 of the table)
    for (int k = 1; k <= kmax; ++k) {
        launch_kth_column(I.topv, I.topk, n, kmax, k, X.tau, X.tau_id, st);
        run_prefix(T, X, n, m, ec.c2, st, false);
        run_bound(U, X, B, Wd, dp, n, m, T.mpad, d, nullptr, nullptr, nullptr,
                  I.table + (size_t)(k - 1) * m, st);
    }
    HIPTRY(hipGetLastError());
    // the build waits for its work and reports its input check itself
    HIPTRY(hipMemcpyAsync(ctx->h_status, T.bad, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    ctx->prof.resolve();
    if (ctx->h_status[0] != 0) return fail(ctx, RMIPS_ENONFINITE, BAD_INPUT);
    int32_t *hdr = ctx->h_status + H_HDR;  // pinned
    int32_t want[INDEX_HDR_WORDS];
    index_header(n, m, d, kmax, prec, dp, want);
    std::memcpy(hdr, want, sizeof(want));
    HIPTRY(hipMemcpyAsync(I.hdr, hdr, sizeof(want), hipMemcpyHostToDevice, st));
    HIPTRY(hipStreamSynchronize(st));
    return RMIPS_OK;
}

rmips_status rmips_index_topn(rmips_ctx *ctx, const float *U, int64_t n, const float *P,
                              int64_t m, int32_t d, int32_t kmax, rmips_prec prec,
                              const void *index, size_t index_bytes, int32_t k, int32_t N,
                              void *ws, size_t ws_bytes, int32_t *top_ids, int32_t *top_scores,
                              rmips_stats *stats) {
    rmips_status s = index_args(ctx, n, m, d, kmax, prec, const_cast<void *>(index), index_bytes);
    if (s != RMIPS_OK) return s;
    if (k < 1 || k > kmax) return fail(ctx, RMIPS_EINVAL, "k out of range (1 <= k <= kmax)");
    if (N < 1 || N > RMIPS_N_MAX || N > m) return fail(ctx, RMIPS_EINVAL, "N out of range");
    if (!U || !P || !ws || !top_ids || !top_scores)
        return fail(ctx, RMIPS_EINVAL, "null pointer");
    if (ws_bytes < rmips_index_workspace_size(n, m, d, kmax, prec))
        return fail(ctx, RMIPS_EWORKSPACE, "workspace too small");
    const int bfirst = ctx->batch_first > 0 ? ctx->batch_first : BATCH_FIRST;
    const int bmax = ctx->batch_max > 0 ? ctx->batch_max : BATCH_MAX;
    HIPTRY(hipSetDevice(ctx->device));
    ProfGuard pguard(ctx);
    hipStream_t st = ctx->stream;
    Carve ci(const_cast<void *>(index)), cw(ws);
    IndexLayout I;
    index_plan(prec, n, m, d, kmax, I, ci);
    PrefixLayout X;
    CountLayout C;
    index_query_plan(n, m, I, X, C, cw);
    s = check_index_header(ctx, I.hdr, n, m, d, kmax, prec);
    if (s != RMIPS_OK) return s;
    const ErrConst ec = err_const(I.T.D, d);
    constexpr int NEV = 5;
    hipEvent_t ev[NEV] = {};
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() { for (int i = 0; i < NEV; ++i) if (e[i]) (void)hipEventDestroy(e[i]); }
    } guard{ev};
    for (auto &e : ev) HIPTRY(hipEventCreate(&e));
    HIPTRY(hipMemsetAsync(C.status, 0, RES_TOP, st));
    HIPTRY(hipEventRecord(ev[0], st));
    // the thresholds of this k from the lists, then the rho order
    launch_kth_column(I.topv, I.topk, n, kmax, k, X.tau, X.tau_id, st);
    run_prefix(I.T, X, n, m, ec.c2, st);
    CountRun cr;
    cr.ev_vis = ev[1]; cr.ev_end = ev[2]; cr.ev_k0 = ev[3]; cr.ev_k1 = ev[4];
    const int32_t *h = nullptr;
    s = run_count_topn(ctx, U, P, I.T, X, C, I.table + (size_t)(k - 1) * m, n, m, d, N, ec,
                       bfirst, bmax, cr, top_ids, top_scores, &h, nullptr);
    if (s != RMIPS_OK) return s;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        const int64_t *hc = reinterpret_cast<const int64_t *>(h);
        stats->visited_items = cr.visited;
        stats->batches = cr.batches;
        stats->recheck_pairs = hc[0];
        stats->count_pairs = cr.screened;
        stats->screened_pairs = cr.screened;
        stats->count_launches = cr.launches;
        float t01 = 0, t12 = 0, t02 = 0;
        (void)hipEventElapsedTime(&t01, ev[0], ev[1]);
        (void)hipEventElapsedTime(&t12, ev[1], ev[2]);
        (void)hipEventElapsedTime(&t02, ev[0], ev[2]);
        stats->ms_bound = t01;
        stats->ms_count = t12;
        stats->ms_total = t02;
        stats->ms_count_kernels = cr.ms_count_k;
    }
    return RMIPS_OK;
}

rmips_status rmips_index_thresholds(rmips_ctx *ctx, int64_t n, int64_t m, int32_t d,
                                    int32_t kmax, rmips_prec prec, const void *index,
                                    size_t index_bytes, int32_t k, double *tau,
                                    int32_t *tau_id) {
    rmips_status s = index_args(ctx, n, m, d, kmax, prec, const_cast<void *>(index), index_bytes);
    if (s != RMIPS_OK) return s;
    if (k < 1 || k > kmax) return fail(ctx, RMIPS_EINVAL, "k out of range (1 <= k <= kmax)");
    if (!tau || !tau_id) return fail(ctx, RMIPS_EINVAL, "null pointer");
    HIPTRY(hipSetDevice(ctx->device));
    ProfGuard pguard(ctx);
    Carve ci(const_cast<void *>(index));
    IndexLayout I;
    index_plan(prec, n, m, d, kmax, I, ci);
    s = check_index_header(ctx, I.hdr, n, m, d, kmax, prec);
    if (s != RMIPS_OK) return s;
    launch_kth_column(I.topv, I.topk, n, kmax, k, tau, tau_id, ctx->stream);
    HIPTRY(hipGetLastError());
    return RMIPS_OK;
}

rmips_status rmips_index_bounds(rmips_ctx *ctx, int64_t n, int64_t m, int32_t d, int32_t kmax,
                                rmips_prec prec, const void *index, size_t index_bytes,
                                int32_t k, int32_t *uscore) {
    rmips_status s = index_args(ctx, n, m, d, kmax, prec, const_cast<void *>(index), index_bytes);
    if (s != RMIPS_OK) return s;
    if (k < 1 || k > kmax) return fail(ctx, RMIPS_EINVAL, "k out of range (1 <= k <= kmax)");
    if (!uscore) return fail(ctx, RMIPS_EINVAL, "null pointer");
    HIPTRY(hipSetDevice(ctx->device));
    ProfGuard pguard(ctx);
    Carve ci(const_cast<void *>(index));
    IndexLayout I;
    index_plan(prec, n, m, d, kmax, I, ci);
    s = check_index_header(ctx, I.hdr, n, m, d, kmax, prec);
    if (s != RMIPS_OK) return s;
    launch_gather_i32(I.table + (size_t)(k - 1) * m, I.inv, m, uscore, ctx->stream);
    HIPTRY(hipGetLastError());
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
    launch_soft(U, n, tau, Q, nq, d, T, nullptr, S, nullptr, nullptr, ws, ctx->stream,
                soft_max_splits());
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
    launch_soft(U, n, tau, Q, nq, d, T, dS, nullptr, nullptr, dQ, ws, ctx->stream,
                soft_max_splits());
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
                    "nq * (d rounded up to 16) exceeds 65536, the size of the static scratch");
    if (!(T > 0.0f) || !std::isfinite(T)) return fail(ctx, RMIPS_EINVAL, "T must be > 0");
    if (!U || !tau || !Q || !dS || !dQ) return fail(ctx, RMIPS_EINVAL, "null pointer");
    HIPTRY(hipSetDevice(ctx->device));
    if (!ctx->soft_scratch) HIPTRY(soft_scratch_init(ctx->device, &ctx->soft_scratch));
    ProfGuard pguard(ctx);
    launch_soft(U, n, tau, Q, nq, d, T, dS, nullptr, nullptr, dQ, ctx->soft_scratch,
                ctx->stream, soft_noalloc_splits());
    HIPTRY(hipGetLastError());
    return RMIPS_OK;
}

rmips_status rmips_soft_fwd_grad(rmips_ctx *ctx, const float *U, int64_t n, const float *tau,
                                 const float *Q, int64_t nq, int32_t d, float T, void *ws,
                                 size_t ws_bytes, float *S, float *G) {
    rmips_status s = soft_common(ctx, U, n, tau, Q, nq, d, T, ws, ws_bytes);
    if (s != RMIPS_OK) return s;
    if (!S || !G) return fail(ctx, RMIPS_EINVAL, "null pointer");
    ProfGuard pguard(ctx);
    launch_soft(U, n, tau, Q, nq, d, T, nullptr, S, G, nullptr, ws, ctx->stream,
                soft_max_splits());
    HIPTRY(hipGetLastError());
    return RMIPS_OK;
}

rmips_status rmips_soft_scale(rmips_ctx *ctx, const float *G, int64_t nq, int32_t d,
                              const float *dS, float *dQ) {
    if (!ctx) return RMIPS_EINVAL;
    if (nq < 1 || nq > (int64_t)INT32_MAX / 2 || d < 1 || d > RMIPS_D_MAX)
        return fail(ctx, RMIPS_EINVAL, "size out of range");
    if (!G || !dS || !dQ) return fail(ctx, RMIPS_EINVAL, "null pointer");
    HIPTRY(hipSetDevice(ctx->device));
    ProfGuard pguard(ctx);
    launch_soft_scale(G, nq, d, dS, dQ, ctx->stream);
    HIPTRY(hipGetLastError());
    return RMIPS_OK;
}

size_t rmips_soft_workspace_size(int64_t n, int64_t nq, int32_t d) {
    if (n < 1 || nq < 1 || d < 1 || d > RMIPS_D_MAX) return 0;
    return soft_ws_bytes(n, nq, d);
}


// ------------------------------------------------------- budgeted index
static bool budget_sizes_ok(int64_t n, int64_t m, int32_t d, int32_t kmax) {
    return n >= 1 && n <= (int64_t)INT32_MAX / 2 && m >= 1 && m <= (int64_t)INT32_MAX / 2 &&
           d >= 1 && d <= RMIPS_D_MAX && kmax >= 1 && kmax <= RMIPS_K_MAX && kmax <= m;
}

size_t rmips_budget_index_size(int64_t n, int64_t m, int32_t d, int32_t kmax) {
    if (!budget_sizes_ok(n, m, d, kmax)) return 0;
    Carve c(nullptr);
    BudgetLayout B;
    budget_plan(n, m, d, kmax, B, c);
    return c.off + 256;
}

size_t rmips_budget_workspace_size(int64_t n, int64_t m, int32_t d, int32_t kmax,
                                   rmips_prec prec) {
    if (!budget_sizes_ok(n, m, d, kmax) || !prec_ok(prec)) return 0;
    Carve c(nullptr);
    BudgetScratch S;
    budget_scratch_plan(prec, n, m, d, kmax, 0, S, c);
    return c.off + 256;
}

static rmips_status budget_args(rmips_ctx *ctx, int64_t n, int64_t m, int32_t d, int32_t kmax,
                                rmips_prec prec, const void *index, size_t index_bytes,
                                const void *ws, size_t ws_bytes) {
    if (!ctx) return RMIPS_EINVAL;
    if (!budget_sizes_ok(n, m, d, kmax))
        return fail(ctx, RMIPS_EINVAL, "sizes out of range (1 <= kmax <= min(m, 32))");
    if (!prec_ok(prec)) return fail(ctx, RMIPS_EUNSUPPORTED, "unknown screening precision");
    if (!index || !ws) return fail(ctx, RMIPS_EINVAL, "null pointer");
    if (index_bytes < rmips_budget_index_size(n, m, d, kmax))
        return fail(ctx, RMIPS_EWORKSPACE, "index buffer too small");
    {
        Carve c(nullptr);
        BudgetScratch S;
        budget_scratch_plan(prec, n, m, d, kmax, ctx->cap_override, S, c);
        if (ws_bytes < c.off + 256) return fail(ctx, RMIPS_EWORKSPACE, "workspace too small");
    }
    return RMIPS_OK;
}

static rmips_status check_budget_header(rmips_ctx *ctx, const int32_t *hdr_dev, int64_t n,
                                        int64_t m, int32_t d, int32_t kmax) {
    HIPTRY(hipMemcpyAsync(ctx->h_status + H_BHDR, hdr_dev, sizeof(int32_t) * BUDGET_HDR_WORDS,
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPTRY(hipStreamSynchronize(ctx->stream));
    int32_t want[BUDGET_HDR_WORDS];
    budget_header(n, m, d, kmax, want);
    if (std::memcmp(ctx->h_status + H_BHDR, want, sizeof(want)) != 0)
        return fail(ctx, RMIPS_EINVAL,
                    "index not built by rmips_budget_build with these n, m, d, kmax");
    return RMIPS_OK;
}

rmips_status rmips_budget_build(rmips_ctx *ctx, const float *U, int64_t n, const float *P,
                                int64_t m, int32_t d, int32_t kmax, rmips_prec prec,
                                const rmips_budget *budget, void *index, size_t index_bytes,
                                void *ws, size_t ws_bytes, rmips_budget_info *info) {
    rmips_status s = budget_args(ctx, n, m, d, kmax, prec, index, index_bytes, ws, ws_bytes);
    if (s != RMIPS_OK) return s;
    if (!U || !P || !budget) return fail(ctx, RMIPS_EINVAL, "null pointer");
    const rmips_budget bud = *budget;
    if (bud.b1 < kmax) return fail(ctx, RMIPS_EINVAL, "b1 below kmax");
    if (bud.B2 < 0 || bud.B2 > ((int64_t)1 << 62)) return fail(ctx, RMIPS_EINVAL, "B2 out of range");
    if (bud.kind < RMIPS_BUDGET_EXP || bud.kind > RMIPS_BUDGET_QUADRATIC)
        return fail(ctx, RMIPS_EINVAL, "unknown budget function");
    if (!(bud.alpha >= 0.0) || !(bud.gamma >= 0.0) || !std::isfinite(bud.alpha) ||
        !std::isfinite(bud.gamma))
        return fail(ctx, RMIPS_EINVAL, "alpha and gamma must be finite and >= 0");
    const int64_t b1 = std::min<int64_t>(bud.b1, m);
    HIPTRY(hipSetDevice(ctx->device));
    ProfGuard pguard(ctx);
    hipStream_t st = ctx->stream;
    Carve ci(index), cw(ws);
    BudgetLayout B;
    budget_plan(n, m, d, kmax, B, ci);
    BudgetScratch S;
    budget_scratch_plan(prec, n, m, d, kmax, ctx->cap_override, S, cw);
    const int dp = budget_dp(d);
    hipEvent_t ev[2] = {};
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() { for (int i = 0; i < 2; ++i) if (e[i]) (void)hipEventDestroy(e[i]); }
    } guard{ev};
    for (auto &e : ev) HIPTRY(hipEventCreate(&e));
    HIPTRY(hipEventRecord(ev[0], st));
    // no valid header until the build has succeeded
    HIPTRY(hipMemsetAsync(B.hdr, 0, sizeof(int32_t) * BUDGET_HDR_WORDS, st));

    // (1) norms and the norm order
    launch_sqnorm64(U, n, d, B.nu2, st);
    launch_sqnorm64(P, m, d, S.np2, st);
    std::vector<double> nu2h(n), np2(m);
    HIPTRY(hipMemcpyAsync(nu2h.data(), B.nu2, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    HIPTRY(hipMemcpyAsync(np2.data(), S.np2, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    const double big = std::ldexp(1.0, 120);  // norms up to 2^60
    for (double x : nu2h)
        if (!(x <= big)) return fail(ctx, RMIPS_ENONFINITE, BAD_INPUT);
    for (double x : np2)
        if (!(x <= big)) return fail(ctx, RMIPS_ENONFINITE, BAD_INPUT);
    std::vector<int32_t> order(m), posof(m);
    for (int64_t j = 0; j < m; ++j) order[j] = (int32_t)j;
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return np2[a] > np2[b] || (np2[a] == np2[b] && a < b);
    });
    std::vector<double> np2s(m);
    for (int64_t j = 0; j < m; ++j) {
        posof[order[j]] = (int32_t)j;
        np2s[j] = np2[order[j]];
    }
    HIPTRY(hipMemcpyAsync(B.order, order.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
    HIPTRY(hipMemcpyAsync(B.posof, posof.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
    HIPTRY(hipMemcpyAsync(B.np2s, np2s.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));

    // (2) the rotation of Eq. (3): the dominant eigenvectors of a sampled
    // Gram matrix of U (any orthonormal rows keep the bound)
    {
        const int64_t ns = std::min<int64_t>(n, GRAM_SAMPLE);
        launch_gram(U, ns, n / ns, d, S.G, S.Gs, st);
        std::vector<double> G((size_t)d * d), W;
        HIPTRY(hipMemcpyAsync(G.data(), S.G, sizeof(double) * d * d, hipMemcpyDeviceToHost, st));
        HIPTRY(hipStreamSynchronize(st));
        top_eigvecs(G, d, dp, W);
        HIPTRY(hipMemcpyAsync(B.W, W.data(), sizeof(double) * dp * d, hipMemcpyHostToDevice, st));
        HIPTRY(hipStreamSynchronize(st));  // W is a local vector
    }
    launch_budget_rotate(U, nullptr, B.nu2, n, d, B.W, dp, B.Ul, B.nru, B.nun, st);
    launch_budget_rotate(P, B.order, S.np2, m, d, B.W, dp, B.Pl, B.nrp, B.npn, st);
    launch_budget_transpose(P, B.order, m, d, S.PgT, st);

    // (3) uniform budget: positions 1..b1 for every user, then U' with its
    // keys j' + 1 - b1
    launch_budget_prefix(U, S.PgT, m, B.order, d, nullptr, nullptr, b1, n, kmax, B.Av, B.Aj, st);
    launch_budget_classify(B.Av, B.nu2, B.np2s, n, m, kmax, b1, B.key, st);
    std::vector<int32_t> key(n);
    HIPTRY(hipMemcpyAsync(key.data(), B.key, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    // U' in ascending (key, user) order: a counting sort over the keys
    std::vector<int64_t> start((size_t)(m + 3), 0);
    int64_t X = 0;
    for (int64_t u = 0; u < n; ++u)
        if (key[u] > 0) {
            ++start[key[u] + 1];
            ++X;
        }
    for (size_t i = 1; i < start.size(); ++i) start[i] += start[i - 1];
    std::vector<int32_t> ux(X);
    for (int64_t u = 0; u < n; ++u)
        if (key[u] > 0) ux[start[key[u]]++] = (int32_t)u;
    const double beta = (bud.kind == RMIPS_BUDGET_EXP && X > 0)
                            ? budget_solve_beta((double)X, (double)bud.B2, bud.alpha, bud.gamma)
                            : 0.0;

    // (4) dynamic budget.  A scan of user i stops at its natural stop t_i:
    // the first position whose Eq. (2) bound is below its exact k_max-th
    // value (stage (a) once over U'), so the budget recurrence with the
    // pooled budget B' needs only t_i.
    std::vector<int32_t> t(X), pos(n, 0), rank(n, 0), u2, lims;
    std::vector<int64_t> b2(n, 0);
    int64_t cert4 = 0, scanned4 = 0;
    if (X > 0) {
        HIPTRY(hipMemcpyAsync(S.ux, ux.data(), sizeof(int32_t) * X, hipMemcpyHostToDevice, st));
        launch_budget_gather(U, S.ux, X, d, S.Ug, st);
        s = run_thresholds(ctx, S.Ug, X, P, m, d, kmax, S.T, S.tau, S.tau_id, S.topk, S.topv);
        if (s != RMIPS_OK) return s;
        launch_budget_tstop(S.ux, S.topv, B.nu2, B.np2s, X, m, kmax, b1, S.t, st);
        HIPTRY(hipMemcpyAsync(t.data(), S.t, sizeof(int32_t) * X, hipMemcpyDeviceToHost, st));
        HIPTRY(hipMemcpyAsync(ctx->h_status, S.T.bad, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPTRY(hipStreamSynchronize(st));
        if (ctx->h_status[0] != 0) return fail(ctx, RMIPS_ENONFINITE, BAD_INPUT);
        int64_t pool = 0;
        for (int64_t r = 0; r < X; ++r) {
            const int32_t u = ux[r];
            rank[u] = (int32_t)(r + 1);
            b2[u] = budget_items(bud.kind, (double)(r + 1), (double)X, (double)bud.B2,
                                 bud.alpha, beta, bud.gamma);
            const int64_t e = b1 + 1 + b2[u] + pool;
            if (t[r] <= e) {  // the scan stops within the budget: its list is exact
                pool = e - t[r];
                ++cert4;
                scanned4 += t[r] - (b1 + 1);
            } else {          // budget spent: pos_i = e (<= m), U''
                pos[u] = (int32_t)e;
                u2.push_back(u);
                lims.push_back((int32_t)e);
                pool = 0;
                scanned4 += e - b1;
            }
        }
    }
    const int64_t nU2 = (int64_t)u2.size();
    HIPTRY(hipMemcpyAsync(B.pos, pos.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    HIPTRY(hipMemcpyAsync(B.rank, rank.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    HIPTRY(hipMemcpyAsync(B.b2, b2.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, st));
    launch_budget_scatter(S.ux, B.pos, S.topv, S.topk, X, kmax, B.Av, B.Aj, st);
    if (nU2 > 0) {
        HIPTRY(hipMemcpyAsync(S.u2, u2.data(), sizeof(int32_t) * nU2, hipMemcpyHostToDevice, st));
        HIPTRY(hipMemcpyAsync(S.lims, lims.data(), sizeof(int32_t) * nU2, hipMemcpyHostToDevice,
                              st));
        launch_budget_prefix(U, S.PgT, m, B.order, d, S.u2, S.lims, 0, nU2, kmax, B.Av, B.Aj,
                             st);
    }

    // (5) lambda_i and uscore_k: Eq. (6) over the unscanned positions of U'',
    // then the first k entries of every list
    launch_fill_f64(B.lam, n, -INFINITY, st);
    HIPTRY(hipMemsetAsync(B.uscore, 0, sizeof(int32_t) * kmax * m, st));
    // users of U'' sorted by the end of their step (5) range
    uint32_t *rkey = reinterpret_cast<uint32_t *>(S.t);
    launch_budget_range(S.u2, B.pos, nU2, B.Av, B.nu2, B.np2s, m, kmax, rkey, S.lims, st);
    if (nU2 > 0)
        HIPTRY(radix_sort_u32(rkey, S.lims, nU2, S.T.usort, st, 0,
                              32 - __builtin_clz((unsigned)(m + 1))));
    launch_budget_step5(S.lims, rkey, B.pos, nU2, B.Av, B.Ul, B.nru, B.nun, B.Pl, B.nrp, B.npn,
                        B.order, m, kmax, dp, B.lam, B.uscore, st);
    launch_budget_hist(B.Aj, n, kmax, m, B.uscore, st);
    launch_budget_prefix_k(B.uscore, m, kmax, st);
    const int64_t cert3 = n - X;
    double inf[8] = {(double)X, (double)nU2, beta, (double)cert3, (double)cert4,
                     (double)scanned4, (double)b1, (double)bud.B2};
    HIPTRY(hipMemcpyAsync(B.info, inf, sizeof(inf), hipMemcpyHostToDevice, st));
    HIPTRY(hipEventRecord(ev[1], st));
    HIPTRY(hipGetLastError());
    HIPTRY(hipStreamSynchronize(st));
    ctx->prof.resolve();
    int32_t *hdr = ctx->h_status + H_BHDR;  // pinned
    int32_t want[BUDGET_HDR_WORDS];
    budget_header(n, m, d, kmax, want);
    std::memcpy(hdr, want, sizeof(want));
    HIPTRY(hipMemcpyAsync(B.hdr, hdr, sizeof(want), hipMemcpyHostToDevice, st));
    HIPTRY(hipStreamSynchronize(st));
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->u_prime = X;
        info->u_dprime = nU2;
        info->cert3 = cert3;
        info->cert4 = cert4;
        info->scanned4 = scanned4;
        info->beta = beta;
        float ms = 0;
        (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
        info->ms_total = ms;
    }
    return RMIPS_OK;
}

rmips_status rmips_budget_topn(rmips_ctx *ctx, const float *U, int64_t n, const float *P,
                               int64_t m, int32_t d, int32_t kmax, rmips_prec prec,
                               const void *index, size_t index_bytes, int32_t k, int32_t N,
                               void *ws, size_t ws_bytes, int32_t *top_ids, int32_t *top_scores,
                               rmips_budget_qstats *stats) {
    rmips_status s = budget_args(ctx, n, m, d, kmax, prec, index, index_bytes, ws, ws_bytes);
    if (s != RMIPS_OK) return s;
    if (k < 1 || k > kmax) return fail(ctx, RMIPS_EINVAL, "k out of range (1 <= k <= kmax)");
    if (N < 1 || N > RMIPS_N_MAX || N > m) return fail(ctx, RMIPS_EINVAL, "N out of range");
    if (!U || !P || !top_ids || !top_scores) return fail(ctx, RMIPS_EINVAL, "null pointer");
    HIPTRY(hipSetDevice(ctx->device));
    ProfGuard pguard(ctx);
    hipStream_t st = ctx->stream;
    Carve ci(const_cast<void *>(index)), cw(ws);
    BudgetLayout B;
    budget_plan(n, m, d, kmax, B, ci);
    BudgetScratch S;
    budget_scratch_plan(prec, n, m, d, kmax, ctx->cap_override, S, cw);
    s = check_budget_header(ctx, B.hdr, n, m, d, kmax);
    if (s != RMIPS_OK) return s;
    const int dp = budget_dp(d);
    hipEvent_t ev[3] = {};
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() { for (int i = 0; i < 3; ++i) if (e[i]) (void)hipEventDestroy(e[i]); }
    } guard{ev};
    for (auto &e : ev) HIPTRY(hipEventCreate(&e));
    HIPTRY(hipEventRecord(ev[0], st));
    // (1) initialisation: certified users into the scores, the others into X
    HIPTRY(hipMemsetAsync(S.base, 0, sizeof(int32_t) * m, st));
    HIPTRY(hipMemsetAsync(S.visited, 0, m, st));
    HIPTRY(hipMemsetAsync(S.xflag, 0, n, st));
    HIPTRY(hipMemsetAsync(S.cnt, 0, sizeof(int32_t) * BUDGET_BATCH_BIG, st));
    HIPTRY(hipMemsetAsync(S.ctr, 0, sizeof(int32_t) * 64, st));
    launch_fill_i32(S.slot, m, -1, st);
    launch_budget_xinit(B.Av, B.Aj, B.lam, n, kmax, k, S.base, S.X, S.ctr, st);
    // (2) the visit order: (uscore_k desc, id asc)
    launch_budget_visit_keys(B.uscore + (size_t)(k - 1) * m, m, S.vkey, S.vval, st);
    HIPTRY(radix_sort_u32(S.vkey, S.vval, m, S.vsort, st));
    std::vector<uint32_t> vkey(m);
    std::vector<int32_t> vval(m);
    HIPTRY(hipMemcpyAsync(vkey.data(), S.vkey, sizeof(uint32_t) * m, hipMemcpyDeviceToHost, st));
    HIPTRY(hipMemcpyAsync(vval.data(), S.vval, sizeof(int32_t) * m, hipMemcpyDeviceToHost, st));
    int32_t *hc = ctx->h_status + H_BCTR;  // pinned
    HIPTRY(hipMemcpyAsync(hc, S.ctr, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPTRY(hipEventRecord(ev[1], st));
    HIPTRY(hipStreamSynchronize(st));
    int64_t xn = hc[0];
    const int64_t x0 = xn;
    auto uscore_at = [&](int64_t i) { return (int64_t)(~vkey[i]); };
    std::vector<std::pair<int32_t, int32_t>> best;  // (score, id), (score desc, id asc)
    std::vector<int32_t> scores;                    // of the processed items, in visit order
    std::vector<int32_t> hs(BUDGET_BATCH_BIG);
    int64_t off = 0, rescanned = 0, rescan_calls = 0, batches = 0;
    int nb_next = 64;
    int32_t *Xc = S.X, *Xn = S.X2;
    while (off < m) {
        if ((int64_t)best.size() == N && uscore_at(off) < best.back().first) break;
        // batches stay small while X holds users (each is tested against
        // all of X); once X is empty a batch is only a lookup
        if (xn == 0) nb_next = std::max(nb_next, BUDGET_BATCH_BIG);
        const int nb = (int)std::min<int64_t>(nb_next, m - off);
        const int32_t *bids = S.vval + off;
        launch_budget_slots(bids, nb, S.slot, st);
        if (xn > 0) {
            HIPTRY(hipMemsetAsync(S.ctr + 1, 0, 2 * sizeof(int32_t), st));
            launch_budget_inc(Xc, xn, bids, nb, S.slot, B.Av, B.Aj, B.lam, B.pos,
                              B.nu2, B.Ul, B.nru, B.nun, B.posof, B.np2s, B.Pl, B.nrp, B.npn,
                              kmax, k, dp, S.cnt, S.R, S.ctr + 1, S.xflag, st);
            HIPTRY(hipMemcpyAsync(hc + 1, S.ctr + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            HIPTRY(hipStreamSynchronize(st));
            const int64_t rn = hc[1];
            if (rn > 0) {
                // rescans: the exact S_k of those users (stage (a)); their
                // items not yet visited are credited now, and they leave X
                launch_budget_gather(U, S.R, rn, d, S.Ug, st);
                s = run_thresholds(ctx, S.Ug, rn, P, m, d, k, S.T, S.tau, S.tau_id, S.topk,
                                   nullptr);
                if (s != RMIPS_OK) return s;
                launch_budget_apply(S.topk, rn, k, S.visited, S.base, st);
                launch_budget_xcompact(Xc, xn, S.xflag, Xn, S.ctr + 2, st);
                HIPTRY(hipMemcpyAsync(hc + 2, S.ctr + 2, sizeof(int32_t), hipMemcpyDeviceToHost,
                                      st));
                HIPTRY(hipStreamSynchronize(st));
                xn = hc[2];
                std::swap(Xc, Xn);
                rescanned += rn;
                ++rescan_calls;
            }
        }
        launch_budget_batch(bids, nb, S.base, S.cnt, S.visited, S.slot, S.score, st);
        HIPTRY(hipMemcpyAsync(hs.data(), S.score, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, st));
        HIPTRY(hipStreamSynchronize(st));
        for (int i = 0; i < nb; ++i) {
            scores.push_back(hs[i]);
            best.emplace_back(hs[i], vval[off + i]);
        }
        std::sort(best.begin(), best.end(), [](const std::pair<int32_t, int32_t> &a,
                                               const std::pair<int32_t, int32_t> &b) {
            return a.first > b.first || (a.first == b.first && a.second < b.second);
        });
        if ((int64_t)best.size() > N) best.resize(N);
        off += nb;
        ++batches;
        nb_next = std::min(2 * nb_next, xn > 0 ? BUDGET_BATCH_MAX : BUDGET_BATCH_BIG);
    }
    HIPTRY(hipEventRecord(ev[2], st));
    HIPTRY(hipGetLastError());
    HIPTRY(hipStreamSynchronize(st));
    ctx->prof.resolve();
    for (int i = 0; i < N; ++i) {
        top_scores[i] = best[i].first;
        top_ids[i] = best[i].second;
    }
    if (stats) {
        // the items Alg. 2 visits one at a time: up to its stop, replayed on
        // the exact scores of the processed batches
        int64_t visited = 0;
        std::vector<int32_t> run;  // the N largest scores so far (desc)
        for (int64_t i = 0; i < (int64_t)scores.size(); ++i) {
            if ((int64_t)run.size() == N && uscore_at(i) < run.back()) break;
            ++visited;
            run.insert(std::upper_bound(run.begin(), run.end(), scores[i], std::greater<int32_t>()),
                       scores[i]);
            if ((int64_t)run.size() > N) run.pop_back();
        }
        std::memset(stats, 0, sizeof(*stats));
        stats->x0 = x0;
        stats->rescanned_users = rescanned;
        stats->rescan_calls = rescan_calls;
        stats->visited_items = visited;
        stats->processed_items = off;
        stats->batches = batches;
        float t01 = 0, t02 = 0;
        (void)hipEventElapsedTime(&t01, ev[0], ev[1]);
        (void)hipEventElapsedTime(&t02, ev[0], ev[2]);
        stats->ms_init = t01;
        stats->ms_total = t02;
    }
    return RMIPS_OK;
}

rmips_status rmips_budget_state(rmips_ctx *ctx, int64_t n, int64_t m, int32_t d, int32_t kmax,
                                const void *index, size_t index_bytes, int32_t *order,
                                int32_t *pos, double *lam, double *Av, int32_t *Aj, int32_t *key,
                                int32_t *rank, int64_t *b2, int32_t *uscore) {
    if (!ctx) return RMIPS_EINVAL;
    if (!budget_sizes_ok(n, m, d, kmax))
        return fail(ctx, RMIPS_EINVAL, "sizes out of range (1 <= kmax <= min(m, 32))");
    if (!index) return fail(ctx, RMIPS_EINVAL, "null pointer");
    if (index_bytes < rmips_budget_index_size(n, m, d, kmax))
        return fail(ctx, RMIPS_EWORKSPACE, "index buffer too small");
    HIPTRY(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    Carve ci(const_cast<void *>(index));
    BudgetLayout B;
    budget_plan(n, m, d, kmax, B, ci);
    rmips_status s = check_budget_header(ctx, B.hdr, n, m, d, kmax);
    if (s != RMIPS_OK) return s;
    auto cp = [&](void *dst, const void *src, size_t bytes) -> rmips_status {
        if (dst) HIPTRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
        return RMIPS_OK;
    };
    if ((s = cp(order, B.order, sizeof(int32_t) * m)) != RMIPS_OK) return s;
    if ((s = cp(pos, B.pos, sizeof(int32_t) * n)) != RMIPS_OK) return s;
    if ((s = cp(lam, B.lam, sizeof(double) * n)) != RMIPS_OK) return s;
    if ((s = cp(Av, B.Av, sizeof(double) * n * kmax)) != RMIPS_OK) return s;
    if ((s = cp(Aj, B.Aj, sizeof(int32_t) * n * kmax)) != RMIPS_OK) return s;
    if ((s = cp(key, B.key, sizeof(int32_t) * n)) != RMIPS_OK) return s;
    if ((s = cp(rank, B.rank, sizeof(int32_t) * n)) != RMIPS_OK) return s;
    if ((s = cp(b2, B.b2, sizeof(int64_t) * n)) != RMIPS_OK) return s;
    if ((s = cp(uscore, B.uscore, sizeof(int32_t) * kmax * m)) != RMIPS_OK) return s;
    return RMIPS_OK;
}

}  // extern "C"

/*
 * librmips -- exact reverse k-MIPS top-N on AMD Instinct MI355X (gfx950).
 *
 * Problem (Amagata et al., "How to Mine Potentially Popular Items? A
 * Reverse MIPS-based Approach"): users U (n x d), items P (m x d).
 *   Def. 1  S_k(u): the k items with the largest inner product u . p.
 *   Def. 2  T_k(p) = {u : p in S_k(u)}   (Eq. 1), score(p) = |T_k(p)|.
 *   Def. 3  the N items with the largest score.
 *
 * Exactness.  The value of u . p is defined as the FP64 sum of the exact
 * products (double)u_i * (double)p_i taken in index order from +0.0.  Every
 * integer output (item ids, scores, counts) is decided on that value, and
 * tau is that value, bit for bit.  Ties are ordered (value desc, item id
 * asc) in k-MIPS and (score desc, item id asc) in top-N, where the paper
 * breaks them arbitrarily.  With that order, item j is in S_k(u) iff
 *     v > tau_u,  or  v == tau_u and j <= tau_id_u.
 * Low-precision screening (FP32, BF16, FP8 e4m3 matrix-core products) only
 * decides pairs that a certified per-pair error bound separates from the
 * threshold; all other pairs are recomputed in FP64 on the GPU.
 *
 * Conventions for every call.
 *   - Matrix arguments are device pointers to caller-owned, contiguous,
 *     row-major FP32 arrays with leading dimension d.  Row i of P has item
 *     id i.  Vectors (tau, tau_id, scores, ...) are device pointers too,
 *     except where a comment says "host".
 *   - The library allocates no device memory.  Scratch space is the
 *     caller's workspace `ws` of `ws_bytes` bytes (device memory, 256-byte
 *     aligned), sized by the matching *_workspace_size query.  Its contents
 *     are undefined after a call.
 *   - Work is enqueued on the context's HIP stream.  rmips_thresholds,
 *     rmips_scores, rmips_soft_fwd and rmips_soft_bwd never wait: they
 *     return once their work is enqueued.  The input check of
 *     rmips_thresholds and rmips_scores (NaN, Inf, a norm above 2^60) runs
 *     on the device and is reported by the next rmips_sync on the context.
 *     rmips_topn synchronises the stream (its bound-ordered loop reads a few
 *     bytes back per batch), checks its own inputs and writes host arrays.
 *   - Arguments are validated before anything is launched.  On error the
 *     outputs are unspecified and rmips_last_error() describes the error.
 *   - A context is not thread-safe; use one context per stream.
 */
#ifndef RMIPS_H
#define RMIPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RMIPS_K_MAX 32      /* largest k accepted (the paper uses k <= 25) */
#define RMIPS_N_MAX 1024    /* largest N accepted by rmips_topn */
#define RMIPS_D_MAX 256     /* largest dimensionality d */

typedef enum {
    RMIPS_OK = 0,
    RMIPS_EINVAL = 1,       /* bad size, pointer or parameter */
    RMIPS_EWORKSPACE = 2,   /* ws_bytes below the *_workspace_size value */
    RMIPS_ENONFINITE = 3,   /* NaN or Inf in an input vector, or a norm above 2^60 */
    RMIPS_EUNSUPPORTED = 4, /* precision or device not supported */
    RMIPS_EDEVICE = 5       /* HIP runtime error */
} rmips_status;

/* Screening precision of the dense products of stages (a) and (b). */
typedef enum {
    RMIPS_FP32 = 0,         /* FP32 inputs, FP32 matrix-core accumulation */
    RMIPS_BF16 = 1,         /* BF16-rounded inputs, FP32 accumulation */
    RMIPS_FP8_E4M3 = 2,     /* OCP e4m3 inputs with a per-vector power-of-two
                               scale, FP32 accumulation */
    RMIPS_FP6_E2M3 = 3,     /* OCP MX FP6 e2m3 element codes (largest 7.5) with a
                               per-vector power-of-two scale, on gfx950's
                               block-scaled f8f6f4 matrix-core instruction */
    RMIPS_FP4_E2M1 = 4      /* OCP MX FP4 e2m1 element codes (largest 6.0), likewise */
} rmips_prec;

typedef struct rmips_ctx rmips_ctx;

/* Counters and per-stage times of the last rmips_topn call. */
typedef struct {
    int64_t visited_items;    /* items whose exact score was computed */
    int64_t batches;          /* bound-ordered batches run */
    int64_t cand_pairs;       /* stage (a): candidates recomputed in FP64 */
    int64_t cand_listed;      /* stage (a): candidates listed by the screen */
    int64_t overflow_users;   /* stage (a): users sent to the exact fallback */
    int64_t refine_users;     /* stage (a): users screened again with a tighter
                                 bound after their candidate lists overflowed */
    int64_t recheck_pairs;    /* stage (b): ambiguous pairs rechecked in FP64 */
    int64_t screened_pairs;   /* stage (a)+(b): pairs through the matrix cores */
    int64_t bound_pairs;      /* stage (c): pairs evaluated by the Eq. 3 bound */
    int64_t thresh_pairs;     /* stage (a): pairs screened by the main pass after
                                 the early exit */
    int64_t count_pairs;      /* stage (b): (item, user) pairs screened */
    int64_t count_launches;   /* stage (b): counting kernel launches */
    int64_t refine_pairs;     /* stage (a): pairs screened by refinement passes */
    float ms_thresh;          /* stage (a), all kernels */
    float ms_bound;           /* stage (c), all kernels and the host rotation */
    float ms_count;           /* stage (b) loop, including host round trips */
    float ms_total;           /* whole call */
    float ms_screen;          /* stage (a) screening kernel alone */
    float ms_count_kernels;   /* stage (b) counting kernels alone, summed */
    float ms_bound_kernel;    /* stage (c) bound-count kernel alone */
    int64_t rebound_items;    /* items given the d' = d bound after a pre-pass */
    int64_t rebound_pairs;    /* pairs of that second bound */
    int32_t prepass_dprime;   /* d' of the pre-pass bound (0: no pre-pass) */
} rmips_stats;

/*
 * Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the context.
 */
rmips_status rmips_create(rmips_ctx **out, int device, void *hip_stream);

/* Destroy a context (NULL is ignored).  Waits for nothing. */
void rmips_destroy(rmips_ctx *ctx);

/* Text of the last error on this context ("" if none).  Owned by ctx. */
const char *rmips_last_error(const rmips_ctx *ctx);

/* Change the stream a context enqueues on. */
rmips_status rmips_set_stream(rmips_ctx *ctx, void *hip_stream);

/*
 * Wait for the context's stream and report the input checks of the
 * rmips_thresholds and rmips_scores calls made since the last rmips_sync:
 * RMIPS_ENONFINITE when any of them saw a NaN or an Inf, or a row norm
 * above 2^60 (the outputs of that call are then unspecified), else
 * RMIPS_OK.  The checks are cleared either way.  (With 63 checks pending,
 * the next such call waits for them itself and returns their result.)
 */
rmips_status rmips_sync(rmips_ctx *ctx);

/*
 * Per-kernel timing.  With on != 0 (which also clears the totals), every
 * kernel launch of the context's calls is bracketed by two HIP events on
 * the context's stream, and their durations are summed per kernel name;
 * on = 0 stops recording and keeps the totals.  Waits for the stream.
 */
rmips_status rmips_set_profiling(rmips_ctx *ctx, int32_t on);

/*
 * Entry i (0, 1, ... in the order the kernels first ran) of the totals:
 * the kernel's name (NUL-terminated, at most name_cap bytes, into the
 * host buffer `name`), its launch count and summed duration in ms (host
 * outputs).  Waits for the stream.  RMIPS_EINVAL past the last entry.
 */
rmips_status rmips_profile_entry(rmips_ctx *ctx, int32_t i, char *name, int32_t name_cap,
                                 int64_t *launches, double *ms_total);

/*
 * Testing knob: capacity of the per-user candidate list of stage (a).
 * 0 restores the default.  A tiny capacity forces the exact per-user
 * fallback path; results do not change.
 */
rmips_status rmips_set_candidate_cap(rmips_ctx *ctx, int32_t cap);

/*
 * Testing knob: first and largest batch size of the bound-ordered loop of
 * rmips_topn (items per batch; 0 = defaults).  Results do not change.
 */
rmips_status rmips_set_batch(rmips_ctx *ctx, int32_t first, int32_t max);

/*
 * Split dimension d' of the Eq. (3) bound (Sec. 4.2; the paper's
 * experiments use d' = 10, Sec. 5.1) for rmips_topn and rmips_index_build.
 * 0 (the default): d' = d, the bound is the inner product itself with its
 * certified slack (no rotation).  1 <= dprime <= 62: both sides are rotated
 * onto the top-d' eigenvectors of a user sample's Gram matrix and the
 * residual norms carry the rest, as in the paper (dprime >= d means d).
 * Results do not change; the bound's tightness (how many items stage (b)
 * counts) and its cost do.  RMIPS_EINVAL outside [0, 62].
 */
rmips_status rmips_set_dprime(rmips_ctx *ctx, int32_t dprime);

/*
 * Pre-pass of rmips_topn's Eq. (3) bound when d' = d (Sec. 4.2): every item
 * is first bounded after a rotation onto the top-`dprime` eigenvectors of a
 * user sample, as rmips_set_dprime describes, and once the first batch has
 * given an N-th score, the items whose pre-pass bound still reaches it (the
 * only ones that can still enter the top-N) are bounded again with d' = d;
 * each keeps the smaller of its two counts.  -1 (the default): automatic,
 * dprime = 62 with FP32 or BF16 screening where the d' = d rows are at
 * least twice as long as the rotated ones (d >= 111); 0: no pre-pass;
 * 1 <= dprime <= 62 (and below d): that d'.  No effect with a rotation chosen by rmips_set_dprime, or in
 * rmips_index_build.  Results do not change; the cost of the bounds does.
 * RMIPS_EINVAL outside [-1, 62].
 */
rmips_status rmips_set_prepass(rmips_ctx *ctx, int32_t dprime);

/*
 * Testing knob: when `uscore` is not NULL (a device array of m int32),
 * rmips_topn also writes the Eq. (3)/(6) bound count of every item in the
 * caller's order (Sec. 4.2; the count over the users of the item's
 * Cauchy-Schwarz prefix, Eq. 2), an upper bound of its exact score by
 * Theorem 2: with a pre-pass (rmips_set_prepass), the pre-pass count, or
 * for the items bounded again the smaller of the two.  NULL stops it.  The
 * array must outlive the rmips_topn call.
 */
rmips_status rmips_set_bound_output(rmips_ctx *ctx, int32_t *uscore);

/* Workspace bytes for rmips_thresholds / rmips_scores / rmips_topn with
 * these sizes (0 if the sizes are invalid). */
size_t rmips_thresholds_workspace_size(int64_t n, int64_t m, int32_t d,
                                       int32_t k, rmips_prec prec);
size_t rmips_scores_workspace_size(int64_t n, int64_t nq, int32_t d,
                                   rmips_prec prec);
size_t rmips_topn_workspace_size(int64_t n, int64_t m, int32_t d, int32_t k,
                                 int32_t N, rmips_prec prec);
size_t rmips_soft_workspace_size(int64_t n, int64_t nq, int32_t d);

/*
 * Stage (a), Def. 1: for every user u, the k-th element of S_k(u).
 *   U [n x d], P [m x d]      device, FP32 row-major.
 *   1 <= k <= min(m, RMIPS_K_MAX), 1 <= d <= RMIPS_D_MAX, n >= 1.
 *   tau    [n]  device FP64 out: the k-th largest u . p (exact value).
 *   tau_id [n]  device int32 out: item id of that k-th element.
 *   topk   [n x k] device int32 out, may be NULL: the ids of S_k(u) in
 *               (value desc, id asc) order.
 */
rmips_status rmips_thresholds(rmips_ctx *ctx, const float *U, int64_t n,
                              const float *P, int64_t m, int32_t d, int32_t k,
                              rmips_prec prec, void *ws, size_t ws_bytes,
                              double *tau, int32_t *tau_id, int32_t *topk);

/*
 * Stage (b), Def. 2 / Eq. 1: score of each query item against users whose
 * k-th neighbours are (tau, tau_id) from rmips_thresholds.
 *   U [n x d] device FP32; tau [n] device FP64; tau_id [n] device int32.
 *   Q [nq x d] device FP32: the query item vectors.
 *   q_ids [nq] device int32: item id of each query in P (its place in the
 *     tie order), or -1 for an item outside P; such an item is placed after
 *     every item of P, so it is counted iff u . q > tau_u.  NULL = all -1.
 *   scores [nq] device int32 out: #{u : q in S_k(u)}.
 */
rmips_status rmips_scores(rmips_ctx *ctx, const float *U, int64_t n,
                          const double *tau, const int32_t *tau_id,
                          const float *Q, const int32_t *q_ids, int64_t nq,
                          int32_t d, rmips_prec prec, void *ws,
                          size_t ws_bytes, int32_t *scores);

/*
 * Def. 3 by the paper's method (Sec. 4, Alg. 2 driven by exact thresholds):
 * stage (a), then the Cauchy-Schwarz (Eq. 2) and incremental-pruning
 * (Eq. 3 / Eq. 6) upper bounds on every score (d' = d unless
 * rmips_set_dprime chose a rotation onto the users' dominant eigenspace;
 * d' = d after a rotated pre-pass where rmips_set_prepass says so),
 * then exact scores of items visited in (bound desc, id asc) order until
 * the next bound is below the current N-th score.
 *   1 <= N <= min(m, RMIPS_N_MAX).
 *   top_ids [N], top_scores [N]: HOST int32 out, (score desc, id asc).
 *   stats: HOST, may be NULL.
 * A NaN or Inf in U or P, or a row norm above 2^60, returns
 * RMIPS_ENONFINITE; on any error top_ids, top_scores and stats are left
 * as they were.  Synchronises the context's stream before returning.
 */
rmips_status rmips_topn(rmips_ctx *ctx, const float *U, int64_t n,
                        const float *P, int64_t m, int32_t d, int32_t k,
                        int32_t N, rmips_prec prec, void *ws, size_t ws_bytes,
                        int32_t *top_ids, int32_t *top_scores,
                        rmips_stats *stats);

/*
 * Relaxed, differentiable score for new-item design (not in the paper; a
 * smooth surrogate of the reverse k-MIPS count for query items q):
 *   S[i] = sum_u sigmoid((u . q_i - tau[u]) / T)         (FP32 in and out)
 *   U [n x d], tau [n] (FP32, e.g. the FP64 thresholds cast), Q [nq x d].
 *   T > 0.  S [nq] device FP32 out.
 */
rmips_status rmips_soft_fwd(rmips_ctx *ctx, const float *U, int64_t n,
                            const float *tau, const float *Q, int64_t nq,
                            int32_t d, float T, void *ws, size_t ws_bytes,
                            float *S);

/*
 * Gradient of the relaxed score:
 *   dQ[i, :] = dS[i] * sum_u sigmoid'(z_ui) / T * u,  z_ui = (u . q_i - tau[u]) / T
 *   dS [nq] device FP32 (upstream gradient), dQ [nq x d] device FP32 out.
 */
rmips_status rmips_soft_bwd(rmips_ctx *ctx, const float *U, int64_t n,
                            const float *tau, const float *Q, int64_t nq,
                            int32_t d, float T, const float *dS, void *ws,
                            size_t ws_bytes, float *dQ);

/*
 * The relaxed score and its unscaled gradient in one pass (the inner
 * products u . q_i are formed once):
 *   S [nq] device FP32 out as rmips_soft_fwd,
 *   G [nq x d] device FP32 out: G[i, :] = sum_u sigmoid'(z_ui) / T * u.
 * A backward pass is then rmips_soft_scale (dQ = dS * G) instead of a second
 * pass over the users.  Workspace: rmips_soft_workspace_size.
 */
rmips_status rmips_soft_fwd_grad(rmips_ctx *ctx, const float *U, int64_t n,
                                 const float *tau, const float *Q, int64_t nq,
                                 int32_t d, float T, void *ws, size_t ws_bytes,
                                 float *S, float *G);

/* dQ[i, :] = dS[i] * G[i, :] (device FP32; G from rmips_soft_fwd_grad). */
rmips_status rmips_soft_scale(rmips_ctx *ctx, const float *G, int64_t nq, int32_t d,
                              const float *dS, float *dQ);

/*
 * k_max index: the paper's offline stage (Sec. 4.2, Alg. 1), which keeps for
 * every user the k_max largest inner products (the lists A_i; k_max = 25 in
 * the paper's experiments, Sec. 5.1) and the upper-bound score uscore_k(p)
 * of every item for every k <= k_max, so that the online stage (Sec. 4.3,
 * Alg. 2) answers any (k <= k_max, N) without recomputing them.  Here the
 * lists are exact (FP64-exact values, tie order as above), so every user is
 * certified and the online stage is the bound-ordered exact scoring of
 * rmips_topn with the thresholds of that k.
 *
 * The index lives in a caller-owned device buffer of rmips_index_size()
 * bytes (256-byte aligned), written by rmips_index_build and read by the
 * calls below; it stays valid while U and P are unchanged.  Every index
 * call takes the same (n, m, d, kmax, prec) as the build; rmips_index_topn
 * also takes the same U and P (it recomputes ambiguous pairs from them).
 * Scratch: a workspace of rmips_index_workspace_size() bytes (for the build
 * and for queries).  1 <= kmax <= min(m, RMIPS_K_MAX).
 */
size_t rmips_index_size(int64_t n, int64_t m, int32_t d, int32_t kmax, rmips_prec prec);
size_t rmips_index_workspace_size(int64_t n, int64_t m, int32_t d, int32_t kmax,
                                  rmips_prec prec);

/*
 * Build the index (Alg. 1's offline stage): stage (a) once with k = kmax
 * (each user's kmax largest values and their ids), then for each k <= kmax
 * the Cauchy-Schwarz prefix (Eq. 2) and the Eq. (3)/(6) bound count of
 * every item.  U [n x d], P [m x d] device FP32.  Synchronises the stream;
 * RMIPS_ENONFINITE for a NaN/Inf or a row norm above 2^60 (the index is then
 * unusable).
 */
rmips_status rmips_index_build(rmips_ctx *ctx, const float *U, int64_t n, const float *P,
                               int64_t m, int32_t d, int32_t kmax, rmips_prec prec,
                               void *index, size_t index_bytes, void *ws, size_t ws_bytes);

/*
 * Def. 3 for one k <= kmax from the index (Alg. 2): items visited in
 * (uscore_k desc, id asc) order, exact scores with the thresholds of S_k,
 * strict stop; results as rmips_topn (host top_ids, top_scores, stats).
 * Synchronises the stream.  The index's header is read back before
 * anything is launched: RMIPS_EINVAL when the buffer does not hold an index
 * that rmips_index_build completed with these sizes and precision.
 */
rmips_status rmips_index_topn(rmips_ctx *ctx, const float *U, int64_t n, const float *P,
                              int64_t m, int32_t d, int32_t kmax, rmips_prec prec,
                              const void *index, size_t index_bytes, int32_t k, int32_t N,
                              void *ws, size_t ws_bytes, int32_t *top_ids,
                              int32_t *top_scores, rmips_stats *stats);

/*
 * The threshold of S_k(u) from the index (Def. 1): tau [n] device FP64 and
 * tau_id [n] device int32, as rmips_thresholds gives them for this k.
 * Waits once, to read the index's header (RMIPS_EINVAL as for
 * rmips_index_topn), then returns without waiting for the copy.
 */
rmips_status rmips_index_thresholds(rmips_ctx *ctx, int64_t n, int64_t m, int32_t d,
                                    int32_t kmax, rmips_prec prec, const void *index,
                                    size_t index_bytes, int32_t k, double *tau,
                                    int32_t *tau_id);

/*
 * The Eq. (3)/(6) bound count uscore_k(p) of every item (Sec. 4.2; an upper
 * bound of score(p) for this k by Theorem 2), caller order: uscore [m]
 * device int32.  Waits once, to read the index's header (RMIPS_EINVAL as
 * for rmips_index_topn), then returns without waiting for the gather.
 */
rmips_status rmips_index_bounds(rmips_ctx *ctx, int64_t n, int64_t m, int32_t d, int32_t kmax,
                                rmips_prec prec, const void *index, size_t index_bytes,
                                int32_t k, int32_t *uscore);

/*
 * Budgeted index: the paper's offline stage under an inner-product budget
 * (Sec. 4.2, Alg. 1) and its online stage with incremental reverse k-MIPS
 * (Sec. 4.3, Alg. 2 with Inc-RMIPS).
 *
 * Positions 1..m are the items in descending order of |p|^2 (the FP64 sum
 * of squares, ties by id).  The build, with B1/n = b1 and the dynamic budget
 * B2:
 *  (3) every user's list A_i = its k_max best items of positions 1..b1
 *      (exact values, order (value desc, id asc)); users whose scan does not
 *      settle there form U', each with key j' + 1 - b1, j' the first later
 *      position whose Cauchy-Schwarz bound (Eq. 2) is below its k_max-th
 *      value (m + 1 if none);
 *  (4) U' in ascending (key, user) order, rank x_i from 1, gets
 *      B_{2,i} = floor(f(x_i)) more positions plus the pooled budget B' that
 *      earlier users left; f is Eq. (4) with beta solved from Eq. (5)
 *      (RMIPS_BUDGET_EXP) or the uniform, linear and quadratic functions of
 *      Sec. 5.2, each integrating to B2 over [0, |U'|].  A user whose scan
 *      ends within b1 + 1 + B_{2,i} + B' has its exact list and leaves the
 *      rest to B'; the others form U'' with pos_i = that position and B' = 0;
 *  (5) lambda_i (Eq. 7) over the positions after pos_i up to the first whose
 *      Eq. (2) bound is below the k_max-th value (Eq. 3 with d' = min(d, 10)
 *      on a rotation), and uscore_k(p) for every k <= kmax: the first k
 *      entries of every list plus the users of U'' with Eq. (6) >= A_i^k.
 * Every "cannot be in" test is strict, so ties follow the id order.  The
 * build reads the exact k_max-th values of U' (stage (a), screened at
 * `prec`) to place each scan's end; the index keeps only what the budget
 * gives (the lists of U'' stop at pos_i).
 *
 * The query (Alg. 2) for k <= kmax: users with A_i^k > lambda_i are counted
 * from their lists; the others form X.  Items are visited in (uscore_k
 * desc, id asc) order in batches, with the strict stop (an item's uscore_k
 * below the N-th score); for each visited item Inc-RMIPS decides every user
 * of X: an item among its first k entries is in when its value exceeds
 * lambda_i; an unscanned item is out by Eq. (2), Eq. (3) or its exact
 * value against the k-th entry; any other pair rescans the user, which
 * gives its exact S_k (stage (a) at `prec`), credits the items not yet
 * visited and removes it from X.  The result is Def. 3 exactly.
 *
 * Index: a caller-owned device buffer of rmips_budget_index_size() bytes
 * (256-byte aligned), valid while U and P are unchanged; the query takes the
 * same U, P, n, m, d, kmax.  Scratch: rmips_budget_workspace_size() bytes
 * (build and query).  1 <= kmax <= min(m, RMIPS_K_MAX), kmax <= b1.
 */
typedef enum {
    RMIPS_BUDGET_EXP = 0,       /* Eq. (4): alpha exp(beta x) + gamma, beta from Eq. (5) */
    RMIPS_BUDGET_UNIFORM = 1,   /* B2 / |U'| */
    RMIPS_BUDGET_LINEAR = 2,    /* 2 B2 x / |U'|^2 */
    RMIPS_BUDGET_QUADRATIC = 3  /* 3 B2 x^2 / |U'|^3 */
} rmips_budget_kind;

typedef struct {
    int64_t b1;     /* B1 / n: positions of step (3), >= kmax (more than m: m) */
    int64_t B2;     /* dynamic budget of step (4), 0 <= B2 <= 2^62 */
    int32_t kind;   /* rmips_budget_kind */
    double alpha;   /* Eq. (4), finite, >= 0 (RMIPS_BUDGET_EXP) */
    double gamma;   /* Eq. (4), finite, >= 0 (RMIPS_BUDGET_EXP) */
} rmips_budget;

typedef struct {
    int64_t u_prime;   /* |U'| */
    int64_t u_dprime;  /* |U''| */
    int64_t cert3;     /* users settled by step (3) */
    int64_t cert4;     /* users of U' settled by step (4) */
    int64_t scanned4;  /* positions scanned in step (4) */
    double beta;       /* Eq. (5)'s solution (-inf: f = gamma; 0 for other kinds) */
    float ms_total;    /* build time, HIP events */
} rmips_budget_info;

typedef struct {
    int64_t x0;               /* |X| at the start */
    int64_t rescanned_users;  /* users rescanned (they leave X) */
    int64_t rescan_calls;     /* batches that rescanned */
    int64_t visited_items;    /* items Alg. 2 visits one by one up to its stop */
    int64_t processed_items;  /* items scored (whole batches) */
    int64_t batches;
    float ms_init;            /* initialisation and visit order */
    float ms_total;
} rmips_budget_qstats;

size_t rmips_budget_index_size(int64_t n, int64_t m, int32_t d, int32_t kmax);
size_t rmips_budget_workspace_size(int64_t n, int64_t m, int32_t d, int32_t kmax,
                                   rmips_prec prec);

/*
 * Build (Alg. 1 under the budget).  U [n x d], P [m x d] device FP32;
 * budget and info (nullable) host.  Synchronises the stream.  RMIPS_EINVAL
 * for a bad budget (b1 < kmax, B2 out of range, unknown kind, alpha or
 * gamma negative or not finite); RMIPS_ENONFINITE for a NaN/Inf or a row
 * norm above 2^60 (the index is then unusable).
 */
rmips_status rmips_budget_build(rmips_ctx *ctx, const float *U, int64_t n, const float *P,
                                int64_t m, int32_t d, int32_t kmax, rmips_prec prec,
                                const rmips_budget *budget, void *index, size_t index_bytes,
                                void *ws, size_t ws_bytes, rmips_budget_info *info);

/*
 * Def. 3 for k <= kmax by Alg. 2 with Inc-RMIPS on the index: top_ids and
 * top_scores (host, N each) in (score desc, id asc) order; stats (host,
 * nullable).  Synchronises the stream (once per batch).  The index's header
 * is read back first: RMIPS_EINVAL when the buffer does not hold an index
 * that rmips_budget_build completed with these n, m, d, kmax.
 */
rmips_status rmips_budget_topn(rmips_ctx *ctx, const float *U, int64_t n, const float *P,
                               int64_t m, int32_t d, int32_t kmax, rmips_prec prec,
                               const void *index, size_t index_bytes, int32_t k, int32_t N,
                               void *ws, size_t ws_bytes, int32_t *top_ids, int32_t *top_scores,
                               rmips_budget_qstats *stats);

/*
 * Copies of the index's state (device pointers, each nullable): order [m]
 * (position j - 1 -> item id), pos [n] (pos_i, 0 outside U''), lam [n]
 * (lambda_i, -inf outside U''), Av / Aj [n x kmax] (the lists: values, item
 * ids), key [n] (j' + 1 - b1, 0 outside U'), rank [n] (x_i, 0 outside U'),
 * b2 [n] (B_{2,i}, 0 outside U'), uscore [kmax x m] (row k - 1: uscore_k by
 * item id).  Waits once to read the header (RMIPS_EINVAL as above), then
 * returns without waiting for the copies.
 */
rmips_status rmips_budget_state(rmips_ctx *ctx, int64_t n, int64_t m, int32_t d, int32_t kmax,
                                const void *index, size_t index_bytes, int32_t *order,
                                int32_t *pos, double *lam, double *Av, int32_t *Aj, int32_t *key,
                                int32_t *rank, int64_t *b2, int32_t *uscore);

/*
 * rmips_soft_bwd without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving or ascent
 * loops, harnesses that forbid allocation).  Same arguments, kernels and
 * results as rmips_soft_bwd.  The partial sums go to a static scratch array
 * of the library (48 MiB per device, held until the process ends), so
 * nq * (d rounded up to 16) must be at most 65536 (e.g. 256 queries of up
 * to 256 dims); larger sizes return RMIPS_EINVAL.  It allocates nothing:
 * no hipMalloc, no allocating library call.  Every call on one device
 * shares that device's array: calls that overlap on one device (two
 * streams, two threads) race and give wrong results.  Does not wait.
 */
rmips_status rmips_soft_bwd_noalloc(rmips_ctx *ctx, const float *U, int64_t n,
                                    const float *tau, const float *Q, int64_t nq,
                                    int32_t d, float T, const float *dS, float *dQ);

#ifdef __cplusplus
}
#endif

#endif /* RMIPS_H */

// Internal launch interfaces of librmips (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rmips {

// ------------------------------------------------------------ profiling
// While a context's profiling is on, each kernel launch records a HIP event
// on its stream before and after itself (a ProfScope around the launch); the
// durations are summed per kernel name once the stream has been waited for.
// With profiling off a scope costs one thread-local load.
struct ProfRecorder;
extern thread_local ProfRecorder *g_prof;  // set by a C-ABI call while it enqueues
void prof_begin(hipStream_t st, const char *name);
void prof_end(hipStream_t st);
struct ProfScope {
    hipStream_t st;
    bool on;
    ProfScope(hipStream_t s, const char *name) : st(s), on(g_prof != nullptr) {
        if (on) prof_begin(s, name);
    }
    ~ProfScope() {
        if (on) prof_end(st);
    }
};
#define RMIPS_PROF(st, name) ::rmips::ProfScope rmips_prof_scope_(st, name)

// ----------------------------------------------------------------- sort
size_t radix_sort_scratch_bytes(int64_t n);
// stable ascending sort by the key bits [lo_bit, hi_bit); the bits above
// must agree in every key
hipError_t radix_sort_u32(uint32_t *keys, int32_t *vals, int64_t n, void *scratch,
                          hipStream_t st, int lo_bit = 0, int hi_bit = 32);

// ----------------------------------------------------------------- prep
// Norm of every row (FP64, rounded up to FP32), zero-padded FP32 copy with
// leading dimension D (may be NULL), and a flag set to 1 on NaN/Inf or a
// norm above 2^60.  key/val (may be NULL): sort key ~bits(norm) (descending
// norm) and the row id.
void launch_rows_prep(const float *X, int64_t rows, int d, int D, float *Xpad,
                      float *norm, uint32_t *key, int32_t *val, int *flag,
                      hipStream_t st);
// Pk[r] = P[perm[r]] for r < m, zero rows for m <= r < rows_pad; Np likewise.
void launch_gather_rows(const float *P, const int32_t *perm, const float *norm_by_id,
                        int64_t m, int64_t rows_pad, int d, int D, float *Pk,
                        float *Np, hipStream_t st);
// inv[perm[r]] = r
void launch_invert_perm(const int32_t *perm, int64_t m, int32_t *inv, hipStream_t st);

// Padded, quantized copy of rows (see k_quant): Xq holds rows_pad rows of
// D elements of the precision's type; group rows share a scale.
void launch_quant(int prec, const float *X, const int32_t *order, int64_t rows,
                  int64_t rows_pad, int d, int D, int group, void *Xq, float *N, float *Nh,
                  float *R, float *sc, unsigned int *rmax, int *flag, hipStream_t st);

// Per-user data of the counting stage, in an order given by `order`
// (sorted position -> user id; NULL = identity).
struct UserSide {
    float *N;        // ||u|| rounded up
    float *Nh;       // ||u_q|| (quantized copy) rounded up
    float *R;        // ||u - u_q|| rounded up
    float *sinv;     // 1 / (power-of-two scale of the quantized copy), exact
    float *tau_hi;   // tau rounded up to FP32
    float *tau_lo;   // tau rounded down to FP32
    double *tau;     // exact tau
    int32_t *tau_id; // item id of the k-th element
    int32_t *uid;    // user id of this position
    // the fields the counting kernel needs per user, in one 16-byte record:
    // {tau_hi, tau_lo, R + c2 N, Nh}; with the items' largest N, Nh, R the
    // bound is E = (R + c2 N) N_p + Nh (R_p + c Nh_p) + e_abs
    float4 *thr;
};
void launch_user_side(const double *tau, const int32_t *tau_id, const float *Nu,
                      const float *Nhu, const float *Ru, const float *su,
                      const int32_t *order, int64_t n, float c2, UserSide out, hipStream_t st);
// tau[u] = topv[u * kmax + k - 1], tau_id likewise (the k-th column of the
// users' lists of their kmax largest values)
void launch_kth_column(const double *topv, const int32_t *topk, int64_t n, int kmax, int k,
                       double *tau, int32_t *tau_id, hipStream_t st);
// Sort keys of the pruning ratio rho_u = tau_u / ||u|| rounded down to FP32
// (-inf when tau_u <= 0 or ||u|| = 0), as ascending uint32 keys; val = user id.
void launch_rho_keys(const double *tau, const float *Nu, int64_t n, uint32_t *key,
                     int32_t *val, hipStream_t st);
// Y[r] = X[order[r]], rows of row_bytes (a multiple of 16)
void launch_gather_padded(const void *X, const int32_t *order, int64_t rows, int row_bytes,
                          void *Y, hipStream_t st);
// cs[j] = number of sorted ratio keys whose bits from lo_bit up are at most
// those of norm[j] * (1 + 2^-18) (keys sorted by those bits)
void launch_cs_prefix(const uint32_t *rho_sorted_keys, int64_t n, const float *norm,
                      int64_t m, int lo_bit, int32_t *cs, hipStream_t st);
// G = sum over sampled rows x x^T (FP64, d x d), rows u = s*stride, s < ns;
// scratch holds gram_scratch_bytes(d) bytes of per-slice partial sums
size_t gram_scratch_bytes(int d);
void launch_gram(const float *X, int64_t ns, int64_t stride, int d, double *G, double *scratch,
                 hipStream_t st);
// Augmented rows for the Eq. (3) bound: the ka FP32 values a = [W x (dp
// values), tail(x), scale * ||x||, 0...] (ka a multiple of 16, dp + 2 <=
// ka), where W (dp x d, FP64, dp <= 62, ka <= 64) has orthonormal rows and
// tail(x) = sqrt(||x||^2 - ||W x||^2) rounded up (W = nullptr: the
// identity, dp = d <= 256, ka <= 288), stored as 2 ka bytes per row: BF16
// rn(a).  Rows are taken from X
// through `order` (NULL = identity); rows from `rows` to `rows_pad` are zero.
void launch_rotate_aug(const float *X, const int32_t *order, int64_t rows,
                       int64_t rows_pad, int d, const double *W, int dp, int ka, float scale,
                       uint4 *out, hipStream_t st);

// ---------------------------------------------------------- stage (a)
struct ThreshArgs {
    int prec;
    // users (caller order): quantized rows, N, Nh, R, scale
    const void *Uq; const float *Nu; const float *Nhu; const float *Ru; const float *su;
    int64_t n;
    // items (norm order): quantized rows (ntiles * 64), N, Nh, R, scale per item
    const void *Pq; const float *Np; const float *Nhp; const float *Rp; const float *sp;
    const float *tmax_nh; const float *tmax_r;  // per tile maxima of Nh and R
    const unsigned int *rmax_bits;              // largest R/N over the items
    const int32_t *perm; int64_t m; int ntiles;
    const float *U; const float *P; int d;      // original FP32 rows (recheck)
    int D; int k; int t0tiles; int nsplit; int cap;
    float c_err; float c2; float e_abs; float g64;
    // candidate lists: (screened value, its error bound E) and the caller's id
    float2 *cand; int32_t *cand_id; int32_t *cand_cnt;
    // outputs: the k-th value and its id; with topk (may be NULL) the ids of
    // S_k(u) in order, and with topv (may be NULL, needs topk) their values
    double *tau; int32_t *tau_id; int32_t *topk; double *topv;
    // overflow handling: lists (3 x n: two refinement lists, the fallback
    // list) with their counters (4 ints), refinement passes (0..2), and the
    // per-user starting bound of the last pass
    int32_t *lists; int32_t *lcnt; int refine; float *Luse;
    // users grouped by their early-exit ratio before the main pass: sort
    // keys, the order, radix-sort scratch, and a device int holding n
    uint32_t *ukey; int32_t *uord; void *usort; int32_t *nall;
    // set per pass by launch_thresh
    const int32_t *ulist; const int32_t *ulist_cnt;  // users of this pass (NULL = all)
    int32_t *rlist; int32_t *rcnt;                   // out: users to screen again
    int32_t *flist; int32_t *fcnt;                   // out: users for the exact fallback
    // statistics (may be NULL), spread over CSTAT_SLOTS addresses:
    // pairs[slot] pairs screened by the main pass, rpairs[slot] by the
    // refinement passes; cstats[slot][4] = candidates, rechecked, fallback
    // users, refined users
    unsigned long long *pairs;
    unsigned long long *rpairs;
    unsigned long long *cstats;
    hipEvent_t ev0, ev1;           // recorded around the first screening pass (may be NULL)
};
constexpr int CSTAT_SLOTS = 32;
void launch_thresh(const ThreshArgs &a, hipStream_t st);
// per-wave list stride of the final selection: the longest list rounded up
// to a power of two (the in-LDS bitonic sorts pad to it)
inline int final_stride(int capT) {
    int p = 1;
    while (p < capT) p <<= 1;
    return p;
}
size_t thresh_screen_lds(int prec, int D);
// LDS bytes per candidate-list entry of the final selection
size_t final_entry_bytes();
// per-tile maxima of Nh and R (64 items per tile)
void launch_tile_max(const float *Nh, const float *R, int ntiles, float *tmax_nh, float *tmax_r,
                     hipStream_t st);

// ---------------------------------------------------------- stage (b)/(c)
struct CountArgs {
    int prec;
    // items (rows): quantized rows gathered through `rows` (NULL = identity),
    // per row N, Nh, R, scale
    const void *Pq; const float *Np; const float *Nhp; const float *Rp; const float *sp;
    const int32_t *rows; int64_t nb;
    const int32_t *item_tie;   // tie id per padded row (NULL = -1: outside P)
    const int32_t *item_orig;  // original row per padded row (NULL = identity)
    const float *Porig;        // original FP32 item rows
    // users (columns): quantized rows, first ulen of them; with ulen_dev
    // the count is read on the device and ulen is only an upper bound
    const void *Us; int64_t ulen; UserSide us;
    const int32_t *ulen_dev;
    const float *Uorig; int d; int D;
    float c_err; float c2; float e_abs;
    int nsplit; int32_t *partial; int64_t *rechecks;
};
void launch_count(const CountArgs &a, hipStream_t st);
// a batch's slots (rows of the norm-ordered item arrays and their caller ids)
// in row order, nb <= 4096
void launch_batch_order(int32_t *rows, int32_t *cid, int64_t nb, hipStream_t st);
// *out = max(x[0], ..., x[n-1]) (0 when n = 0), one workgroup
void launch_max_i32(const int32_t *x, int64_t n, int32_t *out, hipStream_t st);
size_t count_lds(int prec, int D);

struct BoundArgs {
    int ka;                            // augmented row length 16 KS: KS <= 11, or even up to 18
    const uint4 *Pb; int64_t m, mpad;  // augmented item rows (norm order), BF16
    const uint4 *Ub;                   // augmented user rows (rho order), BF16
    const float *tau_lo;               // per sorted user
    float abs_slack;                   // absolute slack of the bound
    const int32_t *cs;                 // CS prefix per item (non-increasing)
    int nsplit; int32_t *partial;
    unsigned long long *pairs;         // stats: evaluated pairs (may be NULL)
};
void launch_bound(const BoundArgs &a, hipStream_t st, const char *prof_name = "k_bound");
int bound_splits(int64_t m, int ka, int smax = 16);

// partial[s][j] summed over s (fixed order) -> out[j]
void launch_colsum(const int32_t *partial, int nsplit, int64_t cols, int32_t *out,
                   hipStream_t st);
// ~uscore keys in id order: key[c] = ~us[inv[c]], val[c] = inv[c]; also
// resets the running top-N status (when not NULL) to {-1, 0}
void launch_visit_keys(const int32_t *uscore, const int32_t *inv, int64_t m,
                       uint32_t *key, int32_t *val, int32_t *status, hipStream_t st);
void launch_gather_i32(const int32_t *src, const int32_t *idx, int64_t n, int32_t *dst,
                       hipStream_t st);
// da[i] = a[idx[i]], db[i] = b[idx[i]], dc[i] = c[idx[i]] in one launch
void launch_gather3_i32(const int32_t *a, const int32_t *b, const int32_t *c,
                        const int32_t *idx, int64_t n, int32_t *da, int32_t *db, int32_t *dc,
                        hipStream_t st);

// key[i] = id[i], val[i] = i for i < n
void launch_seg_init(const int32_t *id, int64_t n, uint32_t *key, int32_t *val, hipStream_t st);
// b[i] = min(b[i], b0[i]) and uscore[rows[i]] = b[i] for i < n
void launch_seg_bound(int32_t *b, const int32_t *b0, const int32_t *rows, int64_t n,
                      int32_t *uscore, hipStream_t st);

// Running top-N: merge the exact scores of a batch into the sorted list
// `top` (keys score<<32 | ~id), keep N.  status[0] = N-th score (-1 while
// fewer than N), status[1] = entries kept.  nb <= 4096, N <= 1024.
void launch_topn_merge(const int32_t *scores, int64_t nb, const int32_t *batch_ids, int N,
                       uint64_t *top, int32_t *status, hipStream_t st);

// ---------------------------------------------------------- relaxed score
// S (may be NULL): the relaxed score; G (may be NULL): its gradient; dQ (may
// be NULL): the gradient scaled by dS per query.  ws holds the per-slice
// partial sums of at most max_splits user slices (soft_ws_bytes for
// soft_max_splits()).
void launch_soft(const float *U, int64_t n, const float *tau, const float *Q, int64_t nq,
                 int d, float T, const float *dS, float *S, float *G, float *dQ, void *ws,
                 hipStream_t st, int max_splits);
int soft_max_splits();
int soft_noalloc_splits();
// dQ[i][:] = dS[i] * G[i][:]
void launch_soft_scale(const float *G, int64_t nq, int d, const float *dS, float *dQ,
                       hipStream_t st);
size_t soft_ws_bytes(int64_t n, int64_t nq, int d);
// Device address of the file-scope scratch array of the relaxed-score
// kernels on `device`, which must be the current device (taken once per
// device, then cached); whether nq queries of d dims fit in it.
hipError_t soft_scratch_init(int device, void **out);
bool soft_noalloc_fits(int64_t nq, int d);


// ------------------------------------------------------ budgeted index
// (Alg. 1 under an inner-product budget, Sec. 4.2; Alg. 2 with Inc-RMIPS,
// Sec. 4.3).  Positions are 1-based in the descending order of the FP64 sum
// of squares (ties by item id); "position order" arrays hold position j at
// index j - 1.
constexpr int BUDGET_DP_MAX = 10;      // d' of the index's Eq. (3) (Sec. 5.1), at most
constexpr int BUDGET_BATCH_MAX = 256;  // items per visited batch while X is not empty
constexpr int BUDGET_BATCH_BIG = 4096; // items per visited batch once X is empty
// x2[r] = FP64 sum of squares of row r (index order)
void launch_sqnorm64(const float *X, int64_t rows, int d, double *x2, hipStream_t st);
// rotated coordinates l = W x (dp values), remaining norm and norm (both
// rounded up) of the rows X[order[r]] (order may be NULL)
void launch_budget_rotate(const float *X, const int32_t *order, const double *x2_by_row,
                          int64_t rows, int d, const double *W, int dp, double *L, double *nr,
                          double *nn, hipStream_t st);
// Y[r] = X[idx[r]], rows of d floats
void launch_budget_gather(const float *X, const int32_t *idx, int64_t rows, int d, float *Y,
                          hipStream_t st);
// the kmax best (value desc, id asc) of positions 1..lim of each listed user
// (users NULL: all; lims NULL: lim0), exact, into the user's row of Av / Aj
void launch_budget_prefix(const float *U, const float *PgT, int64_t m, const int32_t *order,
                          int d, const int32_t *users, const int32_t *lims, int64_t lim0,
                          int64_t nusers, int kmax, double *Av, int32_t *Aj, hipStream_t st);
// PgT (d x m) = the items transposed, in position order
void launch_budget_transpose(const float *P, const int32_t *order, int64_t m, int d,
                             float *PgT, hipStream_t st);
// key[u] = j' + 1 - b1 for a user whose first b1 positions did not settle
// its list, else 0
void launch_budget_classify(const double *Av, const double *nu2, const double *np2s, int64_t n,
                            int64_t m, int kmax, int64_t b1, int32_t *key, hipStream_t st);
// t[r] = natural stop of users[r] from its exact kmax-th value (topv row r)
void launch_budget_tstop(const int32_t *users, const double *topv, const double *nu2,
                         const double *np2s, int64_t X, int64_t m, int kmax, int64_t b1,
                         int32_t *t, hipStream_t st);
// exact lists (rows of topv/topk) to the users among `users` with pos 0
void launch_budget_scatter(const int32_t *users, const int32_t *pos, const double *topv,
                           const int32_t *topk, int64_t X, int kmax, double *Av, int32_t *Aj,
                           hipStream_t st);
// step (5)'s range end of each user of U'' (key) with the user (val)
void launch_budget_range(const int32_t *users, const int32_t *pos, int64_t nusers,
                         const double *Av, const double *nu2, const double *np2s, int64_t m,
                         int kmax, uint32_t *key, int32_t *val, hipStream_t st);
// step (5): lambda of each listed user (sorted by range end hi_pos) and the
// Eq. (6) counts into the difference table diff (kmax x m, by item id)
void launch_budget_step5(const int32_t *users, const uint32_t *hi_pos, const int32_t *pos,
                         int64_t nusers, const double *Av, const double *Ul, const double *nru,
                         const double *nun, const double *Pl, const double *nrp,
                         const double *npn, const int32_t *order, int64_t m, int kmax, int dp,
                         double *lam, int32_t *diff, hipStream_t st);
// the lists' entries into the difference table (entry r -> row r)
void launch_budget_hist(const int32_t *Aj, int64_t n, int kmax, int64_t m, int32_t *diff,
                        hipStream_t st);
// difference table -> uscore (prefix sums over k, in place)
void launch_budget_prefix_k(int32_t *t, int64_t m, int kmax, hipStream_t st);
// query: certified users into base, the others into X (count in *xn)
void launch_budget_xinit(const double *Av, const int32_t *Aj, const double *lam, int64_t n,
                         int kmax, int k, int32_t *base, int32_t *X, int32_t *xn,
                         hipStream_t st);
void launch_budget_slots(const int32_t *bids, int nb, int32_t *slot, hipStream_t st);
// Inc-RMIPS of X against a batch (nb <= BUDGET_BATCH_MAX): ins into cnt (by
// batch slot), users that need a rescan into R (count in *rn), xflag set
void launch_budget_inc(const int32_t *X, int64_t xn, const int32_t *bids, int nb,
                       const int32_t *slot, const double *Av, const int32_t *Aj, const double *lam,
                       const int32_t *pos, const double *nu2, const double *Ul,
                       const double *nru, const double *nun, const int32_t *posof,
                       const double *np2s, const double *Pl, const double *nrp,
                       const double *npn, int kmax, int k, int dp, int32_t *cnt, int32_t *R,
                       int32_t *rn, uint8_t *xflag, hipStream_t st);
// rescanned users' S_k (nr rows of k ids): unvisited items into base
void launch_budget_apply(const int32_t *topk, int64_t nr, int k, const uint8_t *visited,
                         int32_t *base, hipStream_t st);
void launch_budget_xcompact(const int32_t *X, int64_t xn, const uint8_t *xflag, int32_t *Y,
                            int32_t *yn, hipStream_t st);
// score[s] = base + cnt of the batch's items; marks them visited, clears
// their slots and counts
void launch_budget_batch(const int32_t *bids, int nb, const int32_t *base, int32_t *cnt,
                         uint8_t *visited, int32_t *slot, int32_t *score, hipStream_t st);
void launch_budget_visit_keys(const int32_t *us, int64_t m, uint32_t *key, int32_t *val,
                              hipStream_t st);
void launch_fill_i32(int32_t *x, int64_t n, int32_t v, hipStream_t st);
void launch_fill_f64(double *x, int64_t n, double v, hipStream_t st);

}  // namespace rmips

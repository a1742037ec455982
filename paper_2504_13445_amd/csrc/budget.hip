// The budgeted index: Alg. 1 under an inner-product budget (Sec. 4.2) and
// Alg. 2 with Inc-RMIPS (Sec. 4.3).
//
// Positions 1..m name the items in descending order of the FP64 sum of
// squares (ties by item id); arrays "in position order" hold position j at
// index j - 1.  Every value u . p here is the exact one (FP64, products of
// the FP32 inputs summed in index order), and every "cannot be in" test is
// strict, so that an item tying the threshold with a smaller id is kept.
#include "common.h"
#include "kernels.h"

namespace rmips {

namespace {

constexpr double CS_SQ = 1.0 + 0x1p-36;

// Eq. (2) in squares: true when ||u|| ||p|| is certainly below theta, i.e.
// theta > 0 and (|u|^2 |p|^2)(1 + 2^-36) < theta^2 with |x|^2 the FP64 sum
// of squares.  The slack covers the rounding of those sums and of the FP64
// value of u . p for d <= 4096; the products are rounded once each.
__device__ __forceinline__ bool cs_below(double nu2, double np2, double theta) {
    return theta > 0.0 && __dmul_rn(__dmul_rn(nu2, np2), CS_SQ) < __dmul_rn(theta, theta);
}

// (v1, id1) ranks before (v2, id2) in the order (value desc, id asc)
__device__ __forceinline__ bool ranks_before(double v1, int id1, double v2, int id2) {
    return v1 > v2 || (v1 == v2 && id1 < id2);
}

// exact u . p: FP64, products of FP32 values (exact), summed in index order
__device__ __forceinline__ double ip64_rows(const float *u, const float *p, int d) {
    double acc = 0.0;
    for (int i = 0; i < d; ++i) acc = __fma_rn((double)u[i], (double)p[i], acc);
    return acc;
}

// Eq. (3) on rotated coordinates: u^l . p^l + |u^r| |p^r| plus a relative
// slack covering the rotation's rounding and its deviation from
// orthonormality (both far below 2^-30 of |u| |p|)
constexpr double EQ3_SLACK = 0x1p-30;
__device__ __forceinline__ double eq3_bound(const double *ul, double nru, double nun,
                                            const double *pl, double nrp, double npn, int dp) {
    double acc = 0.0;
    for (int t = 0; t < dp; ++t) acc = __fma_rn(ul[t], pl[t], acc);
    return acc + nru * nrp + EQ3_SLACK * (nun * npn);
}

// one compare-exchange of a wave-wide bitonic network on (value, id) keys;
// `first` = this lane keeps the key that ranks first
__device__ __forceinline__ void bitonic_step(double &v, int &id, int j, bool first) {
    const double pv = __shfl_xor(v, j);
    const int pid = __shfl_xor(id, j);
    const bool mine_first = ranks_before(v, id, pv, pid);
    if (mine_first != first) {
        v = pv;
        id = pid;
    }
}

// sort the wave's 64 keys so that lane 0 holds the first in rank
__device__ __forceinline__ void wave_sort64(double &v, int &id, int lane) {
    for (int k = 2; k <= 64; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            const bool asc = (lane & k) == 0;
            const bool lower = (lane & j) == 0;
            bitonic_step(v, id, j, lower == asc);
        }
}

// a bitonic sequence of 64 keys into rank order (lane 0 first)
__device__ __forceinline__ void wave_merge64(double &v, int &id, int lane) {
    for (int j = 32; j > 0; j >>= 1) bitonic_step(v, id, j, (lane & j) == 0);
}

}  // namespace

// ---------------------------------------------------------------- norms
// x2[r] = sum_i x_i^2 (FP64, index order) of row r
__global__ void k_sqnorm64(const float *__restrict__ X, int64_t rows, int d,
                           double *__restrict__ x2) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const float *x = X + r * d;
    double s = 0.0;
    for (int i = 0; i < d; ++i) s = __fma_rn((double)x[i], (double)x[i], s);
    x2[r] = s;
}

void launch_sqnorm64(const float *X, int64_t rows, int d, double *x2, hipStream_t st) {
    RMIPS_PROF(st, "k_sqnorm64");
    k_sqnorm64<<<(unsigned)((rows + 255) / 256), 256, 0, st>>>(X, rows, d, x2);
}

// ------------------------------------------------------------- rotation
// For row r (X row order[r], or r): l = W x (dp values, W dp x d with
// orthonormal rows), the remaining norm sqrt(|x|^2 - |l|^2 + 2^-40 |x|^2)
// and the norm sqrt(|x|^2), both rounded up (the added term covers the
// cancellation of the difference).
__global__ __launch_bounds__(256) void k_budget_rotate(const float *__restrict__ X,
                                                       const int32_t *__restrict__ order,
                                                       const double *__restrict__ x2_by_row,
                                                       int64_t rows, int d,
                                                       const double *__restrict__ W, int dp,
                                                       double *__restrict__ L,
                                                       double *__restrict__ nr,
                                                       double *__restrict__ nn) {
    __shared__ double Ws[BUDGET_DP_MAX * 256];
    for (int i = threadIdx.x; i < dp * d; i += blockDim.x) Ws[i] = W[i];
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int64_t src = order ? order[r] : r;
    const float *x = X + src * d;
    double l[BUDGET_DP_MAX];
#pragma unroll
    for (int t = 0; t < BUDGET_DP_MAX; ++t) l[t] = 0.0;
    for (int i = 0; i < d; ++i) {
        const double xi = (double)x[i];
#pragma unroll
        for (int t = 0; t < BUDGET_DP_MAX; ++t)
            if (t < dp) l[t] = __fma_rn(Ws[t * d + i], xi, l[t]);
    }
    const double x2 = x2_by_row[src];
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < BUDGET_DP_MAX; ++t)
        if (t < dp) {
            L[r * dp + t] = l[t];
            s = __fma_rn(l[t], l[t], s);
        }
    const double up = 1.0 + 0x1p-50;
    nr[r] = sqrt(fmax(x2 - s, 0.0) + 0x1p-40 * x2) * up;
    nn[r] = sqrt(x2) * up;
}

void launch_budget_rotate(const float *X, const int32_t *order, const double *x2_by_row,
                          int64_t rows, int d, const double *W, int dp, double *L, double *nr,
                          double *nn, hipStream_t st) {
    RMIPS_PROF(st, "k_budget_rotate");
    k_budget_rotate<<<(unsigned)((rows + 255) / 256), 256, 0, st>>>(X, order, x2_by_row, rows,
                                                                     d, W, dp, L, nr, nn);
}

// ------------------------------------------------------------- gathers
// Y[r] = X[idx[r]] (rows of d floats); Y2[r] = x2[idx[r]] when both given
__global__ void k_budget_gather(const float *__restrict__ X, const int32_t *__restrict__ idx,
                                int64_t rows, int d, float *__restrict__ Y) {
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows) return;
    const int64_t src = idx[r];
    for (int i = threadIdx.x & 63; i < d; i += 64) Y[r * d + i] = X[src * d + i];
}

void launch_budget_gather(const float *X, const int32_t *idx, int64_t rows, int d, float *Y,
                          hipStream_t st) {
    RMIPS_PROF(st, "k_budget_gather");
    k_budget_gather<<<(unsigned)((rows + 3) / 4), 256, 0, st>>>(X, idx, rows, d, Y);
}

// ------------------------------------------------------- prefix lists
// For user u = users[w] (or w): the kmax best items of positions 1..lim
// (lim = lims[w], or lim0) in the order (value desc, id asc), exact, into
// row u of Av / Aj.  One wave per user: 64 positions per step, one per
// lane, each value summed in index order by its lane; the step's keys are
// sorted across the wave and merged with the 64 best so far.
__global__ __launch_bounds__(256) void k_budget_prefix(
    const float *__restrict__ U, const float *__restrict__ Pg, const int32_t *__restrict__ order,
    int d, const int32_t *__restrict__ users, const int32_t *__restrict__ lims, int64_t lim0,
    int64_t nusers, int kmax, double *__restrict__ Av, int32_t *__restrict__ Aj) {
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= nusers) return;
    const int64_t u = users ? users[w] : w;
    const int64_t lim = lims ? lims[w] : lim0;
    const float *uu = U + u * d;
    double bv = -INFINITY;
    int bid = INT32_MAX;
    for (int64_t c0 = 0; c0 < lim; c0 += 64) {
        const int64_t q = c0 + lane;
        double v = -INFINITY;
        int id = INT32_MAX;
        if (q < lim) {
            id = order[q];
            v = ip64_rows(uu, Pg + q * d, d);
        }
        wave_sort64(v, id, lane);
        // the 64 best of both sorted sequences, as a bitonic sequence
        const double ov = __shfl(bv, 63 - lane);
        const int oid = __shfl(bid, 63 - lane);
        if (ranks_before(ov, oid, v, id)) {
            v = ov;
            id = oid;
        }
        wave_merge64(v, id, lane);
        bv = v;
        bid = id;
    }
    if (lane < kmax) {
        Av[u * kmax + lane] = bv;
        Aj[u * kmax + lane] = bid;
    }
}

void launch_budget_prefix(const float *U, const float *Pg, const int32_t *order, int d,
                          const int32_t *users, const int32_t *lims, int64_t lim0,
                          int64_t nusers, int kmax, double *Av, int32_t *Aj, hipStream_t st) {
    if (nusers <= 0) return;
    RMIPS_PROF(st, "k_budget_prefix");
    k_budget_prefix<<<(unsigned)((nusers + 3) / 4), 256, 0, st>>>(U, Pg, order, d, users, lims,
                                                                   lim0, nusers, kmax, Av, Aj);
}

// first position j in [lo, m] whose Eq. (2) bound is below theta, m + 1
// when there is none (the bound falls with the position)
__device__ __forceinline__ int64_t first_below(double nu2, const double *np2s, int64_t lo,
                                               int64_t m, double theta) {
    int64_t hi = m + 1;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (cs_below(nu2, np2s[mid - 1], theta))
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Step (3)'s outcome per user: key = j' + 1 - b1 for a user whose scan of
// positions 1..b1 did not stop (its list is not known to be exact), with
// j' the first later position whose bound is below its k_max-th value;
// 0 for a user whose scan stopped (or covered all items)
__global__ void k_budget_classify(const double *__restrict__ Av, const double *__restrict__ nu2,
                                  const double *__restrict__ np2s, int64_t n, int64_t m,
                                  int kmax, int64_t b1, int32_t *__restrict__ key) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const double th = Av[u * kmax + kmax - 1];
    int32_t kk = 0;
    if (b1 < m && !cs_below(nu2[u], np2s[b1 - 1], th))
        kk = (int32_t)(first_below(nu2[u], np2s, b1 + 1, m, th) + 1 - b1);
    key[u] = kk;
}

void launch_budget_classify(const double *Av, const double *nu2, const double *np2s, int64_t n,
                            int64_t m, int kmax, int64_t b1, int32_t *key, hipStream_t st) {
    RMIPS_PROF(st, "k_budget_classify");
    k_budget_classify<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(Av, nu2, np2s, n, m, kmax,
                                                                    b1, key);
}

// The natural stop of the scan of user users[r] (in U''s rank order): the
// first position after b1 whose Eq. (2) bound is below the user's exact
// k_max-th value topv[r * kmax + kmax - 1]; m + 1 when there is none.  A
// scan from position 1 stops exactly there (every earlier stop would need
// a bound below a smaller running threshold).
__global__ void k_budget_tstop(const int32_t *__restrict__ users,
                               const double *__restrict__ topv, const double *__restrict__ nu2,
                               const double *__restrict__ np2s, int64_t X, int64_t m, int kmax,
                               int64_t b1, int32_t *__restrict__ t) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= X) return;
    t[r] = (int32_t)first_below(nu2[users[r]], np2s, b1 + 1, m, topv[r * kmax + kmax - 1]);
}

void launch_budget_tstop(const int32_t *users, const double *topv, const double *nu2,
                         const double *np2s, int64_t X, int64_t m, int kmax, int64_t b1,
                         int32_t *t, hipStream_t st) {
    if (X <= 0) return;
    RMIPS_PROF(st, "k_budget_tstop");
    k_budget_tstop<<<(unsigned)((X + 255) / 256), 256, 0, st>>>(users, topv, nu2, np2s, X, m,
                                                                 kmax, b1, t);
}

// rows r of (topv, topk) into the lists of users[r] whose pos is 0 (their
// scan ended within the budget, so the exact lists are theirs)
__global__ void k_budget_scatter(const int32_t *__restrict__ users,
                                 const int32_t *__restrict__ pos,
                                 const double *__restrict__ topv,
                                 const int32_t *__restrict__ topk, int64_t X, int kmax,
                                 double *__restrict__ Av, int32_t *__restrict__ Aj) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= X * kmax) return;
    const int64_t r = i / kmax;
    const int64_t u = users[r];
    if (pos[u] != 0) return;
    const int c = (int)(i - r * kmax);
    Av[u * kmax + c] = topv[i];
    Aj[u * kmax + c] = topk[i];
}

void launch_budget_scatter(const int32_t *users, const int32_t *pos, const double *topv,
                           const int32_t *topk, int64_t X, int kmax, double *Av, int32_t *Aj,
                           hipStream_t st) {
    if (X <= 0) return;
    RMIPS_PROF(st, "k_budget_scatter");
    k_budget_scatter<<<(unsigned)((X * kmax + 255) / 256), 256, 0, st>>>(users, pos, topv, topk,
                                                                          X, kmax, Av, Aj);
}

// ---------------------------------------------------------------- step 5
// For each user of U'' (users[w]): positions pos + 1.. until the first
// whose Eq. (2) bound is below the user's k_max-th value; each gets the
// Eq. (3) bound lam, the user's lambda (Eq. 7) is their maximum (-inf if
// none), and the item counts for every k with lam >= A^k: those k form a
// tail k0..kmax of 1..kmax (the list falls with k), so one count goes to
// row k0 - 1 of the difference table diff (kmax x m, by item id).
__global__ void k_budget_step5(const int32_t *__restrict__ users,
                               const int32_t *__restrict__ pos, int64_t nusers,
                               const double *__restrict__ Av, const double *__restrict__ nu2,
                               const double *__restrict__ Ul, const double *__restrict__ nru,
                               const double *__restrict__ nun,
                               const double *__restrict__ np2s, const double *__restrict__ Pl,
                               const double *__restrict__ nrp, const double *__restrict__ npn,
                               const int32_t *__restrict__ order, int64_t m, int kmax, int dp,
                               double *__restrict__ lam, int32_t *__restrict__ diff) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nusers) return;
    const int64_t u = users[w];
    const double *A = Av + u * kmax;
    const double thk = A[kmax - 1];
    double ul[BUDGET_DP_MAX];
#pragma unroll
    for (int t = 0; t < BUDGET_DP_MAX; ++t) ul[t] = t < dp ? Ul[u * dp + t] : 0.0;
    const double nr = nru[u], nn = nun[u], x2 = nu2[u];
    double best = -INFINITY;
    for (int64_t j = (int64_t)pos[u] + 1; j <= m; ++j) {
        if (cs_below(x2, np2s[j - 1], thk)) break;
        const double l = eq3_bound(ul, nr, nn, Pl + (j - 1) * dp, nrp[j - 1], npn[j - 1], dp);
        best = fmax(best, l);
        if (l >= thk) {
            // smallest k with l >= A^k
            int lo = 1, hi = kmax;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (l >= A[mid - 1])
                    hi = mid;
                else
                    lo = mid + 1;
            }
            atomicAdd(&diff[(int64_t)(lo - 1) * m + order[j - 1]], 1);
        }
    }
    lam[u] = best;
}

void launch_budget_step5(const int32_t *users, const int32_t *pos, int64_t nusers,
                         const double *Av, const double *nu2, const double *Ul,
                         const double *nru, const double *nun, const double *np2s,
                         const double *Pl, const double *nrp, const double *npn,
                         const int32_t *order, int64_t m, int kmax, int dp, double *lam,
                         int32_t *diff, hipStream_t st) {
    if (nusers <= 0) return;
    RMIPS_PROF(st, "k_budget_step5");
    k_budget_step5<<<(unsigned)((nusers + 127) / 128), 128, 0, st>>>(
        users, pos, nusers, Av, nu2, Ul, nru, nun, np2s, Pl, nrp, npn, order, m, kmax, dp, lam,
        diff);
}

// the first k entries of every list count for uscore_k: entry r counts for
// every k > r, i.e. one count in row r of the difference table
__global__ void k_budget_hist(const int32_t *__restrict__ Aj, int64_t n, int kmax, int64_t m,
                              int32_t *__restrict__ diff) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * kmax) return;
    const int r = (int)(i % kmax);
    atomicAdd(&diff[(int64_t)r * m + Aj[i]], 1);
}

void launch_budget_hist(const int32_t *Aj, int64_t n, int kmax, int64_t m, int32_t *diff,
                        hipStream_t st) {
    RMIPS_PROF(st, "k_budget_hist");
    k_budget_hist<<<(unsigned)((n * kmax + 255) / 256), 256, 0, st>>>(Aj, n, kmax, m, diff);
}

// uscore_k(p) = sum of rows 0..k-1 of the difference table (in place)
__global__ void k_budget_prefix_k(int32_t *__restrict__ t, int64_t m, int kmax) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    int32_t acc = 0;
    for (int k = 0; k < kmax; ++k) {
        acc += t[(int64_t)k * m + p];
        t[(int64_t)k * m + p] = acc;
    }
}

void launch_budget_prefix_k(int32_t *t, int64_t m, int kmax, hipStream_t st) {
    RMIPS_PROF(st, "k_budget_prefix_k");
    k_budget_prefix_k<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(t, m, kmax);
}

// ---------------------------------------------------------------- query
// Alg. 2's initialisation for k: a user whose k-th value is above lambda
// has S_k = the first k entries of its list (counted into base); the
// others are appended to X
__global__ void k_budget_xinit(const double *__restrict__ Av, const int32_t *__restrict__ Aj,
                               const double *__restrict__ lam, int64_t n, int kmax, int k,
                               int32_t *__restrict__ base, int32_t *__restrict__ X,
                               int32_t *__restrict__ xn) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    if (Av[u * kmax + k - 1] > lam[u]) {
        for (int r = 0; r < k; ++r) atomicAdd(&base[Aj[u * kmax + r]], 1);
    } else {
        X[atomicAdd(xn, 1)] = (int32_t)u;
    }
}

void launch_budget_xinit(const double *Av, const int32_t *Aj, const double *lam, int64_t n,
                         int kmax, int k, int32_t *base, int32_t *X, int32_t *xn,
                         hipStream_t st) {
    RMIPS_PROF(st, "k_budget_xinit");
    k_budget_xinit<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(Av, Aj, lam, n, kmax, k, base, X,
                                                                 xn);
}

// slot[bids[s]] = s for the batch
__global__ void k_budget_slots(const int32_t *__restrict__ bids, int nb,
                               int32_t *__restrict__ slot) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nb) slot[bids[s]] = s;
}

// Inc-RMIPS (Sec. 4.3) of every user of X against a batch of visited
// items.  Per user: an item of its first k entries whose value is above
// lambda is in; one whose value is not needs a rescan.  An unscanned item
// (position > pos) is out when Eq. (2), then Eq. (3), puts it below the
// k-th value, or when its exact value ranks after the k-th entry; else the
// user needs a rescan (the item is in only if its value exceeds lambda,
// which bounds it).  A user that needs a rescan is appended to R and
// counts nothing here; the others add their ins to the batch counts.
__global__ __launch_bounds__(256) void k_budget_inc(
    const int32_t *__restrict__ X, int64_t xn, const int32_t *__restrict__ bids, int nb,
    const int32_t *__restrict__ slot, const float *__restrict__ U,
    const float *__restrict__ P, int d, const double *__restrict__ Av,
    const int32_t *__restrict__ Aj, const double *__restrict__ lam,
    const int32_t *__restrict__ pos, const double *__restrict__ nu2,
    const double *__restrict__ Ul, const double *__restrict__ nru,
    const double *__restrict__ nun, const int32_t *__restrict__ posof,
    const double *__restrict__ np2s, const double *__restrict__ Pl,
    const double *__restrict__ nrp, const double *__restrict__ npn, int kmax, int k, int dp,
    int32_t *__restrict__ cnt, int32_t *__restrict__ R, int32_t *__restrict__ rn,
    uint8_t *__restrict__ xflag) {
    __shared__ int32_t s_pos[BUDGET_BATCH_MAX], s_id[BUDGET_BATCH_MAX];
    __shared__ double s_np2[BUDGET_BATCH_MAX], s_nrp[BUDGET_BATCH_MAX],
        s_npn[BUDGET_BATCH_MAX], s_pl[BUDGET_BATCH_MAX * BUDGET_DP_MAX];
    for (int s = threadIdx.x; s < nb; s += blockDim.x) {
        const int id = bids[s];
        const int j = posof[id];  // 0-based position
        s_pos[s] = j + 1;
        s_id[s] = id;
        s_np2[s] = np2s[j];
        s_nrp[s] = nrp[j];
        s_npn[s] = npn[j];
        for (int t = 0; t < dp; ++t) s_pl[s * BUDGET_DP_MAX + t] = Pl[(int64_t)j * dp + t];
    }
    __syncthreads();
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= xn) return;
    const int64_t u = X[w];
    const double *A = Av + u * kmax;
    const int32_t *Ajr = Aj + u * kmax;
    const double lu = lam[u], Ak = A[k - 1];
    const int idk = Ajr[k - 1];
    const int64_t pu = pos[u];
    bool rescan = false;
    // scanned items: the first k entries of the list
    for (int r = 0; r < k && !rescan; ++r) {
        const int s = slot[Ajr[r]];
        if (s >= 0 && !(lu < A[r])) rescan = true;
    }
    if (!rescan) {
        double ul[BUDGET_DP_MAX];
#pragma unroll
        for (int t = 0; t < BUDGET_DP_MAX; ++t) ul[t] = t < dp ? Ul[u * dp + t] : 0.0;
        const double x2 = nu2[u], nr = nru[u], nn = nun[u];
        for (int s = 0; s < nb; ++s) {
            if (s_pos[s] <= pu) continue;
            if (cs_below(x2, s_np2[s], Ak)) continue;
            if (eq3_bound(ul, nr, nn, s_pl + s * BUDGET_DP_MAX, s_nrp[s], s_npn[s], dp) < Ak)
                continue;
            const double v = ip64_rows(U + u * d, P + (int64_t)s_id[s] * d, d);
            if (!ranks_before(v, s_id[s], Ak, idk)) continue;
            rescan = true;
            break;
        }
    }
    if (rescan) {
        R[atomicAdd(rn, 1)] = (int32_t)u;
        xflag[u] = 1;
        return;
    }
    for (int r = 0; r < k; ++r) {
        const int s = slot[Ajr[r]];
        if (s >= 0) atomicAdd(&cnt[s], 1);
    }
}

void launch_budget_inc(const int32_t *X, int64_t xn, const int32_t *bids, int nb,
                       const int32_t *slot, const float *U, const float *P, int d,
                       const double *Av, const int32_t *Aj, const double *lam,
                       const int32_t *pos, const double *nu2, const double *Ul,
                       const double *nru, const double *nun, const int32_t *posof,
                       const double *np2s, const double *Pl, const double *nrp,
                       const double *npn, int kmax, int k, int dp, int32_t *cnt, int32_t *R,
                       int32_t *rn, uint8_t *xflag, hipStream_t st) {
    if (xn <= 0) return;
    RMIPS_PROF(st, "k_budget_inc");
    k_budget_inc<<<(unsigned)((xn + 255) / 256), 256, 0, st>>>(
        X, xn, bids, nb, slot, U, P, d, Av, Aj, lam, pos, nu2, Ul, nru, nun, posof, np2s, Pl,
        nrp, npn, kmax, k, dp, cnt, R, rn, xflag);
}

// a rescanned user's exact S_k (rows of topk): items not yet visited are
// credited now; the visited ones were decided exactly before
__global__ void k_budget_apply(const int32_t *__restrict__ topk, int64_t nr, int k,
                               const uint8_t *__restrict__ visited,
                               int32_t *__restrict__ base) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr * k) return;
    const int q = topk[i];
    if (!visited[q]) atomicAdd(&base[q], 1);
}

void launch_budget_apply(const int32_t *topk, int64_t nr, int k, const uint8_t *visited,
                         int32_t *base, hipStream_t st) {
    if (nr <= 0) return;
    RMIPS_PROF(st, "k_budget_apply");
    k_budget_apply<<<(unsigned)((nr * k + 255) / 256), 256, 0, st>>>(topk, nr, k, visited, base);
}

// X without the rescanned users, into Y (count in yn)
__global__ void k_budget_xcompact(const int32_t *__restrict__ X, int64_t xn,
                                  const uint8_t *__restrict__ xflag, int32_t *__restrict__ Y,
                                  int32_t *__restrict__ yn) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= xn) return;
    const int32_t u = X[w];
    if (!xflag[u]) Y[atomicAdd(yn, 1)] = u;
}

void launch_budget_xcompact(const int32_t *X, int64_t xn, const uint8_t *xflag, int32_t *Y,
                            int32_t *yn, hipStream_t st) {
    if (xn <= 0) return;
    RMIPS_PROF(st, "k_budget_xcompact");
    k_budget_xcompact<<<(unsigned)((xn + 255) / 256), 256, 0, st>>>(X, xn, xflag, Y, yn);
}

// the batch's scores (base + the counts of X), then the batch is visited
__global__ void k_budget_batch(const int32_t *__restrict__ bids, int nb,
                               const int32_t *__restrict__ base, int32_t *__restrict__ cnt,
                               uint8_t *__restrict__ visited, int32_t *__restrict__ slot,
                               int32_t *__restrict__ score) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nb) return;
    const int id = bids[s];
    score[s] = base[id] + cnt[s];
    cnt[s] = 0;
    visited[id] = 1;
    slot[id] = -1;
}

void launch_budget_slots(const int32_t *bids, int nb, int32_t *slot, hipStream_t st) {
    RMIPS_PROF(st, "k_budget_slots");
    k_budget_slots<<<1, BUDGET_BATCH_MAX, 0, st>>>(bids, nb, slot);
}

void launch_budget_batch(const int32_t *bids, int nb, const int32_t *base, int32_t *cnt,
                         uint8_t *visited, int32_t *slot, int32_t *score, hipStream_t st) {
    RMIPS_PROF(st, "k_budget_batch");
    k_budget_batch<<<1, BUDGET_BATCH_MAX, 0, st>>>(bids, nb, base, cnt, visited, slot, score);
}

// visit keys: ~uscore (ascending sort = descending uscore), ids as values
__global__ void k_budget_visit_keys(const int32_t *__restrict__ us, int64_t m,
                                    uint32_t *__restrict__ key, int32_t *__restrict__ val) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    key[p] = ~(uint32_t)us[p];
    val[p] = (int32_t)p;
}

void launch_budget_visit_keys(const int32_t *us, int64_t m, uint32_t *key, int32_t *val,
                              hipStream_t st) {
    RMIPS_PROF(st, "k_budget_visit_keys");
    k_budget_visit_keys<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(us, m, key, val);
}

// fills: int32 and double arrays
__global__ void k_fill_i32(int32_t *__restrict__ x, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}
__global__ void k_fill_f64(double *__restrict__ x, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

void launch_fill_i32(int32_t *x, int64_t n, int32_t v, hipStream_t st) {
    if (n <= 0) return;
    k_fill_i32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(x, n, v);
}
void launch_fill_f64(double *x, int64_t n, double v, hipStream_t st) {
    if (n <= 0) return;
    k_fill_f64<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(x, n, v);
}

}  // namespace rmips

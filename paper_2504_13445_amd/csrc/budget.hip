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
// lane, each value summed in index order by its lane (PgT holds the items
// transposed, d x m in position order, so the lanes' loads are adjacent);
// the step's keys are sorted across the wave and merged with the 64 best
// so far.
__global__ __launch_bounds__(256) void k_budget_prefix(
    const float *__restrict__ U, const float *__restrict__ PgT, int64_t m,
    const int32_t *__restrict__ order, int d, const int32_t *__restrict__ users,
    const int32_t *__restrict__ lims, int64_t lim0, int64_t nusers, int kmax,
    double *__restrict__ Av, int32_t *__restrict__ Aj) {
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
            const float *pc = PgT + q;
            double acc = 0.0;
            for (int i = 0; i < d; ++i)
                acc = __fma_rn((double)uu[i], (double)pc[(int64_t)i * m], acc);
            v = acc;
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

void launch_budget_prefix(const float *U, const float *PgT, int64_t m, const int32_t *order,
                          int d, const int32_t *users, const int32_t *lims, int64_t lim0,
                          int64_t nusers, int kmax, double *Av, int32_t *Aj, hipStream_t st) {
    if (nusers <= 0) return;
    RMIPS_PROF(st, "k_budget_prefix");
    k_budget_prefix<<<(unsigned)((nusers + 3) / 4), 256, 0, st>>>(
        U, PgT, m, order, d, users, lims, lim0, nusers, kmax, Av, Aj);
}

// PgT[i * m + q] = P[order[q] * d + i]: the items transposed, position order
__global__ void k_budget_transpose(const float *__restrict__ P, const int32_t *__restrict__ order,
                                   int64_t m, int d, float *__restrict__ PgT) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const float *p = P + (int64_t)order[q] * d;
    for (int i = 0; i < d; ++i) PgT[(int64_t)i * m + q] = p[i];
}

void launch_budget_transpose(const float *P, const int32_t *order, int64_t m, int d,
                             float *PgT, hipStream_t st) {
    RMIPS_PROF(st, "k_budget_transpose");
    k_budget_transpose<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(P, order, m, d, PgT);
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
// The range of step (5) for each user of U'' (users[w]): positions pos + 1
// up to, not including, the first whose Eq. (2) bound is below the user's
// k_max-th value (m + 1 if none): key[w] = that end, val[w] = the user.
__global__ void k_budget_range(const int32_t *__restrict__ users,
                               const int32_t *__restrict__ pos, int64_t nusers,
                               const double *__restrict__ Av, const double *__restrict__ nu2,
                               const double *__restrict__ np2s, int64_t m, int kmax,
                               uint32_t *__restrict__ key, int32_t *__restrict__ val) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nusers) return;
    const int64_t u = users[w];
    key[w] = (uint32_t)first_below(nu2[u], np2s, (int64_t)pos[u] + 1, m,
                                   Av[u * kmax + kmax - 1]);
    val[w] = (int32_t)u;
}

void launch_budget_range(const int32_t *users, const int32_t *pos, int64_t nusers,
                         const double *Av, const double *nu2, const double *np2s, int64_t m,
                         int kmax, uint32_t *key, int32_t *val, hipStream_t st) {
    if (nusers <= 0) return;
    RMIPS_PROF(st, "k_budget_range");
    k_budget_range<<<(unsigned)((nusers + 255) / 256), 256, 0, st>>>(users, pos, nusers, Av, nu2,
                                                                      np2s, m, kmax, key, val);
}

// Step (5) over those ranges, users sorted by the range's end (similar
// ranges share a wave).  Per tile of S5_TILE positions the items' Eq. (3)
// data sit in LDS and a wave's lanes (one user each) take the positions in
// step.  lambda (Eq. 7) is the largest bound over a user's range (-inf if
// empty).  An item counts for user u and every k with the bound >= A_u^k;
// per position the wave counts its lanes for each k (ballots), keeping the
// count for k in lane k - 1, and adds them to the tile's LDS table (row
// k - 1, no two lanes on one entry).  The table goes to the difference
// table diff (kmax x m, by item id) as differences of consecutive rows,
// once per tile.  A^k is compared rounded down to FP32: a lower threshold
// can only add counts, so uscore_k stays an upper bound (Theorem 3).
constexpr int S5_TILE = 256;
constexpr int S5_THREADS = 512;
__global__ __launch_bounds__(S5_THREADS) void k_budget_step5(
    const int32_t *__restrict__ users, const uint32_t *__restrict__ hi_pos,
    const int32_t *__restrict__ pos, int64_t nusers, const double *__restrict__ Av,
    const double *__restrict__ Ul, const double *__restrict__ nru,
    const double *__restrict__ nun, const double *__restrict__ Pl,
    const double *__restrict__ nrp, const double *__restrict__ npn,
    const int32_t *__restrict__ order, int64_t m, int kmax, int dp, double *__restrict__ lam,
    int32_t *__restrict__ diff) {
    __shared__ double t_pl[S5_TILE * BUDGET_DP_MAX];
    __shared__ double t_nrp[S5_TILE], t_npn[S5_TILE];
    __shared__ int32_t t_id[S5_TILE];
    __shared__ int32_t cnt[KMAX * S5_TILE];
    __shared__ int64_t s_lo, s_hi;
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t w = (int64_t)blockIdx.x * S5_THREADS + tid;
    const bool valid = w < nusers;
    int64_t u = 0, lo = INT64_MAX, hi = 0;
    if (valid) {
        u = users[w];
        lo = (int64_t)pos[u] + 1;
        hi = hi_pos[w];
    }
    if (tid == 0) {
        s_lo = INT64_MAX;
        s_hi = 0;
    }
    __syncthreads();
    if (valid && lo < hi) {
        atomicMin((unsigned long long *)&s_lo, (unsigned long long)lo);
        atomicMax((unsigned long long *)&s_hi, (unsigned long long)hi);
    }
    __syncthreads();
    const int64_t blo = s_lo, bhi = s_hi;
    double ul[BUDGET_DP_MAX];
#pragma unroll
    for (int t = 0; t < BUDGET_DP_MAX; ++t) ul[t] = (valid && t < dp) ? Ul[u * dp + t] : 0.0;
    const double nr = valid ? nru[u] : 0.0, nn = valid ? nun[u] : 0.0;
    float af[KMAX];
#pragma unroll
    for (int r = 0; r < KMAX; ++r)
        af[r] = (valid && r < kmax) ? __double2float_rd(Av[u * kmax + r]) : -INFINITY;
    const double thk = valid ? Av[u * kmax + kmax - 1] : INFINITY;
    double best = -INFINITY;
    for (int64_t t0 = blo; t0 < bhi; t0 += S5_TILE) {
        const int tn = (int)min<int64_t>(S5_TILE, m + 1 - t0);
        for (int i = tid; i < tn; i += S5_THREADS) {
            const int64_t j = t0 + i - 1;  // 0-based position
            t_id[i] = order[j];
            t_nrp[i] = nrp[j];
            t_npn[i] = npn[j];
            for (int t = 0; t < dp; ++t) t_pl[i * BUDGET_DP_MAX + t] = Pl[j * dp + t];
        }
        for (int e = tid; e < kmax * S5_TILE; e += S5_THREADS) cnt[e] = 0;
        __syncthreads();
        // the wave's positions: the union of its lanes' ranges in the tile
        int64_t wa = valid ? max(lo, t0) : INT64_MAX, wb = valid ? min(hi, t0 + tn) : 0;
        for (int o = 32; o > 0; o >>= 1) {
            wa = min(wa, __shfl_xor(wa, o));
            wb = max(wb, __shfl_xor(wb, o));
        }
        for (int64_t j = wa; j < wb; ++j) {
            const int i = (int)(j - t0);
            const bool act = valid && j >= lo && j < hi;
            int k0 = KMAX + 1;
            if (act) {
                const double l =
                    eq3_bound(ul, nr, nn, t_pl + i * BUDGET_DP_MAX, t_nrp[i], t_npn[i], dp);
                best = fmax(best, l);
                if (l >= thk) {
                    // af[r] > lf >= l: a lower count, so a smaller k0 (safe)
                    const float lf = __double2float_ru(l);
                    k0 = 1;
#pragma unroll
                    for (int r = 0; r < KMAX; ++r) k0 += (af[r] > lf) ? 1 : 0;
                }
            }
            if (__ballot(k0 <= kmax) == 0) continue;
            int mine = 0;
            for (int k = 1; k <= kmax; ++k) {
                const int c = __popcll(__ballot(k0 <= k));
                if (lane == k - 1) mine = c;
            }
            if (lane < kmax && mine) atomicAdd(&cnt[lane * S5_TILE + i], mine);
        }
        __syncthreads();
        for (int e = tid; e < kmax * S5_TILE; e += S5_THREADS) {
            const int r = e / S5_TILE, i = e - r * S5_TILE;
            const int c = cnt[e] - (r ? cnt[e - S5_TILE] : 0);
            if (c && i < tn) atomicAdd(&diff[(int64_t)r * m + t_id[i]], c);
        }
        __syncthreads();
    }
    if (valid) lam[u] = best;
}

void launch_budget_step5(const int32_t *users, const uint32_t *hi_pos, const int32_t *pos,
                         int64_t nusers, const double *Av, const double *Ul, const double *nru,
                         const double *nun, const double *Pl, const double *nrp,
                         const double *npn, const int32_t *order, int64_t m, int kmax, int dp,
                         double *lam, int32_t *diff, hipStream_t st) {
    if (nusers <= 0) return;
    RMIPS_PROF(st, "k_budget_step5");
    k_budget_step5<<<(unsigned)((nusers + S5_THREADS - 1) / S5_THREADS), S5_THREADS, 0, st>>>(
        users, hi_pos, pos, nusers, Av, Ul, nru, nun, Pl, nrp, npn, order, m, kmax, dp, lam,
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
// k-th value; any other unscanned item needs a rescan.  (The paper first
// computes that pair's exact value, which can still rule it out; here the
// rescan, one screened stage (a) pass for all flagged users, settles the
// user's S_k for every later batch at once and costs less than exact
// products against each of them.)  A user that needs a rescan is appended
// to R and counts nothing here; the others add their ins to the counts.
__global__ __launch_bounds__(256) void k_budget_inc(
    const int32_t *__restrict__ X, int64_t xn, const int32_t *__restrict__ bids, int nb,
    const int32_t *__restrict__ slot, const double *__restrict__ Av,
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
                       const int32_t *slot, const double *Av, const int32_t *Aj, const double *lam,
                       const int32_t *pos, const double *nu2, const double *Ul,
                       const double *nru, const double *nun, const int32_t *posof,
                       const double *np2s, const double *Pl, const double *nrp,
                       const double *npn, int kmax, int k, int dp, int32_t *cnt, int32_t *R,
                       int32_t *rn, uint8_t *xflag, hipStream_t st) {
    if (xn <= 0) return;
    RMIPS_PROF(st, "k_budget_inc");
    k_budget_inc<<<(unsigned)((xn + 255) / 256), 256, 0, st>>>(
        X, xn, bids, nb, slot, Av, Aj, lam, pos, nu2, Ul, nru, nun, posof, np2s, Pl,
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
    k_budget_slots<<<(nb + 255) / 256, 256, 0, st>>>(bids, nb, slot);
}

void launch_budget_batch(const int32_t *bids, int nb, const int32_t *base, int32_t *cnt,
                         uint8_t *visited, int32_t *slot, int32_t *score, hipStream_t st) {
    RMIPS_PROF(st, "k_budget_batch");
    k_budget_batch<<<(nb + 255) / 256, 256, 0, st>>>(bids, nb, base, cnt, visited, slot, score);
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

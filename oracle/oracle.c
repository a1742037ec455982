/*
 * Plain, slow, obviously correct CPU FP64 oracle for reverse k-MIPS top-N.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links or calls this;
 * only the tests, the smoke check and the CPU baseline of the benchmark do.
 *
 * The exact value of an inner product is defined here (the paper leaves
 * the arithmetic unspecified, Sec. 5.1): inputs are FP32, each product
 * (double)u_i * (double)p_i is exact in FP64, and the products are added
 * in FP64 in index order starting from +0.0.  Every decision below is
 * taken on that value.
 *
 * Ties: k-MIPS (Def. 1) and top-N (Def. 3) break ties arbitrarily in the
 * paper; here ties are ordered by (value descending, item index ascending)
 * and (score descending, item index ascending).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Def. 1: inner product u . p, FP64, summed in index order from +0.0. */
static double ip64(const float *u, const float *p, int d)
{
    double acc = 0.0;
    for (int i = 0; i < d; ++i)
        acc += (double)u[i] * (double)p[i];
    return acc;
}

/* The same sum for nb <= 4 consecutive item rows; each value is its own
 * index-ordered chain, identical to ip64 (the chains are only interleaved). */
static void ip64_block(const float *u, const float *p, int d, int nb, double *v)
{
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (nb == 4) {
        for (int i = 0; i < d; ++i) {
            double ui = (double)u[i];
            a0 += ui * (double)p[i];
            a1 += ui * (double)p[d + i];
            a2 += ui * (double)p[2 * d + i];
            a3 += ui * (double)p[3 * d + i];
        }
        v[0] = a0; v[1] = a1; v[2] = a2; v[3] = a3;
        return;
    }
    for (int b = 0; b < nb; ++b)
        v[b] = ip64(u, p + b * d, d);
}

/* Full n x m matrix of exact inner products (small inputs only). */
void orc_inner_products(const float *U, const float *P, int64_t n, int64_t m,
                        int d, double *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t u = 0; u < n; ++u)
        for (int64_t j = 0; j < m; ++j)
            out[u * m + j] = ip64(U + u * d, P + j * d, d);
}

/*
 * Def. 1 (k-MIPS) for every user: a linear scan over the items in index
 * order keeping the k best by (value desc, index asc).  Because items
 * arrive in increasing index, a new item with a value equal to the k-th
 * kept one ranks after it and is not inserted.
 *   tau[u]    = value of the k-th element,
 *   tau_id[u] = its item index,
 *   topk[u*k + r] = item index of the r-th element (may be NULL),
 *   topv[u*k + r] = its value (may be NULL): the r-th largest value, which
 *                   is the threshold of S_{r+1}(u), so one scan with k =
 *                   k_max gives the thresholds of every k <= k_max (the
 *                   per-user lists A_i of Alg. 1, Sec. 4.2).
 */
void orc_kmips(const float *U, const float *P, int64_t n, int64_t m, int d,
               int k, double *tau, int32_t *tau_id, int32_t *topk, double *topv)
{
#pragma omp parallel
    {
        double *bv = (double *)malloc(sizeof(double) * (size_t)k);
        int32_t *bj = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
#pragma omp for schedule(dynamic, 8)
        for (int64_t u = 0; u < n; ++u) {
            const float *uu = U + u * d;
            int cnt = 0;
            for (int64_t j0 = 0; j0 < m; j0 += 4) {
              /* four items at a time, each summed on its own in index order */
              double v4[4];
              int nb = (m - j0 < 4) ? (int)(m - j0) : 4;
              ip64_block(uu, P + j0 * d, d, nb, v4);
              for (int b = 0; b < nb; ++b) {
                int64_t j = j0 + b;
                double v = v4[b];
                if (cnt == k && !(v > bv[k - 1]))
                    continue;
                /* insertion position: after every kept entry with value >= v */
                int pos = (cnt < k) ? cnt : k - 1;
                while (pos > 0 && bv[pos - 1] < v) {
                    bv[pos] = bv[pos - 1];
                    bj[pos] = bj[pos - 1];
                    --pos;
                }
                bv[pos] = v;
                bj[pos] = (int32_t)j;
                if (cnt < k)
                    ++cnt;
              }
            }
            tau[u] = bv[k - 1];
            tau_id[u] = bj[k - 1];
            if (topk)
                for (int r = 0; r < k; ++r)
                    topk[u * k + r] = bj[r];
            if (topv)
                for (int r = 0; r < k; ++r)
                    topv[u * k + r] = bv[r];
        }
        free(bv);
        free(bj);
    }
}

/*
 * Def. 2 / Eq. (1): |T_k(q)| for query items q against users whose k-th
 * neighbour is (tau[u], tau_id[u]).  Item q with index j belongs to
 * S_k(u) iff (v, -j) >= (tau_u, -tau_id_u) lexicographically.  A query
 * with q_ids[i] < 0 is an item outside P, taken to have the largest index
 * so that it loses every tie: it is counted iff v > tau_u.
 */
void orc_reverse_counts(const float *U, int64_t n, int d, const double *tau,
                        const int32_t *tau_id, const float *Q,
                        const int32_t *q_ids, int64_t nq, int32_t *out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nq; ++i) {
        const float *q = Q + i * d;
        int64_t c = 0;
        for (int64_t u = 0; u < n; ++u) {
            double v = ip64(U + u * d, q, d);
            if (v > tau[u])
                ++c;
            else if (v == tau[u] && q_ids[i] >= 0 && q_ids[i] <= tau_id[u])
                ++c;
        }
        out[i] = (int32_t)c;
    }
}

/* l2 norm in FP64 of an FP32 vector, summed in index order. */
static double norm64(const float *x, int d)
{
    double s = 0.0;
    for (int i = 0; i < d; ++i)
        s += (double)x[i] * (double)x[i];
    return sqrt(s);
}

/*
 * Eq. (2) bound count: uscore_cs[j] = #{u : ||u|| ||p_j|| (1+s) >= tau_u},
 * the Cauchy-Schwarz upper bound on score(p_j) (Sec. 4.1) taken with the
 * exact k-th values tau_u, in FP64; the relative slack s keeps it a bound
 * where the inequality is tight.
 */
void orc_uscore_cs(const float *U, const float *P, int64_t n, int64_t m,
                   int d, const double *tau, double rel_slack, int32_t *out)
{
    double *nu = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t u = 0; u < n; ++u)
        nu[u] = norm64(U + u * d, d);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < m; ++j) {
        double np_ = norm64(P + j * d, d);
        int64_t c = 0;
        for (int64_t u = 0; u < n; ++u)
            if (nu[u] * np_ * (1.0 + rel_slack) >= tau[u])
                ++c;
        out[j] = (int32_t)c;
    }
    free(nu);
}

/* ==========================================================================
 * Alg. 1 (Sec. 4.2): the offline stage under an inner-product budget.
 *
 * Positions j = 1..m refer to the items in descending order of norm (ties
 * by item index), as Alg. 1 assumes after its first two lines.  A user's
 * list A_i holds its k_max best items seen so far in the tie order
 * (value desc, item index asc); theta is the value of its k_max-th entry,
 * -inf while the list is not full.
 *
 * Readings of the listing (each one also in the design notes):
 *  - Every "cannot be in the result" test is strict, so that an item whose
 *    value equals the threshold and whose index is smaller is never lost:
 *    the scans stop at the first item whose Cauchy-Schwarz bound (Eq. 2) is
 *    certainly below theta, and Eq. (3) skips an inner product only when
 *    its bound is below theta.
 *  - Eq. (2) is tested in squares with a relative slack,
 *        cs_below(u, p, theta) := theta > 0 and (|u|^2 |p|^2) (1 + 2^-36) < theta^2,
 *    where |x|^2 is the FP64 sum of squares in index order; it implies that
 *    the FP64 value u . p is below theta for d <= 4096.
 *  - theta starts at -inf (the listing's 0 would never admit negative values).
 *  - A scan that reaches the end of P (the virtual position m + 1) stops
 *    there: the user's list is then exact.
 *  - Step 4 pools what a user leaves unused (the listing's B' update) and a
 *    user that runs out of budget consumes the pool (B' = 0 after it).
 *  - lambda_i starts at -inf; users outside U'' keep lambda_i = -inf.
 *  - In step 5 the scan of a user of U'' ends at the first item whose
 *    Cauchy-Schwarz bound is below the user's own k_max-th value.
 *  - x_i is the 1-based rank in U' ordered by (j' + 1 - b1 asc, user asc);
 *    the budget of a user of U' is floor(f(x_i)), at most 2^40.
 * ========================================================================== */

#define CS_SQ_SLACK (1.0 + 0x1p-36)

static int cs_below(double nu2, double np2, double theta)
{
    return theta > 0.0 && (nu2 * np2) * CS_SQ_SLACK < theta * theta;
}

static double sqsum64(const float *x, int d)
{
    double s = 0.0;
    for (int i = 0; i < d; ++i)
        s += (double)x[i] * (double)x[i];
    return s;
}

/* insert (v, id) into a list sorted by (value desc, id asc) holding *cnt of
 * at most cap entries; an entry that ranks after a full list is dropped */
static void list_insert(double *Lv, int32_t *Lj, int *cnt, int cap, double v, int32_t id)
{
    if (*cnt == cap && !(v > Lv[cap - 1] || (v == Lv[cap - 1] && id < Lj[cap - 1])))
        return;
    int pos = (*cnt < cap) ? *cnt : cap - 1;
    while (pos > 0 && (Lv[pos - 1] < v || (Lv[pos - 1] == v && Lj[pos - 1] > id))) {
        Lv[pos] = Lv[pos - 1];
        Lj[pos] = Lj[pos - 1];
        --pos;
    }
    Lv[pos] = v;
    Lj[pos] = id;
    if (*cnt < cap)
        ++*cnt;
}

/* Eq. (3): u^l . p^l + |u^r| |p^r| on rotated coordinates, plus a slack
 * s |u| |p| covering the rounding of the rotation and of the sums */
static double eq3_bound(const double *ul, double nru, double nu, const double *pl,
                        double nrp, double np_, int dp, double s)
{
    double acc = 0.0;
    for (int t = 0; t < dp; ++t)
        acc += ul[t] * pl[t];
    return acc + nru * nrp + s * (nu * np_);
}

/* Eq. (5): alpha (exp(beta X) - 1) / beta + gamma X = B2, solved for beta
 * by bisection (the left side increases with beta); -inf when no beta
 * reaches B2 (B2 <= gamma X), so that f(x) = gamma. */
static double budget_beta(double X, double B2, double alpha, double gamma)
{
    double target = B2 - gamma * X;
    if (!(target > 0.0) || !(alpha > 0.0))
        return -INFINITY;
#define G_OF(b) ((b) == 0.0 ? alpha * X : alpha * expm1((b) * X) / (b))
    double lo, hi;
    if (G_OF(0.0) == target)
        return 0.0;
    if (G_OF(0.0) < target) {
        lo = 0.0;
        hi = 1.0 / X;
        while (G_OF(hi) < target)
            hi *= 2.0;
    } else {
        hi = 0.0;
        lo = -1.0 / X;
        while (G_OF(lo) > target)
            lo *= 2.0;
    }
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi)
            break;
        if (G_OF(mid) < target)
            lo = mid;
        else
            hi = mid;
    }
#undef G_OF
    return 0.5 * (lo + hi);
}

/* the budget of the user of rank x (1-based) among X users of U':
 * kind 0 = Eq. (4), 1 = uniform, 2 = linear, 3 = quadratic (Sec. 5.2's
 * comparison); each integrates to B2 over [0, X] */
static int64_t budget_of(int kind, double x, double X, double B2, double alpha,
                         double beta, double gamma)
{
    double f;
    if (kind == 0)
        f = alpha * exp(beta * x) + gamma;
    else if (kind == 1)
        f = B2 / X;
    else if (kind == 2)
        f = 2.0 * B2 * x / (X * X);
    else
        f = 3.0 * B2 * x * x / (X * X * X);
    if (!(f > 0.0))
        return 0;
    if (f >= 1099511627776.0)
        return 1099511627776LL;
    return (int64_t)floor(f);
}

typedef struct {
    int64_t n;
    int64_t key;
} orc_ukey;

static int cmp_ukey(const void *a, const void *b)
{
    const orc_ukey *x = (const orc_ukey *)a, *y = (const orc_ukey *)b;
    if (x->key != y->key)
        return x->key < y->key ? -1 : 1;
    return x->n < y->n ? -1 : (x->n > y->n);
}

static const double *g_np2_sort;
static int cmp_item_norm(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    if (g_np2_sort[x] != g_np2_sort[y])
        return g_np2_sort[x] > g_np2_sort[y] ? -1 : 1;
    return x < y ? -1 : (x > y);
}

/* one inner product of the scan: Eq. (3)'s test first when the list is
 * full, then the exact value and the list update; returns 1 when computed */
static int scan_item(const float *uu, const float *P, int d, int32_t p, double *Lv,
                     int32_t *Lj, int *cnt, int kmax, const double *ul, double nru,
                     double nu, const double *pl, const double *nrp, const double *npn,
                     int dp, double s)
{
    if (*cnt == kmax) {
        double lam = eq3_bound(ul, nru, nu, pl + (int64_t)p * dp, nrp[p], npn[p], dp, s);
        if (lam < Lv[kmax - 1])
            return 0;
    }
    list_insert(Lv, Lj, cnt, kmax, ip64(uu, P + (int64_t)p * d, d), p);
    return 1;
}

/*
 * Alg. 1.  Inputs: U (n x d), P (m x d), k_max, b1 = B1/n (kmax <= b1),
 * the dynamic budget B2, the budget kind, alpha and gamma of Eq. (4), and
 * the rotated coordinates of Eq. (3) computed by the caller with one
 * orthogonal matrix: ul (n x dp), pl (m x dp), the norms of the remaining
 * coordinates nru, nrp, and the norms nu, npn, with the slack s.
 * Outputs:
 *   order[m]          item indices in the norm order (position j is order[j-1]);
 *   Av, Aj [n x kmax] the lists A_i (values, item indices);
 *   pos[n]            pos_i for users of U'', else 0;
 *   lam[n]            lambda_i (Eq. 7) for users of U'', else -inf;
 *   uscore[kmax x m]  uscore_k(p) for k = 1..kmax (row k-1, by item index);
 *   key[n]            j' + 1 - b1 for users of U', else 0;
 *   rank[n]           x_i for users of U', else 0;
 *   b2[n]             B_{2,i} for users of U', else 0;
 *   info[8]           |U'|, |U''|, beta, inner products of step 3,
 *                     inner products of step 4, positions scanned in step 4,
 *                     users certified in step 3, users certified in step 4.
 */
int orc_budget_pre(const float *U, const float *P, int64_t n, int64_t m, int d, int kmax,
                   int64_t b1, int64_t B2, int kind, double alpha, double gamma,
                   const double *ul, const double *nru, const double *nu,
                   const double *pl, const double *nrp, const double *npn, int dp,
                   double s, int32_t *order, double *Av, int32_t *Aj, int64_t *pos,
                   double *lam, int32_t *uscore, int64_t *key, int64_t *rank,
                   int64_t *b2, double *info)
{
    if (kmax < 1 || kmax > m || b1 < kmax || n < 1 || d < 1)
        return 1;
    if (b1 > m)
        b1 = m;
    double *nu2 = (double *)malloc(sizeof(double) * (size_t)n);
    double *np2 = (double *)malloc(sizeof(double) * (size_t)m);
    int *cnt = (int *)malloc(sizeof(int) * (size_t)n);
    /* (1) norms, then the items in descending order of norm */
    for (int64_t u = 0; u < n; ++u)
        nu2[u] = sqsum64(U + u * d, d);
    for (int64_t j = 0; j < m; ++j) {
        np2[j] = sqsum64(P + j * d, d);
        order[j] = (int32_t)j;
    }
    g_np2_sort = np2;
    qsort(order, (size_t)m, sizeof(int32_t), cmp_item_norm);
    /* (3) uniform budget: the first b1 positions for every user */
    int64_t ips3 = 0, cert3 = 0;
    for (int64_t u = 0; u < n; ++u) {
        const float *uu = U + u * d;
        double *Lv = Av + u * kmax;
        int32_t *Lj = Aj + u * kmax;
        int c = 0, broke = 0;
        pos[u] = 0;
        lam[u] = -INFINITY;
        key[u] = 0;
        rank[u] = 0;
        b2[u] = 0;
        for (int64_t j = 1; j <= b1; ++j) {
            int32_t p = order[j - 1];
            double theta = (c == kmax) ? Lv[kmax - 1] : -INFINITY;
            if (cs_below(nu2[u], np2[p], theta)) {
                broke = 1;
                break;
            }
            ips3 += scan_item(uu, P, d, p, Lv, Lj, &c, kmax, ul + u * dp, nru[u], nu[u], pl,
                              nrp, npn, dp, s);
        }
        cnt[u] = c;
        if (broke || b1 == m) {
            ++cert3;
            continue;
        }
        /* j': the first position whose bound is below theta (binary search,
         * the bound falls with the position), m + 1 when there is none */
        double theta = Lv[kmax - 1];
        int64_t lo = b1 + 1, hi = m + 1;
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (cs_below(nu2[u], np2[order[mid - 1]], theta))
                hi = mid;
            else
                lo = mid + 1;
        }
        key[u] = lo + 1 - b1;
    }
    /* U' in ascending order of j' + 1 - b1; beta of Eq. (5) */
    int64_t X = 0;
    for (int64_t u = 0; u < n; ++u)
        X += key[u] > 0;
    orc_ukey *ux = (orc_ukey *)malloc(sizeof(orc_ukey) * (size_t)(X > 0 ? X : 1));
    for (int64_t u = 0, t = 0; u < n; ++u)
        if (key[u] > 0) {
            ux[t].n = u;
            ux[t].key = key[u];
            ++t;
        }
    qsort(ux, (size_t)X, sizeof(orc_ukey), cmp_ukey);
    double beta = (kind == 0 && X > 0) ? budget_beta((double)X, (double)B2, alpha, gamma) : 0.0;
    /* (4) dynamic budget, in that order, with the pooled budget B' */
    int64_t Bp = 0, ips4 = 0, scanned4 = 0, cert4 = 0, nU2 = 0;
    for (int64_t t = 0; t < X; ++t) {
        int64_t u = ux[t].n;
        const float *uu = U + u * d;
        double *Lv = Av + u * kmax;
        int32_t *Lj = Aj + u * kmax;
        rank[u] = t + 1;
        b2[u] = budget_of(kind, (double)(t + 1), (double)X, (double)B2, alpha, beta, gamma);
        int64_t e = b1 + 1 + b2[u] + Bp;
        int64_t brk = 0;
        for (int64_t j = b1 + 1; j <= e; ++j) {
            if (j == m + 1) {
                brk = j;
                break;
            }
            int32_t p = order[j - 1];
            if (cs_below(nu2[u], np2[p], Lv[kmax - 1])) {
                brk = j;
                break;
            }
            ++scanned4;
            ips4 += scan_item(uu, P, d, p, Lv, Lj, &cnt[u], kmax, ul + u * dp, nru[u], nu[u],
                              pl, nrp, npn, dp, s);
        }
        if (brk) {
            Bp = e - brk;
            ++cert4;
        } else {
            pos[u] = e;
            Bp = 0;
            ++nU2;
        }
    }
    /* (5) upper-bound scores: Eq. (6) over the unscanned positions of the
     * users of U'', then the first k entries of every list */
    memset(uscore, 0, sizeof(int32_t) * (size_t)kmax * (size_t)m);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t u = 0; u < n; ++u) {
        if (pos[u] == 0)
            continue;
        const double *Lv = Av + u * kmax;
        double best = -INFINITY;
        for (int64_t j = pos[u] + 1; j <= m; ++j) {
            int32_t p = order[j - 1];
            if (cs_below(nu2[u], np2[p], Lv[kmax - 1]))
                break;
            double l = eq3_bound(ul + u * dp, nru[u], nu[u], pl + (int64_t)p * dp, nrp[p],
                                 npn[p], dp, s);
            if (l > best)
                best = l;
            for (int k = 1; k <= kmax; ++k)
                if (l >= Lv[k - 1]) {
#pragma omp atomic
                    uscore[(int64_t)(k - 1) * m + p] += 1;
                }
        }
        lam[u] = best;
    }
    for (int64_t u = 0; u < n; ++u)
        for (int k = 1; k <= kmax; ++k)
            for (int r = 0; r < k; ++r)
                uscore[(int64_t)(k - 1) * m + Aj[u * kmax + r]] += 1;
    info[0] = (double)X;
    info[1] = (double)nU2;
    info[2] = beta;
    info[3] = (double)ips3;
    info[4] = (double)ips4;
    info[5] = (double)scanned4;
    info[6] = (double)cert3;
    info[7] = (double)cert4;
    free(ux);
    free(cnt);
    free(np2);
    free(nu2);
    return 0;
}

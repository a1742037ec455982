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

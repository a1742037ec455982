"""Plain, slow, obviously correct FP64 oracle (test infrastructure only).

Each function restates a definition of the paper "How to Mine Potentially
Popular Items? A Reverse MIPS-based Approach" (Amagata et al.) in numpy or
calls the plain C in oracle.c for sizes numpy cannot hold.

Exact value of an inner product (the paper leaves precision open): FP32
inputs up-cast to FP64, products exact, summed in index order from +0.0.
Ties: (value desc, item index asc) for k-MIPS, (score desc, item index asc)
for top-N.  See the functions for the passage each follows.

parity unpinned: none -- every function is pinned by tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "inner_products", "inner_products_c", "kmips", "kmips_c", "kmips_table",
    "kmips_table_c", "topn_from_table", "histogram_scores",
    "reverse_counts", "reverse_counts_c", "topn_from_scores", "topn",
    "uscore_cs", "uscore_cs_c", "uscore_eq3", "topn_bound_ordered",
    "temperature", "soft_score", "soft_grad", "sigmoid",
    "budget_rotation", "budget_preprocess", "budget_query", "BUDGET_KINDS",
]

# --------------------------------------------------------------------- C part
_lib = None


def _c():
    global _lib
    if _lib is None:
        from .build import LIB, build
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64, i32 = ctypes.c_int64, ctypes.c_int
        lib.orc_inner_products.argtypes = [f32p, f32p, i64, i64, i32, f64p]
        lib.orc_kmips.argtypes = [f32p, f32p, i64, i64, i32, i32, f64p, i32p,
                                  ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_reverse_counts.argtypes = [f32p, i64, i32, f64p, i32p, f32p,
                                           i32p, i64, i32p]
        lib.orc_uscore_cs.argtypes = [f32p, f32p, i64, i64, i32, f64p,
                                      ctypes.c_double, i32p]
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        dbl = ctypes.c_double
        lib.orc_budget_pre.restype = ctypes.c_int
        lib.orc_budget_pre.argtypes = [f32p, f32p, i64, i64, i32, i32, i64, i64, i32, dbl,
                                       dbl, f64p, f64p, f64p, f64p, f64p, f64p, i32, dbl,
                                       i32p, f64p, i32p, i64p, f64p, i32p, i64p, i64p,
                                       i64p, f64p]
        _lib = lib
    return _lib


def _f32(x):
    return np.ascontiguousarray(x, dtype=np.float32)


# ------------------------------------------------------------ definitions
def inner_products(U, P):
    """All u . p (Def. 1) in FP64: acc += u_i * p_i for i = 0..d-1, acc0 = +0.

    Vectorised over (u, p) pairs, sequential over i, exactly as the
    definition reads.  Small inputs only (n*m doubles)."""
    U = _f32(U).astype(np.float64)
    P = _f32(P).astype(np.float64)
    acc = np.zeros((U.shape[0], P.shape[0]), dtype=np.float64)
    for i in range(U.shape[1]):
        acc += U[:, i, None] * P[None, :, i]
    return acc


def inner_products_c(U, P):
    """inner_products in plain C."""
    U, P = _f32(U), _f32(P)
    out = np.empty((U.shape[0], P.shape[0]), np.float64)
    _c().orc_inner_products(U, P, U.shape[0], P.shape[0], U.shape[1], out)
    return out


def _order_desc_id_asc(v):
    """Row-wise item order by (value desc, index asc): a full sort."""
    m = v.shape[1]
    ids = np.broadcast_to(np.arange(m), v.shape)
    return np.lexsort((ids, -v), axis=-1)


def kmips(U, P, k, V=None):
    """Def. 1: S_k(u) for every user, by fully sorting each user's row.

    Returns (tau, tau_id, topk): tau[u] is the k-th largest value, tau_id[u]
    the item index at that position, topk[u] the k item indices in order."""
    if V is None:
        V = inner_products(U, P)
    order = _order_desc_id_asc(V)
    topk = order[:, :k].astype(np.int32)
    tau_id = topk[:, k - 1].copy()
    tau = V[np.arange(V.shape[0]), tau_id]
    return tau, tau_id, topk


def kmips_c(U, P, k, with_topk=True):
    """Def. 1 by a linear scan per user in plain C (large inputs)."""
    U, P = _f32(U), _f32(P)
    n, d = U.shape
    m = P.shape[0]
    tau = np.empty(n, np.float64)
    tau_id = np.empty(n, np.int32)
    topk = np.empty((n, k), np.int32) if with_topk else None
    _c().orc_kmips(U, P, n, m, d, k, tau, tau_id,
                   topk.ctypes.data if with_topk else None, None)
    return tau, tau_id, topk


def kmips_table(U, P, kmax, V=None):
    """Def. 1 for every k <= kmax at once (the per-user lists A_i of Alg. 1,
    Sec. 4.2, with k_max entries): by fully sorting each user's row,
    topv[u, r] is the (r+1)-th largest value and topk[u, r] its item index,
    so (topv[u, k-1], topk[u, k-1]) is (tau_u, tau_id_u) for k and
    topk[u, :k] is S_k(u)."""
    if V is None:
        V = inner_products(U, P)
    order = _order_desc_id_asc(V)
    topk = order[:, :kmax].astype(np.int32)
    topv = np.take_along_axis(V, topk.astype(np.int64), axis=1)
    return topv, topk


def kmips_table_c(U, P, kmax):
    """kmips_table by the linear scan in plain C (large inputs)."""
    U, P = _f32(U), _f32(P)
    n, d = U.shape
    m = P.shape[0]
    tau = np.empty(n, np.float64)
    tau_id = np.empty(n, np.int32)
    topk = np.empty((n, kmax), np.int32)
    topv = np.empty((n, kmax), np.float64)
    _c().orc_kmips(U, P, n, m, d, kmax, tau, tau_id, topk.ctypes.data, topv.ctypes.data)
    return topv, topk


def topn_from_table(topk_table, k, N, m):
    """Def. 3 for one k <= kmax from the k_max lists: S_k(u) is the first k
    entries of S_kmax(u) (the same tie order), then Baseline 1 and top-N."""
    return topn_from_scores(histogram_scores(np.asarray(topk_table)[:, :k], m), N)


def histogram_scores(topk, m):
    """Baseline 1 (Sec. 2.2): score(p) = number of users whose S_k holds p."""
    return np.bincount(np.asarray(topk).ravel(), minlength=m).astype(np.int64)


def reverse_counts(U, tau, tau_id, Q, q_ids=None, V=None):
    """Def. 2 / Eq. (1) per query item: |T_k(q)| = #{u : q in S_k(u)}.

    With the tie order above, item q of index j is in S_k(u) iff
    v > tau_u, or v == tau_u and j <= tau_id_u.  q_ids[i] < 0 marks an item
    outside P, placed after every item of P: counted iff v > tau_u."""
    Q = _f32(Q)
    if q_ids is None:
        q_ids = np.full(Q.shape[0], -1, np.int64)
    q_ids = np.asarray(q_ids, np.int64)
    if V is None:
        V = inner_products(U, Q)
    tau = np.asarray(tau, np.float64)[:, None]
    tid = np.asarray(tau_id, np.int64)[:, None]
    inside = (V > tau) | ((V == tau) & (q_ids[None, :] >= 0) & (q_ids[None, :] <= tid))
    return inside.sum(axis=0).astype(np.int64)


def reverse_counts_c(U, tau, tau_id, Q, q_ids=None):
    """reverse_counts in plain C (large inputs)."""
    U, Q = _f32(U), _f32(Q)
    nq = Q.shape[0]
    if q_ids is None:
        q_ids = np.full(nq, -1, np.int32)
    out = np.empty(nq, np.int32)
    _c().orc_reverse_counts(U, U.shape[0], U.shape[1],
                            np.ascontiguousarray(tau, np.float64),
                            np.ascontiguousarray(tau_id, np.int32), Q,
                            np.ascontiguousarray(q_ids, np.int32), nq, out)
    return out.astype(np.int64)


def topn_from_scores(scores, N):
    """Def. 3: the N items with the largest score, ordered (score desc, id asc)."""
    scores = np.asarray(scores, np.int64)
    order = np.lexsort((np.arange(scores.size), -scores))[:N]
    return order.astype(np.int32), scores[order]


def topn(U, P, k, N):
    """Brute force for Def. 3: every S_k, histogram, then top-N."""
    _, _, topk = kmips(U, P, k)
    return topn_from_scores(histogram_scores(topk, P.shape[0]), N)


# ---------------------------------------------------------------- bounds
# Relative slack added to the FP64 bound evaluations: far above the FP64
# rounding of a rotation and a d <= 256 term sum (about 1e-13 relative).
REL_SLACK = 1e-12

def _norms(X):
    X = _f32(X).astype(np.float64)
    s = np.zeros(X.shape[0])
    for i in range(X.shape[1]):
        s += X[:, i] * X[:, i]
    return np.sqrt(s)


def uscore_cs(U, P, tau, rel_slack=REL_SLACK):
    """Eq. (2) bound count with exact thresholds (Sec. 4.1):
    uscore(p) = #{u : ||u|| ||p|| (1 + rel_slack) >= tau_u}, FP64.
    The slack keeps the FP64 evaluation an upper bound where the
    inequality is tight (vectors that are parallel)."""
    nu, npp = _norms(U), _norms(P)
    tau = np.asarray(tau, np.float64)
    lhs = (nu[:, None] * npp[None, :]) * (1.0 + rel_slack)
    return (lhs >= tau[:, None]).sum(0).astype(np.int64)


def uscore_cs_c(U, P, tau, rel_slack=REL_SLACK):
    """uscore_cs in plain C (large inputs)."""
    U, P = _f32(U), _f32(P)
    out = np.empty(P.shape[0], np.int32)
    _c().orc_uscore_cs(U, P, U.shape[0], P.shape[0], U.shape[1],
                       np.ascontiguousarray(tau, np.float64), float(rel_slack), out)
    return out.astype(np.int64)


def uscore_eq3(U, P, tau, Vrot, dprime, rel_slack=REL_SLACK):
    """Eq. (3)/(6) bound count: after rotating both sides by the orthogonal
    Vrot, split at d':
        uscore(p) = #{u : u^l . p^l + ||u^r|| ||p^r|| + s ||u|| ||p|| >= tau_u}
    with s = rel_slack covering the FP64 rounding of the rotation and the
    sums, so the count stays an upper bound where the bound is tight (the
    k-th item itself has u . p = tau_u).  dprime = 0 gives the
    Cauchy-Schwarz count."""
    Ur = _f32(U).astype(np.float64) @ Vrot
    Pr = _f32(P).astype(np.float64) @ Vrot
    lam = Ur[:, :dprime] @ Pr[:, :dprime].T
    lam += np.sqrt((Ur[:, dprime:] ** 2).sum(1))[:, None] * \
        np.sqrt((Pr[:, dprime:] ** 2).sum(1))[None, :]
    lam += rel_slack * (_norms(U)[:, None] * _norms(P)[None, :])
    return (lam >= np.asarray(tau, np.float64)[:, None]).sum(0).astype(np.int64)


def topn_bound_ordered(scores, uscore, N):
    """Alg. 2 with exact per-item scores supplied: visit items in
    (uscore desc, id asc) order, keep the running top-N, and stop at the
    first item whose bound is strictly below the current N-th score.

    The paper stops on uscore <= tau (Alg. 2); with ties ordered by item
    index an item whose bound equals tau can still displace the N-th entry,
    so the stop here is strict.  Returns (ids, scores, visited)."""
    scores = np.asarray(scores, np.int64)
    uscore = np.asarray(uscore, np.int64)
    m = scores.size
    order = np.lexsort((np.arange(m), -uscore))
    best = []  # list of (score, id), kept sorted by (score desc, id asc)
    visited = 0
    for j in order:
        if len(best) == N and uscore[j] < best[-1][0]:
            break
        visited += 1
        best.append((int(scores[j]), int(j)))
        best.sort(key=lambda t: (-t[0], t[1]))
        best = best[:N]
    ids = np.array([b[1] for b in best], np.int32)
    sc = np.array([b[0] for b in best], np.int64)
    return ids, sc, visited


# ----------------------------------------------------------- relaxed score
def temperature(U, P, factor=0.05):
    """T = factor x population std of u . p over all n x m pairs, in FP64 by
    the Gram identities mean = (sum u).(sum p)/(nm),
    E[(u.p)^2] = trace((U^T U)(P^T P))/(nm)."""
    U = _f32(U).astype(np.float64)
    P = _f32(P).astype(np.float64)
    n, m = U.shape[0], P.shape[0]
    mean = U.sum(0) @ P.sum(0) / (n * m)
    e2 = np.trace((U.T @ U) @ (P.T @ P)) / (n * m)
    return factor * np.sqrt(e2 - mean * mean)


def sigmoid(z):
    """Logistic function in the form that never overflows."""
    z = np.asarray(z, np.float64)
    out = np.empty_like(z)
    pos = z >= 0
    out[pos] = 1.0 / (1.0 + np.exp(-z[pos]))
    ez = np.exp(z[~pos])
    out[~pos] = ez / (1.0 + ez)
    return out


def _soft_chunks(U, tau, Q, T, chunk=1 << 16):
    U = _f32(U)
    Qd = _f32(Q).astype(np.float64)
    tau = np.asarray(tau, np.float64)
    for s in range(0, U.shape[0], chunk):
        Ud = U[s:s + chunk].astype(np.float64)
        Z = (Qd @ Ud.T - tau[None, s:s + chunk]) / T
        yield Ud, sigmoid(Z)


def soft_score(U, tau, Q, T):
    """Relaxed score S(q) = sum_u sigmoid((u . q - tau_u) / T), FP64."""
    S = np.zeros(np.asarray(Q).shape[0])
    for _, s in _soft_chunks(U, tau, Q, T):
        S += s.sum(1)
    return S


def soft_grad(U, tau, Q, T):
    """dS/dq = sum_u sigmoid(z)(1 - sigmoid(z)) / T * u, FP64."""
    G = np.zeros(np.asarray(Q).shape, np.float64)
    for Ud, s in _soft_chunks(U, tau, Q, T):
        G += (s * (1.0 - s) / T) @ Ud
    return G


# ------------------------------------------- budgeted offline stage (Alg. 1)
BUDGET_KINDS = {"exp": 0, "uniform": 1, "linear": 2, "quadratic": 3}


def budget_rotation(U, P):
    """The orthogonal matrix of Alg. 1's second step (Sec. 4.2, "SVD
    transformation"): the right singular vectors of U and P stacked, from
    the eigenvectors of U^T U + P^T P by decreasing eigenvalue, so that the
    first coordinates carry most of the energy.  Any orthogonal matrix keeps
    Eq. (3) a bound; this one makes it tight."""
    U64 = _f32(U).astype(np.float64)
    P64 = _f32(P).astype(np.float64)
    w, V = np.linalg.eigh(U64.T @ U64 + P64.T @ P64)
    return V[:, np.argsort(-w, kind="stable")]


def budget_preprocess(U, P, kmax, b1, B2, kind="exp", alpha=1.0, gamma=0.0, dprime=10,
                      V=None, rel_slack=REL_SLACK):
    """Alg. 1 (Sec. 4.2) under the budget B = b1 * n + B2: the uniform
    step over the first b1 = B1/n items in norm order, U' and its ranks,
    beta of Eq. (5), the dynamic step with Eq. (4)'s budgets and the pooled
    budget B', U'' with pos_i, lambda_i of Eq. (7) and uscore_k for every
    k <= kmax (Eq. 6 over the positions after pos_i, then the first k
    entries of every list A_i).  kind: "exp" (Eq. 4), or Sec. 5.2's
    "uniform", "linear", "quadratic".  The rotation V (default
    budget_rotation) and the split d' = dprime define Eq. (3).

    The steps run in plain C (oracle.c, orc_budget_pre) in the order of the
    listing; the readings of its unclear points are stated there.  Returns a
    dict of numpy arrays: order, Av, Aj, pos, lam, uscore (kmax x m), key,
    rank, b2, nu2, np2, and the scalars of info."""
    U, P = _f32(U), _f32(P)
    n, d = U.shape
    m = P.shape[0]
    if V is None:
        V = budget_rotation(U, P)
    V = np.asarray(V, np.float64)
    dp = int(min(dprime, d))
    Ur = U.astype(np.float64) @ V
    Pr = P.astype(np.float64) @ V
    ul = np.ascontiguousarray(Ur[:, :dp])
    pl = np.ascontiguousarray(Pr[:, :dp])
    nru = np.sqrt((Ur[:, dp:] ** 2).sum(1))
    nrp = np.sqrt((Pr[:, dp:] ** 2).sum(1))
    nu, npn = _norms(U), _norms(P)
    out = {
        "order": np.empty(m, np.int32), "Av": np.empty((n, kmax), np.float64),
        "Aj": np.empty((n, kmax), np.int32), "pos": np.empty(n, np.int64),
        "lam": np.empty(n, np.float64), "uscore": np.empty((kmax, m), np.int32),
        "key": np.empty(n, np.int64), "rank": np.empty(n, np.int64),
        "b2": np.empty(n, np.int64),
    }
    info = np.zeros(8, np.float64)
    rc = _c().orc_budget_pre(U, P, n, m, d, int(kmax), int(b1), int(B2), BUDGET_KINDS[kind],
                             float(alpha), float(gamma), ul, np.ascontiguousarray(nru),
                             np.ascontiguousarray(nu), pl, np.ascontiguousarray(nrp),
                             np.ascontiguousarray(npn), dp, float(rel_slack), out["order"],
                             out["Av"], out["Aj"], out["pos"], out["lam"], out["uscore"],
                             out["key"], out["rank"], out["b2"], info)
    if rc != 0:
        raise ValueError("budget_preprocess: kmax <= b1 and kmax <= m are required")
    out["uscore"] = out["uscore"].astype(np.int64)
    U64, P64 = U.astype(np.float64), P.astype(np.float64)
    out["nu2"] = _sqsum(U64)
    out["np2"] = _sqsum(P64)
    out["rot"] = {"ul": ul, "pl": pl, "nru": nru, "nrp": nrp, "nu": nu, "np": npn,
                  "s": float(rel_slack)}
    out["U_prime"], out["U_dprime"], out["beta"] = int(info[0]), int(info[1]), float(info[2])
    out["ips3"], out["ips4"], out["scanned4"] = int(info[3]), int(info[4]), int(info[5])
    out["cert3"], out["cert4"] = int(info[6]), int(info[7])
    out["b1"], out["B2"], out["kind"], out["kmax"] = int(min(b1, m)), int(B2), kind, int(kmax)
    return out


def _sqsum(X64):
    s = np.zeros(X64.shape[0])
    for i in range(X64.shape[1]):
        s += X64[:, i] * X64[:, i]
    return s


def _cs_below(nu2, np2, theta):
    """Eq. (2) in squares with the oracle's relative slack 2^-36: true when
    |u| |p| is certainly below theta (theta > 0)."""
    return theta > 0.0 and (nu2 * np2) * (1.0 + 2.0 ** -36) < theta * theta


def _ip64(u, p):
    acc = 0.0
    for a, b in zip(u.astype(np.float64), p.astype(np.float64)):
        acc += a * b
    return acc


def budget_query(U, P, pre, k, N):
    """Alg. 2 with Inc-RMIPS (Sec. 4.3) on the state of budget_preprocess.

    (1) A user whose k-th value exceeds lambda_i (strictly: an unscanned
    item with an equal value and a smaller index would outrank it) has
    S_k = the first k entries of A_i, which are counted; the others form X.
    (2) Items are visited by (uscore_k desc, index asc); the visit stops at
    the first item whose uscore_k is below the N-th score (strict, for the
    index order of ties).  The score of a visited item adds, for each user
    of X, the decision of Inc-RMIPS:
      - a scanned item (position <= pos_i) outside the first k entries of
        A_i is out; one inside them, at rank r, is in when lambda_i is below
        its value, else the user is rescanned;
      - an unscanned item is out when Eq. (2), then Eq. (3), puts it below
        the k-th value, or when its exact value ranks after the k-th entry;
        otherwise it is in when lambda_i is below its value, else the user
        is rescanned.
    A rescan continues the user's scan from pos_i + 1 as in Alg. 1 (kmax
    list, Eq. 2 stop on the k-th value, Eq. 3 filter) to the exact S_k;
    the user leaves X, and the items of S_k not yet visited are credited
    now (the visited ones were decided exactly before).
    Small inputs only (pure Python over the pairs).
    Returns (ids, scores, stats)."""
    U, P = _f32(U), _f32(P)
    n, m = U.shape[0], P.shape[0]
    Av, Aj, pos, lam = pre["Av"], pre["Aj"], pre["pos"], pre["lam"]
    order, nu2, np2 = pre["order"], pre["nu2"], pre["np2"]
    rot = pre["rot"]
    kmax = pre["kmax"]
    posof = np.empty(m, np.int64)
    posof[order] = np.arange(1, m + 1)
    us = pre["uscore"][k - 1]
    score = np.zeros(m, np.int64)
    X = []
    for i in range(n):
        if Av[i, k - 1] > lam[i]:
            score[Aj[i, :k]] += 1
        else:
            X.append(i)
    x0 = len(X)

    def eq3(u, p):
        return float(rot["ul"][u] @ rot["pl"][p]) + rot["nru"][u] * rot["nrp"][p] + \
            rot["s"] * (rot["nu"][u] * rot["np"][p])

    def ranks_before(v1, i1, v2, i2):
        return v1 > v2 or (v1 == v2 and i1 < i2)

    def decide(u, p):
        Ak, idk = Av[u, k - 1], int(Aj[u, k - 1])
        if posof[p] <= pos[u]:
            hit = np.nonzero(Aj[u, :k] == p)[0]
            if hit.size == 0:
                return "out"
            return "in" if lam[u] < Av[u, hit[0]] else "rescan"
        if _cs_below(nu2[u], np2[p], Ak):
            return "out"
        if eq3(u, p) < Ak:
            return "out"
        v = _ip64(U[u], P[p])
        if not ranks_before(v, p, Ak, idk):
            return "out"
        return "in" if lam[u] < v else "rescan"

    def rescan(u):
        Lv, Lj = list(Av[u]), [int(x) for x in Aj[u]]
        for j in range(int(pos[u]) + 1, m + 1):
            p = int(order[j - 1])
            if _cs_below(nu2[u], np2[p], Lv[k - 1]):
                break
            if eq3(u, p) < Lv[kmax - 1]:
                continue
            v = _ip64(U[u], P[p])
            if ranks_before(v, p, Lv[-1], Lj[-1]):
                t = len(Lv) - 1
                while t > 0 and ranks_before(v, p, Lv[t - 1], Lj[t - 1]):
                    Lv[t], Lj[t] = Lv[t - 1], Lj[t - 1]
                    t -= 1
                Lv[t], Lj[t] = v, p
        return Lj[:k]

    visit = np.lexsort((np.arange(m), -us))
    visited = np.zeros(m, bool)
    best = []
    rescans = 0
    nvis = 0
    for p in visit:
        p = int(p)
        if len(best) == N and us[p] < best[-1][0]:
            break
        nvis += 1
        c = int(score[p])
        for u in list(X):
            r = decide(u, p)
            if r == "in":
                c += 1
            elif r == "rescan":
                rescans += 1
                X.remove(u)
                for q in rescan(u):
                    if q == p:
                        c += 1
                    elif not visited[q]:
                        score[q] += 1
        visited[p] = True
        best.append((c, p))
        best.sort(key=lambda t: (-t[0], t[1]))
        best = best[:N]
    ids = np.array([b[1] for b in best], np.int32)
    sc = np.array([b[0] for b in best], np.int64)
    return ids, sc, {"X0": x0, "rescans": rescans, "visited": nvis, "X_end": len(X)}

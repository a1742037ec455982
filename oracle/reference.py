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

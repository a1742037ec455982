"""Pins of the budgeted offline stage (Alg. 1, Sec. 4.2) and of the query
with Inc-RMIPS (Alg. 2, Sec. 4.3) in the oracle, against facts the paper
and the mathematics fix: a case worked by hand, Theorem 3 (uscore_k is an
upper bound of score_k), the exact lists of the users whose scan stopped,
Eq. (8)'s bound on the unscanned items, the solution of Eq. (5), the limit
cases of the budget, and Def. 3 computed by brute force."""
import json
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "budget_onehot_case.json")


def _instance(seed, n=300, m=240, d=12, clustered=False):
    rng = np.random.default_rng(seed)
    if clustered:
        C = rng.standard_normal((6, d))
        U = C[rng.integers(0, 6, n)] + 0.5 * rng.standard_normal((n, d))
    else:
        U = rng.standard_normal((n, d))
    U = U / np.linalg.norm(U, axis=1, keepdims=True) * rng.lognormal(0, 0.25, (n, 1))
    P = rng.standard_normal((m, d))
    P = P / np.linalg.norm(P, axis=1, keepdims=True) * rng.lognormal(0, 0.8, (m, 1))
    return U.astype(np.float32), P.astype(np.float32)


def test_hand_worked_case():
    g = json.load(open(GOLD))
    U = np.array(g["U"], np.float32)
    P = np.array(g["P"], np.float32)
    pre = oracle.budget_preprocess(U, P, g["kmax"], g["b1"], g["B2"], g["kind"], dprime=2,
                                   V=np.eye(2))
    for key in ("order", "key", "rank", "b2", "pos", "Aj"):
        assert pre[key].tolist() == g[key], key
    assert pre["Av"].tolist() == g["Av"]
    lam = [None if not np.isfinite(x) else x for x in pre["lam"].tolist()]
    assert lam[:3] == g["lam"][:3]
    assert lam[3] == pytest.approx(g["lam"][3], abs=1e-15)
    assert pre["uscore"][0].tolist() == g["uscore_1"]
    for key, val in g["info"].items():
        assert pre[key] == val, key
    for N, want in g["query"].items():
        ids, sc, st = oracle.budget_query(U, P, pre, 1, int(N))
        assert ids.tolist() == want["ids"] and sc.tolist() == want["scores"]
        for key in ("X0", "rescans", "visited"):
            assert st[key] == want[key], (N, key)
    ids, sc = oracle.topn(U, P, 1, 5)
    assert oracle.histogram_scores(oracle.kmips(U, P, 1)[2], 5).tolist() == g["scores_1"]


CASES = [
    # seed, kind, b1, B2 per user, kmax, clustered
    (1, "exp", 8, 4, 5, False),
    (2, "uniform", 8, 4, 5, True),
    (3, "linear", 10, 20, 6, False),
    (4, "quadratic", 6, 40, 6, True),
    (5, "exp", 6, 200, 4, True),
]


@pytest.mark.parametrize("seed,kind,b1,per,kmax,clu", CASES)
def test_lists_bounds_and_theorem3(seed, kind, b1, per, kmax, clu):
    U, P = _instance(seed, clustered=clu)
    n, m = U.shape[0], P.shape[0]
    pre = oracle.budget_preprocess(U, P, kmax, b1, per * n, kind)
    V = oracle.inner_products(U, P)
    topv, topk = oracle.kmips_table(U, P, kmax, V)
    order = pre["order"]
    posof = np.empty(m, np.int64)
    posof[order] = np.arange(1, m + 1)
    # the norm order
    np2 = (P.astype(np.float64) ** 2).sum(1)
    assert np.all(np.diff(np2[order]) <= 1e-9 * np2.max())
    dprime = pre["pos"] > 0
    assert dprime.sum() == pre["U_dprime"]
    # users outside U'': the exact k_max lists (Def. 1)
    assert np.array_equal(pre["Aj"][~dprime], topk[~dprime])
    assert np.array_equal(pre["Av"][~dprime], topv[~dprime])
    # users of U'': the k_max best of their first pos_i positions
    for u in np.nonzero(dprime)[0]:
        pref = order[: pre["pos"][u]]
        o = np.lexsort((pref, -V[u, pref]))[:kmax]
        assert pre["Aj"][u].tolist() == pref[o].tolist()
        assert np.array_equal(pre["Av"][u], V[u, pref[o]])
        # Eq. (8): every unscanned item is below lambda_i or below A^kmax
        rest = order[pre["pos"][u]:]
        ok = (V[u, rest] <= pre["lam"][u]) | (V[u, rest] < pre["Av"][u, kmax - 1])
        assert ok.all()
    assert np.all(np.isneginf(pre["lam"][~dprime]))
    # Theorem 3 for every k
    for k in range(1, kmax + 1):
        sc = oracle.histogram_scores(topk[:, :k], m)
        assert np.all(pre["uscore"][k - 1] >= sc), k
    # the budget of step 4: positions scanned at most sum(B2_i + 1)
    up = pre["key"] > 0
    assert up.sum() == pre["U_prime"]
    assert pre["scanned4"] <= int((pre["b2"][up] + 1).sum())
    assert sorted(pre["rank"][up].tolist()) == list(range(1, up.sum() + 1))
    # ranks follow (key, user)
    uu = np.nonzero(up)[0]
    o = np.lexsort((uu, pre["key"][uu]))
    assert pre["rank"][uu[o]].tolist() == list(range(1, uu.size + 1))


@pytest.mark.parametrize("seed,kind,b1,per,kmax,clu", CASES[:4])
def test_query_equals_definition(seed, kind, b1, per, kmax, clu):
    U, P = _instance(seed + 10, n=160, m=120, d=10, clustered=clu)
    pre = oracle.budget_preprocess(U, P, kmax, b1, per * U.shape[0], kind)
    for k in sorted({1, 2, kmax}):
        for N in (1, 7, 120):
            ids, sc, st = oracle.budget_query(U, P, pre, k, N)
            i2, s2 = oracle.topn(U, P, k, N)
            assert np.array_equal(ids, i2) and np.array_equal(sc, s2), (k, N)


def test_eq5_beta():
    U, P = _instance(21)
    n = U.shape[0]
    for alpha, gamma, per in ((1.0, 0.0, 3), (2.0, 1.0, 10), (0.5, 0.0, 0.2)):
        B2 = int(per * n)
        pre = oracle.budget_preprocess(U, P, 4, 6, B2, "exp", alpha=alpha, gamma=gamma)
        X, b = pre["U_prime"], pre["beta"]
        lhs = alpha * np.expm1(b * X) / b + gamma * X if b != 0 else (alpha + gamma) * X
        assert lhs == pytest.approx(B2, rel=1e-9)
        up = pre["key"] > 0
        x = pre["rank"][up].astype(np.float64)
        assert np.array_equal(pre["b2"][up], np.floor(alpha * np.exp(b * x) + gamma))
    # no beta reaches B2 <= gamma |U'|: f = gamma
    pre = oracle.budget_preprocess(U, P, 4, 6, 10, "exp", alpha=1.0, gamma=3.0)
    assert np.isneginf(pre["beta"])
    assert np.all(pre["b2"][pre["key"] > 0] == 3)


def test_budget_kinds_integrate_to_B2():
    U, P = _instance(22)
    B2 = 5000
    for kind, f in (("uniform", lambda x, X: B2 / X), ("linear", lambda x, X: 2 * B2 * x / X**2),
                    ("quadratic", lambda x, X: 3 * B2 * x * x / X**3)):
        pre = oracle.budget_preprocess(U, P, 4, 6, B2, kind)
        up = pre["key"] > 0
        X = up.sum()
        x = pre["rank"][up].astype(np.float64)
        assert np.all(pre["b2"][up] == np.floor(f(x, float(X))))
        assert abs(pre["b2"][up].sum() - B2) <= B2 * 3.0 / X + X


def test_limits():
    U, P = _instance(23, n=200, m=150)
    m = P.shape[0]
    topv, topk = oracle.kmips_table(U, P, 5)
    # an unbounded budget: every scan ends by itself, U'' is empty and
    # uscore_k is the exact score (Baseline 1, Sec. 2.2)
    pre = oracle.budget_preprocess(U, P, 5, 5, 10**9, "uniform")
    assert pre["U_dprime"] == 0 and np.all(pre["pos"] == 0)
    for k in range(1, 6):
        assert np.array_equal(pre["uscore"][k - 1], oracle.histogram_scores(topk[:, :k], m))
    # b1 = m: step 3 scans everything, U' is empty
    pre = oracle.budget_preprocess(U, P, 5, m, 0, "exp")
    assert pre["U_prime"] == 0 and pre["cert3"] == U.shape[0]
    assert np.array_equal(pre["Aj"], topk)
    # no dynamic budget: each user of U' scans one more position at most
    pre = oracle.budget_preprocess(U, P, 5, 8, 0, "uniform")
    up = pre["key"] > 0
    assert np.all(pre["b2"][up] == 0)
    assert np.all(pre["pos"][pre["pos"] > 0] == 9)
    with pytest.raises(ValueError):
        oracle.budget_preprocess(U, P, 5, 4, 0, "uniform")


def _tie_instance():
    """Items that share a value with a user but sit later in the norm order
    with a smaller index: p = (c, t_j) with the same c and decreasing t_j,
    indices assigned in reverse, so equal values meet the bound exactly and
    only the index decides.  Plus users opposite to everything (all values
    negative, their scans never stop early)."""
    rng = np.random.default_rng(7)
    m, d = 60, 4
    P = np.zeros((m, d), np.float32)
    for j in range(m):
        g = j // 4            # groups of four items with one value for e1
        t = j % 4             # larger index -> larger norm -> earlier in the norm order
        P[j, 0] = 8.0 - g * 0.25
        P[j, 1] = float(t)
    U = np.zeros((40, d), np.float32)
    U[:20, 0] = rng.integers(1, 4, 20)
    U[20:30] = rng.integers(-3, 4, (10, d)).astype(np.float32)
    U[30:, 0] = -rng.integers(1, 4, 10)
    U[30:, 1] = -1.0
    return U, P


def test_exact_ties_at_the_bound():
    U, P = _tie_instance()
    m = P.shape[0]
    topv, topk = oracle.kmips_table(U, P, 6)
    for b1, per, kind in ((6, 3, "uniform"), (6, 0, "uniform"), (10, 50, "exp")):
        pre = oracle.budget_preprocess(U, P, 6, b1, per * U.shape[0], kind)
        cert = pre["pos"] == 0
        assert np.array_equal(pre["Aj"][cert], topk[cert])
        for k in (1, 3, 6):
            sc = oracle.histogram_scores(topk[:, :k], m)
            assert np.all(pre["uscore"][k - 1] >= sc)
            for N in (1, 4, 20):
                ids, s, _ = oracle.budget_query(U, P, pre, k, N)
                i2, s2 = oracle.topn(U, P, k, N)
                assert np.array_equal(ids, i2) and np.array_equal(s, s2), (b1, k, N)


@pytest.mark.parametrize("seed,kind", [(31, "exp"), (32, "quadratic")])
def test_identity_rotation_closed_form(seed, kind):
    """With the identity rotation and d' = d, Eq. (3)'s bound is the exact
    product plus the slack s |u| |p|, so lambda_i (Eq. 7) is the largest of
    these over the positions after pos_i up to the first Cauchy-Schwarz
    stop, and uscore_k(p) (Eq. 6, step 5) counts the first k entries of the
    lists plus the users of U'' whose range holds p with a bound >= A^k."""
    U, P = _instance(seed, n=150, m=120, d=6)
    U = np.vstack([U, -np.abs(U[:5]) - 0.1, np.zeros((1, 6), np.float32)]).astype(np.float32)
    P = np.abs(P).astype(np.float32)
    n, m, kmax, s = U.shape[0], P.shape[0], 4, 1e-12
    pre = oracle.budget_preprocess(U, P, kmax, 5, 2 * n, kind, dprime=6, V=np.eye(6),
                                   rel_slack=s)
    V = oracle.inner_products(U, P)
    U64, P64 = U.astype(np.float64), P.astype(np.float64)
    nu2 = (U64 ** 2).sum(1)
    np2 = (P64 ** 2).sum(1)
    nu, npn = np.sqrt(nu2), np.sqrt(np2)
    order = pre["order"]
    want = np.zeros((kmax, m), np.int64)
    for u in range(n):
        for k in range(1, kmax + 1):
            want[k - 1, pre["Aj"][u, :k]] += 1
    neg = 0
    for u in np.nonzero(pre["pos"] > 0)[0]:
        th = pre["Av"][u, kmax - 1]
        best = -np.inf
        for j in range(pre["pos"][u] + 1, m + 1):
            p = order[j - 1]
            if th > 0 and nu2[u] * np2[p] * (1 + 2.0 ** -36) < th * th:
                break
            lam = V[u, p] + s * nu[u] * npn[p]
            best = max(best, lam)
            want[:, p] += lam >= pre["Av"][u]
        assert pre["lam"][u] == pytest.approx(best, rel=1e-12, abs=1e-13)
        neg += best < 0
    assert neg > 0   # the instance holds users whose lambda is negative
    assert np.array_equal(pre["uscore"], want)

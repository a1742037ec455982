"""Pins for the CPU FP64 oracle: hand-worked cases, closed forms,
invariants and brute force, each independent of the oracle's own code."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle as orc
import synth


def _rand(seed, n, m, d, su=0.3, sp=0.5):
    rng = np.random.default_rng(seed)
    return (synth.isotropic(rng, n, d, su), synth.isotropic(rng, m, d, sp))


# ------------------------------------------------------------ inner product
def test_inner_product_integer_closed_form():
    # small integers: every partial sum is exact, so the FP64 value equals
    # the integer dot product whatever the order
    rng = np.random.default_rng(1)
    Ui = rng.integers(-50, 50, size=(37, 23))
    Pi = rng.integers(-50, 50, size=(41, 23))
    V = orc.inner_products(Ui.astype(np.float32), Pi.astype(np.float32))
    assert np.array_equal(V, (Ui @ Pi.T).astype(np.float64))


def test_inner_product_is_index_ordered_sum():
    # values whose sum depends on the order: 1, 2^-60, -1 gives 0 in index
    # order (the 2^-60 is absorbed), 2^-60 in reverse order
    U = np.array([[1.0, 1.0, 1.0]], np.float32)
    P = np.array([[1.0, 2.0 ** -60, -1.0]], np.float32)
    assert orc.inner_products(U, P)[0, 0] == 0.0
    P2 = P[:, ::-1].copy()
    U2 = U[:, ::-1].copy()
    assert orc.inner_products(U2, P2)[0, 0] == 0.0  # -1 + 2^-60 + 1 -> 0 too
    P3 = np.array([[2.0 ** -60, 1.0, -1.0]], np.float32)
    assert orc.inner_products(U, P3)[0, 0] == 0.0
    P4 = np.array([[1.0, -1.0, 2.0 ** -60]], np.float32)
    assert orc.inner_products(U, P4)[0, 0] == 2.0 ** -60


def test_products_exact_in_fp64():
    # FP32 x FP32 fits in FP64: a single product is exact
    rng = np.random.default_rng(2)
    a = rng.standard_normal(1000).astype(np.float32)
    b = rng.standard_normal(1000).astype(np.float32)
    from fractions import Fraction
    for x, y in zip(a[:50], b[:50]):
        exact = Fraction(float(x)) * Fraction(float(y))
        V = orc.inner_products(np.array([[x]], np.float32), np.array([[y]], np.float32))
        assert Fraction(V[0, 0]) == exact


def test_numpy_and_c_inner_products_bit_equal():
    U, P = _rand(3, 300, 257, 37)
    V1 = orc.inner_products(U, P)
    V2 = orc.inner_products_c(U, P)
    assert np.array_equal(V1.view(np.uint64), V2.view(np.uint64))


# ------------------------------------------------------------ hand-worked
def _golden(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


def test_onehot_hand_worked(golden_dir):
    g = _golden(golden_dir, "onehot_case.json")
    U = np.array(g["U"], np.float32)
    P = np.array(g["P"], np.float32)
    assert np.array_equal(orc.inner_products(U, P), np.array(g["inner_products"], float))
    for ks, e in g["k"].items():
        k = int(ks)
        for fn in (orc.kmips, lambda a, b, c: orc.kmips_c(a, b, c)):
            tau, tid, topk = fn(U, P, k)
            assert np.array_equal(tau, np.array(e["tau"], float)), (k, tau)
            assert np.array_equal(tid, e["tau_id"]), (k, tid)
            assert np.array_equal(topk, np.array(e["topk"])), (k, topk)
        sc = orc.histogram_scores(topk, P.shape[0])
        assert np.array_equal(sc, e["scores"])
        rc = orc.reverse_counts(U, tau, tid, P, np.arange(P.shape[0]))
        assert np.array_equal(rc, e["scores"])
        if "top3_ids" in e:
            ids, s = orc.topn_from_scores(sc, 3)
            assert ids.tolist() == e["top3_ids"] and s.tolist() == e["top3_scores"]
            assert orc.uscore_cs(U, P, tau).tolist() == e["uscore_cs"]
            assert orc.uscore_cs_c(U, P, tau).tolist() == e["uscore_cs"]
            q = np.array([e["external_query"]], np.float32)
            assert orc.reverse_counts(U, tau, tid, q, [-1]).tolist() == [e["external_query_count"]]
            assert orc.reverse_counts_c(U, tau, tid, q, [-1]).tolist() == [e["external_query_count"]]
            assert orc.reverse_counts(U, tau, tid, P[2:3], [2]).tolist() == [e["p2_as_member_count"]]


def test_strict_stop_hand_worked(golden_dir):
    g = _golden(golden_dir, "strict_stop_case.json")
    ids, sc, visited = orc.topn_bound_ordered(g["scores"], g["uscore"], g["N"])
    assert ids.tolist() == g["expected_ids"]
    assert sc.tolist() == g["expected_scores"]
    assert visited == g["expected_visited_strict"]
    bi, bs = orc.topn_from_scores(g["scores"], g["N"])
    assert bi.tolist() == g["expected_ids"]


# ------------------------------------------------------------ brute force
def _brute_kmips(U, P, k):
    taus, tids, tops = [], [], []
    for u in range(U.shape[0]):
        vals = []
        for j in range(P.shape[0]):
            s = 0.0
            for i in range(U.shape[1]):
                s = s + float(U[u, i]) * float(P[j, i])
            vals.append((s, j))
        vals.sort(key=lambda t: (-t[0], t[1]))
        taus.append(vals[k - 1][0])
        tids.append(vals[k - 1][1])
        tops.append([t[1] for t in vals[:k]])
    return np.array(taus), np.array(tids), np.array(tops)


@pytest.mark.parametrize("seed,k", [(0, 1), (1, 3), (2, 7)])
def test_kmips_matches_python_brute_force(seed, k):
    U, P = _rand(10 + seed, 12, 40, 6)
    bt, bj, bk = _brute_kmips(U, P, k)
    for fn in (orc.kmips, lambda a, b, c: orc.kmips_c(a, b, c)):
        tau, tid, topk = fn(U, P, k)
        assert np.array_equal(tau, bt)
        assert np.array_equal(tid, bj)
        assert np.array_equal(topk, bk)


def test_ties_resolved_by_index():
    # duplicated items and a zero user: exact ties everywhere
    U = np.array([[1, 0], [0, 0], [1, 1]], np.float32)
    P = np.array([[1, 0], [1, 0], [0, 1], [1, 0], [0, 0]], np.float32)
    tau, tid, topk = orc.kmips(U, P, 2)
    assert topk.tolist() == [[0, 1], [0, 1], [0, 1]]
    assert tid.tolist() == [1, 1, 1]
    tau, tid, topk = orc.kmips_c(U, P, 4)
    # user 0: values 1,1,0,1,0 -> 0,1,3 then 2 (0, index 2)
    assert topk.tolist()[0] == [0, 1, 3, 2]
    assert topk.tolist()[1] == [0, 1, 2, 3]          # all zero: by index
    assert topk.tolist()[2] == [0, 1, 2, 3]          # all one except item 4
    sc = orc.histogram_scores(topk, 5)
    assert sc.sum() == 3 * 4
    # plain "v >= tau" would count item 4 for user 1 and break the sum
    rc = orc.reverse_counts(U, tau, tid, P, np.arange(5))
    assert np.array_equal(rc, sc)


def test_orthogonal_with_duplicates():
    d = 6
    U = np.eye(d, dtype=np.float32)
    c = np.array([3, 1, 4, 1, 5, 9], np.float32)
    P = np.vstack([np.diag(c), np.diag(c)]).astype(np.float32)  # item j and j+d equal
    tau, tid, topk = orc.kmips(U, P, 2)
    # user a sees c_a at items a and a+d, zero elsewhere
    assert topk.tolist() == [[a, a + d] for a in range(d)]
    assert tau.tolist() == c.tolist()
    sc = orc.histogram_scores(topk, 2 * d)
    assert sc.tolist() == [1] * (2 * d)
    tau3, tid3, topk3 = orc.kmips(U, P, 3)
    # third place is a zero; the smallest index with value 0 wins
    assert topk3[:, 2].tolist() == [1, 0, 0, 0, 0, 0]


# ------------------------------------------------------------ k_max table
def test_kmax_table_onehot_golden(golden_dir):
    # one scan with k_max = 3 (the per-user lists of Alg. 1, Sec. 4.2) holds
    # the hand-worked answers of k = 1, 2 and 3
    g = _golden(golden_dir, "onehot_case.json")
    U = np.array(g["U"], np.float32)
    P = np.array(g["P"], np.float32)
    m = P.shape[0]
    for fn in (orc.kmips_table, orc.kmips_table_c):
        topv, topk = fn(U, P, 3)
        for ks, e in g["k"].items():
            k = int(ks)
            assert topv[:, k - 1].tolist() == e["tau"], (k, topv)
            assert topk[:, k - 1].tolist() == e["tau_id"], (k, topk)
            assert topk[:, :k].tolist() == e["topk"], k
            assert orc.histogram_scores(topk[:, :k], m).tolist() == e["scores"], k
            if "top3_ids" in e:
                ids, sc = orc.topn_from_table(topk, k, 3, m)
                assert ids.tolist() == e["top3_ids"] and sc.tolist() == e["top3_scores"]


@pytest.mark.parametrize("seed,kmax", [(0, 9), (1, 4)])
def test_kmax_table_matches_python_brute_force(seed, kmax):
    U, P = _rand(30 + seed, 10, 35, 5)
    topv, topk = orc.kmips_table(U, P, kmax)
    topv_c, topk_c = orc.kmips_table_c(U, P, kmax)
    assert np.array_equal(topv_c.view(np.uint64), topv.view(np.uint64))
    assert np.array_equal(topk_c, topk)
    for k in range(1, kmax + 1):
        bt, bj, bk = _brute_kmips(U, P, k)
        assert np.array_equal(topv[:, k - 1], bt), k
        assert np.array_equal(topk[:, k - 1], bj), k
        assert np.array_equal(topk[:, :k], bk), k


def test_kmax_table_sum_of_scores_every_k():
    # Eq. (1): every S_k(u) holds k items, so the scores sum to n k for
    # every k <= k_max; the k-th values do not increase with k
    U, P = _rand(23, 400, 150, 7)
    n, m, kmax = U.shape[0], P.shape[0], 25
    topv, topk = orc.kmips_table_c(U, P, kmax)
    assert (np.diff(topv, axis=1) <= 0).all()
    for k in range(1, kmax + 1):
        assert orc.histogram_scores(topk[:, :k], m).sum() == n * k, k
    # with ties everywhere (small integers) as well
    rng = np.random.default_rng(3)
    Ui = rng.integers(-2, 3, size=(300, 4)).astype(np.float32)
    Pi = rng.integers(-2, 3, size=(60, 4)).astype(np.float32)
    tv, tk = orc.kmips_table_c(Ui, Pi, 25)
    for k in (1, 7, 25):
        assert orc.histogram_scores(tk[:, :k], 60).sum() == 300 * k
        t, j, kk = orc.kmips(Ui, Pi, k)
        assert np.array_equal(tk[:, :k], kk) and np.array_equal(tv[:, k - 1], t)


# ------------------------------------------------------------ invariants
def test_sum_of_scores_is_nk_and_special_k():
    U, P = _rand(5, 150, 80, 9)
    n, m = U.shape[0], P.shape[0]
    for k in (1, 5, m):
        tau, tid, topk = orc.kmips(U, P, k)
        sc = orc.histogram_scores(topk, m)
        assert sc.sum() == n * k
        if k == m:
            assert (sc == n).all()
        if k == 1:
            V = orc.inner_products(U, P)
            assert np.array_equal(sc, np.bincount(V.argmax(1), minlength=m))
    tau, tid, topk = orc.kmips(U[:1], P, 4)
    sc = orc.histogram_scores(topk, m)
    assert set(np.unique(sc)) <= {0, 1} and sc.sum() == 4


def test_power_of_two_scaling():
    U, P = _rand(6, 60, 70, 11)
    t0, j0, k0 = orc.kmips(U, P, 5)
    t1, j1, k1 = orc.kmips((U * 2.0 ** 7).astype(np.float32), P, 5)
    t2, j2, k2 = orc.kmips(U, (P * 2.0 ** -9).astype(np.float32), 5)
    assert np.array_equal(k0, k1) and np.array_equal(k0, k2)
    assert np.array_equal(t1, t0 * 2.0 ** 7) and np.array_equal(t2, t0 * 2.0 ** -9)


def test_user_and_item_permutation():
    U, P = _rand(7, 90, 60, 8)
    n, m = U.shape[0], P.shape[0]
    k = 4
    sc = orc.histogram_scores(orc.kmips(U, P, k)[2], m)
    rng = np.random.default_rng(0)
    pu = rng.permutation(n)
    assert np.array_equal(orc.histogram_scores(orc.kmips(U[pu], P, k)[2], m), sc)
    pi = rng.permutation(m)  # continuous data: no ties, scores follow the items
    sc2 = orc.histogram_scores(orc.kmips(U, P[pi], k)[2], m)
    assert np.array_equal(sc2, sc[pi])


def test_histogram_equals_reverse_counts_and_c():
    U, P = _rand(8, 200, 120, 10)
    m = P.shape[0]
    tau, tid, topk = orc.kmips(U, P, 6)
    sc = orc.histogram_scores(topk, m)
    assert np.array_equal(orc.reverse_counts(U, tau, tid, P, np.arange(m)), sc)
    assert np.array_equal(orc.reverse_counts_c(U, tau, tid, P, np.arange(m)), sc)
    tc, jc, kc = orc.kmips_c(U, P, 6)
    assert np.array_equal(tc, tau) and np.array_equal(jc, tid) and np.array_equal(kc, topk)


def test_external_query_is_appended_item():
    U, P = _rand(9, 40, 30, 5)
    rng = np.random.default_rng(3)
    Q = rng.standard_normal((7, 5)).astype(np.float32)
    Q[0] = P[3]          # an exact duplicate of an item of P: must lose ties
    k = 3
    tau, tid, _ = orc.kmips(U, P, k)
    got = orc.reverse_counts(U, tau, tid, Q, None)
    for i in range(Q.shape[0]):
        PP = np.vstack([P, Q[i:i + 1]])
        _, _, topk = orc.kmips(U, PP, k)
        assert got[i] == int((topk == P.shape[0]).any(1).sum())


# ------------------------------------------------------------ bounds
def _random_orthogonal(d, seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((d, d)))
    return q * np.sign(np.diag(r))


def test_theorem2_bounds_dominate_scores():
    U, P = _rand(11, 300, 150, 12, 0.25, 0.6)
    m = P.shape[0]
    tau, tid, topk = orc.kmips(U, P, 5)
    sc = orc.histogram_scores(topk, m)
    cs = orc.uscore_cs(U, P, tau)
    assert (cs >= sc).all()
    assert np.array_equal(orc.uscore_cs_c(U, P, tau), cs)
    for seed, dp in [(0, 3), (1, 6), (2, 0), (3, 11)]:
        V = _random_orthogonal(12, seed)
        e3 = orc.uscore_eq3(U, P, tau, V, dp)
        assert (e3 >= sc).all(), dp
        assert (e3 <= cs).all(), dp       # Eq. (3) is never looser than Eq. (2)
    # d' = 0 with V = I is the Cauchy-Schwarz count
    assert np.array_equal(orc.uscore_eq3(U, P, tau, np.eye(12), 0), cs)
    # d' = d with V = I is #{u : v >= tau_u}; integer data keeps every sum exact
    rng = np.random.default_rng(9)
    Ui = rng.integers(-4, 5, size=(60, 5)).astype(np.float32)
    Pi = rng.integers(-4, 5, size=(30, 5)).astype(np.float32)
    ti, _, _ = orc.kmips(Ui, Pi, 3)
    Vi = orc.inner_products(Ui, Pi)
    assert np.array_equal(orc.uscore_eq3(Ui, Pi, ti, np.eye(5), 5),
                          (Vi >= ti[:, None]).sum(0))


def test_bound_ordered_topn_equals_brute_force():
    U, P = _rand(12, 400, 300, 8, 0.25, 0.7)
    m = P.shape[0]
    for k, N in [(3, 1), (5, 10), (10, 25)]:
        tau, tid, topk = orc.kmips(U, P, k)
        sc = orc.histogram_scores(topk, m)
        bi, bs = orc.topn_from_scores(sc, N)
        for ub in (orc.uscore_cs(U, P, tau), sc, np.full(m, U.shape[0]),
                   orc.uscore_eq3(U, P, tau, _random_orthogonal(8, 5), 3)):
            ids, s, visited = orc.topn_bound_ordered(sc, ub, N)
            assert np.array_equal(ids, bi) and np.array_equal(s, bs)
            assert N <= visited <= m
        # the tightest bound (the scores themselves) visits the fewest items
        _, _, v_tight = orc.topn_bound_ordered(sc, sc, N)
        _, _, v_cs = orc.topn_bound_ordered(sc, orc.uscore_cs(U, P, tau), N)
        assert v_tight <= v_cs


# ------------------------------------------------------------ relaxed score
def test_temperature_gram_identity():
    U, P = _rand(13, 120, 90, 7)
    V = orc.inner_products(U, P)
    assert abs(orc.temperature(U, P) - 0.05 * V.std()) <= 1e-12 * V.std()


def test_soft_closed_form_identical_users():
    d = 9
    rng = np.random.default_rng(4)
    u = rng.standard_normal(d).astype(np.float32)
    U = np.repeat(u[None], 50, 0)
    tau = np.full(50, 0.3)
    Q = rng.standard_normal((5, d)).astype(np.float32)
    T = 0.7
    z = (Q.astype(np.float64) @ u.astype(np.float64) - 0.3) / T
    s = 1.0 / (1.0 + np.exp(-z))
    np.testing.assert_allclose(orc.soft_score(U, tau, Q, T), 50 * s, rtol=1e-13)
    np.testing.assert_allclose(orc.soft_grad(U, tau, Q, T),
                               (50 * s * (1 - s) / T)[:, None] * u.astype(np.float64)[None],
                               rtol=1e-12)


def test_soft_zero_temperature_limit_is_count():
    U, P = _rand(14, 200, 50, 6)
    tau, tid, _ = orc.kmips(U, P, 4)
    rng = np.random.default_rng(5)
    Q = rng.standard_normal((6, 6)).astype(np.float32)
    cnt = orc.reverse_counts(U, tau, tid, Q, None)
    S = orc.soft_score(U, tau, Q, 1e-9)
    assert np.array_equal(np.rint(S).astype(np.int64), cnt)


def test_soft_gradient_central_differences():
    U, P = _rand(15, 300, 50, 6)
    tau, _, _ = orc.kmips(U, P, 4)
    T = orc.temperature(U, P) * 4
    rng = np.random.default_rng(6)
    Q = (rng.standard_normal((3, 6)) * 0.5).astype(np.float32)
    G = orc.soft_grad(U, tau, Q, T)
    h = 1e-6
    for i in range(3):
        for _ in range(4):
            v = rng.standard_normal(6)
            v /= np.linalg.norm(v)
            # differentiate in FP64 through the same definition
            Ud = U.astype(np.float64)
            def S(q):
                return orc.sigmoid((Ud @ q - tau) / T).sum()
            fd = (S(Q[i].astype(np.float64) + h * v) - S(Q[i].astype(np.float64) - h * v)) / (2 * h)
            assert abs(fd - G[i] @ v) <= 1e-6 * np.linalg.norm(G[i]) + 1e-12


def test_numpy_and_c_oracles_agree_on_tiny_workload():
    # the 2,000 x 1,000 x 16 workload in full: numpy full sort vs C scan
    U, P = synth.make_config(0)
    t1, j1, k1 = orc.kmips(U, P, 10)
    t2, j2, k2 = orc.kmips_c(U, P, 10)
    assert np.array_equal(t1.view(np.uint64), t2.view(np.uint64))
    assert np.array_equal(j1, j2) and np.array_equal(k1, k2)
    sc = orc.histogram_scores(k1, P.shape[0])
    assert sc.sum() == U.shape[0] * 10
    assert np.array_equal(orc.reverse_counts_c(U, t2, j2, P, np.arange(P.shape[0])), sc)


def test_generator_is_deterministic_and_shaped():
    for i in range(5):
        cfg = synth.CONFIGS[i]
        U, P = synth.make_config(cfg, n=300, m=200)
        U2, P2 = synth.make_config(cfg, n=300, m=200)
        assert U.dtype == np.float32 and U.shape == (300, cfg.d) and P.shape == (200, cfg.d)
        assert np.array_equal(U, U2) and np.array_equal(P, P2)
        assert U.flags.c_contiguous and P.flags.c_contiguous
    sub = synth.subsample_users(3)
    assert sub.size == synth.CONFIGS[3].n // 100 and (np.diff(sub) > 0).all()

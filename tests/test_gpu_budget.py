"""GPU parity of the budgeted index (Alg. 1 under an inner-product budget,
Sec. 4.2) and of its query (Alg. 2 with Inc-RMIPS, Sec. 4.3) against the CPU
oracle.

Exact on both sides, element by element: the norm order, U' with its keys
and ranks, every budget B_2,i, U'' with pos_i, and every list A_i (values
bit for bit, ids); the top-N of the query equals Def. 3.  The rotation of
Eq. (3) differs between the two sides (any orthogonal one is valid), so
lambda_i and uscore_k are checked by what the paper fixes for any valid
bound: Eq. (8) (no unscanned item outranks lambda_i unless it is below the
k_max-th value), Theorem 3 (uscore_k >= score_k), and the lists' part of
uscore_k exactly."""
import json
import os

import numpy as np
import pytest

import oracle as orc
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _g(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(_dev())


def _state(bi):
    return {k: v.cpu().numpy() for k, v in bi.state().items()}


def _check_state(U, P, bi, pre, kmax, V=None, topk=None):
    """GPU index state against the oracle's Alg. 1 (exact parts) and the
    bound properties (Eq. 8, Theorem 3)."""
    n, m = U.shape[0], P.shape[0]
    g = _state(bi)
    assert np.array_equal(g["order"], pre["order"])
    assert np.array_equal(g["key"], pre["key"].astype(np.int32))
    assert np.array_equal(g["rank"], pre["rank"].astype(np.int32))
    assert np.array_equal(g["b2"], pre["b2"])
    assert np.array_equal(g["pos"], pre["pos"].astype(np.int32))
    assert np.array_equal(g["Aj"], pre["Aj"])
    assert np.array_equal(g["Av"].view(np.uint64), pre["Av"].view(np.uint64))
    info = bi.info
    assert info["u_prime"] == pre["U_prime"] and info["u_dprime"] == pre["U_dprime"]
    assert info["cert3"] == pre["cert3"] and info["cert4"] == pre["cert4"]
    assert info["scanned4"] == pre["scanned4"]
    if pre["kind"] == "exp" and pre["U_prime"] > 0:
        assert info["beta"] == pytest.approx(pre["beta"], rel=1e-12, abs=1e-300)
    u2 = g["pos"] > 0
    assert np.all(np.isneginf(g["lam"][~u2]))
    # uscore: the lists' part exactly, the rest within the users of U''
    hist = np.zeros((kmax, m), np.int64)
    for k in range(1, kmax + 1):
        hist[k - 1] = orc.histogram_scores(g["Aj"][:, :k], m)
    us = g["uscore"].astype(np.int64)
    assert np.all(us >= hist) and np.all(us - hist <= u2.sum())
    assert np.all(np.diff(us, axis=0) >= 0)
    if topk is not None:
        for k in range(1, kmax + 1):   # Theorem 3
            assert np.all(us[k - 1] >= orc.histogram_scores(topk[:, :k], m)), k
    if V is not None:
        order = g["order"]
        for u in np.nonzero(u2)[0]:   # Eq. (8)
            rest = order[g["pos"][u]:]
            ok = (V[u, rest] <= g["lam"][u]) | (V[u, rest] < g["Av"][u, kmax - 1])
            assert ok.all(), u
    return g


def _check_query(bi, topk, m, ks, Ns):
    for k in ks:
        for N in Ns:
            print("[case] budget query k", k, "N", N, flush=True)
            ri, rs = orc.topn_from_table(topk, k, N, m)
            ids, sc, st = bi.topn(k, N)
            assert ids.tolist() == ri.tolist() and sc.tolist() == rs.tolist(), (k, N, st)
            assert st["visited_items"] <= st["processed_items"] <= m
            assert st["rescanned_users"] <= st["x0"]


KINDS = ["exp", "uniform", "linear", "quadratic"]


@pytest.mark.parametrize("kind", KINDS)
def test_budget_tiny_workload(kind):
    import paper_2504_13445_amd as rm
    U, P = synth.make_config(0)
    # norms of this workload spread little, so most users need nearly every
    # item: a budget of 300 positions per user settles some of them
    kmax, b1, B2 = 25, 30, 300 * U.shape[0]
    print("[case] budget tiny", kind, flush=True)
    pre = orc.budget_preprocess(U, P, kmax, b1, B2, kind)
    V = orc.inner_products_c(U, P)
    topv, topk = orc.kmips_table(U, P, kmax, V)
    bi = rm.BudgetIndex(_g(U), _g(P), kmax, b1, B2, kind)
    g = _check_state(U, P, bi, pre, kmax, V, topk)
    if kind == "exp":   # both kinds of users (the others settle none here)
        assert g["pos"].max() > 0 and (g["pos"] == 0).sum() > 0
    _check_query(bi, topk, P.shape[0], (1, 10, 25), (10, 37))


@pytest.mark.parametrize("prec", ["bf16", "fp8", "fp6", "fp4"])
def test_budget_screened_stage_a(prec):
    # the exact k_max-th values and rescans come from stage (a) screened at
    # this precision: the index and the results do not change
    import paper_2504_13445_amd as rm
    U, P = synth.make_config(0)
    kmax, b1, B2 = 25, 26, 5 * U.shape[0]
    pre = orc.budget_preprocess(U, P, kmax, b1, B2, "exp", alpha=2.0, gamma=1.0)
    topv, topk = orc.kmips_table(U, P, kmax)
    bi = rm.BudgetIndex(_g(U), _g(P), kmax, b1, B2, "exp", alpha=2.0, gamma=1.0, prec=prec)
    _check_state(U, P, bi, pre, kmax, None, topk)
    _check_query(bi, topk, P.shape[0], (5, 25), (20,))


def test_budget_limits():
    import paper_2504_13445_amd as rm
    U, P = synth.make_config(0)
    n, m, kmax = U.shape[0], P.shape[0], 12
    topv, topk = orc.kmips_table(U, P, kmax)
    # an unbounded budget: U'' is empty and uscore_k is the exact score
    bi = rm.BudgetIndex(_g(U), _g(P), kmax, kmax, 10**12, "uniform")
    g = _check_state(U, P, bi, orc.budget_preprocess(U, P, kmax, kmax, 10**12, "uniform"),
                     kmax, None, topk)
    assert bi.info["u_dprime"] == 0
    for k in range(1, kmax + 1):
        assert np.array_equal(g["uscore"][k - 1], orc.histogram_scores(topk[:, :k], m))
    _check_query(bi, topk, m, (1, 12), (10,))
    # b1 = m: every user settled in step (3)
    bi = rm.BudgetIndex(_g(U), _g(P), kmax, m + 5, 0, "exp")
    assert bi.info["u_prime"] == 0 and bi.info["cert3"] == n
    _check_state(U, P, bi, orc.budget_preprocess(U, P, kmax, m + 5, 0, "exp"), kmax)
    # no dynamic budget: one more position per user of U'
    pre = orc.budget_preprocess(U, P, kmax, kmax, 0, "linear")
    bi = rm.BudgetIndex(_g(U), _g(P), kmax, kmax, 0, "linear")
    _check_state(U, P, bi, pre, kmax, None, topk)
    _check_query(bi, topk, m, (3, 12), (1, 25))


def test_budget_exact_ties():
    """Items that tie a user's value at the Cauchy-Schwarz bound, later in the
    norm order with a smaller id, and users opposite to every item."""
    import paper_2504_13445_amd as rm
    rng = np.random.default_rng(7)
    m, d = 64, 4
    P = np.zeros((m, d), np.float32)
    for j in range(m):
        P[j, 0] = 8.0 - (j // 4) * 0.25
        P[j, 1] = float(j % 4)
    U = np.zeros((48, d), np.float32)
    U[:20, 0] = rng.integers(1, 4, 20)
    U[20:36] = rng.integers(-3, 4, (16, d)).astype(np.float32)
    U[36:, 0] = -rng.integers(1, 4, 12)
    U[36:, 1] = -1.0
    kmax = 6
    V = orc.inner_products(U, P)
    topv, topk = orc.kmips_table(U, P, kmax, V)
    for b1, per, kind in ((6, 3, "uniform"), (6, 0, "uniform"), (10, 50, "exp")):
        pre = orc.budget_preprocess(U, P, kmax, b1, per * U.shape[0], kind)
        bi = rm.BudgetIndex(_g(U), _g(P), kmax, b1, per * U.shape[0], kind)
        _check_state(U, P, bi, pre, kmax, V, topk)
        _check_query(bi, topk, m, (1, 3, 6), (1, 4, 20))


def test_budget_mf_workload():
    # the 100,000 x 20,000 x 50 workload, k_max = 10 (its k)
    import paper_2504_13445_amd as rm
    cfg = synth.CONFIGS[1]
    U, P = synth.make_config(cfg)
    kmax, b1, B2 = 10, 20, 30 * U.shape[0]
    print("[case] budget mf oracle", flush=True)
    pre = orc.budget_preprocess(U, P, kmax, b1, B2, "exp")
    topv, topk = orc.kmips_table_c(U, P, kmax)
    print("[case] budget mf gpu", flush=True)
    bi = rm.BudgetIndex(_g(U), _g(P), kmax, b1, B2, "exp")
    _check_state(U, P, bi, pre, kmax, None, topk)
    _check_query(bi, topk, P.shape[0], (1, 10), (10, 100))


def test_budget_bf16_workload_golden():
    # the 500,000 x 50,000 x 100 workload: the query's top-50 at k = 20
    # against the full-oracle golden (all scores from the FP64 oracle)
    import paper_2504_13445_amd as rm
    gold = json.load(open(os.path.join(HERE, "golden", "bf16_workload_scores.json")))
    cfg = synth.CONFIGS[2]
    U, P = synth.make_config(cfg)
    import hashlib
    assert hashlib.sha256(np.ascontiguousarray(U).tobytes()).hexdigest() == gold["sha256_U"]
    n, m = U.shape[0], P.shape[0]
    print("[case] budget bf16 workload", flush=True)
    bi = rm.BudgetIndex(_g(U), _g(P), 25, 50, 40 * n, "exp", prec="bf16")
    ids, sc, st = bi.topn(cfg.k, cfg.N)
    assert ids.tolist() == gold["top_ids"] and sc.tolist() == gold["top_scores"], st
    # Theorem 3 at k = 20 against the golden's exact scores
    us = bi.state()["uscore"][cfg.k - 1].cpu().numpy()
    assert np.all(us >= np.asarray(gold["scores"]))
    # sampled users: the lists against the definition
    g = _state(bi)
    rng = np.random.default_rng(5)
    sample = rng.choice(n, 300, replace=False)
    order = g["order"]
    Vs = orc.inner_products_c(U[sample], P)
    for i, u in enumerate(sample):
        if g["pos"][u] == 0:
            want = np.lexsort((np.arange(m), -Vs[i]))[:25]
        else:
            pref = order[: g["pos"][u]]
            want = pref[np.lexsort((pref, -Vs[i, pref]))[:25]]
        assert g["Aj"][u].tolist() == want.tolist(), u
        assert np.array_equal(g["Av"][u], Vs[i, want])


def test_budget_rejects_bad_arguments():
    import paper_2504_13445_amd as rm
    U, P = synth.make_config(0)
    Ug, Pg = _g(U), _g(P)
    for kw in ({"b1": 5}, {"kind": "cubic"}, {"alpha": -1.0}, {"B2": -3}):
        args = {"b1": 30, "B2": 100, "kind": "exp", "alpha": 1.0}
        args.update(kw)
        if args["kind"] not in rm._lib.BUDGET_KINDS:
            with pytest.raises(KeyError):
                rm.BudgetIndex(Ug, Pg, 10, **args)
            continue
        with pytest.raises(rm.RmipsError):
            rm.BudgetIndex(Ug, Pg, 10, **args)
    bi = rm.BudgetIndex(Ug, Pg, 10, 30, 1000, "exp")
    with pytest.raises(rm.RmipsError):
        bi.topn(11, 10)          # k > kmax
    bi.kmax = 9                  # another kmax than the build's: the header check
    with pytest.raises(rm.RmipsError):
        bi.topn(5, 10)
    bi.kmax = 10
    topv, topk = orc.kmips_table(U, P, 10)
    _check_query(bi, topk, P.shape[0], (10,), (10,))

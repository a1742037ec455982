"""GPU parity: every librmips output against the CPU FP64 oracle.

Integer outputs (ids, scores) and the FP64 thresholds must match bit for
bit; inputs are the seeded synthetic workloads plus hand-built tie cases.
"""
import numpy as np
import pytest

import oracle as orc
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)


def _rm():
    import paper_2504_13445_amd as rm
    return rm


def _g(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(_dev())


PRECS = ["fp32", "bf16", "fp8", "fp6", "fp4"]


def _check_thresholds(U, P, k, **kw):
    rm = _rm()
    tau, tid, topk = rm.thresholds(_g(U), _g(P), k, with_topk=True, **kw)
    t, j, tk = orc.kmips_c(U, P, k)
    tau, tid, topk = tau.cpu().numpy(), tid.cpu().numpy(), topk.cpu().numpy()
    bad = np.nonzero((tau.view(np.uint64) != t.view(np.uint64)) | (tid != j))[0]
    assert bad.size == 0, (bad[:10], tau[bad[:5]], t[bad[:5]], tid[bad[:5]], j[bad[:5]])
    assert np.array_equal(topk, tk)
    return t, j, tk


def _check_topn(U, P, k, N, topk_ref=None, **kw):
    rm = _rm()
    if topk_ref is None:
        _, _, topk_ref = orc.kmips_c(U, P, k)
    ri, rs = orc.topn_from_scores(orc.histogram_scores(topk_ref, P.shape[0]), N)
    ids, sc, st = rm.topn(_g(U), _g(P), k, N, **kw)
    assert ids.tolist() == ri.tolist() and sc.tolist() == rs.tolist(), (ids, ri, sc, rs)
    return st


# ------------------------------------------------------------ stage (a)
@pytest.mark.parametrize("prec", PRECS)
def test_thresholds_tiny_workload(prec):
    _say("thresholds tiny 2000x1000x16 k=10", prec)
    U, P = synth.make_config(0)
    _check_thresholds(U, P, 10, prec=prec)


@pytest.mark.parametrize("n,m,d,k", [(1, 1, 1, 1), (7, 3, 5, 3), (130, 65, 17, 32),
                                     (300, 64, 8, 1), (257, 129, 33, 7), (64, 500, 255, 20),
                                     (1000, 4097, 50, 10)])
@pytest.mark.parametrize("prec", PRECS)
def test_thresholds_shapes(n, m, d, k, prec):
    _say("thresholds shape", n, m, d, k, prec)
    rng = np.random.default_rng(n * 7 + m)
    U = synth.isotropic(rng, n, d, 0.3)
    P = synth.isotropic(rng, m, d, 0.6)
    _check_thresholds(U, P, k, prec=prec)


@pytest.mark.parametrize("prec", PRECS)
def test_thresholds_forced_fallback(prec):
    _say("thresholds forced fallback cap=1", prec)
    U, P = synth.make_config(0, n=600, m=900)
    _check_thresholds(U, P, 10, cand_cap=1, prec=prec)


@pytest.mark.parametrize("prec", PRECS)
def test_thresholds_ties_and_zeros(prec):
    _say("thresholds ties", prec)
    rng = np.random.default_rng(5)
    P = rng.integers(-2, 3, size=(200, 6)).astype(np.float32)
    P[100:150] = P[0:50]          # exact duplicates
    P[150:160] = 0.0              # zero items
    U = rng.integers(-2, 3, size=(300, 6)).astype(np.float32)
    U[:5] = 0.0                   # zero users: every item ties at 0
    for k in (1, 5, 17):
        _check_thresholds(U, P, k, prec=prec)


def test_thresholds_onehot_golden(golden_dir):
    import json, os
    g = json.load(open(os.path.join(golden_dir, "onehot_case.json")))
    U = np.array(g["U"], np.float32)
    P = np.array(g["P"], np.float32)
    rm = _rm()
    for ks, e in g["k"].items():
        _say("onehot k", ks)
        tau, tid, topk = rm.thresholds(_g(U), _g(P), int(ks), with_topk=True)
        assert tau.cpu().numpy().tolist() == e["tau"]
        assert tid.cpu().numpy().tolist() == e["tau_id"]
        assert topk.cpu().numpy().tolist() == e["topk"]


@pytest.mark.parametrize("prec", PRECS)
def test_thresholds_tiny_magnitudes(prec):
    # entries of about 1e-20 (normal FP32 values) whose products, about
    # 1e-40, fall into the FP32 subnormal range: the absolute term of the
    # screen's bound must cover the rounding there
    _say("thresholds inputs with subnormal products", prec)
    rng = np.random.default_rng(8)
    U = (synth.isotropic(rng, 200, 12, 0.3).astype(np.float64) * 1e-20).astype(np.float32)
    P = (synth.isotropic(rng, 300, 12, 0.3).astype(np.float64) * 1e-20).astype(np.float32)
    _check_thresholds(U, P, 5, prec=prec)


# ------------------------------------------------------------ subnormal operands
def _subnormal(rng, shape):
    """FP32 subnormal values: magnitudes log-uniform in [1e-45, 1e-38]
    (1e-45 rounds to the smallest subnormal, 2^-149), random signs."""
    mag = 10.0 ** rng.uniform(-45.0, -38.0, size=shape)
    x = (mag * rng.choice([-1.0, 1.0], size=shape)).astype(np.float32)
    x[x == 0] = np.float32(2.0 ** -149)
    assert (np.abs(x) < np.float32(2.0 ** -126)).all()
    return x


def _subnormal_case(kind):
    rng = np.random.default_rng({"all": 11, "users": 12, "mixed": 13}[kind])
    d = 12
    if kind == "all":            # every entry of every vector subnormal
        return _subnormal(rng, (150, d)), _subnormal(rng, (200, d))
    if kind == "users":
        # all-subnormal user rows beside ordinary ones, against unit-norm
        # items and items of norm about 2^40 (products up to ~1e-26, far
        # above the bound's absolute term: only the residual term of the
        # subnormal rows can cover them)
        U = synth.isotropic(rng, 160, d, 0.3)
        U[::2] = _subnormal(rng, (80, d))
        P = synth.isotropic(rng, 240, d, 0.5)
        P[::3] = (P[::3].astype(np.float64) * 2.0 ** 40).astype(np.float32)
        return U, P
    # mixed rows: a third of the entries subnormal, and items that differ
    # from an earlier item in one subnormal entry only
    U = synth.isotropic(rng, 200, d, 0.3)
    P = synth.isotropic(rng, 260, d, 0.5)
    for X in (U, P):
        mask = rng.random(X.shape) < 1.0 / 3.0
        X[mask] = _subnormal(rng, (int(mask.sum()),))
    P[200:230] = P[0:30]
    P[200:230, 5] = _subnormal(rng, (30,))
    return U, P


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kind", ["all", "users", "mixed"])
def test_subnormal_operands(kind, prec):
    """Subnormal inputs are zero in the screening copies and counted in the
    residual R, so thresholds, scores and top-N stay exact whatever the
    matrix cores do with subnormal operands."""
    _say("subnormal operands", kind, prec)
    U, P = _subnormal_case(kind)
    m = P.shape[0]
    for k in (1, 5):
        t, j, tk = _check_thresholds(U, P, k, prec=prec)
        rm = _rm()
        s = rm.scores(_g(U), _g(t), _g(j), _g(P),
                      torch.arange(m, dtype=torch.int32, device=_dev()), prec=prec)
        h = orc.histogram_scores(tk, m)
        assert np.array_equal(s.cpu().numpy(), h), kind
        _check_topn(U, P, k, 10, topk_ref=tk, prec=prec)


# ------------------------------------------------------------ stage (b)
@pytest.mark.parametrize("prec", PRECS)
def test_scores_all_items_equal_histogram(prec):
    _say("scores of all items, tiny workload", prec)
    U, P = synth.make_config(0)
    rm = _rm()
    k = 10
    t, j, tk = orc.kmips_c(U, P, k)
    Ug = _g(U)
    tau, tid = rm.thresholds(Ug, _g(P), k, prec=prec)
    s = rm.scores(Ug, tau, tid, _g(P), torch.arange(P.shape[0], dtype=torch.int32,
                                                      device=_dev()), prec=prec)
    h = orc.histogram_scores(tk, P.shape[0])
    assert np.array_equal(s.cpu().numpy(), h)
    assert int(s.sum()) == U.shape[0] * k


@pytest.mark.parametrize("prec", PRECS)
def test_scores_external_and_duplicate_queries(prec):
    _say("scores external queries", prec)
    U, P = synth.make_config(0, n=800, m=300)
    rm = _rm()
    k = 7
    t, j, _ = orc.kmips_c(U, P, k)
    rng = np.random.default_rng(3)
    Q = (rng.standard_normal((40, U.shape[1])) * 0.8).astype(np.float32)
    Q[:10] = P[:10]                       # duplicates of items: lose every tie
    qid = np.full(40, -1, np.int32)
    qid[10:20] = np.arange(10, 20)        # members of P: tie rule by id
    Q[10:20] = P[10:20]
    ref = orc.reverse_counts_c(U, t, j, Q, qid)
    s = rm.scores(_g(U), _g(t), _g(j), _g(Q), _g(qid), prec=prec)
    assert np.array_equal(s.cpu().numpy(), ref)


# ------------------------------------------------------------ top-N
@pytest.mark.parametrize("prec", PRECS)
def test_topn_tiny_workload(prec):
    _say("topn tiny", prec)
    U, P = synth.make_config(0)
    st = _check_topn(U, P, 10, 10, prec=prec)
    assert st["visited_items"] <= P.shape[0]


@pytest.mark.parametrize("batch", [(1, 1), (16, 64), (4096, 4096)])
def test_topn_batch_invariance(batch):
    _say("topn batch", batch)
    U, P = synth.make_config(0, n=1200, m=400)
    _check_topn(U, P, 5, 20, batch=batch)


@pytest.mark.parametrize("k,N", [(1, 1), (32, 50), (3, 400)])
def test_topn_parameters(k, N):
    _say("topn k N", k, N)
    U, P = synth.make_config(1, n=3000, m=400)
    _check_topn(U, P, k, N)


@pytest.mark.parametrize("prec", PRECS)
def test_topn_ties(prec):
    _say("topn ties", prec)
    rng = np.random.default_rng(6)
    P = rng.integers(-2, 3, size=(120, 5)).astype(np.float32)
    P[60:] = P[:60]
    U = rng.integers(-2, 3, size=(500, 5)).astype(np.float32)
    for k, N in ((3, 10), (8, 60)):
        _check_topn(U, P, k, N, prec=prec)


@pytest.mark.parametrize("prec", PRECS)
def test_topn_forced_fallback_and_small_batches(prec):
    _say("topn forced fallback", prec)
    U, P = synth.make_config(0, n=700, m=500)
    _check_topn(U, P, 10, 10, cand_cap=2, batch=(8, 32), prec=prec)


def _bound_case(shape):
    if shape == "d50":
        return synth.make_config(1, n=3000, m=2000), 10
    if shape == "d100":
        return synth.make_config(2, n=4000, m=1500), 20
    if shape == "d200":
        return synth.make_config(3, n=3000, m=1000), 10
    if shape in ("d240", "d256"):
        # the longest augmented rows (ka = 256 and 272: the bound kernel's
        # two- and one-step read groups)
        d = int(shape[1:])
        rng = np.random.default_rng(d)
        U = rng.standard_normal((2000, d)) * rng.lognormal(0.0, 0.25, (2000, 1))
        P = rng.standard_normal((700, d)) * rng.lognormal(0.0, 0.8, (700, 1))
        return (U.astype(np.float32), P.astype(np.float32)), 10
    # subnormal range: the bound's absolute slack
    (U, P), k = synth.make_config(2, n=2000, m=800), 10
    return (U * np.float32(1e-19), P * np.float32(1e-19)), k


@pytest.mark.parametrize("dprime", [0, 10, 62])
@pytest.mark.parametrize("shape", ["d50", "d100", "d200", "d240", "d256", "tiny_values"])
def test_topn_bound_counts_dominate_scores(shape, dprime):
    """The Eq. (3)/(6) bound count of every item (BF16 products with a
    certified slack) is at least its exact score (Theorem 2), with d' = d
    (dprime 0: no rotation) and with the users' top-d' eigenvectors (d' = 10,
    62); with d' = d it counts no user whose exact value is below tau_u by
    more than twice the relative slack 2^-7 of ||u|| ||p|| (the bound is then
    the inner product plus that slack, up to BF16 rounding that the slack
    covers).  The top-N is the same for every d'."""
    _say("topn bound counts", shape, "dprime", dprime)
    rm = _rm()
    (U, P), k = _bound_case(shape)
    m = P.shape[0]
    tau, _, tk = orc.kmips_c(U, P, k)
    score = orc.histogram_scores(tk, m)
    us = torch.zeros(m, dtype=torch.int32, device=_dev())
    ri, rs = orc.topn_from_scores(score, 10)
    # (no pre-pass: the d' = d bound of every item)
    ids, sc, _ = rm.topn(_g(U), _g(P), k, 10, prec="bf16", bound_out=us, dprime=dprime,
                         prepass=0)
    assert ids.tolist() == ri.tolist() and sc.tolist() == rs.tolist()
    us = us.cpu().numpy().astype(np.int64)
    bad = np.nonzero(us < score)[0]
    assert bad.size == 0, (bad[:10], us[bad[:10]], score[bad[:10]])
    assert us.max() <= U.shape[0]
    if dprime == 0:
        U64, P64 = U.astype(np.float64), P.astype(np.float64)
        V = U64 @ P64.T
        slack = 2.0 ** -6 * np.linalg.norm(U64, axis=1)[:, None] * np.linalg.norm(P64, axis=1)
        reach = (V + slack + 2.0 ** -59 >= tau[:, None]).sum(axis=0)
        over = np.nonzero(us > reach)[0]
        assert over.size == 0, (over[:10], us[over[:10]], reach[over[:10]])


@pytest.mark.parametrize("d", [20, 33, 70, 130, 150, 190, 230])
def test_topn_bound_counts_every_row_length(d):
    """The bound kernels of every augmented row length in between (ka = 32
    to 256: register-resident users, LDS stages of 256 and 128 users, the
    32x32 and the 16x16 matrix-core forms): bound counts at or above the
    exact scores and the exact top-N, with d' = d (every item, no pre-pass)."""
    _say("topn bound counts, d", d)
    rm = _rm()
    rng = np.random.default_rng(1000 + d)
    U = (rng.standard_normal((1500, d)) * rng.lognormal(0.0, 0.25, (1500, 1))).astype(np.float32)
    P = (rng.standard_normal((1100, d)) * rng.lognormal(0.0, 0.8, (1100, 1))).astype(np.float32)
    m = P.shape[0]
    _, _, tk = orc.kmips_c(U, P, 10)
    score = orc.histogram_scores(tk, m)
    us = torch.zeros(m, dtype=torch.int32, device=_dev())
    ri, rs = orc.topn_from_scores(score, 20)
    ids, sc, _ = rm.topn(_g(U), _g(P), 10, 20, prec="bf16", bound_out=us, prepass=0)
    assert ids.tolist() == ri.tolist() and sc.tolist() == rs.tolist()
    us = us.cpu().numpy().astype(np.int64)
    bad = np.nonzero(us < score)[0]
    assert bad.size == 0, (bad[:10], us[bad[:10]], score[bad[:10]])
    assert us.max() <= U.shape[0]


@pytest.mark.parametrize("d,prepass,batch,prec", [
    (50, 10, (16, 64), "bf16"), (130, -1, (16, 64), "bf16"), (200, -1, (16, 64), "fp32"),
    (200, 30, (4, 8), "bf16"), (240, 62, (16, 64), "fp8"), (256, -1, None, "bf16")])
def test_topn_prepass(d, prepass, batch, prec):
    """The rotated pre-pass before the d' = d bound (Eq. 3 with a rotation,
    then with the identity for the items it leaves open once the first
    batches give an N-th score): the exact top-N, bound counts at or above
    the exact scores, and every item's count either the pre-pass one (the
    bound of the same rotation alone) or, for the items bounded again, the
    smaller of that and the d' = d count (the bound without a pre-pass).  A
    first batch of 4 items (N = 10) takes the N-th score from a later
    batch."""
    _say("topn prepass, d", d, "prepass", prepass, "batch", batch, prec)
    rm = _rm()
    rng = np.random.default_rng(2000 + d)
    C = rng.standard_normal((12, d))
    U = (C[rng.integers(0, 12, 3000)] + 0.7 * rng.standard_normal((3000, d)))
    U = (U * rng.lognormal(0.0, 0.25, (3000, 1))).astype(np.float32)
    P = (rng.standard_normal((1500, d)) * rng.lognormal(0.0, 0.8, (1500, 1))).astype(np.float32)
    m = P.shape[0]
    _, _, tk = orc.kmips_c(U, P, 10)
    score = orc.histogram_scores(tk, m)
    ri, rs = orc.topn_from_scores(score, 10)
    us = torch.zeros(m, dtype=torch.int32, device=_dev())
    u0 = torch.zeros(m, dtype=torch.int32, device=_dev())
    ids, sc, st = rm.topn(_g(U), _g(P), 10, 10, prec=prec, bound_out=us, prepass=prepass,
                          batch=batch)
    print("stats", st, flush=True)
    assert ids.tolist() == ri.tolist() and sc.tolist() == rs.tolist()
    assert st["prepass_dprime"] == (62 if prepass == -1 else prepass)
    if prepass == -1:  # automatic: FP32 and BF16 screening only
        _, _, s8 = rm.topn(_g(U), _g(P), 10, 10, prec="fp8")
        assert s8["prepass_dprime"] == 0 and s8["rebound_items"] == 0
    assert st["rebound_items"] > 0 and st["rebound_pairs"] > 0
    ids0, sc0, st0 = rm.topn(_g(U), _g(P), 10, 10, prec=prec, bound_out=u0, prepass=0,
                             batch=batch)
    assert st0["prepass_dprime"] == 0 and st0["rebound_items"] == 0
    assert ids0.tolist() == ri.tolist() and sc0.tolist() == rs.tolist()
    dpre = st["prepass_dprime"]
    ur = torch.zeros(m, dtype=torch.int32, device=_dev())
    ids1, sc1, _ = rm.topn(_g(U), _g(P), 10, 10, prec=prec, bound_out=ur, dprime=dpre,
                           batch=batch)
    assert ids1.tolist() == ri.tolist() and sc1.tolist() == rs.tolist()
    us = us.cpu().numpy().astype(np.int64)
    u0 = u0.cpu().numpy().astype(np.int64)
    ur = ur.cpu().numpy().astype(np.int64)
    bad = np.nonzero(us < score)[0]
    assert bad.size == 0, (bad[:10], us[bad[:10]], score[bad[:10]])
    assert us.max() <= U.shape[0]
    ok = (us == ur) | (us == np.minimum(ur, u0))
    assert ok.all(), np.nonzero(~ok)[0][:10]
    assert (us < ur).any()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("cap", [2, 4])
def test_topn_refinement_passes(prec, cap):
    """Short candidate lists: users whose lists overflow are screened again
    from the k-th largest lower bound among their stored candidates, the
    rest go to the exact fallback; results stay exact either way."""
    _say("topn refinement passes", prec, cap)
    U, P = synth.make_config(1, n=3000, m=4000)
    _, _, tk = orc.kmips_c(U, P, 10)
    st = _check_topn(U, P, 10, 10, topk_ref=tk, cand_cap=cap, prec=prec)
    print("stats", st, flush=True)
    assert st["refine_users"] + st["overflow_users"] > 0
    if cap >= 4 and prec != "fp4":
        # (with e2m1's band the lower bounds among a few stored candidates
        # never improve on the starting bound: every overflowing user goes
        # to the exact fallback instead)
        assert st["refine_users"] > 0
    _check_thresholds(U, P, 10, cand_cap=cap, prec=prec)


# ------------------------------------------------------------ full sizes
@pytest.fixture(scope="module")
def mf_workload():
    U, P = synth.make_config(1)
    t, j, tk = orc.kmips_c(U, P, 10)
    return U, P, t, j, tk


@pytest.mark.parametrize("prec", PRECS)
def test_mf_thresholds_full(mf_workload, prec):
    _say("mf thresholds 100000x20000x50", prec)
    U, P, t, j, tk = mf_workload
    rm = _rm()
    tau, tid, topk = rm.thresholds(_g(U), _g(P), 10, with_topk=True, prec=prec)
    assert np.array_equal(tau.cpu().numpy().view(np.uint64), t.view(np.uint64))
    assert np.array_equal(tid.cpu().numpy(), j)
    assert np.array_equal(topk.cpu().numpy(), tk)


@pytest.mark.parametrize("prec", PRECS)
def test_mf_topn_full(mf_workload, prec):
    _say("mf topn 100000x20000x50 k=10 N=10", prec)
    U, P, t, j, tk = mf_workload
    h = orc.histogram_scores(tk, P.shape[0])
    assert h.sum() == U.shape[0] * 10
    st = _check_topn(U, P, 10, 10, topk_ref=tk, prec=prec)
    print("stats", st, flush=True)

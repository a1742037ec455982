"""GPU parity of the k_max index (Alg. 1's offline stage, Sec. 4.2; the
online stage of Alg. 2, Sec. 4.3) against the CPU FP64 oracle: the
thresholds of every k from one build bit for bit, the bound of every item
for every k above its exact score (Theorem 2), and the top-N of any
(k <= k_max, N) identical to the oracle's."""
import numpy as np
import pytest

import oracle as orc
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KMAX = 25


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _g(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(_dev())


def _check_index(U, P, prec, ks, Ns, kmax=KMAX, dprime=None):
    import paper_2504_13445_amd as rm
    n, m = U.shape[0], P.shape[0]
    topv, topk = orc.kmips_table_c(U, P, kmax)
    idx = rm.Index(_g(U), _g(P), kmax, prec, dprime=dprime)
    prev = None
    for k in range(1, kmax + 1):
        score = orc.histogram_scores(topk[:, :k], m)
        us = idx.bounds(k).cpu().numpy().astype(np.int64)
        bad = np.nonzero(us < score)[0]
        assert bad.size == 0, (k, bad[:10], us[bad[:10]], score[bad[:10]])
        assert us.max() <= n
        if prev is not None:
            assert (us >= prev).all(), k   # thresholds fall with k: bounds grow
        prev = us
        if k in ks:
            print("[case] index", prec, n, m, "k", k, flush=True)
            tau, tid = idx.thresholds(k)
            assert np.array_equal(tau.cpu().numpy().view(np.uint64),
                                  topv[:, k - 1].view(np.uint64)), k
            assert np.array_equal(tid.cpu().numpy(), topk[:, k - 1]), k
            for N in Ns:
                ri, rs = orc.topn_from_table(topk, k, N, m)
                ids, sc, st = idx.topn(k, N)
                assert ids.tolist() == ri.tolist() and sc.tolist() == rs.tolist(), (k, N)
                assert st["visited_items"] <= m
    return idx


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8", "fp6", "fp4"])
def test_index_tiny_workload(prec):
    U, P = synth.make_config(0)
    _check_index(U, P, prec, (1, 10, 25), (10, 37))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_index_mf_workload(prec):
    U, P = synth.make_config(1)
    _check_index(U, P, prec, (1, 10, 25), (10,))


@pytest.mark.parametrize("dprime", [None, 62])
def test_index_rotation_and_ties(dprime):
    # d = 200: the bound table on the full rows (d' = d) and on the rotated,
    # split rows (d' = 62); integer inputs with duplicated items give exact
    # ties everywhere
    U, P = synth.make_config(3, n=3000, m=900)
    _check_index(U, P, "bf16", (1, 7, 25), (10,), dprime=dprime)
    rng = np.random.default_rng(4)
    Pi = rng.integers(-2, 3, size=(90, 5)).astype(np.float32)
    Pi[45:] = Pi[:45]
    Ui = rng.integers(-2, 3, size=(700, 5)).astype(np.float32)
    _check_index(Ui, Pi, "fp32", (1, 3, 8), (10, 60), kmax=8)


def test_index_rejects_bad_arguments():
    import paper_2504_13445_amd as rm
    from paper_2504_13445_amd import _lib
    U, P = synth.make_config(0, n=500, m=200)
    idx = rm.Index(_g(U), _g(P), 8, "fp32")
    with pytest.raises(rm.RmipsError) as e:
        idx.topn(9, 5)                                 # k above kmax
    assert e.value.status == _lib.RMIPS_EINVAL
    idx.kmax = 7                                       # not the sizes it was built with
    with pytest.raises(rm.RmipsError) as e:
        idx.topn(3, 5)
    assert e.value.status == _lib.RMIPS_EINVAL
    idx.kmax = 8
    t, j, tk = orc.kmips_c(U, P, 3)
    ri, rs = orc.topn_from_scores(orc.histogram_scores(tk, 200), 5)
    ids, sc, _ = idx.topn(3, 5)
    assert ids.tolist() == ri.tolist() and sc.tolist() == rs.tolist()

"""Error paths of librmips on the GPU.

Inputs the library must reject: a NaN or an Inf in a vector, a vector whose
norm exceeds 2^60 (the bound on norms that keeps the screening arithmetic
finite), and sizes out of range.  Each rejection is followed by a valid call
on the same context, whose results must still match the FP64 oracle: stage
(b) of rmips_topn starts before the input check is read on the host, so a
rejected call must leave nothing behind that a later call could see.
"""
import numpy as np
import pytest

import oracle as orc
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PRECS = ["fp32", "bf16", "fp8", "fp6", "fp4"]
BAD = ["nan_user", "inf_item", "huge_user", "huge_item"]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)


def _rm():
    import paper_2504_13445_amd as rm
    from paper_2504_13445_amd import _lib
    return rm, _lib


def _g(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(_dev())


def _poison(U, P, kind):
    """One bad entry in a copy of U or P."""
    U, P = U.copy(), P.copy()
    if kind == "nan_user":
        U[17, 3] = np.nan
    elif kind == "inf_item":
        P[5, 0] = np.inf
    elif kind == "huge_user":   # finite, norm 2^61 > 2^60
        U[0, :] = 0.0
        U[0, 0] = 2.0 ** 61
    elif kind == "huge_item":
        P[P.shape[0] - 1, :] = 0.0
        P[P.shape[0] - 1, 1] = -(2.0 ** 61)
    return U, P


def _topn_ref(U, P, k, N):
    _, _, topk = orc.kmips_c(U, P, k)
    return orc.topn_from_scores(orc.histogram_scores(topk, P.shape[0]), N)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kind", BAD)
def test_topn_rejects_then_recovers(kind, prec):
    _say("topn rejects", kind, prec)
    rm, lib = _rm()
    U, P = synth.make_config(0, n=600, m=300)
    Ub, Pb = _poison(U, P, kind)
    with pytest.raises(rm.RmipsError) as e:
        rm.topn(_g(Ub), _g(Pb), 5, 10, prec=prec)
    assert e.value.status == lib.RMIPS_ENONFINITE
    ri, rs = _topn_ref(U, P, 5, 10)
    ids, sc, _ = rm.topn(_g(U), _g(P), 5, 10, prec=prec)
    assert ids.tolist() == ri.tolist() and sc.tolist() == rs.tolist()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kind", BAD)
def test_thresholds_rejects_then_recovers(kind, prec):
    _say("thresholds rejects", kind, prec)
    rm, lib = _rm()
    U, P = synth.make_config(0, n=500, m=200)
    Ub, Pb = _poison(U, P, kind)
    with pytest.raises(rm.RmipsError) as e:
        rm.thresholds(_g(Ub), _g(Pb), 4, prec=prec)
    assert e.value.status == lib.RMIPS_ENONFINITE
    tau_ref, id_ref, _ = orc.kmips_c(U, P, 4)
    tau, tid = rm.thresholds(_g(U), _g(P), 4, prec=prec)
    assert np.array_equal(tau.cpu().numpy().view(np.uint64), tau_ref.view(np.uint64))
    assert np.array_equal(tid.cpu().numpy(), id_ref)


@pytest.mark.parametrize("prec", PRECS)
def test_scores_rejects_bad_query(prec):
    _say("scores rejects", prec)
    rm, lib = _rm()
    U, P = synth.make_config(0, n=400, m=100)
    tau, tid, _ = orc.kmips_c(U, P, 3)
    Q = P[:20].copy()
    Q[7, 2] = np.nan
    with pytest.raises(rm.RmipsError) as e:
        rm.scores(_g(U), _g(tau), _g(tid.astype(np.int32)), _g(Q), prec=prec)
    assert e.value.status == lib.RMIPS_ENONFINITE


def test_topn_rejects_sizes_out_of_range():
    _say("topn sizes out of range")
    rm, lib = _rm()
    U, P = synth.make_config(0, n=100, m=50)
    cases = [dict(k=51, N=5),              # k > m
             dict(k=5, N=51),              # N > m
             dict(k=0, N=5),               # k < 1
             dict(k=5, N=0)]               # N < 1
    for c in cases:
        with pytest.raises((rm.RmipsError, ValueError)) as e:
            rm.topn(_g(U), _g(P), c["k"], c["N"])
        if isinstance(e.value, rm.RmipsError):
            assert e.value.status == lib.RMIPS_EINVAL, c
    ri, rs = _topn_ref(U, P, 5, 5)
    ids, sc, _ = rm.topn(_g(U), _g(P), 5, 5)
    assert ids.tolist() == ri.tolist() and sc.tolist() == rs.tolist()


def test_set_prepass_rejects_out_of_range():
    """rmips_set_prepass takes -1 (automatic), 0 (none) or 1..62."""
    _say("set_prepass out of range")
    rm, lib = _rm()
    U, P = synth.make_config(0, n=100, m=50)
    for dp in (-2, 63):
        with pytest.raises(rm.RmipsError) as e:
            rm.topn(_g(U), _g(P), 5, 5, prepass=dp)
        assert e.value.status == lib.RMIPS_EINVAL, dp
    ri, rs = _topn_ref(U, P, 5, 5)
    for dp in (None, 0, 3):
        ids, sc, _ = rm.topn(_g(U), _g(P), 5, 5, prepass=dp)
        assert ids.tolist() == ri.tolist() and sc.tolist() == rs.tolist(), dp


def test_set_dprime_rejects_out_of_range():
    """rmips_set_dprime takes 0 (d' = d) or a rotation to 1..62 dimensions."""
    _say("set_dprime out of range")
    rm, lib = _rm()
    U, P = synth.make_config(0, n=100, m=50)
    for dp in (-1, 63):
        with pytest.raises(rm.RmipsError) as e:
            rm.topn(_g(U), _g(P), 5, 5, dprime=dp)
        assert e.value.status == lib.RMIPS_EINVAL, dp
    ri, rs = _topn_ref(U, P, 5, 5)
    for dp in (None, 3):
        ids, sc, _ = rm.topn(_g(U), _g(P), 5, 5, dprime=dp)
        assert ids.tolist() == ri.tolist() and sc.tolist() == rs.tolist(), dp

"""The relaxed-score gradient entry point that allocates nothing
(rmips_soft_bwd_noalloc: partial sums in the library's static per-device
scratch) against the workspace entry point rmips_soft_bwd, through the C
ABI, on two calls in a row, the second with a smaller input."""
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


def _g(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(_dev())


def _case(n, m, d, nq, seed):
    rng = np.random.default_rng(seed)
    U = synth.clustered(rng, n, d, 0.25, 64, 0.5)
    P = synth.isotropic(rng, m, d, 0.8)
    Q = (rng.standard_normal((nq, d)) / np.sqrt(d)).astype(np.float32)
    tau = orc.kmips_c(U, P, 10, with_topk=False)[0].astype(np.float32)
    T = float(orc.temperature(U, P))
    dS = np.linspace(0.5, 1.5, nq).astype(np.float32)
    return U, Q, tau, T, dS


def test_soft_bwd_noalloc_matches_workspace_entry_point():
    import paper_2504_13445_amd as rm
    from paper_2504_13445_amd import _lib
    # second call smaller in every size: users, queries and dims
    for (n, m, d, nq, seed) in ((6000, 800, 100, 256, 1), (2500, 300, 40, 37, 2)):
        print("[case] soft_bwd_noalloc", n, m, d, nq, flush=True)
        U, Q, tau, T, dS = _case(n, m, d, nq, seed)
        Ug, Qg, tg, dSg = _g(U), _g(Q), _g(tau), _g(dS)
        ref = rm.soft_bwd(Ug, tg, Qg, T, dSg).cpu().numpy()
        got = _lib.soft_bwd_noalloc(Ug, tg, Qg, T, dSg).cpu().numpy()
        # the same kernels in the same fixed order: identical bits
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (n, nq, d)
        G64 = orc.soft_grad(U, tau.astype(np.float64), Q, T) * dS[:, None]
        num = np.linalg.norm(got.astype(np.float64) - G64, axis=1)
        den = np.linalg.norm(G64, axis=1)
        ok = den > 1e-30
        assert (num[ok] <= 1e-4 * den[ok]).all(), (num[ok] / den[ok]).max()


def test_soft_bwd_noalloc_rejects_oversize():
    import paper_2504_13445_amd as rm
    from paper_2504_13445_amd import _lib
    U, Q, tau, T, dS = _case(500, 100, 256, 257, 3)   # 257 * 256 > 65536
    with pytest.raises(rm.RmipsError) as e:
        _lib.soft_bwd_noalloc(_g(U), _g(tau), _g(Q), T, _g(dS))
    assert e.value.status == _lib.RMIPS_EINVAL

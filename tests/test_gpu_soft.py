"""GPU parity of the relaxed score S(q) and its gradient against the FP64
oracle (tolerance 1e-4 relative), plus central finite differences."""
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


def _case(n, m, d, nq, seed=4, k=10):
    cfg = synth.CONFIGS[4]
    rng = np.random.default_rng(seed)
    U = synth.clustered(rng, n, d, cfg.user_sigma, 64, 0.5)
    P = synth.isotropic(rng, m, d, cfg.item_sigma)
    Q = (rng.standard_normal((nq, d)) / np.sqrt(d)).astype(np.float32)
    tau64, _, _ = orc.kmips_c(U, P, k, with_topk=False)
    tau = tau64.astype(np.float32)           # the soft calls take FP32 thresholds
    T = float(orc.temperature(U, P))
    return U, P, Q, tau, T


def _check(U, Q, tau, T, tol=1e-4):
    import paper_2504_13445_amd as rm
    Ug, Qg, tg = _g(U), _g(Q), _g(tau)
    S = rm.soft_fwd(Ug, tg, Qg, T).cpu().numpy().astype(np.float64)
    S64 = orc.soft_score(U, tau.astype(np.float64), Q, T)
    rel = np.abs(S - S64) / np.maximum(S64, 1e-300)
    assert (rel[S64 > 1e-30] <= tol).all(), (rel.max(), S[:4], S64[:4])
    dS = np.linspace(0.5, 1.5, Q.shape[0]).astype(np.float32)
    G = rm.soft_bwd(Ug, tg, Qg, T, _g(dS)).cpu().numpy().astype(np.float64)
    G64 = orc.soft_grad(U, tau.astype(np.float64), Q, T) * dS[:, None]
    num = np.linalg.norm(G - G64, axis=1)
    den = np.linalg.norm(G64, axis=1)
    ok = den > 1e-30
    assert (num[ok] <= tol * den[ok]).all(), (num[ok] / den[ok]).max()
    return S, G


@pytest.mark.parametrize("n,m,d,nq", [(3000, 500, 100, 70), (1000, 300, 16, 5),
                                      (2049, 400, 50, 64), (700, 200, 200, 33)])
def test_soft_matches_fp64(n, m, d, nq):
    print("[case] soft", n, m, d, nq, flush=True)
    U, P, Q, tau, T = _case(n, m, d, nq)
    _check(U, Q, tau, T)


@pytest.mark.parametrize("n,m,d,nq", [(3000, 500, 100, 70), (900, 200, 8, 65), (1500, 300, 1, 3),
                                      (1200, 300, 128, 40), (800, 200, 129, 9),
                                      (700, 200, 256, 33), (4100, 300, 64, 128)])
def test_soft_fwd_grad_matches_fp64(n, m, d, nq):
    """S and its unscaled gradient from one pass (rmips_soft_fwd_grad), and
    the backward pass as rmips_soft_scale of that gradient."""
    print("[case] soft fwd+grad", n, m, d, nq, flush=True)
    import paper_2504_13445_amd as rm
    U, P, Q, tau, T = _case(n, m, d, nq)
    Ug, Qg, tg = _g(U), _g(Q), _g(tau)
    S, G = rm.soft_fwd_grad(Ug, tg, Qg, T)
    S64 = orc.soft_score(U, tau.astype(np.float64), Q, T)
    G64 = orc.soft_grad(U, tau.astype(np.float64), Q, T)
    S = S.cpu().numpy().astype(np.float64)
    rel = np.abs(S - S64) / np.maximum(S64, 1e-300)
    assert (rel[S64 > 1e-30] <= 1e-4).all(), rel.max()
    Gn = G.cpu().numpy().astype(np.float64)
    num = np.linalg.norm(Gn - G64, axis=1)
    den = np.linalg.norm(G64, axis=1)
    ok = den > 1e-30
    assert (num[ok] <= 1e-4 * den[ok]).all(), (num[ok] / den[ok]).max()
    dS = np.linspace(0.5, 1.5, nq).astype(np.float32)
    dQ = rm.soft_scale(G, _g(dS)).cpu().numpy()
    assert np.array_equal(dQ, (G.cpu().numpy() * dS[:, None]).astype(np.float32))
    # the fused pass forms the same sums as the separate calls
    S1 = rm.soft_fwd(Ug, tg, Qg, T).cpu().numpy()
    assert np.array_equal(S1.astype(np.float64), S)
    G1 = rm.soft_bwd(Ug, tg, Qg, T, torch.ones(nq, device=_dev())).cpu().numpy()
    assert np.array_equal(G1, G.cpu().numpy())


def test_soft_closed_form_identical_users():
    print("[case] soft identical users", flush=True)
    rng = np.random.default_rng(1)
    d = 24
    u = rng.standard_normal(d).astype(np.float32)
    U = np.repeat(u[None], 777, 0)
    tau = np.full(777, 0.25, np.float32)
    Q = (rng.standard_normal((9, d)) * 0.2).astype(np.float32)
    _check(U, Q, tau, 0.5)


def test_soft_autograd_and_finite_differences():
    print("[case] soft autograd + FD", flush=True)
    import paper_2504_13445_amd as rm
    U, P, Q, tau, T = _case(2000, 400, 32, 4)
    Ug, tg = _g(U), _g(tau)
    q = _g(Q).requires_grad_(True)
    S = rm.SoftScore.apply(q, Ug, tg, T)
    S.sum().backward()
    g = q.grad.cpu().numpy().astype(np.float64)
    Ud = U.astype(np.float64)
    rng = np.random.default_rng(2)
    h = 1e-6
    for i in range(Q.shape[0]):
        gn = np.linalg.norm(g[i])
        for _ in range(8):
            v = rng.standard_normal(Q.shape[1])
            v /= np.linalg.norm(v)
            q0 = Q[i].astype(np.float64)
            fd = (orc.sigmoid((Ud @ (q0 + h * v) - tau) / T).sum() -
                  orc.sigmoid((Ud @ (q0 - h * v) - tau) / T).sum()) / (2 * h)
            assert abs(fd - g[i] @ v) <= 1e-4 * gn + 1e-300, (fd, g[i] @ v, gn)


def test_soft_relaxed_workload_subsample():
    # the relaxed-score workload: users from the 1,000,000-user generator,
    # thresholds over its 50,000 items at k = 10, 256 queries; the FP64
    # oracle runs on a seeded subsample of the users
    print("[case] soft relaxed workload subsample", flush=True)
    cfg = synth.CONFIGS[4]
    U, P = synth.make_config(cfg)
    T = float(orc.temperature(U, P))
    sub = synth.subsample_users(cfg, 0.01)
    Us = np.ascontiguousarray(U[sub])
    tau = orc.kmips_c(Us, P, cfg.k, with_topk=False)[0].astype(np.float32)
    Q = synth.make_queries(cfg)
    S, G = _check(Us, Q, tau, T)
    assert np.isfinite(S).all() and (S > 0).all()


def test_soft_ascent_iterates_subsample():
    """The relaxed-score workload's 50 projected gradient-ascent steps
    (each query ascends its own S: q <- proj(q + eta g / ||g||), eta =
    0.02 R, proj(q) = q min(1, R / ||q||), R = median item norm) on the
    seeded 1% user subsample: S and dS/dq against the FP64 oracle at
    iterates 0, 10, 25 and 50 (1e-4 relative), and ||q|| <= R after every
    step."""
    print("[case] soft ascent iterates, 1% of the relaxed-score workload", flush=True)
    import paper_2504_13445_amd as rm
    cfg = synth.CONFIGS[4]
    U, P = synth.make_config(cfg)
    T = float(orc.temperature(U, P))
    R = float(np.median(np.sqrt((P.astype(np.float64) ** 2).sum(1))))
    sub = synth.subsample_users(cfg, 0.01)
    Us = np.ascontiguousarray(U[sub])
    del U
    tau = orc.kmips_c(Us, P, cfg.k, with_topk=False)[0].astype(np.float32)
    Ug, tg = _g(Us), _g(tau)
    q = _g(synth.make_queries(cfg))
    ones = torch.ones(q.shape[0], dtype=torch.float32, device=_dev())
    checked = []
    for it in range(51):
        if it in (0, 10, 25, 50):
            print("[case] ascent iterate", it, flush=True)
            _check(Us, q.cpu().numpy(), tau, T)
            checked.append(it)
        if it == 50:
            break
        g = rm.soft_bwd(Ug, tg, q, T, ones)
        gn = g.norm(dim=1, keepdim=True)
        step = torch.where(gn > 0, (0.02 * R) * g / gn.clamp_min(1e-30), torch.zeros_like(g))
        q = q + step
        qn = q.norm(dim=1, keepdim=True)
        q = (q * torch.clamp(R / qn.clamp_min(1e-30), max=1.0)).contiguous()
        qn64 = np.sqrt((q.cpu().numpy().astype(np.float64) ** 2).sum(1))
        assert (qn64 <= R * (1.0 + 1e-6)).all(), (it, qn64.max(), R)
    assert checked == [0, 10, 25, 50]

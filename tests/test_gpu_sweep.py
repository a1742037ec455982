"""GPU parity over a seeded sweep of small random problems: rmips_topn's
ids and scores and rmips_thresholds' tau (bit for bit) and tau ids against
the CPU FP64 oracle, at every screening precision, with d' = d and with the
paper's rotation, with and without a rotated pre-pass before the d' = d
bound, with default and small batches, on Gaussian, integer-valued (exact
ties, duplicated items), wide-scale and clustered inputs, at n, m, d, k and
N drawn across their ranges (d up to 256, k up to 32)."""
import numpy as np
import pytest

import oracle as orc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PRECS = ["fp32", "bf16", "fp8", "fp6", "fp4"]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _g(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(_dev())


def _case(seed):
    rng = np.random.default_rng(7000 + seed)
    n, m, d = int(rng.integers(40, 2500)), int(rng.integers(16, 1800)), int(rng.integers(1, 257))
    k = int(rng.integers(1, min(32, m) + 1))
    N = int(rng.integers(1, min(m, 64) + 1))
    prec = PRECS[seed % 5]
    dprime = 0 if rng.random() < 0.6 else int(rng.integers(1, 63))
    kind = seed % 4
    if kind == 0:    # Gaussian directions, log-normal norms
        U = rng.standard_normal((n, d)) * rng.lognormal(0, 0.3, (n, 1))
        P = rng.standard_normal((m, d)) * rng.lognormal(0, 0.8, (m, 1))
    elif kind == 1:  # small integers, the second half of the items a copy of the first
        U = rng.integers(-2, 3, (n, d)).astype(np.float64)
        P = rng.integers(-2, 3, (m, d)).astype(np.float64)
        P[m // 2:] = P[: m - m // 2]
    elif kind == 2:  # row norms spread over 16 decades
        U = rng.standard_normal((n, d)) * 10.0 ** rng.uniform(-8, 8, (n, 1))
        P = rng.standard_normal((m, d)) * 10.0 ** rng.uniform(-8, 8, (m, 1))
    else:            # users from 8 clusters
        C = rng.standard_normal((8, d))
        U = C[rng.integers(0, 8, n)] + 0.3 * rng.standard_normal((n, d))
        P = rng.standard_normal((m, d)) * rng.lognormal(0, 0.6, (m, 1))
    # the bound's pre-pass and the batch sizes of the counting loop, from a
    # stream of their own (the problems above stay as they were): automatic,
    # none or a rotation to 1..62 dimensions; first batches from 1 item, so
    # that the items still open are often re-bounded after a later batch
    r2 = np.random.default_rng(17000 + seed)
    prepass = -1 if r2.random() < 0.4 else (0 if r2.random() < 0.3 else int(r2.integers(1, 63)))
    batch = None
    if r2.random() < 0.5:
        first = int(r2.integers(1, 65))
        batch = (first, int(r2.integers(first, 257)))
    return U.astype(np.float32), P.astype(np.float32), k, N, prec, dprime, prepass, batch


@pytest.mark.parametrize("seed", range(100))
def test_random_problem(seed):
    import paper_2504_13445_amd as rm
    U, P, k, N, prec, dprime, prepass, batch = _case(seed)
    print("[case] sweep", seed, U.shape, P.shape, k, N, prec, dprime, prepass, batch, flush=True)
    tau, tid, tk = orc.kmips_c(U, P, k)
    ri, rs = orc.topn_from_scores(orc.histogram_scores(tk, P.shape[0]), N)
    ids, sc, _ = rm.topn(_g(U), _g(P), k, N, prec=prec, dprime=dprime, prepass=prepass,
                         batch=batch)
    assert ids.tolist() == ri.tolist() and sc.tolist() == rs.tolist()
    t, j = rm.thresholds(_g(U), _g(P), k, prec=prec)
    assert np.array_equal(t.cpu().numpy().view(np.uint64), tau.view(np.uint64))
    assert np.array_equal(j.cpu().numpy(), tid)

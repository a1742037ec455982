"""Parity at the full sizes of the screened workloads.

The FP64 oracle checks tau and S_k(u) bit for bit on a seeded 1% user
subsample; properties that hold at any size check the rest: every user's
S_k has k items (sum of scores over all items = n k), the pruned top-N
equals the top-N of the exact scores of all items (the unpruned method),
and the integer outputs agree across screening precisions.  On the
500,000-user workload the score of every item and the top-N are also
compared with the full oracle, stored by tests/golden/make_bf16_workload_scores.py.
"""
import hashlib
import json
import os

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


def _run_workload(idx, precs):
    import paper_2504_13445_amd as rm
    cfg = synth.CONFIGS[idx]
    print("[case] generate", cfg.name, flush=True)
    U, P = synth.make_config(cfg)
    n, m, k, N = U.shape[0], P.shape[0], cfg.k, cfg.N
    sub = synth.subsample_users(cfg, 0.01)
    print("[case] oracle on", sub.size, "users", flush=True)
    t_ref, j_ref, tk_ref = orc.kmips_c(np.ascontiguousarray(U[sub]), P, k)
    Ug = torch.from_numpy(U).to(_dev())
    Pg = torch.from_numpy(P).to(_dev())
    del U
    sub_g = torch.from_numpy(sub).to(_dev())
    results = {}
    for prec in precs:
        print("[case]", cfg.name, prec, "thresholds", flush=True)
        tau, tid, topk = rm.thresholds(Ug, Pg, k, prec=prec, with_topk=True)
        ts = tau[sub_g].cpu().numpy()
        assert np.array_equal(ts.view(np.uint64), t_ref.view(np.uint64)), prec
        assert np.array_equal(tid[sub_g].cpu().numpy(), j_ref), prec
        assert np.array_equal(topk[sub_g].cpu().numpy(), tk_ref), prec
        print("[case]", cfg.name, prec, "scores of all items", flush=True)
        sc = rm.scores(Ug, tau, tid, Pg, torch.arange(m, dtype=torch.int32, device=_dev()),
                       prec=prec).cpu().numpy().astype(np.int64)
        assert sc.sum() == n * k, prec
        hist = np.bincount(topk.cpu().numpy().ravel(), minlength=m)
        assert np.array_equal(sc, hist), prec
        ui, us = orc.topn_from_scores(sc, N)
        print("[case]", cfg.name, prec, "topn", flush=True)
        ids, tsc, st = rm.topn(Ug, Pg, k, N, prec=prec)
        print("stats", prec, st, flush=True)
        assert ids.tolist() == ui.tolist() and tsc.tolist() == us.tolist(), prec
        results[prec] = (ids.tolist(), tsc.tolist(), tau.cpu().numpy(), tid.cpu().numpy())
        del tau, tid, topk
        torch.cuda.empty_cache()
    base = precs[0]
    for prec in precs[1:]:
        assert results[prec][0] == results[base][0] and results[prec][1] == results[base][1]
        assert np.array_equal(results[prec][2].view(np.uint64), results[base][2].view(np.uint64))
        assert np.array_equal(results[prec][3], results[base][3])


def test_bf16_workload_500k_users():
    _run_workload(2, ["bf16", "fp32"])


def test_fp8_workload_2m_users():
    _run_workload(3, ["fp8", "bf16", "fp6"])


@pytest.mark.parametrize("prec", ["bf16", "fp32", "fp8", "fp6"])
def test_bf16_workload_full_oracle(golden_dir, prec):
    """Score of each of the 50,000 items and the top-50 of the 500,000-user
    workload, element by element against the full FP64 oracle (Def. 2 and
    Def. 3; expected values written by the oracle alone)."""
    import paper_2504_13445_amd as rm
    g = json.load(open(os.path.join(golden_dir, "bf16_workload_scores.json")))
    cfg = synth.CONFIGS[2]
    print("[case] full-oracle scores", cfg.name, prec, flush=True)
    U, P = synth.make_config(cfg)
    assert hashlib.sha256(U.tobytes()).hexdigest() == g["sha256_U"], "generator changed"
    assert hashlib.sha256(P.tobytes()).hexdigest() == g["sha256_P"], "generator changed"
    n, m, k, N = U.shape[0], P.shape[0], g["k"], g["N"]
    ref = np.array(g["scores"], np.int64)
    Ug = torch.from_numpy(U).to(_dev())
    Pg = torch.from_numpy(P).to(_dev())
    del U, P
    tau, tid = rm.thresholds(Ug, Pg, k, prec=prec)
    sc = rm.scores(Ug, tau, tid, Pg, torch.arange(m, dtype=torch.int32, device=_dev()),
                   prec=prec).cpu().numpy().astype(np.int64)
    bad = np.nonzero(sc != ref)[0]
    assert bad.size == 0, (prec, bad[:10], sc[bad[:10]], ref[bad[:10]])
    ids, tsc, st = rm.topn(Ug, Pg, k, N, prec=prec)
    print("stats", prec, st, flush=True)
    assert ids.tolist() == g["top_ids"] and tsc.tolist() == g["top_scores"], prec

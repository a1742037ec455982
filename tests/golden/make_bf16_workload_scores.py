"""Write the exact scores of every item of the 500,000-user workload.

Workload: n = 500,000 users (64-cluster directions, LogNormal(0, 0.25)
norms), m = 50,000 items (isotropic, LogNormal(0, 0.8) norms), d = 100,
k = 20, N = 50, seed 2.  The expected values come from the CPU FP64
oracle alone (oracle.kmips_c: Def. 1 by a linear scan per user;
oracle.histogram_scores: Baseline 1 of Sec. 2.2; oracle.topn_from_scores:
Def. 3), never from the library.  The SHA-256 of the generated U and P is
stored with them, so a test can tell whether the generator still produces
the same inputs.

Run from the repository root:  python tests/golden/make_bf16_workload_scores.py
(about two minutes on 8 cores).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bf16_workload_scores.json")


def sha256(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    cfg = synth.CONFIGS[2]
    U, P = synth.make_config(cfg)
    n, m = U.shape[0], P.shape[0]
    t = time.time()
    _, _, topk = oracle.kmips_c(U, P, cfg.k, with_topk=True)
    scores = oracle.histogram_scores(topk, m)
    ids, top = oracle.topn_from_scores(scores, cfg.N)
    assert int(scores.sum()) == n * cfg.k
    rec = {
        "workload": f"{cfg.name}: n={n} users, m={m} items, d={cfg.d}, k={cfg.k}, "
                    f"N={cfg.N}, seed {cfg.seed}",
        "generator": "synth.make_config(2)",
        "sha256_U": sha256(U), "sha256_P": sha256(P),
        "n": n, "m": m, "d": cfg.d, "k": cfg.k, "N": cfg.N,
        "oracle": "oracle.kmips_c + histogram_scores + topn_from_scores (FP64)",
        "oracle_seconds": round(time.time() - t, 1),
        "top_ids": ids.tolist(), "top_scores": top.tolist(),
        "scores": scores.tolist(),
    }
    with open(OUT, "w") as fh:
        json.dump(rec, fh, separators=(",", ":"))
    print(OUT, rec["oracle_seconds"], "s")


if __name__ == "__main__":
    main()

"""Write tests/golden/tiny_search.json with the oracle only (no GPU code).

A seeded 300-vector mixture, PQ 8x256 over d = 32, level-0 degree 32, k = 4,
a 16-entry regression codebook; 8 queries searched with efSearch 16, short-list
16, top-5 (Sec. 2 walk, Sec. 4.1 short-list, Sec. 4.2 Eq. 5 and Sec. 4.3
Eq. 7 refinement).  The fixture freezes the oracle's outputs: a later change
to its arithmetic must regenerate it, naming the passage that justifies it.

    python -m tests.golden.make_golden
"""
import json
import os

import numpy as np

import datagen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
W = datagen.small(name="golden", n=300, nq=8, d=32, m=8, n_train=1024, n_beta=16, n_beta_train=300, k_reg=4,
                  ef=16, shortlist=16, topk=5)


def build():
    return oracle.build_workload(W, nthreads=1)


def main():
    ix, db, q = build()
    r = ix.search(q, W.ef, W.shortlist, W.topk, nthreads=1)
    out = {
        "what": "oracle search of a seeded 300-vector index (Sec. 2, Sec. 4.1-4.3), written by make_golden.py",
        "workload": {k: getattr(W, k) for k in ("name", "n", "nq", "d", "m", "k_reg", "n_beta", "ef", "shortlist",
                                                  "topk", "seed")},
        "entry": int(ix.entry), "max_level": int(ix.max_level),
        "ids": r["ids"].tolist(), "d": [[float(x).hex() for x in row] for row in r["d"]],
        "cand_ids": r["cand_ids"].tolist(), "cand_n": r["cand_n"].tolist(), "stats": r["stats"].tolist(),
        "beta_idx_head": ix.beta_idx[:32].tolist(), "codes_head": ix.codes[:4].tolist(),
    }
    with open(os.path.join(HERE, "tiny_search.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", os.path.join(HERE, "tiny_search.json"))


if __name__ == "__main__":
    main()

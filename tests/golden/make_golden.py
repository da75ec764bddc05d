"""Writes tests/golden/tiny_oracle.json: a digest of the FP64 oracle's outputs on
the tiny configuration (event seeds 1-5, weight seed 0).  It calls only the
oracle and the input generator; the file guards the oracle against unnoticed
changes of its arithmetic.  Run:  python tests/golden/make_golden.py"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from gen import TINY, make_weights, generate_event  # noqa: E402


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def summarise(seed):
    ev = generate_event(seed, 1)
    r = oracle.event(ev.x, make_weights(TINY, 0), TINY)
    return {
        "seed": seed, "n_hits": int(ev.n),
        "n_cand": int(r["src"].size), "n_filt": int(r["fsrc"].size),
        "n_kept": int((r["gnn_scores"] > np.float32(TINY.score_cut)).sum()),
        "n_saturated": int((r["nbr_count"] > TINY.k_max).sum()),
        "cand_digest": digest(np.stack([r["src"], r["dst"]]).astype(np.int64)),
        "filt_digest": digest(np.stack([r["fsrc"], r["fdst"]]).astype(np.int64)),
        "labels_digest": digest(r["labels"].astype(np.int32)),
        "emb_sum": float(r["emb"].sum()),
        "filter_score_sum": float(r["filter_scores"].sum()),
        "gnn_score_sum": float(r["gnn_scores"].sum()),
    }


if __name__ == "__main__":
    out = {"config": TINY.as_dict(), "events": [summarise(s) for s in range(1, 6)]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)

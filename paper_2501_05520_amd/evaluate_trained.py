"""Track-finding quality of a chain against the generator truth: runs seeded events
through the library and matches the track candidates to the generated particles.

A candidate (a component with at least `min_hits` hits) is matched to a particle
when that particle owns more than half of the candidate's hits and the candidate
holds more than half of the particle's hits (double-majority matching).  Reported
per event: the efficiency (matched particles over particles with at least
`min_hits` hits), the number of candidates, the fake candidates (unmatched), and
the purity of the candidate graph (share of candidate edges joining two hits of the
same particle).

  python -m paper_2501_05520_amd.evaluate_trained --weights trained_mu200.npz --mu 20
"""
import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def match_candidates(labels, pid, min_hits=3):
    """(matched particles, particles with >= min_hits hits, candidates, fake candidates)."""
    labels = np.asarray(labels)
    pid = np.asarray(pid)
    order = np.argsort(labels, kind="stable")
    bounds = np.flatnonzero(np.diff(labels[order])) + 1
    groups = np.split(order, bounds) if labels.size else []
    ids, counts = np.unique(pid[pid > 0], return_counts=True)
    n_of = dict(zip(ids.tolist(), counts.tolist()))
    found, n_cand, fake = set(), 0, 0
    for hits in groups:
        if hits.size < min_hits:
            continue
        n_cand += 1
        vals, cnt = np.unique(pid[hits], return_counts=True)
        k = int(np.argmax(cnt))
        p = int(vals[k])
        if p > 0 and 2 * cnt[k] > hits.size and 2 * cnt[k] > n_of[p]:
            found.add(p)
        else:
            fake += 1
    n_true = sum(1 for v in n_of.values() if v >= min_hits)
    return len(found), n_true, n_cand, fake


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--weights", required=True, help=".npz written by paper_2501_05520_amd.train_weights")
    ap.add_argument("--config", default="mu200")
    ap.add_argument("--mu", type=int, default=20, help="pile-up of the evaluation events")
    ap.add_argument("--events", type=int, default=3)
    ap.add_argument("--seed", type=int, default=200, help="first event seed")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--min-hits", type=int, default=3)
    a = ap.parse_args()
    from gen import CONFIGS, generate_event, load_trained
    from paper_2501_05520_amd.trk import Pipeline
    cfg, nets = load_trained(a.weights, CONFIGS[a.config])
    evs = [generate_event(a.seed + k, a.mu) for k in range(a.events)]
    p = Pipeline(cfg, nets, a.precision, max_hits=max(ev.n for ev in evs))
    out = []
    for ev in evs:
        labels, info = p.event(ev.x)
        src, dst, _ = p.build_graph(p.embed(ev.x))
        s, d = src.cpu().numpy(), dst.cpu().numpy()
        purity = float(np.mean((ev.pid[s] == ev.pid[d]) & (ev.pid[s] > 0))) if s.size else 0.0
        found, n_true, n_cand, fake = match_candidates(labels.cpu().numpy(), ev.pid, a.min_hits)
        out.append({"hits": int(ev.n), "cand_edges": int(info["n_cand_edges"]), "graph_purity": round(purity, 4),
                    "kept_edges": int(info["n_kept_edges"]), "candidates": n_cand, "fake": fake,
                    "efficiency": round(found / max(1, n_true), 4)})
    p.close()
    print(json.dumps({"precision": a.precision, "mu": a.mu, "events": out}))


if __name__ == "__main__":
    main()

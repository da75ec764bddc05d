"""Seeded training run that produces trained weights for a configuration, in
three phases on generated events:
  1. metric learning of the embedding;
  2. the filter on the candidate edges of the trained embedding;
  3. the filter cut is calibrated to keep --keep of the true candidate edges of
     held-out events, then the interaction network is trained on the edges that
     pass it.
The filter's and the output head's last layers start without the output gains of
the seeded initial weights.  Every event comes from the seeded generator, the
initial weights from gen.make_weights (seed 0), each phase starts a fresh Adam
state, and every reduction in the library is in a fixed order, so a rerun on the
same device gives the same weights.  The output .npz holds the weights in
gen.weights' layout and the calibrated 'filter_cut'.

  python -m paper_2501_05520_amd.train_weights --config mu200 --mu 200 \
      --emb-steps 600 --filter-steps 300 --gnn-steps 400 --out trained_mu200.npz

At the end the chain is evaluated against the generator truth on held-out events
(--eval-events, seeds 300000+): track efficiency and fake candidates by
double-majority matching (evaluate_trained.match_candidates).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="mu200")
    ap.add_argument("--mu", type=int, default=200, help="pile-up of the training events")
    ap.add_argument("--max-cand", type=int, default=6_000_000, help="candidate-edge capacity of the training context")
    ap.add_argument("--max-kept", type=int, default=3_000_000, help="filtered-edge capacity of the training context")
    ap.add_argument("--eval-events", type=int, default=2, help="held-out events evaluated at the end")
    ap.add_argument("--emb-steps", type=int, default=600)
    ap.add_argument("--filter-steps", type=int, default=200)
    ap.add_argument("--gnn-steps", type=int, default=300)
    ap.add_argument("--keep", type=float, default=0.95, help="fraction of true candidate edges the filter cut keeps")
    ap.add_argument("--lr", type=float, default=3e-4, help="learning rate of the filter + GNN phase")
    ap.add_argument("--emb-lr", type=float, default=1e-3, help="learning rate of the embedding phase")
    ap.add_argument("--emb-warmup", type=int, default=100, help="steps of linear learning-rate warm-up")
    ap.add_argument("--neg-weight", type=float, default=10.0, help="weight of the negative-pair term")
    ap.add_argument("--seed", type=int, default=20000, help="first event seed")
    ap.add_argument("--init", default=None, help="continue from a .npz this script wrote (its filter cut too)")
    ap.add_argument("--reset", default="", help="comma list of 'filter', 'gnn': restart those networks from the seeded "
                                                 "weights (output gain divided out) instead of the --init values")
    ap.add_argument("--pair-std", action="store_true",
                    help="start the untrained filter and interaction network with first layers that read the "
                         "standardised mean and difference of an edge's two ends (statistics of held-out events)")
    ap.add_argument("--gnn-lr", type=float, default=None, help="learning rate of the interaction-network phase")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    import torch  # noqa: F401
    from gen import CONFIGS, make_weights, generate_event, load_trained
    from paper_2501_05520_amd import trk
    from paper_2501_05520_amd.training import (TrainContext, embedding_step, pipeline_step, filter_scores_on,
                                               pair_samples, standardised_start)
    cfg = CONFIGS[a.config]
    nets = make_weights(cfg, 0)
    # networks already trained (embedding, filter, interaction network): a network
    # starts from the seeded weights with its output gain divided out until trained
    done = np.zeros(3, bool)
    if a.init:
        cfg, nets = load_trained(a.init, cfg)
        with np.load(a.init, allow_pickle=False) as z:
            done = z["trained"].astype(bool) if "trained" in z.files else np.ones(3, bool)
    n_max = 60 * a.mu * 12 + 1000
    caps = dict(max_hits=n_max, max_cand_edges=min(a.max_cand, n_max * cfg.k_max),
                max_kept_edges=min(a.max_kept, n_max * cfg.k_max))
    seeded = make_weights(cfg, 0)
    for grp, names, k in (("filter", ("filt",), 1), ("gnn", ("node_enc", "edge_enc", "edge_net", "node_net", "out"), 2)):
        if grp in a.reset.split(","):
            for name in names:
                nets[name] = seeded[name]
            done[k] = False
    rng = np.random.default_rng(a.seed)
    log = []
    t0 = time.time()

    def note(rec):
        log.append(rec)
        print(json.dumps(rec), flush=True)

    def restart(tc, cfg_now, unscale=None):
        # a fresh context (and Adam state) from the current parameters
        cur = trk.unflatten_params(tc.params.cpu().numpy(), nets) if tc is not None else nets
        cur = {k: [(np.asarray(w, np.float32), np.asarray(b, np.float32)) for w, b in v] for k, v in cur.items()}
        if unscale is not None:
            name, gain = unscale
            w, b = cur[name][-1]
            cur[name][-1] = ((w / gain).astype(np.float32), (b / gain).astype(np.float32))
        if tc is not None:
            tc.close()
        return TrainContext(cfg_now, cur, **caps)

    seed = a.seed
    tc = restart(None, cfg)
    for k in range(a.emb_steps):
        meas = k % 20 == 0 or k == a.emb_steps - 1
        lr = a.emb_lr * min(1.0, (k + 1) / max(1, a.emb_warmup))
        r = embedding_step(tc, generate_event(seed, a.mu), rng, float(cfg.radius), lr,
                           neg_weight=a.neg_weight, measure=meas)
        seed += 1
        if meas:
            note({"phase": "embedding", "step": k, "loss": r[0], "true_frac_cand": r[1], "n_cand": r[2],
                  "pair_efficiency": r[3], "s": round(time.time() - t0, 1)})
    done[0] |= a.emb_steps > 0
    if a.pair_std and (a.filter_steps > 0 or a.gnn_steps > 0):
        # data-dependent start of the untrained first layers (training.standardised_start),
        # statistics over the candidate edges of two held-out events of the current chain
        cur = trk.unflatten_params(tc.params.cpu().numpy(), nets)
        cur = {k: [(np.asarray(w, np.float32), np.asarray(b, np.float32)) for w, b in v] for k, v in cur.items()}
        tc.close()
        pipe = trk.Pipeline(cfg, cur, "fp32", max_hits=caps["max_hits"], max_cand_edges=caps["max_cand_edges"],
                            max_kept_edges=caps["max_kept_edges"])
        ep, xp, xa = pair_samples(pipe, [generate_event(a.seed + 200000 + k, a.mu) for k in range(2)])
        pipe.close()
        nets.update(standardised_start(cur, ep, xp, xa, filter=a.filter_steps > 0 and not done[1],
                                       gnn=a.gnn_steps > 0 and not done[2]))
        note({"phase": "pair_std", "emb_diff_sd": float(np.std(ep[0] - ep[1])), "x_diff_sd": float(np.std(xp[0] - xp[1]))})
        tc = restart(None, cfg)
    if a.filter_steps > 0:
        tc = restart(tc, cfg, None if done[1] else ("filt", cfg.filt_out_gain))
        done[1] = True
    for k in range(a.filter_steps):
        lf, _, fc, _ = pipeline_step(tc, generate_event(seed, a.mu), a.lr, filter=True, gnn=False)
        seed += 1
        if k % 20 == 0 or k == a.filter_steps - 1:
            note({"phase": "filter", "step": k, "loss_filter": lf, "true_frac_cand": fc, "s": round(time.time() - t0, 1)})
    if a.filter_steps > 0 or (a.gnn_steps > 0 and not done[2] and not a.init):
        scores, truth = [], []
        for k in range(4):
            sc, y = filter_scores_on(tc, generate_event(a.seed + 100000 + k, a.mu))
            scores.append(sc)
            truth.append(y)
        sc, y = np.concatenate(scores), np.concatenate(truth)
        cut = float(np.quantile(sc[y > 0.5], 1.0 - a.keep)) if (y > 0.5).any() else float(cfg.filter_cut)
        note({"phase": "filter_cut", "filter_cut": cut, "kept_fraction": float(np.mean(sc > cut)),
              "true_kept": float(np.mean(sc[y > 0.5] > cut)), "fake_kept": float(np.mean(sc[y < 0.5] > cut))})
        cfg = cfg.with_(filter_cut=cut)
    if a.gnn_steps > 0:
        tc = restart(tc, cfg, None if done[2] else ("out", cfg.gnn_out_gain))
        done[2] = True
    for k in range(a.gnn_steps):
        _, lg, fc, ff = pipeline_step(tc, generate_event(seed, a.mu), a.gnn_lr or a.lr, filter=False, gnn=True)
        seed += 1
        if k % 20 == 0 or k == a.gnn_steps - 1:
            note({"phase": "gnn", "step": k, "loss_gnn": lg, "true_frac_filt": ff, "s": round(time.time() - t0, 1)})
    params = tc.params.cpu().numpy()
    trained = trk.unflatten_params(params, nets)
    out = {}
    for name, layers in trained.items():
        for li, (w, b) in enumerate(layers):
            out[f"{name}.{li}.w"] = np.asarray(w, np.float32)
            out[f"{name}.{li}.b"] = np.asarray(b, np.float32)
    out["filter_cut"] = np.float32(cfg.filter_cut)
    out["trained"] = done.astype(np.int8)
    np.savez(a.out, **out)
    tc.close()
    print("wrote", a.out, flush=True)
    if a.eval_events > 0:
        from paper_2501_05520_amd.evaluate_trained import match_candidates
        from paper_2501_05520_amd.trk import Pipeline
        evs = [generate_event(300000 + k, a.mu) for k in range(a.eval_events)]
        p = Pipeline(cfg, trk.unflatten_params(params, nets), "fp32", max_hits=max(e.n for e in evs),
                     max_cand_edges=a.max_cand, max_kept_edges=a.max_kept)
        for ev in evs:
            try:
                labels, info = p.event(ev.x)
            except trk.TrkError as e:
                note({"phase": "evaluation", "error": str(e)})
                continue
            found, n_true, n_cand, fake = match_candidates(labels.cpu().numpy(), ev.pid)
            note({"phase": "evaluation", "hits": int(ev.n), "cand_edges": info["n_cand_edges"],
                  "filt_edges": info["n_filt_edges"], "kept_edges": info["n_kept_edges"], "candidates": n_cand,
                  "fake": fake, "efficiency": round(found / max(1, n_true), 4)})
        p.close()
    with open(os.path.splitext(a.out)[0] + ".json", "w") as f:
        json.dump({"args": vars(a), "seconds": time.time() - t0, "log": log}, f, indent=1)


if __name__ == "__main__":
    main()

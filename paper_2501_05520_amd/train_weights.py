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

  python -m paper_2501_05520_amd.train_weights --config mu200 --mu 20 \
      --emb-steps 600 --filter-steps 200 --gnn-steps 300 --out trained_mu200.npz
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
    ap.add_argument("--mu", type=int, default=20, help="pile-up of the training events")
    ap.add_argument("--emb-steps", type=int, default=600)
    ap.add_argument("--filter-steps", type=int, default=200)
    ap.add_argument("--gnn-steps", type=int, default=300)
    ap.add_argument("--keep", type=float, default=0.95, help="fraction of true candidate edges the filter cut keeps")
    ap.add_argument("--lr", type=float, default=3e-4, help="learning rate of the filter + GNN phase")
    ap.add_argument("--emb-lr", type=float, default=1e-3, help="learning rate of the embedding phase")
    ap.add_argument("--neg-weight", type=float, default=10.0, help="weight of the negative-pair term")
    ap.add_argument("--seed", type=int, default=20000, help="first event seed")
    ap.add_argument("--init", default=None, help="continue from a .npz this script wrote (its filter cut too)")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    import torch  # noqa: F401
    from gen import CONFIGS, make_weights, generate_event, load_trained
    from paper_2501_05520_amd import trk
    from paper_2501_05520_amd.training import TrainContext, embedding_step, pipeline_step, filter_scores_on
    cfg = CONFIGS[a.config]
    nets = make_weights(cfg, 0)
    if a.init:
        cfg, nets = load_trained(a.init, cfg)
    n_max = 60 * a.mu * 12 + 1000
    caps = dict(max_hits=n_max, max_cand_edges=n_max * cfg.k_max, max_kept_edges=n_max * cfg.k_max)
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
        loss, frac, ncand = embedding_step(tc, generate_event(seed, a.mu), rng, float(cfg.radius), a.emb_lr,
                                           neg_weight=a.neg_weight)
        seed += 1
        if k % 20 == 0 or k == a.emb_steps - 1:
            note({"phase": "embedding", "step": k, "loss": loss, "true_frac_cand": frac, "n_cand": ncand})
    if a.filter_steps > 0:
        tc = restart(tc, cfg, None if a.init else ("filt", cfg.filt_out_gain))
    for k in range(a.filter_steps):
        lf, _, fc, _ = pipeline_step(tc, generate_event(seed, a.mu), a.lr, filter=True, gnn=False)
        seed += 1
        if k % 20 == 0 or k == a.filter_steps - 1:
            note({"phase": "filter", "step": k, "loss_filter": lf, "true_frac_cand": fc})
    if a.filter_steps > 0 or not a.init:
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
    tc = restart(tc, cfg, None if a.init else ("out", cfg.gnn_out_gain))
    for k in range(a.gnn_steps):
        _, lg, fc, ff = pipeline_step(tc, generate_event(seed, a.mu), a.lr, filter=False, gnn=True)
        seed += 1
        if k % 20 == 0 or k == a.gnn_steps - 1:
            note({"phase": "gnn", "step": k, "loss_gnn": lg, "true_frac_filt": ff})
    params = tc.params.cpu().numpy()
    trained = trk.unflatten_params(params, nets)
    out = {}
    for name, layers in trained.items():
        for li, (w, b) in enumerate(layers):
            out[f"{name}.{li}.w"] = np.asarray(w, np.float32)
            out[f"{name}.{li}.b"] = np.asarray(b, np.float32)
    out["filter_cut"] = np.float32(cfg.filter_cut)
    np.savez(a.out, **out)
    with open(os.path.splitext(a.out)[0] + ".json", "w") as f:
        json.dump({"args": vars(a), "seconds": time.time() - t0, "log": log}, f, indent=1)
    tc.close()
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()

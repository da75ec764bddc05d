"""Seeded training run that produces trained weights for a configuration:
metric learning of the embedding on generated events, then the filter and the
interaction network on the edge sets the trained embedding yields.  Every event
comes from the seeded generator, the initial weights from gen.make_weights
(seed 0), and the optimiser is the library's Adam, so the run is reproducible up
to floating-point reduction order.

  python -m paper_2501_05520_amd.train_weights --config mu200 --mu 20 \
      --emb-steps 600 --pipe-steps 300 --out trained_mu200.npz
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
    ap.add_argument("--emb-steps", type=int, default=400)
    ap.add_argument("--pipe-steps", type=int, default=200)
    ap.add_argument("--lr", type=float, default=3e-4, help="learning rate of the filter + GNN phase")
    ap.add_argument("--emb-lr", type=float, default=1e-3, help="learning rate of the embedding phase")
    ap.add_argument("--neg-weight", type=float, default=10.0, help="weight of the negative-pair term")
    ap.add_argument("--seed", type=int, default=20000, help="first event seed")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    import torch  # noqa: F401
    from gen import CONFIGS, make_weights, generate_event
    from paper_2501_05520_amd import trk
    from paper_2501_05520_amd.training import TrainContext, embedding_step, pipeline_step
    cfg = CONFIGS[a.config]
    nets = make_weights(cfg, 0)
    n_max = 60 * a.mu * 12 + 1000
    tc = TrainContext(cfg, nets, max_hits=n_max, max_cand_edges=n_max * cfg.k_max, max_kept_edges=n_max * cfg.k_max)
    rng = np.random.default_rng(a.seed)
    log = []
    t0 = time.time()
    for k in range(a.emb_steps):
        ev = generate_event(a.seed + k, a.mu)
        loss, frac, ncand = embedding_step(tc, ev, rng, float(cfg.radius), a.emb_lr, neg_weight=a.neg_weight)
        if k % 20 == 0 or k == a.emb_steps - 1:
            log.append({"phase": "embedding", "step": k, "loss": loss, "true_frac_cand": frac, "n_cand": ncand})
            print(json.dumps(log[-1]), flush=True)
    for k in range(a.pipe_steps):
        ev = generate_event(a.seed + a.emb_steps + k, a.mu)
        lf, lg, fc, ff = pipeline_step(tc, ev, a.lr)
        if k % 20 == 0 or k == a.pipe_steps - 1:
            log.append({"phase": "filter+gnn", "step": k, "loss_filter": lf, "loss_gnn": lg,
                        "true_frac_cand": fc, "true_frac_filt": ff})
            print(json.dumps(log[-1]), flush=True)
    params = tc.params.cpu().numpy()
    trained = trk.unflatten_params(params, nets)
    out = {}
    for name, layers in trained.items():
        for li, (w, b) in enumerate(layers):
            out[f"{name}.{li}.w"] = np.asarray(w, np.float32)
            out[f"{name}.{li}.b"] = np.asarray(b, np.float32)
    np.savez(a.out, **out)
    with open(os.path.splitext(a.out)[0] + ".json", "w") as f:
        json.dump({"args": vars(a), "seconds": time.time() - t0, "log": log}, f, indent=1)
    tc.close()
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()

"""Loss curve of the training configuration: the filter MLP and the interaction
network trained together (one summed BCE objective, hand-written backward with
per-iteration recomputation, Adam) on a fresh pile-up-200 event per step (event
seeds 10000 + step), BF16 or FP32 products with FP32 master weights.

The edge sets of each step come from an inference context with the weights of
--weights (an .npz of train_weights: its trained embedding gives candidate edges
that contain true pairs, so the truth labels are not degenerate); the filter and
the interaction network start from the seeded weights with their output gains
divided out and their first layers reading standardised inputs
(training.standardised_start, statistics of two events outside the curve's seeds).
Prints one JSON line per logged step and writes the whole curve as JSON.

  python -m paper_2501_05520_amd.train_curve --weights weights/trained_mu200.npz \\
      --steps 200 --precision bf16 --out curve.json
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
    ap.add_argument("--weights", required=True)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--precision", default="bf16", choices=("fp32", "bf16"))
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--mu", type=int, default=200)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    import torch
    from gen import MU200, make_weights, generate_event, load_trained
    from paper_2501_05520_amd import trk
    from paper_2501_05520_amd.training import (TrainContext, train_step, edge_truth, pair_samples,
                                               standardised_start)
    tcfg, tnets = load_trained(a.weights, MU200)
    init = make_weights(MU200, 0)
    nets = dict(tnets)
    for name, gain in (("filt", MU200.filt_out_gain), ("out", MU200.gnn_out_gain)):
        layers = list(init[name])
        w, b = layers[-1]
        layers[-1] = ((w / gain).astype(np.float32), (b / gain).astype(np.float32))
        nets[name] = layers
    for name in ("node_enc", "edge_enc", "edge_net", "node_net"):
        nets[name] = init[name]
    pipe = trk.Pipeline(tcfg, tnets, "fp32", max_hits=120000, max_cand_edges=6_000_000, max_kept_edges=3_000_000)
    # the seeded first layers read standardised inputs (training.standardised_start)
    ep, xp, xa = pair_samples(pipe, [generate_event(a.mu * 1000 + 900 + k, a.mu) for k in range(2)])
    nets = standardised_start(nets, ep, xp, xa)
    free0 = torch.cuda.mem_get_info()[0]
    tc = TrainContext(tcfg, nets, max_hits=120000, max_cand_edges=6_000_000, max_kept_edges=3_000_000,
                      precision=a.precision)
    held = free0 - torch.cuda.mem_get_info()[0]
    log, t0 = [], time.time()
    for k in range(a.steps):
        ev = generate_event(10000 + k, a.mu)
        x = torch.as_tensor(ev.x).cuda()
        emb = pipe.embed(x)
        cs, cd, _ = pipe.build_graph(emb)
        _, fs, fd = pipe.filter(emb, cs, cd, cap=3_000_000)
        yc = torch.as_tensor(edge_truth(ev.pid, cs.cpu().numpy(), cd.cpu().numpy())).cuda()
        yf = torch.as_tensor(edge_truth(ev.pid, fs.cpu().numpy(), fd.cpu().numpy())).cuda()
        torch.cuda.synchronize()
        s = time.perf_counter()
        lf, lg = train_step(tc, x, emb, (cs, cd), (fs, fd), yc, yf, lr=a.lr)
        torch.cuda.synchronize()
        rec = {"step": k, "loss_filter": round(lf, 5), "loss_gnn": round(lg, 5),
               "step_ms": round((time.perf_counter() - s) * 1e3, 2), "n_cand": int(cs.numel()),
               "n_filt": int(fs.numel()), "true_frac_cand": round(float(yc.mean()), 4),
               "true_frac_filt": round(float(yf.mean()), 4)}
        log.append(rec)
        if k % 10 == 0 or k == a.steps - 1:
            print(json.dumps(dict(rec, s=round(time.time() - t0, 1))), flush=True)
    tc.close()
    pipe.close()
    out = {"precision": a.precision, "steps": a.steps, "lr": a.lr, "weights": a.weights,
           "device_memory_gb": round(held / 2**30, 2), "curve": log}
    with open(a.out, "w") as f:
        json.dump(out, f)
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()

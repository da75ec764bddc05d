"""Throughput benchmark of the tracking chain on one MI355X.

Workload: synthetic pile-up-200 events (200 overlaid collisions x 50 helical
tracks x 10 barrel layers + 10 % noise = 110,000 hits, event seeds 200-209),
the full-size network (embedding 3->3x1024->12, radius 0.2, <= 256 neighbours,
filter 24->3x512->1, interaction network H=128 with 8 iterations), seeded
random-init weights (seed 0).  A step is one event through the whole chain
(trk_event: embedding, radius graph, filter, interaction network, score cut and
components), inputs resident in HBM before the timed region.  Prints one JSON
line.  The FP64 CPU oracle is timed on a bounded sample as a reference point.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FILTER_FLOP_PER_EDGE = 2 * (2 * 512 * 512 + 512)     # hidden 512x512 layers + output dot
EMBED_FLOP_PER_HIT = 2 * (3 * 1024 + 2 * 1024 * 1024 + 1024 * 12)
# interaction network, H = 128, T = 8, first edge layers factorised per node
GNN_H, GNN_T = 128, 8
GNN_FLOP_EDGE_ITER = 2 * 2 * GNN_H * GNN_H                                  # e W_c, then W_2
GNN_FLOP_NODE_ITER = 2 * (2 * GNN_H * GNN_H + GNN_H * GNN_H + GNN_H * 2 * GNN_H)  # node net + next projections
GNN_FLOP_EDGE_ONCE = 2 * (6 * GNN_H + GNN_H * GNN_H) + 2 * (GNN_H * GNN_H + GNN_H)  # edge encoder, output head
GNN_FLOP_NODE_ONCE = 2 * (3 * GNN_H + GNN_H * GNN_H + GNN_H * 2 * GNN_H)            # node encoder + projections
HBM_PEAK_GBS = 8000.0
# bytes per stored interaction-network state element (FP8: E4M3 edge states and projections)
ACT_BYTES = {"fp32": 4, "bf16": 2, "fp8": 1, "fp8all": 1, "bf16emb32": 2, "bf16x3": 4, "bf16x3gnn16": 2}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "filter_kernel_mu200_traffic.md")
TRAINED_WEIGHTS = os.path.join(ROOT, "weights", "trained_mu200.npz")
SERVED_FORMS = ("bf16", "bf16emb32", "bf16x3", "bf16x3gnn16", "fp8", "fp8all")
FILTER_SOURCES = ["mlp.hip", "mfma_tile.h", "common.h", "layers.h", "kernels.h"]


def filter_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in FILTER_SOURCES:
        with open(os.path.join(ROOT, "paper_2501_05520_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(precision):
    """HBM bytes per launch of the FP32 filter kernel from the committed counter
    summary, if the kernel sources are still the ones it was measured on."""
    if precision != "fp32" or not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        text = fh.read()
    # the machine-readable block of the counter summary
    t = json.loads(text[text.index("```json") + len("```json"):text.rindex("```")])
    return t["hbm_bytes_per_launch"] if t.get("sources_sha256") == filter_sources_digest() else None


def gnn_work(n_nodes, n_edges, prec):
    """Algorithmic FLOPs and minimal HBM bytes of the interaction network per event:
    per iteration each edge state is read and written once, node states (FP32) are
    read, messages read and written once, projections written and read once."""
    b = ACT_BYTES[prec]
    flops = n_edges * (GNN_T * GNN_FLOP_EDGE_ITER + GNN_FLOP_EDGE_ONCE) + \
        n_nodes * (GNN_T * GNN_FLOP_NODE_ITER + GNN_FLOP_NODE_ONCE)
    per_iter = 2 * n_edges * GNN_H * b + n_nodes * GNN_H * 4 * 4 + 2 * n_nodes * 2 * GNN_H * b
    once = n_edges * (GNN_H * b * 2 + 8 * 2 + 4) + n_nodes * (12 + GNN_H * 4)
    return flops, GNN_T * per_iter + once


def stage_rooflines(st, counts, prec, peak):
    n, ec, ef, ek = counts["n_hits"], counts["n_cand_edges"], counts["n_filt_edges"], counts["n_kept_edges"]
    gf, gb = gnn_work(n, ef, prec)
    # components: read the kept-edge ends and scores once, write the labels a few times
    cc_bytes = ef * 12 + n * 4 * 4
    # radius graph: embeddings read and sorted once, edges written twice (rows, sorted)
    graph_bytes = n * (12 * 4 * 3 + 32) + ec * 8 * 2
    return {
        "embed": {"bound": "mfma", "frac": round(n * EMBED_FLOP_PER_HIT / (st["embed"] * 1e-3) / 1e12 / peak, 4)},
        "filter": {"bound": "mfma", "frac": round(ec * FILTER_FLOP_PER_EDGE / (st["filter"] * 1e-3) / 1e12 / peak, 4)},
        "gnn": {"bound": "mfma" if prec == "fp32" else "hbm",
                "mfma_frac": round(gf / (st["gnn"] * 1e-3) / 1e12 / peak, 4),
                "hbm_frac": round(gb / (st["gnn"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "tflop": round(gf / 1e12, 4), "min_gbytes": round(gb / 1e9, 3)},
        "graph": {"bound": "latency", "hbm_frac": round(graph_bytes / (st["graph"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "components": {"bound": "latency", "hbm_frac": round(cc_bytes / (st["components"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
    }
# split BF16 issues three BF16 products per algorithmic product: its fraction is of
# the BF16 peak counted in algorithmic FLOPs (at most 1/3)
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0, "fp8all": 5000.0, "bf16emb32": 2500.0,
               "bf16x3": 2500.0, "bf16x3gnn16": 2500.0}
EVENT_SEEDS = list(range(200, 210))


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--precision", default="fp32", choices=list(PEAK_TFLOPS))
    p.add_argument("--no-variant", action="store_true", help="skip the BF16 comparison run")
    p.add_argument("--no-trained", action="store_true", help="skip the chain on the trained weights")
    p.add_argument("--serving-long", choices=("mix", "mu200"), default=None,
                   help="long serving runs with fixed request counts (mix: 10,000 requests per load; mu200: 2,000 "
                        "per form), after 200 warm-up requests each")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--events", type=int, default=len(EVENT_SEEDS))
    p.add_argument("--latency-events", type=int, default=200,
                   help="events run one at a time after the timed steps for the p50/p99 latency")
    p.add_argument("--serve-seconds", type=float, default=6.0, help="0 skips the serving measurement")
    p.add_argument("--train-steps", type=int, default=3, help="0 skips the training-step measurement")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run a plain 256 MiB device-to-device copy (to scale HBM counters)")
    return p.parse_args()


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def run_precision(prec, cfg, nets, xs, steps, warmup, torch, trk, latency_events=0):
    """Times `steps` events (cycling over xs) back to back; then, when
    latency_events > 0, that many more one at a time for the latency percentiles
    (each trk_event call returns after its event's labels are complete)."""
    progress(f"{prec}: {steps} timed events, then {latency_events} one at a time")
    max_hits = max(x.shape[0] for x in xs)
    pipe = trk.Pipeline(cfg, nets, prec, max_hits=max_hits, stage_timing=True)
    dev = [torch.as_tensor(x).cuda() for x in xs]
    labels = [torch.empty(x.shape[0], dtype=torch.int32, device="cuda") for x in xs]
    for i in range(warmup):
        k = i % len(dev)
        trk.trk_event(pipe.ctx, dev[k], labels[k])
    torch.cuda.synchronize()
    lat, infos = [], []
    t0 = time.perf_counter()
    for i in range(steps):
        k = i % len(dev)
        s = time.perf_counter()
        infos.append(trk.trk_event(pipe.ctx, dev[k], labels[k]))
        lat.append(time.perf_counter() - s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if latency_events > 0:
        lat = []
        for i in range(latency_events):
            k = i % len(dev)
            s = time.perf_counter()
            trk.trk_event(pipe.ctx, dev[k], labels[k])
            lat.append(time.perf_counter() - s)
    # events that no run above reached (fewer steps than events) get their labels
    # here, untimed, so that every event's labels are compared
    for k in range(max(warmup, steps, latency_events), len(dev)):
        trk.trk_event(pipe.ctx, dev[k], labels[k])
    out_labels = [l.cpu().numpy() for l in labels]
    pipe.close()
    return wall, np.array(lat), infos, out_labels


def margin_counts(cfg, nets, xs, trk, tol=1e-4):
    """Per event: edges whose FP32 filter score lies within tol of the filter cut,
    and edges whose FP32 interaction-network score lies within tol of the score cut
    (the decisions a last-bit difference can flip)."""
    pipe = trk.Pipeline(cfg, nets, "fp32", max_hits=max(x.shape[0] for x in xs))
    out = []
    for x in xs:
        emb = pipe.embed(x)
        cs, cd, _ = pipe.build_graph(emb)
        pf, fs, fd = pipe.filter(emb, cs, cd)
        q = pipe.gnn(x, fs, fd)
        pf, q = pf.cpu().numpy(), q.cpu().numpy()
        out.append({"filter": int(np.sum(np.abs(pf - np.float32(cfg.filter_cut)) <= tol)),
                    "score": int(np.sum(np.abs(q - np.float32(cfg.score_cut)) <= tol))})
    pipe.close()
    return out


def score_errors(cfg, nets, precisions, trk, seed=300, mu=10):
    """Score error of each precision against the FP64 oracle on one pile-up-10 event
    (5,500 hits), stage-isolated: the filter on the oracle's candidate edges and
    embedding (rounded to FP32), the interaction network on the oracle's filtered
    edges; max and 99th percentile of |p - p_oracle|."""
    import oracle
    from gen import generate_event
    progress("score errors against the FP64 oracle on a pile-up-10 event")
    ev = generate_event(seed, mu)
    r = oracle.event(ev.x, nets, cfg)
    e32 = r["emb"].astype(np.float32)
    out = {}
    for prec in precisions:
        p = trk.Pipeline(cfg, nets, prec, max_hits=ev.n)
        pf = p.filter(e32, r["src"], r["dst"])[0].cpu().numpy()
        q = p.gnn(ev.x, r["fsrc"], r["fdst"]).cpu().numpy()
        p.close()
        df, dq = np.abs(pf - r["filter_scores"]), np.abs(q - r["gnn_scores"])
        out[prec] = {"filter_dp_max": float(df.max()), "filter_dp_p99": float(np.percentile(df, 99)),
                     "gnn_dp_max": float(dq.max()) if dq.size else 0.0,
                     "gnn_dp_p99": float(np.percentile(dq, 99)) if dq.size else 0.0}
    return {"event": f"pile-up {mu}, seed {seed}, {ev.n} hits, {r['src'].size} candidate and {r['fsrc'].size} "
                     "filtered edges (oracle)", "precisions": out}


def trained_chain(cfg, evs, args, torch, trk):
    """The chain on the trained weights (weights/trained_mu200.npz): FP32 and every
    served form on the pile-up-200 events, with candidate agreement against FP32,
    margin counts, track efficiency and fake candidates against the generator truth
    (double-majority matching), and score errors against the FP64 oracle."""
    import hashlib
    from gen import load_trained
    from paper_2501_05520_amd.evaluate_trained import match_candidates
    if not os.path.exists(TRAINED_WEIGHTS):
        return {"error": f"no trained weights at {os.path.relpath(TRAINED_WEIGHTS, ROOT)}"}
    progress("trained chain")
    with open(TRAINED_WEIGHTS, "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    tcfg, tnets = load_trained(TRAINED_WEIGHTS, cfg)
    xs = [e.x for e in evs]

    def quality(labels):
        m = [match_candidates(l, e.pid) for l, e in zip(labels, evs)]
        return {"efficiency": round(float(np.mean([f / max(1, t) for f, t, _, _ in m])), 4),
                "candidates": int(np.mean([c for _, _, c, _ in m])),
                "fake_fraction": round(float(np.mean([k / max(1, c) for _, _, c, k in m])), 4)}

    wall, lat, infos, labels = run_precision("fp32", tcfg, tnets, xs, args.steps, args.warmup, torch, trk,
                                             args.latency_events)
    out = {"weights": os.path.relpath(TRAINED_WEIGHTS, ROOT), "sha256": digest, "filter_cut": tcfg.filter_cut,
           "fp32": {"value": round(args.steps / wall, 3), "unit": "events/s",
                    "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                                   "p99": round(float(np.percentile(lat, 99)) * 1e3, 3), "events": int(lat.size)},
                    "stage_ms": {k: round(v, 4) for k, v in stage_means(infos).items()},
                    "counts": {k: int(np.mean([i[k] for i in infos])) for k in
                               ("n_cand_edges", "n_filt_edges", "n_kept_edges")},
                    "truth": quality(labels)},
           "margin_edges_per_event": margin_counts(tcfg, tnets, xs, trk), "forms": {}}
    for prec in SERVED_FORMS:
        w2, lat2, inf2, lab2 = run_precision(prec, tcfg, tnets, xs, args.steps, args.warmup, torch, trk,
                                             args.latency_events)
        agr = [agreement(a, b) for a, b in zip(labels, lab2)]
        out["forms"][prec] = {
            "value": round(args.steps / w2, 3), "unit": "events/s",
            "latency_ms": {"p50": round(float(np.percentile(lat2, 50)) * 1e3, 3),
                           "p99": round(float(np.percentile(lat2, 99)) * 1e3, 3)},
            "hit_agreement_vs_fp32": round(float(np.mean([a[0] for a in agr])), 6),
            "candidate_jaccard_vs_fp32": round(float(np.mean([a[1] for a in agr])), 6),
            "candidate_jaccard_vs_fp32_min": round(float(np.min([a[1] for a in agr])), 6),
            "truth": quality(lab2)}
    out["score_errors_vs_fp64"] = score_errors(tcfg, tnets, ("fp32",) + SERVED_FORMS, trk)
    return out


def host_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    return {"cpu_model": model, "cores": cores}


def cpu_baseline_tiny(runs=20):
    """The FP64 oracle on the tiny configuration (550 hits, event seed 1): median
    wall time of `runs` whole-chain runs with every host core for NumPy's BLAS,
    and with one thread."""
    import oracle
    from gen import TINY, make_weights, generate_event
    from threadpoolctl import threadpool_limits
    progress("FP64 oracle on the tiny event")
    nets = make_weights(TINY, 0)
    x = generate_event(1, 1).x

    def med():
        t = []
        for _ in range(runs):
            s = time.perf_counter()
            oracle.event(x, nets, TINY)
            t.append(time.perf_counter() - s)
        return float(np.median(t))
    all_cores = med()
    with threadpool_limits(limits=1):
        one = med()
    return {"config": "tiny (550 hits, emb 3-64-64-8, filter 16-64-64-1, IN H=32 T=4)", "runs": runs,
            "median_ms_all_cores": round(all_cores * 1e3, 2), "median_ms_one_thread": round(one * 1e3, 2)}


def stage_means(infos):
    keys = infos[0]["stage_ms"].keys()
    return {k: float(np.mean([i["stage_ms"][k] for i in infos])) for k in keys}


def agreement(la, lb, min_hits=3):
    """hit-level label agreement and exact-match Jaccard of candidates (>= min_hits)"""
    hit = float(np.mean(la == lb))

    def cands(lab):
        order = np.argsort(lab, kind="stable")
        ls = lab[order]
        cuts = np.flatnonzero(np.diff(ls)) + 1
        return {tuple(g.tolist()) for g in np.split(order, cuts) if len(g) >= min_hits}

    ca, cb = cands(la), cands(lb)
    u = ca | cb
    return hit, (len(ca & cb) / len(u) if u else 1.0)


def serve_load(cfg, nets, precision, seconds, load_frac, trk, n_clients=32, seed=7, pool=6, mus=None, rate=None,
               n_slots=3, max_batch_events=8, requests=None, warmup_requests=0, budget_events=None):
    """Serving mix: client threads with Poisson arrivals submit events whose
    pile-up is drawn uniformly from `mus` (default {50, 100, 140, 200}); one
    collector harvests results.  First a burst measures the saturated rate, then
    the offered load is load_frac x that rate (or `rate` events/s when given) for
    `seconds`, or, when `requests` is given, until warmup_requests + requests have
    been submitted (the first warmup_requests submissions are not measured).
    Latency = submission -> labels on host."""
    import queue
    import random
    import threading
    from gen import SERVE_MUS, generate_event
    mus = list(mus or SERVE_MUS)
    progress(f"serving {precision}, pile-up {mus}, " + (f"{seconds} s" if requests is None else f"{requests} requests"))
    pools = {mu: [generate_event(9000 + 97 * mu + k, mu).x for k in range(pool)] for mu in mus}
    # default admission: a 64 GB budget against each slot's measured bytes per hit; with
    # budget_events, a forced-small budget of that many pile-up-200 events in flight
    # (4 KiB per hit each), so that admission queues requests
    per_hit = 0 if budget_events is None else 4096
    budget = (64 << 30) if budget_events is None else int(budget_events * 110000 * per_hit)
    srv = trk.Server(cfg, nets, precision, n_slots=n_slots, max_batch_events=max_batch_events, max_batch_hits=330000,
                     mem_budget_bytes=budget, bytes_per_hit=per_hit)
    # warm-up and saturated rate: a burst of 48 requests
    burst = [pools[mus[k % len(mus)]][k % pool] for k in range(48)]
    t0 = time.perf_counter()
    tickets = [(srv.submit(x), x.shape[0]) for x in burst]
    for t, n in tickets:
        srv.wait(t, n)
    sat = len(burst) / (time.perf_counter() - t0)
    rate = load_frac * sat if rate is None else float(rate)
    done = queue.Queue()
    lat, status = [], []
    stop_at = time.perf_counter() + (seconds if requests is None else 1e9)
    total = None if requests is None else warmup_requests + requests
    lock = threading.Lock()
    submitted = [0]

    def client(c):
        rng = random.Random(seed * 1000 + c)
        nxt = time.perf_counter()
        while True:
            nxt += rng.expovariate(rate / n_clients)
            if nxt > stop_at:
                break
            d = nxt - time.perf_counter()
            if d > 0:
                time.sleep(d)
            with lock:
                idx = submitted[0]
                submitted[0] += 1
            if total is not None and idx >= total:
                break
            x = pools[rng.choice(mus)][rng.randrange(pool)]
            done.put((idx, srv.submit(x), x.shape[0]))
        done.put(None)

    def collector():
        ended = 0
        while ended < n_clients:
            item = done.get()
            if item is None:
                ended += 1
                continue
            idx, t, n = item
            rc, _, _, ms = srv.wait(t, n)
            if idx >= warmup_requests:
                status.append(rc)
                lat.append(ms)
                if requests is not None and len(lat) % 500 == 0:
                    progress(f"  {len(lat)} of {requests} requests measured")

    st0 = srv.stats()
    threads = [threading.Thread(target=client, args=(c,)) for c in range(n_clients)]
    col = threading.Thread(target=collector)
    t1 = time.perf_counter()
    for t in threads + [col]:
        t.start()
    for t in threads + [col]:
        t.join()
    wall = time.perf_counter() - t1
    st = srv.stats()
    srv.close()
    lat = np.array(lat)
    nb = st["batches"] - st0["batches"]
    return {"precision": precision, "saturated_events_per_s": round(sat, 2), "offered_events_per_s": round(rate, 2),
            "achieved_events_per_s": round(len(lat) / wall, 2), "requests": int(len(lat)),
            "errors": int(sum(1 for r in status if r != 0)),
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 2), "p90": round(float(np.percentile(lat, 90)), 2),
                           "p99": round(float(np.percentile(lat, 99)), 2)},
            "mean_batch_events": round((st["batched_events"] - st0["batched_events"]) / max(nb, 1), 2),
            "max_batch_events": max_batch_events,
            "waited_for_memory": st["waited_for_memory"] - st0["waited_for_memory"],
            "slots": n_slots, "clients": n_clients, "mix_mu": mus, "warmup_requests": warmup_requests,
            "mem_budget_bytes": budget, "bytes_per_hit": per_hit or "measured per slot"}


def service_load(cfg, nets, precision, seconds, rate, trk, n_conn=8, seed=11, pool=6, mu=200):
    """The socket front end on 127.0.0.1: n_conn client connections (one thread
    each, requests in order per connection) with Poisson arrivals at `rate`
    events/s in total; client latency (send to last label received) beside the
    server's own (submission to completion): their difference is what the
    transfer adds."""
    import random
    import threading
    from gen import generate_event
    xs = [generate_event(9100 + k, mu).x for k in range(pool)]
    srv = trk.Server(cfg, nets, precision, n_slots=1, max_batch_events=8, max_batch_hits=330000,
                     mem_budget_bytes=64 << 30)
    svc, port = trk.trk_service_start(srv.h, "127.0.0.1", 0)
    warm = trk.ServiceClient("127.0.0.1", port)
    for x in xs[:2]:
        warm.request(x)
    warm.close()
    client_ms, server_ms, status = [], [], []
    lock = threading.Lock()
    stop_at = time.perf_counter() + seconds

    def conn(c):
        rng = random.Random(seed * 100 + c)
        cl = trk.ServiceClient("127.0.0.1", port)
        nxt = time.perf_counter()
        while True:
            nxt += rng.expovariate(rate / n_conn)
            if nxt > stop_at:
                break
            d = nxt - time.perf_counter()
            if d > 0:
                time.sleep(d)
            t0 = time.perf_counter()
            st, _, _, lat = cl.request(xs[rng.randrange(pool)])
            with lock:
                client_ms.append((time.perf_counter() - t0) * 1e3)
                server_ms.append(lat)
                status.append(st)
        cl.close()

    th = [threading.Thread(target=conn, args=(c,)) for c in range(n_conn)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    trk.trk_service_stop(svc)
    srv.close()
    cm, sm = np.array(client_ms), np.array(server_ms)
    pct = lambda a, q: round(float(np.percentile(a, q)), 2)
    return {"precision": precision, "connections": n_conn, "offered_events_per_s": round(rate, 2), "mu": mu,
            "requests": int(cm.size), "errors": int(sum(1 for s in status if s != 0)),
            "client_latency_ms": {"p50": pct(cm, 50), "p99": pct(cm, 99)},
            "server_latency_ms": {"p50": pct(sm, 50), "p99": pct(sm, 99)},
            "transfer_ms": {"p50": pct(cm - sm, 50), "p99": pct(cm - sm, 99)},
            "payload_bytes": {"request": int(24 + 12 * xs[0].shape[0]), "response": int(96 + 4 * xs[0].shape[0])}}


def fit_measure(cfg, nets, ev, labels_chain, torch, trk, reps=5):
    """Downstream helix fit (trk_fit) of one pile-up-200 event: on the chain's own
    candidates, on the generator's particles as candidates (which gives the pT
    resolution against the generated values) and, where the trained weights are
    present, on the trained chain's candidates (pT against the generated value of
    each candidate's majority particle)."""
    pipe = trk.Pipeline(cfg, nets, "fp32", max_hits=ev.n + 64)
    x = torch.as_tensor(ev.x, device="cuda")
    lab_truth = np.arange(ev.n)
    for p in np.unique(ev.pid[ev.pid > 0]):
        idx = np.flatnonzero(ev.pid == p)
        lab_truth[idx] = idx.min()
    inputs = [("chain_candidates", labels_chain), ("generated_particles", lab_truth)]
    if os.path.exists(TRAINED_WEIGHTS):
        # the trained chain's own track candidates on the same event
        from gen import load_trained
        tcfg, tnets = load_trained(TRAINED_WEIGHTS, cfg)
        tp = trk.Pipeline(tcfg, tnets, "fp32", max_hits=ev.n + 64)
        lab_t, _ = tp.event(ev.x)
        tp.close()
        inputs.append(("trained_chain_candidates", lab_t.cpu().numpy()))
    out = {}
    for name, lab in inputs:
        l = torch.as_tensor(np.asarray(lab, np.int32), device="cuda")
        trk.trk_fit(pipe.ctx, x, l)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            cl, cn, par = trk.trk_fit(pipe.ctx, x, l)
        torch.cuda.synchronize()
        out[name] = {"candidates": int(cl.numel()), "ms": round((time.perf_counter() - t0) / reps * 1e3, 3)}
        if name == "generated_particles":
            par = par.cpu().numpy()
            pid = ev.pid[cl.cpu().numpy()] - 1
            rel = par[:, 0] / ev.truth["pt"][pid] - 1.0
            out[name]["pt_rel_error_rms"] = float(np.sqrt(np.mean(rel ** 2)))
            out[name]["charge_correct"] = float(np.mean(par[:, 4] == ev.truth["q"][pid]))
        if name == "trained_chain_candidates":
            # candidates whose majority particle owns more than half of their hits: the
            # fitted pT against that particle's generated pT
            par, cl = par.cpu().numpy(), cl.cpu().numpy()
            lab = np.asarray(lab, np.int64)
            pid = np.asarray(ev.pid, np.int64)
            size = np.bincount(lab, minlength=ev.n)
            keys, cnt = np.unique(lab * (pid.max() + 1) + pid, return_counts=True)
            kl, kp = keys // (pid.max() + 1), keys % (pid.max() + 1)
            order = np.lexsort((-cnt, kl))                   # per label, largest count first
            first = order[np.r_[True, kl[order][1:] != kl[order][:-1]]]
            major = np.full(ev.n, -1, np.int64)
            mcnt = np.zeros(ev.n, np.int64)
            major[kl[first]], mcnt[kl[first]] = kp[first], cnt[first]
            ok = (major[cl] > 0) & (2 * mcnt[cl] > size[cl])
            mp = major[cl][ok] - 1
            rels = par[ok, 0] / ev.truth["pt"][mp] - 1.0
            qok = par[ok, 4] == ev.truth["q"][mp]
            out[name]["matched"] = int(rels.size)
            out[name]["pt_rel_error_median_abs"] = float(np.median(np.abs(rels))) if rels.size else None
            out[name]["pt_rel_error_p90_abs"] = float(np.percentile(np.abs(rels), 90)) if rels.size else None
            out[name]["charge_correct"] = float(np.mean(qok)) if qok.size else None
    pipe.close()
    return out


def train_measure(cfg, nets, steps, torch, trk, precision="fp32"):
    """Training configuration: filter + interaction network on a fresh pile-up-200
    event per step (seeds 10000+step), BCE on generator truth, hand-written
    backward with per-iteration recomputation, Adam.  The edge sets come from the
    trained chain (weights/trained_mu200.npz, whose embedding puts true pairs in the
    candidate graph; the seeded random chain's graph holds none) and the trained
    networks start from the seeded weights.  Reports the step time, a training
    roofline (algorithmic FLOPs: forward, twice the forward for the backward, and one
    more forward of the iterations for the recomputation), the device memory the
    context holds (HIP's free-memory counter) and what storing every iteration's
    internals instead of recomputing them would add."""
    from gen import generate_event, load_trained
    from paper_2501_05520_amd.training import (TrainContext, train_step, edge_truth, pair_samples,
                                               standardised_start)
    progress(f"training steps ({precision})")
    src = "seeded random chain (candidate graph without true pairs)"
    pcfg, pnets = cfg, nets
    if os.path.exists(TRAINED_WEIGHTS):
        pcfg, pnets = load_trained(TRAINED_WEIGHTS, cfg)
        src = os.path.relpath(TRAINED_WEIGHTS, ROOT)
    pipe = trk.Pipeline(pcfg, pnets, "fp32", max_hits=120000, max_cand_edges=6_000_000, max_kept_edges=3_000_000)
    # the trained networks start as in the loss-curve command: seeded weights, output
    # gains divided out, first layers on standardised inputs
    start = dict(pnets)
    for name, gain in (("filt", cfg.filt_out_gain), ("out", cfg.gnn_out_gain)):
        layers = list(nets[name])
        w, b = layers[-1]
        layers[-1] = ((w / gain).astype(np.float32), (b / gain).astype(np.float32))
        start[name] = layers
    for name in ("node_enc", "edge_enc", "edge_net", "node_net"):
        start[name] = nets[name]
    ep, xp, xa = pair_samples(pipe, [generate_event(cfg.n_collisions * 1000 + 900 + k, cfg.n_collisions)
                                     for k in range(2)])
    start = standardised_start(start, ep, xp, xa)
    free0 = torch.cuda.mem_get_info()[0]
    tc = TrainContext(pcfg, start, max_hits=120000, max_cand_edges=6_000_000, max_kept_edges=3_000_000,
                      precision=precision)
    held = free0 - torch.cuda.mem_get_info()[0]
    times, losses, ec, ef, nh, tf = [], [], [], [], [], []
    for k in range(steps + 1):
        ev = generate_event(10000 + k, cfg.n_collisions)
        emb = pipe.embed(ev.x)
        cs, cd, _ = pipe.build_graph(emb)
        _, fs, fd = pipe.filter(emb, cs, cd, cap=3_000_000)
        x = torch.as_tensor(ev.x).cuda()
        yc = torch.as_tensor(edge_truth(ev.pid, cs.cpu().numpy(), cd.cpu().numpy())).cuda()
        yf = torch.as_tensor(edge_truth(ev.pid, fs.cpu().numpy(), fd.cpu().numpy())).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lf, lg = train_step(tc, x, emb, (cs, cd), (fs, fd), yc, yf, lr=3e-4)
        torch.cuda.synchronize()
        if k > 0:                      # the first step includes one-time warm-up
            times.append(time.perf_counter() - t0)
            ec.append(cs.numel()); ef.append(fs.numel()); nh.append(ev.n); tf.append(float(yf.mean()))
        losses.append(round(lf + lg, 5))
    tc.close()
    pipe.close()
    step_s = float(np.mean(times)) if times else float("nan")
    E_c, E_f, N = float(np.mean(ec)), float(np.mean(ef)), float(np.mean(nh))
    filt_fwd = E_c * 2 * (2 * cfg.emb_dim * 512 + 2 * 512 * 512 + 512)
    gnn_fwd, _ = gnn_work(N, E_f, "fp32")
    flops = 3 * filt_fwd + 3 * gnn_fwd + gnn_fwd
    peak = PEAK_TFLOPS["bf16" if precision == "bf16" else "fp32"]
    H, T = GNN_H, GNN_T
    extra = T * (E_f * 3 * H + N * 7 * H) * 4      # per iteration: pre, t1, v per edge; P, msg, nin, q1, q2 per node
    return {"steps": steps, "step_ms": round(step_s * 1e3, 2), "edge_sets": src,
            "loss": losses, "n_cand_edges": int(E_c), "n_filt_edges": int(E_f),
            "true_frac_filt": round(float(np.mean(tf)), 4) if tf else None,
            "roofline": {"bound": "mfma", "tflop_per_step": round(flops / 1e12, 3),
                         "achieved_tflops": round(flops / step_s / 1e12, 2), "peak": peak,
                         "frac": round(flops / step_s / 1e12 / peak, 4)},
            "device_memory_gb": round(held / 2**30, 2),
            "device_memory_gb_without_recompute": round((held + extra) / 2**30, 2),
            "precision": {"fp32": "fp32 (activations and master weights)",
                          "bf16": "bf16 operands of every product and bf16 stored activations (hidden "
                                  "layers, per-iteration node and edge states), fp32 accumulation, deltas, "
                                  "master weights and Adam moments"}[precision]}


# The paper's own figures for its served chain (Section 4), on its hardware and workload:
# context only, not comparable (trained models of unstated precision on ~350k ACTS
# spacepoints per event, with the connected components on the CPU).
PAPER_CONTEXT = {
    "hardware": "one NVIDIA A100-SXM4 behind Triton (Perlmutter)",
    "workload": "ttbar at mu=200, about 350k spacepoints per event, trained models",
    "max_throughput_events_per_s": 1.75,
    "seconds_per_event": {"cpu_direct": 9.65, "gpu_direct": 2.42, "gpu_as_a_service": 2.24},
    "comparable": False,
}


def measured_peaks(torch, trk):
    """Dense MFMA rate of each precision from independent MFMA chains on every CU,
    and the HBM bandwidth of a 1 GiB device-to-device copy (read + write)."""
    out = {"fp32_mfma_tflops": round(trk.trk_probe_mfma("fp32", 100_000), 1),
           "bf16_mfma_tflops": round(trk.trk_probe_mfma("bf16", 200_000), 1),
           "fp8_mfma_tflops": round(trk.trk_probe_mfma("fp8", 100_000), 1)}
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    out["hbm_copy_gbs"] = round(trk.trk_probe_copy(a, b, reps=5), 1)
    del a, b
    out["published"] = {"fp32_mfma_tflops": PEAK_TFLOPS["fp32"], "bf16_mfma_tflops": PEAK_TFLOPS["bf16"],
                        "fp8_mfma_tflops": PEAK_TFLOPS["fp8"], "hbm_gbs": HBM_PEAK_GBS}
    return out


def cpu_baseline(cfg, nets, x):
    """FP64 oracle on a bounded sample of one event, scaled to events/s:
    embedding on 1/8 of the hits, the radius graph in full, the filter on 1/16
    of the candidate edges, the interaction network on all nodes with 1/16 of
    the filtered edges minus its cost with no edges (its cost is linear in
    nodes and edges), components in full."""
    import oracle
    progress("FP64 oracle on a bounded sample of one pile-up-200 event")
    t = {}
    n = x.shape[0]
    s = time.perf_counter(); emb8 = oracle.embed(x[: n // 8], nets); t["embed"] = (time.perf_counter() - s) * 8
    emb = oracle.embed(x, nets)          # untimed: the graph needs the whole embedding
    s = time.perf_counter(); src, dst, _ = oracle.radius_graph(emb, np.float32(cfg.radius), cfg.k_max)
    t["graph"] = time.perf_counter() - s
    m16 = src.size // 16
    s = time.perf_counter(); pf16 = oracle.filter_scores(emb, src[:m16], dst[:m16], nets)
    t["filter"] = (time.perf_counter() - s) * 16
    pf = pf16  # the kept edges of the sample feed the GNN timing below
    fs, fd = oracle.filter_edges(pf, src[:m16], dst[:m16], np.float32(cfg.filter_cut))
    e_f = int(fs.size) * 16
    s = time.perf_counter(); oracle.interaction_network(x, fs[:0], fd[:0], nets, cfg.gnn_iters)
    t0 = time.perf_counter() - s
    s = time.perf_counter(); p = oracle.interaction_network(x, fs, fd, nets, cfg.gnn_iters)
    t1 = time.perf_counter() - s
    t["gnn"] = t0 + (t1 - t0) * 16
    s = time.perf_counter(); oracle.components(n, fs, fd, p, np.float32(cfg.score_cut)); t["components"] = time.perf_counter() - s
    total = sum(t.values())
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    return {"value": 1.0 / total, "unit": "events/s", "cores": cores, "kind": "oracle",
            "sample": (f"one mu=200 event ({n} hits, {src.size} candidate edges, ~{e_f} filtered): embedding on "
                       "1/8 of hits, radius graph in full, filter on 1/16 of candidate edges, GNN on all nodes with "
                       "1/16 of filtered edges (edge part scaled x16), components in full; FP64 NumPy"),
            "stage_s": {k: round(v, 3) for k, v in t.items()}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the tracking chain shards by whole events with no exchange "
              f"between GPUs, and this benchmark measures a single MI355X (--gpus {args.gpus} requested)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from gen import MU200, make_weights, generate_event
    from paper_2501_05520_amd import trk

    cfg = MU200
    nets = make_weights(cfg, 0)
    evs = [generate_event(s, cfg.n_collisions) for s in EVENT_SEEDS[: args.events]]
    xs = [e.x for e in evs]

    if args.copy_calibration:
        # a plain copy of known size: the hardware byte counters of this dispatch give the
        # factor between counter units and bytes moved
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    wall, lat, infos, labels = run_precision(args.precision, cfg, nets, xs, args.steps, args.warmup, torch, trk,
                                             args.latency_events)
    st = stage_means(infos)
    n_cand = float(np.mean([i["n_cand_edges"] for i in infos]))
    filt_tflops = n_cand * FILTER_FLOP_PER_EDGE / (st["filter"] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    value = args.steps / wall
    result = {
        "metric": "events/s and p50/p99 latency per mu=200 event; per-stage MFMA/HBM roofline %",
        "value": round(value, 3), "unit": "events/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp32": "f32", "bf16": "bf16", "fp8": "fp8-e4m3", "fp8all": "fp8-e4m3", "bf16emb32": "bf16", "bf16x3": "bf16x3", "bf16x3gnn16": "bf16x3+bf16"}[args.precision],
        "data": "synthetic helical-track events (seeded), random-init weights (seed 0)",
        "config": {"workload": "mu200 event: 110000 hits, emb 3-1024x3-12, r=0.2 K=256, filter 24-512x3-1, "
                               "IN H=128 T=8, trk_event per event", "events": len(xs),
                   "precision": args.precision},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 3), "events": int(lat.size)},
        "stage_ms": {k: round(v, 4) for k, v in st.items()},
        "counts": {"n_hits": int(np.mean([i["n_hits"] for i in infos])), "n_cand_edges": int(n_cand),
                   "n_filt_edges": int(np.mean([i["n_filt_edges"] for i in infos])),
                   "n_kept_edges": int(np.mean([i["n_kept_edges"] for i in infos])),
                   "n_saturated": int(np.mean([i["n_saturated"] for i in infos]))},
        "roofline": {"kernel": "filter_kernel", "bound": "mfma", "achieved": round(filt_tflops, 2),
                     "peak": peak, "unit": "TFLOP/s", "frac": round(filt_tflops / peak, 4),
                     "traffic": measured_traffic(args.precision),
                     "flop_per_edge": FILTER_FLOP_PER_EDGE},
        "stage_roofline": None,
    }
    result["stage_roofline"] = stage_rooflines(st, result["counts"], args.precision, peak)
    result["margin_edges_per_event"] = margin_counts(cfg, nets, xs, trk)
    result["host"] = host_info()
    if not args.no_variant:
        result["score_errors_vs_fp64"] = score_errors(cfg, nets, ("fp32",) + SERVED_FORMS, trk)
        result["variants"] = {}
        for other in [p for p in ("fp32", "bf16", "bf16emb32", "bf16x3", "bf16x3gnn16", "fp8", "fp8all") if p != args.precision]:
            w2, lat2, inf2, lab2 = run_precision(other, cfg, nets, xs, args.steps, args.warmup, torch, trk,
                                                 args.latency_events)
            agr = [agreement(a, b) for a, b in zip(labels, lab2)]
            st2 = stage_means(inf2)
            nc2 = float(np.mean([i["n_cand_edges"] for i in inf2]))
            ft2 = nc2 * FILTER_FLOP_PER_EDGE / (st2["filter"] * 1e-3) / 1e12
            result["variants"][other] = {
                "value": round(args.steps / w2, 3), "unit": "events/s",
                "latency_ms": {"p50": round(float(np.percentile(lat2, 50)) * 1e3, 3),
                               "p99": round(float(np.percentile(lat2, 99)) * 1e3, 3)},
                "stage_ms": {k: round(v, 4) for k, v in st2.items()},
                "filter_tflops": round(ft2, 2), "filter_frac_of_peak": round(ft2 / PEAK_TFLOPS[other], 4),
                "stage_roofline": stage_rooflines(st2, {
                    "n_hits": int(np.mean([i["n_hits"] for i in inf2])), "n_cand_edges": int(nc2),
                    "n_filt_edges": int(np.mean([i["n_filt_edges"] for i in inf2])),
                    "n_kept_edges": int(np.mean([i["n_kept_edges"] for i in inf2]))}, other, PEAK_TFLOPS[other]),
                "hit_agreement_vs_primary": round(float(np.mean([a[0] for a in agr])), 5),
                "candidate_jaccard_vs_primary": round(float(np.mean([a[1] for a in agr])), 5),
                "n_cand_edges": int(nc2), "n_filt_edges": int(np.mean([i["n_filt_edges"] for i in inf2])),
            }
    if not args.no_trained:
        try:
            result["trained"] = trained_chain(cfg, evs, args, torch, trk)
        except trk.TrkError as e:
            result["trained"] = {"error": str(e)}
    # roofline denominators measured on this device, beside the published peaks
    try:
        pm = measured_peaks(torch, trk)
        result["peaks_measured"] = pm
        key = {"fp32": "fp32_mfma_tflops", "bf16x3": "bf16_mfma_tflops", "bf16x3gnn16": "bf16_mfma_tflops",
               "fp8": "fp8_mfma_tflops", "fp8all": "fp8_mfma_tflops"}.get(args.precision, "bf16_mfma_tflops")
        result["roofline"]["peak_measured"] = pm[key]
        result["roofline"]["frac_measured"] = round(filt_tflops / pm[key], 4)
    except trk.TrkError as e:
        result["peaks_measured"] = {"error": str(e)}
    if args.serving_long == "mix":
        # BF16 at 0.5 and 0.8 of its saturated rate, 10,000 measured requests each; the
        # FP32 pipeline offered the same rates (it saturates below them: 1,000 requests)
        result["serving_long"] = []
        for frac in (0.5, 0.8):
            sv = serve_load(cfg, nets, "bf16", 0, frac, trk, requests=10000, warmup_requests=200)
            result["serving_long"].append(sv)
            result["serving_long"].append(serve_load(cfg, nets, "fp32", 0, 1.0, trk, rate=sv["offered_events_per_s"],
                                                     requests=1000, warmup_requests=200))
        # a forced-small memory budget (two and a half pile-up-200 events in flight):
        # requests queue for admission instead of overlapping freely
        result["serving_long"].append(serve_load(cfg, nets, "bf16", 0, 0.8, trk, requests=2000, warmup_requests=200,
                                                 budget_events=2.5))
    if args.serving_long == "mu200":
        # pile-up-200 events only, offered half the FP32 pipeline's own rate, one slot,
        # batches of one event: 2,000 measured requests per form
        result["serving_long"] = [serve_load(cfg, nets, prec, 0, 1.0, trk, mus=[200], rate=0.5 * value, n_slots=1,
                                             max_batch_events=1, requests=2000, warmup_requests=200)
                                  for prec in ("fp32", "bf16", "bf16x3", "fp8")]
    if args.serve_seconds > 0:
        try:
            result["serving"] = serve_load(cfg, nets, "bf16", args.serve_seconds, 0.8, trk)
        except trk.TrkError as e:
            result["serving"] = {"error": str(e)}
        try:
            # the same load under a forced-small memory budget: admission queues requests
            result["serving_small_budget"] = serve_load(cfg, nets, "bf16", args.serve_seconds, 0.8, trk,
                                                        budget_events=2.5)
        except trk.TrkError as e:
            result["serving_small_budget"] = {"error": str(e)}
        # the served BF16 forms on pile-up-200 events only, offered the plain FP32
        # pipeline's own event rate (and half of it): p99 beside the FP32 p99 (host
        # buffers, PCIe included; Poisson arrivals queue, the FP32 figure is back to
        # back) and the saturated rate beside the FP32 rate.  Three slots overlap
        # events on the device (throughput); one slot runs them one after another.
        # The FP32 pipeline served at half its own rate gives its queueing tail under
        # the same arrivals.  Batches of one event (no batching of queued pile-up-200
        # events, which only delays the first of them) give the latency-oriented form.
        result["serving_mu200"] = []
        for prec, slots, frac, mb in (("bf16", 3, 1.0, 8), ("bf16", 1, 1.0, 8), ("bf16", 1, 0.5, 8),
                                      ("bf16emb32", 1, 1.0, 8), ("bf16emb32", 1, 0.5, 8), ("bf16x3", 1, 1.0, 8),
                                      ("bf16x3", 1, 0.5, 8), ("bf16x3", 1, 1.0, 1), ("bf16x3", 1, 0.5, 1),
                                      ("bf16x3gnn16", 1, 1.0, 8), ("fp32", 1, 0.5, 8), ("fp32", 1, 0.5, 1)):
            try:
                sv = serve_load(cfg, nets, prec, args.serve_seconds, 1.0, trk, mus=[200], rate=frac * value,
                                n_slots=slots, max_batch_events=mb)
                if args.precision == "fp32":
                    sv["vs_fp32_pipeline"] = {"offered_fraction_of_fp32_rate": frac,
                                              "fp32_events_per_s": round(value, 3),
                                              "fp32_p99_ms": result["latency_ms"]["p99"]}
            except trk.TrkError as e:
                sv = {"precision": prec, "slots": slots, "error": str(e)}
            result["serving_mu200"].append(sv)
    if args.serve_seconds > 0:
        try:
            # the socket front end: what the transfer adds to each request
            result["service_mu200"] = service_load(cfg, nets, "bf16", args.serve_seconds, 0.5 * value, trk)
        except (trk.TrkError, OSError) as e:
            result["service_mu200"] = {"error": str(e)}
    try:
        result["downstream_fit"] = fit_measure(cfg, nets, evs[0], labels[0], torch, trk)
    except trk.TrkError as e:
        result["downstream_fit"] = {"error": str(e)}
    if args.train_steps > 0:
        try:
            result["training"] = train_measure(cfg, nets, args.train_steps, torch, trk)
        except trk.TrkError as e:
            result["training"] = {"error": str(e)}
        try:
            result["training_bf16"] = train_measure(cfg, nets, args.train_steps, torch, trk, "bf16")
        except trk.TrkError as e:
            result["training_bf16"] = {"error": str(e)}
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(cfg, nets, xs[0])
        result["cpu_baseline_tiny"] = cpu_baseline_tiny()
    result["paper_context"] = PAPER_CONTEXT
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

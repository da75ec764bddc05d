"""Training of the filter MLP and the interaction network through the library's
hand-written backward passes, exposed as torch.autograd.Function objects.  The
forward, backward, loss and Adam update all run in libtrk.so; torch only holds
the device tensors and chains the gradients."""
import numpy as np
import torch

from . import trk


class TrainContext:
    """A context with training buffers and a flat FP32 parameter vector.
    precision "fp32": FP32 products; "bf16": every product with BF16 operands and
    FP32 accumulation (FP32 master parameters, moments and stored activations)."""

    def __init__(self, cfg, nets, device=0, max_hits=None, max_cand_edges=None, max_kept_edges=None,
                 precision="fp32"):
        if precision not in ("fp32", "bf16"):
            raise ValueError("training runs in fp32 or bf16")
        self.cfg = cfg
        self.precision = precision
        self.device = torch.device("cuda", device)
        self.config = trk.make_config(cfg, precision, max_hits, max_cand_edges, max_kept_edges, 1, False, True)
        self.ctx = trk.trk_create(self.config, trk.pack_weights(cfg, nets), device)
        self.n_params = trk.trk_train_param_count(self.config)
        flat = trk.flatten_params(nets)
        assert flat.size == self.n_params
        self.params = torch.tensor(flat, device=self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step_count = 0
        self.sync_params()

    def sync_params(self):
        trk.trk_train_set_params(self.ctx, self.params)

    def close(self):
        if self.ctx is not None:
            trk.trk_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def adam_step(self, grads, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        trk.trk_adam_update(self.ctx, self.params, grads, self.m, self.v, lr, beta1, beta2, eps, self.step_count)
        self.sync_params()


class FilterLogits(torch.autograd.Function):
    """z_f = MLP_f([emb_src, emb_dst]) with gradient with respect to the flat parameters."""

    @staticmethod
    def forward(ctx, params, emb, src, dst, tctx):
        logits = torch.empty(src.numel(), dtype=torch.float32, device=emb.device)
        trk.trk_filter_train_fwd(tctx.ctx, emb, src, dst, logits)
        ctx.save_for_backward(emb, src, dst)
        ctx.tctx = tctx
        return logits

    @staticmethod
    def backward(ctx, dlogits):
        emb, src, dst = ctx.saved_tensors
        grads = torch.zeros(ctx.tctx.n_params, dtype=torch.float32, device=emb.device)
        trk.trk_filter_train_bwd(ctx.tctx.ctx, emb, src, dst, dlogits.contiguous(), grads)
        return grads, None, None, None, None


class GnnLogits(torch.autograd.Function):
    """z_o of the interaction network with gradient with respect to the flat parameters."""

    @staticmethod
    def forward(ctx, params, x, src, dst, tctx):
        logits = torch.empty(src.numel(), dtype=torch.float32, device=x.device)
        trk.trk_gnn_train_fwd(tctx.ctx, x, src, dst, logits)
        ctx.save_for_backward(x, src, dst)
        ctx.tctx = tctx
        return logits

    @staticmethod
    def backward(ctx, dlogits):
        x, src, dst = ctx.saved_tensors
        grads = torch.zeros(ctx.tctx.n_params, dtype=torch.float32, device=x.device)
        trk.trk_gnn_train_bwd(ctx.tctx.ctx, x, src, dst, dlogits.contiguous(), grads)
        return grads, None, None, None, None


class BCEWithLogits(torch.autograd.Function):
    """Mean binary cross-entropy with logits, evaluated by the library kernel."""

    @staticmethod
    def forward(ctx, logits, targets, tctx):
        dz = torch.empty_like(logits)
        loss = trk.trk_bce_with_logits(tctx.ctx, logits.contiguous(), targets.contiguous(), dz)
        ctx.save_for_backward(dz)
        return torch.tensor(loss, device=logits.device)

    @staticmethod
    def backward(ctx, g):
        (dz,) = ctx.saved_tensors
        return dz * g, None, None


def edge_truth(pid, src, dst):
    pid = np.asarray(pid)
    src = np.asarray(src)
    dst = np.asarray(dst)
    return ((pid[src] == pid[dst]) & (pid[src] != 0)).astype(np.float32)


def train_step(tctx, x, emb, cand, filt, y_cand, y_filt, lr=1e-3, filter=True, gnn=True):
    """One step: forward of the selected networks, summed loss, hand-written
    backward, Adam update; returns (loss_filter, loss_gnn)."""
    params = tctx.params.detach().requires_grad_(True)
    total, lf, lg = None, torch.zeros(()), torch.zeros(())
    if filter and cand[0].numel():
        zf = FilterLogits.apply(params, emb, cand[0], cand[1], tctx)
        lf = BCEWithLogits.apply(zf, y_cand, tctx)
        total = lf
    if gnn and filt[0].numel():
        zg = GnnLogits.apply(params, x, filt[0], filt[1], tctx)
        lg = BCEWithLogits.apply(zg, y_filt, tctx)
        total = lg if total is None else total + lg
    if total is not None:
        total.backward()
        tctx.adam_step(params.grad, lr)
    return float(lf), float(lg)


# ---------------------------------------------------------------------------
# metric learning of the embedding, then the filter and the interaction network
# ---------------------------------------------------------------------------
def positive_pairs(pid, layer, reach=2):
    """Same-particle hit pairs on layers up to `reach` apart (generator truth)."""
    pid = np.asarray(pid)
    layer = np.asarray(layer).astype(np.int64)
    order = np.lexsort((layer, pid))
    pa, pb = [], []
    for k in range(1, reach + 1):
        s, t = order[:-k], order[k:]
        ok = (pid[s] == pid[t]) & (pid[s] > 0)
        pa.append(s[ok])
        pb.append(t[ok])
    return np.concatenate(pa), np.concatenate(pb)


def embedding_step(tc, ev, rng, margin, lr, n_random=2.0, max_hard=2.0, neg_weight=10.0, measure=False):
    """One metric-learning step on event ev: positives from the truth, hard
    negatives from the current radius graph, uniform random negatives, the
    negative term weighted by neg_weight (without it the positive term dominates
    and the embedding contracts: every point ends up within r of ~100 others);
    returns (loss, true-edge fraction of the current candidate graph, its edge
    count) and, with measure, the fraction of the positive pairs that the current
    candidate graph holds."""
    dev = tc.device
    x = torch.as_tensor(ev.x, device=dev)
    emb = torch.empty((ev.n, tc.cfg.emb_dim), device=dev)
    trk.trk_embed_train_fwd(tc.ctx, x, emb)
    cap = int(tc.config.max_cand_edges)
    cs = torch.empty(cap, dtype=torch.int32, device=dev)
    cd = torch.empty_like(cs)
    # a graph above the capacity still yields its first `cap` edges (the rows of the
    # lowest ids, a random subset of hits since ids are shuffled): hard negatives
    # keep coming when the embedding contracts, which is when they are needed most
    total, _ = trk.trk_build_graph(tc.ctx, emb, cs, cd, truncate_ok=True)
    ne = min(total, cap)
    cs_h, cd_h = cs[:ne].cpu().numpy(), cd[:ne].cpu().numpy()
    yc = edge_truth(ev.pid, cs_h, cd_h) if ne else np.zeros(0, np.float32)
    true_frac = float(yc.mean()) if ne else 0.0
    pa, pb = positive_pairs(ev.pid, ev.layer)
    npos = pa.size
    hard = np.flatnonzero(yc < 0.5)
    if hard.size > max_hard * npos:
        hard = rng.choice(hard, int(max_hard * npos), replace=False)
    nr = int(n_random * npos)
    ra = rng.integers(0, ev.n, nr)
    rb = rng.integers(0, ev.n, nr)
    keep = ra != rb
    allA = np.concatenate([pa, cs_h[hard], ra[keep]])
    allB = np.concatenate([pb, cd_h[hard], rb[keep]])
    y = np.concatenate([np.ones(npos, np.float32), np.zeros(hard.size, np.float32),
                        edge_truth(ev.pid, ra[keep], rb[keep])])
    allA, allB, y = allA[:cap], allB[:cap], y[:cap]
    A = torch.as_tensor(allA.astype(np.int32), device=dev)
    B = torch.as_tensor(allB.astype(np.int32), device=dev)
    Y = torch.as_tensor(y, device=dev)
    demb = torch.empty_like(emb)
    loss = trk.trk_pair_loss(tc.ctx, emb, A, B, Y, margin, demb, neg_weight=neg_weight)
    grads = torch.zeros(tc.n_params, device=dev)
    trk.trk_embed_train_bwd(tc.ctx, x, demb, grads)
    tc.adam_step(grads, lr)
    if not measure:
        return loss, true_frac, int(total)
    n = np.int64(ev.n)
    pos = np.minimum(pa, pb).astype(np.int64) * n + np.maximum(pa, pb)
    cand = cs_h.astype(np.int64) * n + cd_h
    eff = float(np.isin(pos, cand).mean()) if pos.size and total <= cap else float("nan")
    return loss, true_frac, int(total), eff


def pipeline_step(tc, ev, lr, filter=True, gnn=True):
    """One filter and/or interaction-network step on the edge sets the current
    parameters produce for event ev (embedding frozen)."""
    dev = tc.device
    x = torch.as_tensor(ev.x, device=dev)
    emb = torch.empty((ev.n, tc.cfg.emb_dim), device=dev)
    trk.trk_embed(tc.ctx, x, emb)
    cap = int(tc.config.max_cand_edges)
    cs = torch.empty(cap, dtype=torch.int32, device=dev)
    cd = torch.empty_like(cs)
    ne, _ = trk.trk_build_graph(tc.ctx, emb, cs, cd)
    cs, cd = cs[:ne], cd[:ne]
    scores = torch.empty(ne, device=dev)
    kcap = int(tc.config.max_kept_edges)
    ks = torch.empty(max(kcap, 1), dtype=torch.int32, device=dev)
    kd = torch.empty_like(ks)
    nk = trk.trk_filter(tc.ctx, emb, cs, cd, scores, ks[:kcap], kd[:kcap])
    ks, kd = ks[:nk], kd[:nk]
    yc = torch.as_tensor(edge_truth(ev.pid, cs.cpu().numpy(), cd.cpu().numpy()), device=dev)
    yf = torch.as_tensor(edge_truth(ev.pid, ks.cpu().numpy(), kd.cpu().numpy()), device=dev)
    lf, lg = train_step(tc, x, emb, (cs, cd), (ks, kd), yc, yf, lr, filter=filter, gnn=gnn)
    return lf, lg, float(yc.mean()) if ne else 0.0, float(yf.mean()) if nk else 0.0


def filter_scores_on(tc, ev):
    """Filter scores of the candidate edges of event ev under the current
    parameters, with their truth (host arrays)."""
    dev = tc.device
    x = torch.as_tensor(ev.x, device=dev)
    emb = torch.empty((ev.n, tc.cfg.emb_dim), device=dev)
    trk.trk_embed(tc.ctx, x, emb)
    cap = int(tc.config.max_cand_edges)
    cs = torch.empty(cap, dtype=torch.int32, device=dev)
    cd = torch.empty_like(cs)
    ne, _ = trk.trk_build_graph(tc.ctx, emb, cs, cd)
    cs, cd = cs[:ne], cd[:ne]
    scores = torch.empty(ne, device=dev)
    kcap = int(tc.config.max_kept_edges)
    ks = torch.empty(max(kcap, 1), dtype=torch.int32, device=dev)
    kd = torch.empty_like(ks)
    trk.trk_filter(tc.ctx, emb, cs, cd, scores, ks[:kcap], kd[:kcap])
    return scores.cpu().numpy(), edge_truth(ev.pid, cs.cpu().numpy(), cd.cpu().numpy())


# ---------------------------------------------------------------------------
# data-dependent start of the first layers that read an edge's two ends
# ---------------------------------------------------------------------------
def fold_pair_standardisation(w, b, a_s, a_t):
    """First-layer weights acting on u = [a_s, a_t] that compute the seeded layer
    (w, b) of the standardised pair mean m = (a_s + a_t) / 2 and difference
    d = a_s - a_t (statistics over the rows of a_s, a_t): with A, B the two halves of
    w, W_s = A / (2 sd_m) + B / sd_d, W_t = A / (2 sd_m) - B / sd_d and
    b' = b - (A mu_m / sd_m + B mu_d / sd_d).  The small difference between the two
    ends of an edge, which carries the track signal, is then seen at unit scale."""
    a_s = np.asarray(a_s, np.float64)
    a_t = np.asarray(a_t, np.float64)
    m, d = (a_s + a_t) / 2, a_s - a_t
    mu_m, sd_m = m.mean(0), m.std(0) + 1e-9
    mu_d, sd_d = d.mean(0), d.std(0) + 1e-9
    w = np.asarray(w, np.float64)
    D = w.shape[0] // 2
    A, B = w[:D], w[D:]
    ws = A / (2 * sd_m[:, None]) + B / sd_d[:, None]
    wt = A / (2 * sd_m[:, None]) - B / sd_d[:, None]
    b2 = np.asarray(b, np.float64) - (mu_m / sd_m) @ A - (mu_d / sd_d) @ B
    return np.concatenate([ws, wt]).astype(np.float32), b2.astype(np.float32)


def pair_samples(pipe, events):
    """Embedding pairs, feature pairs (over the candidate edges) and the features
    of the given events, from an inference Pipeline (host arrays)."""
    emb_pairs, x_pairs, xs = [], [], []
    for ev in events:
        e = pipe.embed(ev.x)
        s, d, _ = pipe.build_graph(e)
        s, d = s.cpu().numpy(), d.cpu().numpy()
        en = e.cpu().numpy()
        emb_pairs.append((en[s], en[d]))
        x_pairs.append((ev.x[s], ev.x[d]))
        xs.append(ev.x)
    cat = lambda ps, i: np.concatenate([p[i] for p in ps])
    return (cat(emb_pairs, 0), cat(emb_pairs, 1)), (cat(x_pairs, 0), cat(x_pairs, 1)), np.concatenate(xs)


def standardised_start(nets, emb_pairs, x_pairs, x, filter=True, gnn=True):
    """nets with the filter's first layer (filter) and the edge and node encoders'
    first layers (gnn) reading standardised inputs: pair mean and difference for the
    layers that read both ends of an edge, the features themselves for the node
    encoder."""
    out = dict(nets)
    if filter:
        w, b = fold_pair_standardisation(*nets["filt"][0], *emb_pairs)
        out["filt"] = [(w, b)] + list(nets["filt"][1:])
    if gnn:
        w, b = fold_pair_standardisation(*nets["edge_enc"][0], *x_pairs)
        out["edge_enc"] = [(w, b)] + list(nets["edge_enc"][1:])
        xa = np.asarray(x, np.float64)
        mu, sd = xa.mean(0), xa.std(0) + 1e-9
        w0, b0 = [np.asarray(v, np.float64) for v in nets["node_enc"][0]]
        out["node_enc"] = [((w0 / sd[:, None]).astype(np.float32), (b0 - (mu / sd) @ w0).astype(np.float32))] + \
            list(nets["node_enc"][1:])
    return out

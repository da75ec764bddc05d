"""Training of the filter MLP and the interaction network through the library's
hand-written backward passes, exposed as torch.autograd.Function objects.  The
forward, backward, loss and Adam update all run in libtrk.so; torch only holds
the device tensors and chains the gradients."""
import numpy as np
import torch

from . import trk


class TrainContext:
    """An FP32 context with training buffers and a flat FP32 parameter vector."""

    def __init__(self, cfg, nets, device=0, max_hits=None, max_cand_edges=None, max_kept_edges=None):
        self.cfg = cfg
        self.device = torch.device("cuda", device)
        self.config = trk.make_config(cfg, "fp32", max_hits, max_cand_edges, max_kept_edges, 1, False, True)
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


def train_step(tctx, x, emb, cand, filt, y_cand, y_filt, lr=1e-3):
    """One step: forward of both networks, summed loss, hand-written backward,
    Adam update; returns (loss_filter, loss_gnn)."""
    params = tctx.params.detach().requires_grad_(True)
    zf = FilterLogits.apply(params, emb, cand[0], cand[1], tctx)
    lf = BCEWithLogits.apply(zf, y_cand, tctx)
    zg = GnnLogits.apply(params, x, filt[0], filt[1], tctx)
    lg = BCEWithLogits.apply(zg, y_filt, tctx)
    (lf + lg).backward()
    tctx.adam_step(params.grad, lr)
    return float(lf), float(lg)

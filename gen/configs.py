"""Model and workload configurations (the sizes of the two event classes, the
pipeline constants, and the output-layer gains of the seeded weights).

Widths are written as the layer sequence of each network:
  embedding  3 -> hidden x emb_layers -> emb_dim          (tanh on hidden layers)
  filter     2*emb_dim -> hidden x filt_layers -> 1       (tanh on hidden layers)
  interaction network with hidden size H:
      node encoder [3, H, H], edge encoder [6, H, H],
      edge network [3H, H, H], node network [2H, H, H]   (tanh after every layer)
      output head  [3H, H, 1]                             (last layer linear)
"""
from dataclasses import dataclass, replace, asdict


@dataclass(frozen=True)
class TrkConfig:
    name: str
    n_collisions: int          # pile-up mu: 50 particles per collision
    emb_hidden: int
    emb_layers: int
    emb_dim: int
    filt_hidden: int
    filt_layers: int
    gnn_hidden: int
    gnn_iters: int
    radius: float
    k_max: int
    filter_cut: float
    score_cut: float = 0.5
    min_track_hits: int = 3
    # gains applied to the last layer (weights and bias) of each seeded network
    emb_out_gain: float = 1.0
    filt_out_gain: float = 1.0
    gnn_out_gain: float = 1.0

    def with_(self, **kw):
        return replace(self, **kw)

    def as_dict(self):
        return asdict(self)


# 50 tracks x 10 layers + 10 % noise = 550 hits
TINY = TrkConfig(name="tiny", n_collisions=1,
                 emb_hidden=64, emb_layers=2, emb_dim=8,
                 filt_hidden=64, filt_layers=2,
                 gnn_hidden=32, gnn_iters=4,
                 radius=0.5, k_max=64, filter_cut=0.2,
                 emb_out_gain=4.0, filt_out_gain=14.0, gnn_out_gain=14.0)

# pile-up 200: 10,000 tracks x 10 layers + 10 % noise = 110,000 hits
MU200 = TrkConfig(name="mu200", n_collisions=200,
                  emb_hidden=1024, emb_layers=3, emb_dim=12,
                  filt_hidden=512, filt_layers=3,
                  gnn_hidden=128, gnn_iters=8,
                  radius=0.2, k_max=256, filter_cut=0.38,
                  emb_out_gain=20.0, filt_out_gain=25.0, gnn_out_gain=6.0)

CONFIGS = {"tiny": TINY, "mu200": MU200}

# pile-up values of the serving mix
SERVE_MUS = (50, 100, 140, 200)


def mlp_dims(cfg):
    """Layer widths of every network, in weight-blob order."""
    H = cfg.gnn_hidden
    return [
        ("emb", [3] + [cfg.emb_hidden] * cfg.emb_layers + [cfg.emb_dim]),
        ("filt", [2 * cfg.emb_dim] + [cfg.filt_hidden] * cfg.filt_layers + [1]),
        ("node_enc", [3, H, H]),
        ("edge_enc", [6, H, H]),
        ("edge_net", [3 * H, H, H]),
        ("node_net", [2 * H, H, H]),
        ("out", [3 * H, H, 1]),
    ]

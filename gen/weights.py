"""Seeded random initialisation of every network's weights.

Each Linear layer of fan-in f gets W [f, out] and b [out] drawn uniform on
(-1/sqrt(f), +1/sqrt(f)) from its own SplitMix64 stream, computed in double and
rounded to float32 (round-to-nearest-even).  The last layer of the embedding,
the filter and the output head is scaled by the configured gain.  These are the
inputs both pipelines receive; no step of the tracking method is computed here.
"""
import numpy as np

from . import splitmix as sm
from .configs import mlp_dims

_GAIN_OF = {"emb": "emb_out_gain", "filt": "filt_out_gain", "out": "gnn_out_gain"}


def make_weights(cfg, seed=0):
    """Ordered dict name -> list of (W float32 [in, out], b float32 [out])."""
    nets = {}
    tag = 0
    for name, dims in mlp_dims(cfg):
        layers = []
        for li in range(len(dims) - 1):
            fi, fo = dims[li], dims[li + 1]
            bound = 1.0 / np.sqrt(fi)
            w = sm.uniform(seed, 1000 + tag, fi * fo, -bound, bound).reshape(fi, fo)
            b = sm.uniform(seed, 2000 + tag, fo, -bound, bound)
            tag += 1
            if li == len(dims) - 2 and name in _GAIN_OF:
                g = float(getattr(cfg, _GAIN_OF[name]))
                w, b = w * g, b * g
            layers.append((w.astype(np.float32), b.astype(np.float32)))
        nets[name] = layers
    return nets


def n_params(nets):
    return sum(w.size + b.size for layers in nets.values() for (w, b) in layers)


def load_weights(path, cfg):
    """Weights written by paper_2501_05520_amd.train_weights (an .npz of float32
    arrays named '<net>.<layer>.w' / '.b'), in make_weights' layout."""
    from .configs import mlp_dims
    z = np.load(path, allow_pickle=False)
    nets = {}
    for name, dims in mlp_dims(cfg):
        nets[name] = [(z[f"{name}.{li}.w"].astype(np.float32), z[f"{name}.{li}.b"].astype(np.float32))
                      for li in range(len(dims) - 1)]
    return nets


def load_trained(path, cfg):
    """Trained weights and the configuration they were calibrated for: the .npz
    written by paper_2501_05520_amd.train_weights carries its filter cut."""
    z = np.load(path, allow_pickle=False)
    cut = float(z["filter_cut"]) if "filter_cut" in z.files else float(cfg.filter_cut)
    return cfg.with_(filter_cut=cut), load_weights(path, cfg)

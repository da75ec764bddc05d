"""CPU checks of the committed trained weight set: the file matches the sha256 its
record states, loads through gen.load_trained with the record's configuration and its
calibrated filter cut, and holds finite weights of the configured shapes."""
import hashlib
import json
import os

import numpy as np

from gen import MU200, load_trained, make_weights

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "weights", "trained_mu200.npz")
RECORD = os.path.join(ROOT, "weights", "trained_mu200.json")


def test_record_matches_file():
    with open(RECORD) as fh:
        rec = json.load(fh)
    with open(WEIGHTS, "rb") as fh:
        assert hashlib.sha256(fh.read()).hexdigest() == rec["sha256"]
    assert rec["file"] == "weights/trained_mu200.npz"
    assert len(rec["recipe"]) >= 1 and all("train_weights" in c for c in rec["recipe"])


def test_weights_load_with_the_configured_shapes():
    cfg, nets = load_trained(WEIGHTS, MU200)
    seeded = make_weights(MU200, 0)
    assert set(nets) == set(seeded)
    for name, layers in seeded.items():
        assert len(nets[name]) == len(layers)
        for (w, b), (w0, b0) in zip(nets[name], layers):
            assert w.shape == w0.shape and b.shape == b0.shape
            assert np.all(np.isfinite(w)) and np.all(np.isfinite(b))
    with np.load(WEIGHTS, allow_pickle=False) as z:
        assert np.isclose(float(cfg.filter_cut), float(z["filter_cut"]))
        assert z["trained"].astype(bool).all()

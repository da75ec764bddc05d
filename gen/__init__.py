"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path: events,
weights and the configuration constants.  Nothing here computes a step of the
tracking pipeline."""
from .configs import TrkConfig, TINY, MU200, CONFIGS, SERVE_MUS, mlp_dims
from .events import Event, generate_event, pack_events, LAYER_RADII_MM, B_FIELD_T
from .weights import make_weights, n_params, load_weights, load_trained

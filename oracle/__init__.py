"""FP64 CPU oracle of the tracking chain.  Test infrastructure only: the library
and its binding never import it; tests, the smoke check and the benchmark's
CPU-baseline leg do."""
from .pipeline import (sigmoid, mlp, embed, radius_pairs, select_neighbours, radius_graph,
                       filter_scores, filter_edges, interaction_network, components,
                       candidates, event)

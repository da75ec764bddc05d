"""Pins for the oracle's connected components: hand graphs with known labels,
a pure-Python breadth-first search, networkx, and label invariants."""
import numpy as np
import networkx as nx
from hypothesis import given, settings, strategies as st

import oracle


def _bfs_labels(n, edges):
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    lab = [-1] * n
    for s in range(n):
        if lab[s] >= 0:
            continue
        lab[s] = s                        # s is the smallest unvisited id: the component minimum
        stack = [s]
        while stack:
            u = stack.pop()
            for v in adj[u]:
                if lab[v] < 0:
                    lab[v] = s
                    stack.append(v)
    return lab


def _cc(n, edges, scores=None, cut=0.5):
    s = np.array([a for a, _ in edges], np.int64)
    d = np.array([b for _, b in edges], np.int64)
    return oracle.components(n, s, d, scores, cut).tolist()


def test_hand_graphs():
    assert _cc(5, [(3, 4), (2, 3), (1, 2), (0, 1)]) == [0] * 5          # path, edges in reverse order
    assert _cc(6, [(5, 0), (5, 1), (5, 2)]) == [0, 0, 0, 3, 4, 0]       # star + isolated
    assert _cc(4, [(0, 1), (1, 2), (2, 3), (3, 0)]) == [0] * 4           # cycle
    two = [(a, b) for a in range(3) for b in range(a + 1, 3)] + [(a, b) for a in range(3, 7) for b in range(a + 1, 7)]
    assert _cc(8, two) == [0, 0, 0, 3, 3, 3, 3, 7]                       # two cliques + isolated
    assert _cc(3, []) == [0, 1, 2]
    assert _cc(0, []) == []
    # a long chain with ids descending along it
    n = 5000
    chain = [(i, i - 1) for i in range(n - 1, 0, -1)]
    assert _cc(n, chain) == [0] * n


def test_score_cut_is_strict():
    edges = [(0, 1), (1, 2), (3, 4)]
    assert _cc(5, edges, np.array([0.5, 0.9, 0.51]), 0.5) == [0, 1, 1, 3, 3]


@settings(max_examples=40, deadline=None)
@given(n=st.integers(1, 80), m=st.integers(0, 120), seed=st.integers(0, 2**31 - 1))
def test_random_graphs_against_bfs_and_networkx(n, m, seed):
    rng = np.random.default_rng(seed)
    edges = [tuple(map(int, rng.integers(0, n, 2))) for _ in range(m)]
    lab = _cc(n, edges)
    assert lab == _bfs_labels(n, edges)
    g = nx.Graph()
    g.add_nodes_from(range(n))
    g.add_edges_from(edges)
    comps = list(nx.connected_components(g))
    want = [0] * n
    for c in comps:
        for v in c:
            want[v] = min(c)
    assert lab == want
    lab = np.array(lab)
    assert np.all(lab <= np.arange(n)) and np.array_equal(lab[lab], lab)
    for a, b in edges:
        assert lab[a] == lab[b]
    assert np.unique(lab).size == len(comps)


def test_candidates_min_size():
    lab = np.array([0, 0, 0, 3, 3, 5, 0, 5, 5, 9])
    assert oracle.candidates(lab, 3) == [(0, 1, 2, 6), (5, 7, 8)]

"""Pins for the oracle's fixed-radius graph: brute-force all pairs, the K-cap
by explicit per-point sorting, symmetry and monotonicity invariants."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from gen import TINY, make_weights, generate_event


def _brute_pairs(e, r):
    e = e.astype(np.float64)
    n = e.shape[0]
    out = []
    for i in range(n):
        d2 = ((e[i + 1:] - e[i]) ** 2).sum(axis=1)
        for k in np.flatnonzero(d2 < r * r):
            out.append((i, i + 1 + k, d2[k]))
    return out


def _brute_graph(e, r, kmax):
    e = e.astype(np.float64)
    n = e.shape[0]
    edges = set()
    for i in range(n):
        d2 = ((e - e[i]) ** 2).sum(axis=1)
        cand = sorted((d2[j], j) for j in range(n) if j != i and d2[j] < r * r)
        for _, j in cand[:kmax]:
            edges.add((min(i, j), max(i, j)))
    return sorted(edges)


def _tiny_emb(seed=1):
    nets = make_weights(TINY, 0)
    return oracle.embed(generate_event(seed, 1).x, nets).astype(np.float32)


def test_pairs_match_brute_force_tiny_event():
    e = _tiny_emb()
    r = float(np.float32(TINY.radius))
    lo, hi, d2 = oracle.radius_pairs(e, r)
    got = sorted(zip(lo.tolist(), hi.tolist()))
    want = [(i, j) for i, j, _ in _brute_pairs(e, r)]
    assert got == want and len(got) > 1000


@pytest.mark.parametrize("seed,kmax", [(1, 64), (2, 64), (3, 5), (4, 1)])
def test_capped_graph_matches_brute_force(seed, kmax):
    e = _tiny_emb(seed)
    r = float(np.float32(TINY.radius))
    s, d, count = oracle.radius_graph(e, r, kmax)
    want = _brute_graph(e, r, kmax)
    assert list(zip(s.tolist(), d.tolist())) == want
    assert np.all(s < d)
    if kmax == 64:
        assert np.any(count > kmax), "the K-cap must be exercised"


@settings(max_examples=25, deadline=None)
@given(n=st.integers(0, 60), dim=st.integers(1, 12), r=st.floats(0.05, 1.5),
       kmax=st.integers(1, 70), seed=st.integers(0, 2**31 - 1))
def test_random_clouds(n, dim, r, kmax, seed):
    rng = np.random.default_rng(seed)
    e = rng.uniform(-1, 1, size=(n, dim)).astype(np.float32)
    s, d, _ = oracle.radius_graph(e, r, kmax)
    assert list(zip(s.tolist(), d.tolist())) == _brute_graph(e, r, kmax)


def test_uncapped_is_symmetric_and_monotone():
    e = _tiny_emb(2)
    big = 10**6
    s1, d1, c1 = oracle.radius_graph(e, 0.3, big)
    s2, d2, _ = oracle.radius_graph(e, 0.5, big)
    a = set(zip(s1.tolist(), d1.tolist()))
    b = set(zip(s2.tolist(), d2.tolist()))
    assert a <= b and len(a) < len(b)
    # uncapped selection is symmetric: every within-r pair appears, and the
    # per-point count equals the degree in the undirected graph
    deg = np.bincount(s1, minlength=e.shape[0]) + np.bincount(d1, minlength=e.shape[0])
    assert np.array_equal(deg, c1)


def test_strict_radius_and_ties():
    # points on a line at exact binary distances: d = r is excluded (strict <)
    e = np.array([[0.0], [0.5], [1.0], [1.25]], np.float32)
    s, d, c = oracle.radius_graph(e, 0.5, 10)
    assert list(zip(s.tolist(), d.tolist())) == [(2, 3)]
    # equal distances: the lower id wins the last slot of the cap
    e = np.array([[0.0], [-0.25], [0.25], [0.1]], np.float32)
    s, d, _ = oracle.radius_graph(e, 1.0, 2)
    # point 0 keeps 3 (d=.1) and 1 (d=.25, id 1 < 2); 2 keeps 3 and 0; 1 keeps 0 and 3;
    # 3 keeps 0 and 2
    assert list(zip(s.tolist(), d.tolist())) == [(0, 1), (0, 2), (0, 3), (1, 3), (2, 3)]


def test_empty_and_single():
    s, d, c = oracle.radius_graph(np.zeros((0, 8), np.float32), 0.5, 4)
    assert s.size == 0 and c.size == 0
    s, d, c = oracle.radius_graph(np.zeros((1, 8), np.float32), 0.5, 4)
    assert s.size == 0 and c.tolist() == [0]

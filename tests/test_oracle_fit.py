"""Pins of the FP64 helix-fit oracle (oracle/fit.py) against what the generator
fixes, not against the oracle itself: the helix parameters each particle was
generated with (pT, phi0, eta, z0, charge), exact circles, and the degenerate
cases (too few hits, collinear points)."""
import numpy as np

from gen import generate_event
from oracle import fit as F


def _truth_labels(ev):
    # one label per particle (its smallest hit index), noise hits on their own
    lab = np.arange(ev.n)
    for p in np.unique(ev.pid[ev.pid > 0]):
        idx = np.flatnonzero(ev.pid == p)
        lab[idx] = idx.min()
    return lab


def test_recovers_generated_helices():
    ev = generate_event(8, 3)
    lab = _truth_labels(ev)
    labels, nh, par = F.fit_candidates(ev.x, lab, min_hits=3, b_field=2.0)
    assert len(labels) == 150 and np.all(nh == 10)       # every particle, no noise singleton
    pid = ev.pid[labels] - 1
    t = ev.truth
    # features are float32 (relative rounding 6e-8): the fitted parameters agree with
    # the generated ones far below the spread of the sample
    assert np.max(np.abs(par[:, 0] / t["pt"][pid] - 1.0)) < 1e-3
    dphi = (par[:, 1] - t["phi0"][pid] + np.pi) % (2 * np.pi) - np.pi
    assert np.max(np.abs(dphi)) < 1e-4
    assert np.max(np.abs(par[:, 2] - t["eta"][pid])) < 1e-4
    assert np.max(np.abs(par[:, 3] - t["z0"][pid])) < 0.05            # mm
    assert np.array_equal(par[:, 4], t["q"][pid])
    assert np.max(par[:, 5]) < 1e-6                                    # mm^2: the hits lie on the circle


def test_exact_circle_and_line():
    # a circle of radius 2000 mm through the origin, clockwise (q = +1), phi0 = 0.3
    R, phi0, q, tl, z0 = 2000.0, 0.3, 1.0, 0.5, 12.0
    rho = np.array([40.0, 150.0, 300.0, 500.0, 800.0])
    a = np.arcsin(rho / (2 * R))
    phi = phi0 - q * a
    z = z0 + 2 * R * a * tl
    x = np.stack([rho / 1000, phi / np.pi, z / 1000], axis=1)
    _, _, par = F.fit_candidates(x, np.zeros(5, int), min_hits=3, b_field=2.0)
    pt, p0, eta, zz, qq, chi2 = par[0]
    assert abs(pt - 0.3 * 2.0 * R / 1000) < 1e-9 and abs(p0 - phi0) < 1e-12
    assert abs(eta - np.arcsinh(tl)) < 1e-12 and abs(zz - z0) < 1e-9 and qq == q and chi2 < 1e-18


def test_min_hits_and_ordering():
    ev = generate_event(9, 1)
    lab = _truth_labels(ev)
    l3, n3, _ = F.fit_candidates(ev.x, lab, min_hits=3)
    l11, _, _ = F.fit_candidates(ev.x, lab, min_hits=11)
    assert np.all(np.diff(l3) > 0) and len(l11) == 0 and np.all(n3 >= 3)


def test_degenerate_candidates_are_nan():
    # three hits on one line through the origin, and three coincident hits
    line = np.array([[0.1, 0.25, 0.0], [0.2, 0.25, 0.1], [0.3, 0.25, 0.2]], np.float32)
    same = np.tile(np.array([[0.5, 0.1, 0.0]], np.float32), (3, 1))
    x = np.concatenate([line, same])
    _, _, par = F.fit_candidates(x, [0, 0, 0, 3, 3, 3], min_hits=3)
    assert np.all(np.isnan(par))

"""FP64 oracle of the downstream helix fit of track candidates.  TEST
INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).

The tracking chain ends with track candidates, lists of spacepoints
(Section 2.2.2); what consumes them next is a fit of the track parameters.  The
reading taken here, for a solenoid field B along z:

* spacepoints from the features: rho = 1000 x0 mm, phi = pi x1, z = 1000 x2 mm,
  X = rho cos(phi), Y = rho sin(phi);
* a candidate is a label value carried by at least min_hits spacepoints;
* transverse plane: the algebraic circle fit, the least-squares solution of
      X^2 + Y^2 + D X + E Y + F = 0   over the candidate's hits,
  centre (a, b) = (-D/2, -E/2), radius R = sqrt(a^2 + b^2 - F);
  pT = 0.3 B R [GeV, T, m]; charge q = +1 when the hits turn clockwise about the
  centre as rho grows (the sign of (x_far - x_near) x (c - x_near) is negative), else -1;
  phi0 = the direction of motion at the point of closest approach to the origin,
  atan2(b, a) + q pi / 2;
* longitudinal: s = 2 R asin(min(1, rho / 2R)) (transverse arc length from the
  origin), least-squares line z = z0 + s tan(lambda); eta = asinh(tan(lambda));
* chi2_xy = mean over hits of (|x - c| - R)^2 in mm^2;
* collinear or coincident transverse positions define no circle: all six
  parameters are NaN.

Returns, for candidates in ascending label order: label, n_hits and
params = (pT, phi0, eta, z0 [mm], q, chi2_xy).
"""
import numpy as np


def positions(x):
    x = np.asarray(x, np.float64)
    rho, phi, z = 1000.0 * x[:, 0], np.pi * x[:, 1], 1000.0 * x[:, 2]
    return rho * np.cos(phi), rho * np.sin(phi), z, rho


def fit_candidate(X, Y, Z, rho, b_field):
    A = np.stack([X, Y, np.ones_like(X)], axis=1)
    if np.linalg.matrix_rank(A) < 3:
        # collinear or coincident transverse positions: no circle is defined
        return np.full(6, np.nan)
    (D, E, F), *_ = np.linalg.lstsq(A, -(X * X + Y * Y), rcond=None)
    a, b = -D / 2.0, -E / 2.0
    R = np.sqrt(max(a * a + b * b - F, 0.0))
    pt = 0.3 * b_field * R / 1000.0
    near, far = np.argmin(rho), np.argmax(rho)
    cross = (X[far] - X[near]) * (b - Y[near]) - (Y[far] - Y[near]) * (a - X[near])
    q = 1.0 if cross < 0.0 else -1.0
    phi0 = np.arctan2(b, a) + q * np.pi / 2.0
    phi0 = (phi0 + np.pi) % (2.0 * np.pi) - np.pi
    s = 2.0 * R * np.arcsin(np.minimum(1.0, rho / (2.0 * R))) if R > 0 else rho
    Bm = np.stack([np.ones_like(s), s], axis=1)
    (z0, tl), *_ = np.linalg.lstsq(Bm, Z, rcond=None)
    chi2 = float(np.mean((np.hypot(X - a, Y - b) - R) ** 2))
    return np.array([pt, phi0, np.arcsinh(tl), z0, q, chi2])


def fit_candidates(x, labels, min_hits=3, b_field=2.0):
    labels = np.asarray(labels)
    X, Y, Z, rho = positions(x)
    vals, counts = np.unique(labels, return_counts=True)
    out_l, out_n, out_p = [], [], []
    for v, c in zip(vals, counts):
        if c < min_hits:
            continue
        idx = np.flatnonzero(labels == v)
        out_l.append(int(v))
        out_n.append(int(c))
        out_p.append(fit_candidate(X[idx], Y[idx], Z[idx], rho[idx], b_field))
    return (np.array(out_l, np.int64), np.array(out_n, np.int64),
            np.array(out_p, np.float64).reshape(-1, 6))

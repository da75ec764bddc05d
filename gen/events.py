"""Synthetic helical-track events: the stand-in for the paper's simulated ttbar
events at pile-up 200 (Section 2.2.2 describes spacepoints with three features
each; the paper's Fatras/Pythia sample is not available, so seeded helices of
the same form are generated instead).

Geometry: ten barrel layers, unbounded cylinders at radii rho_k = 30 + k*970/9 mm,
solenoid field B = 2 T along z.  A particle of transverse momentum pT [GeV] and
charge q moves on a circle of radius R = pT / (0.3 B) [m] through the origin in
the transverse plane, so at cylinder radius rho it has

    phi(rho) = phi0 - q * asin(rho / 2R)
    s(rho)   = 2R * asin(rho / 2R)            (transverse arc length)
    z(rho)   = z0 + s(rho) * sinh(eta)        (cot(theta) = sinh(eta))

Each collision shares a vertex z0 ~ N(0, 50 mm) and emits 50 particles with
pT ~ U[1, 10] GeV, eta ~ U[-2, 2], phi0 ~ U[-pi, pi), q = +-1.  The smallest
helix diameter (2R = 3.33 m at 1 GeV) exceeds the outer layer radius, so every
particle crosses all ten layers and leaves exactly one hit per layer.  Noise
hits, round(0.1 * track hits) of them, are uniform in layer, phi and
z in [-Z_k, Z_k] with Z_k = 1.05 * rho_k * sinh(2) + 150 mm, particle id 0.

Features per hit: (rho / 1000 mm, phi / pi, z / 1000 mm) as float32, the
generated hit order shuffled by the seed so that ids carry no track order.
This module holds no step of the tracking method itself.
"""
from dataclasses import dataclass

import numpy as np

from . import splitmix as sm

B_FIELD_T = 2.0
N_LAYERS = 10
PARTICLES_PER_COLLISION = 50
NOISE_FRACTION = 0.1
VERTEX_SIGMA_MM = 50.0
LAYER_RADII_MM = 30.0 + np.arange(N_LAYERS, dtype=np.float64) * (970.0 / 9.0)

# stream tags: one independent SplitMix64 stream per drawn quantity
_T_Z0, _T_PT, _T_ETA, _T_PHI, _T_Q = 1, 2, 3, 4, 5
_T_NLAY, _T_NPHI, _T_NZ, _T_SHUF = 11, 12, 13, 14


@dataclass
class Event:
    x: np.ndarray        # float32 [N, 3] = (rho/1000, phi/pi, z/1000)
    pid: np.ndarray      # int32 [N], 1-based particle id, 0 = noise
    layer: np.ndarray    # int8 [N]
    xyz_mm: np.ndarray   # float64 [N, 3], exact generated positions (for generator checks)
    truth: dict          # per-particle parameters, for generator checks

    @property
    def n(self):
        return self.x.shape[0]


def generate_event(seed, n_collisions=1, particles_per_collision=PARTICLES_PER_COLLISION,
                   noise_fraction=NOISE_FRACTION, sigma_mm=0.0):
    """One event of n_collisions overlaid collisions (pile-up mu = n_collisions)."""
    n_coll = int(n_collisions)
    n_part = n_coll * int(particles_per_collision)
    z0_coll = sm.normal(seed, _T_Z0, n_coll, 0.0, VERTEX_SIGMA_MM)
    pt = sm.uniform(seed, _T_PT, n_part, 1.0, 10.0)
    eta = sm.uniform(seed, _T_ETA, n_part, -2.0, 2.0)
    phi0 = sm.uniform(seed, _T_PHI, n_part, -np.pi, np.pi)
    q = np.where(sm.uniform(seed, _T_Q, n_part) < 0.5, -1.0, 1.0)
    z0 = np.repeat(z0_coll, int(particles_per_collision))

    radius_mm = pt / (0.3 * B_FIELD_T) * 1000.0                     # [P]
    rho = LAYER_RADII_MM[None, :]                                    # [1, L]
    a = np.arcsin(rho / (2.0 * radius_mm[:, None]))                  # [P, L]
    phi = phi0[:, None] - q[:, None] * a
    s = 2.0 * radius_mm[:, None] * a
    z = z0[:, None] + s * np.sinh(eta)[:, None]
    rho_t = np.broadcast_to(rho, phi.shape)
    if sigma_mm > 0.0:
        # optional Gaussian smearing of the transverse position and z
        dphi = sm.normal(seed, 21, phi.size).reshape(phi.shape) * sigma_mm / rho_t
        phi = phi + dphi
        z = z + sm.normal(seed, 22, z.size).reshape(z.shape) * sigma_mm
    pid_t = np.repeat(np.arange(1, n_part + 1, dtype=np.int32), N_LAYERS)
    lay_t = np.tile(np.arange(N_LAYERS, dtype=np.int8), n_part)

    n_track_hits = n_part * N_LAYERS
    n_noise = int(np.floor(noise_fraction * n_track_hits + 0.5))
    nl = np.minimum((sm.uniform(seed, _T_NLAY, n_noise) * N_LAYERS).astype(np.int64), N_LAYERS - 1)
    nrho = LAYER_RADII_MM[nl]
    nphi = sm.uniform(seed, _T_NPHI, n_noise, -np.pi, np.pi)
    zmax = 1.05 * nrho * np.sinh(2.0) + 150.0
    nz = -zmax + 2.0 * zmax * sm.uniform(seed, _T_NZ, n_noise)

    rho_all = np.concatenate([rho_t.reshape(-1), nrho])
    phi_all = np.concatenate([phi.reshape(-1), nphi])
    z_all = np.concatenate([z.reshape(-1), nz])
    pid_all = np.concatenate([pid_t, np.zeros(n_noise, np.int32)])
    lay_all = np.concatenate([lay_t, nl.astype(np.int8)])

    phi_w = np.mod(phi_all + np.pi, 2.0 * np.pi) - np.pi             # wrap to [-pi, pi)
    order = np.argsort(sm.bits(seed, _T_SHUF, rho_all.size), kind="stable")
    rho_all, phi_w, z_all = rho_all[order], phi_w[order], z_all[order]
    x = np.stack([rho_all / 1000.0, phi_w / np.pi, z_all / 1000.0], axis=1).astype(np.float32)
    xyz = np.stack([rho_all * np.cos(phi_w), rho_all * np.sin(phi_w), z_all], axis=1)
    truth = dict(pt=pt, eta=eta, phi0=phi0, q=q, z0=z0, radius_mm=radius_mm)
    return Event(x=x, pid=pid_all[order].astype(np.int32), layer=lay_all[order], xyz_mm=xyz, truth=truth)


def pack_events(events):
    """Concatenate events into one packed hit array with int64 offsets [B+1]."""
    offs = np.zeros(len(events) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([e.n for e in events])
    x = np.concatenate([e.x for e in events], axis=0) if events else np.zeros((0, 3), np.float32)
    return np.ascontiguousarray(x), offs

"""Equispaced orientation library and nearest-neighbour disorientations
(oracle; test only).

Section "SO(3) Spacing" and Figure 2: the library is an S^2 x S^1 sampling of
SO(3) reduced to the cubic fundamental zone; the sphere is split into
equidistant polar rings with as many azimuths on each ring as its
circumference needs, the circle linearly.  Its quality is measured by the
disorientation (Equation 6) from each library orientation to its nearest
neighbour in the library.

Readings (the paper delegates the construction to MTEX and states only the
split):

* spacing d (radians); m = max(1, round(pi / d)) polar intervals, rings at
  theta_i = pi i / m (i = 0 .. m); ring i carries n_i = max(1, round(2 m
  sin theta_i)) azimuths phi_j = 2 pi j / n_i; the circle carries
  n_psi = max(1, round(2 pi / d)) angles psi_k = 2 pi k / n_psi;
* the orientation of (theta, phi, psi) is Rz(phi) Ry(theta) Rz(psi - phi):
  the sphere point is where the rotation takes +z, and psi turns about that
  point with the azimuth taken out, so that the circle coordinate does not
  wind as phi goes round near the poles (these Euler angles cover SO(3)
  once);
* fundamental-zone reduction: keep an orientation q if no cubic equivalent
  s (x) q has a larger |w| (a smaller rotation angle) by more than
  eps = 1e-12; among equivalents tied with it within eps keep only the one
  whose canonical quaternion (w >= 0; at w = 0 the first non-zero component
  positive) is lexicographically smallest, components compared with the
  same eps;
* the nearest-neighbour disorientation of k is the smallest disorientation
  angle to any other library orientation, ties to the smallest index.
"""

import numpy as np

from . import rotations

EPS = 1e-12


def grid_counts(spacing_deg):
    """(m, ring azimuth counts n_i, n_psi) of the construction."""
    d = np.deg2rad(spacing_deg)
    m = max(1, int(np.round(np.pi / d)))
    theta = np.pi * np.arange(m + 1) / m
    n_ring = np.maximum(1, np.round(2 * m * np.sin(theta)).astype(np.int64))
    n_psi = max(1, int(np.round(2 * np.pi / d)))
    return m, n_ring, n_psi


def full_grid(spacing_deg):
    """Every grid orientation over SO(3) as matrices [N, 3, 3], ordered by
    (ring, azimuth, circle angle)."""
    m, n_ring, n_psi = grid_counts(spacing_deg)
    out = []
    for i in range(m + 1):
        theta = np.pi * i / m
        for j in range(n_ring[i]):
            phi = 2 * np.pi * j / n_ring[i]
            for k in range(n_psi):
                psi = 2 * np.pi * k / n_psi
                out.append(rotations.rot_z(phi) @ rotations.rot_y(theta) @ rotations.rot_z(psi - phi))
    return np.array(out)


def canonical(q):
    q = np.array(q, dtype=np.float64)
    if abs(q[0]) <= EPS:
        nz = np.nonzero(np.abs(q) > EPS)[0]
        if len(nz) and q[nz[0]] < 0:
            q = -q
    elif q[0] < 0:
        q = -q
    return q


def key_less_equal(a, b):
    """Lexicographic a <= b with components equal within EPS."""
    for x, y in zip(a, b):
        if abs(x - y) > EPS:
            return x < y
    return True


def in_fundamental_zone(r, ops):
    cand = [canonical(rotations.matrix_to_quat(s @ r)) for s in ops]
    w = np.array([abs(c[0]) for c in cand])
    best = w.max()
    if w[0] < best - EPS:
        return False
    return all(key_less_equal(cand[0], cand[i]) for i in range(1, len(ops)) if w[i] >= best - EPS)


def library(spacing_deg):
    """Fundamental-zone library, unit quaternions [L, 4] (w >= 0), in grid order.

    |w| of every equivalent comes from its trace, |w| = sqrt(1 + tr) / 2;
    the per-orientation rule above is applied where an equivalent ties."""
    ops = rotations.cubic_operators()
    rs = full_grid(spacing_deg)
    tr = np.einsum("sij,nji->ns", ops, rs)
    w = 0.5 * np.sqrt(np.clip(1.0 + tr, 0.0, None))
    best = w.max(axis=1)
    keep = w[:, 0] >= best - EPS
    tied = keep & np.any(w[:, 1:] >= best[:, None] - EPS, axis=1)
    for n in np.nonzero(tied)[0]:
        keep[n] = in_fundamental_zone(rs[n], ops)
    return np.array([canonical(q) for q in rotations.matrix_to_quat(rs[keep])])


def nn_disorientation(q):
    """(angle_deg [L], index [L]) of each orientation's nearest neighbour
    (Equation 6 disorientation, ties to the smallest index)."""
    r = rotations.quat_to_matrix(np.asarray(q, dtype=np.float64))
    n = len(r)
    ang = np.empty(n)
    idx = np.empty(n, dtype=np.int64)
    ops = rotations.cubic_operators()
    for a in range(n):
        d = rotations.disorientation(r[a][None], r, ops)
        d[a] = np.inf
        idx[a] = int(np.argmin(d))
        ang[a] = np.rad2deg(d[idx[a]])
    return ang, idx

"""Orientation sets (input generator).

Quaternions are (w, x, y, z), w >= 0, encoding the rotation matrix that maps
detector-frame directions to crystal directions.  Uniform SO(3) samples use
Shoemake's subgroup algorithm (Graphics Gems III, 1992).  Libraries are
reduced to the cubic fundamental zone by picking, among the 24 equivalents
q_S * q, the one with the largest |w| (smallest rotation angle).
"""

import numpy as np

_S = np.sqrt(0.5)


def _cubic_quats():
    q = [(1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1)]
    for i in range(1, 4):
        for s in (1, -1):
            v = [_S, 0, 0, 0]
            v[i] = s * _S
            q.append(tuple(v))
    for sx in (1, -1):
        for sy in (1, -1):
            for sz in (1, -1):
                q.append((0.5, 0.5 * sx, 0.5 * sy, 0.5 * sz))
    for a, b in ((1, 2), (1, 3), (2, 3)):
        for s in (1, -1):
            v = [0, 0, 0, 0]
            v[a] = _S
            v[b] = s * _S
            q.append(tuple(v))
    return np.array(q, dtype=np.float64)


CUBIC_Q = _cubic_quats()


def qmul(a, b):
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], axis=-1)


def canon(q):
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    return np.where(q[..., :1] < 0, -q, q)


def random_quats(rng, n):
    u1, u2, u3 = rng.random((3, n))
    a, b = np.sqrt(1 - u1), np.sqrt(u1)
    q = np.stack([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                  b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)], axis=-1)
    return canon(q)


def fz_reduce(q):
    q = np.asarray(q, dtype=np.float64)
    eq = qmul(CUBIC_Q[None, :, :], q[:, None, :])          # [n, 24, 4]
    k = np.argmax(np.abs(eq[..., 0]), axis=1)
    return canon(eq[np.arange(q.shape[0]), k])


def random_fz_quats(rng, n):
    return fz_reduce(random_quats(rng, n))


def axis_angle_quat(axis, angle):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis, axis=-1, keepdims=True)
    half = 0.5 * np.asarray(angle, dtype=np.float64)[..., None]
    return np.concatenate([np.cos(half), np.sin(half) * axis], axis=-1)


def perturb_quats(rng, q, max_deg):
    """q * dq with dq a rotation about a uniform random axis by U[0, max_deg]."""
    n = q.shape[0]
    ax = rng.normal(size=(n, 3))
    ang = np.deg2rad(rng.uniform(0.0, max_deg, n))
    return canon(qmul(q, axis_angle_quat(ax, ang)))


def voronoi_map(rng, rows, cols, n_grains):
    """Grain id per map point from n_grains uniform seeds (nearest seed)."""
    seeds = rng.uniform([0, 0], [rows, cols], size=(n_grains, 2))
    yy, xx = np.mgrid[0:rows, 0:cols]
    d2 = (yy[..., None] - seeds[:, 0]) ** 2 + (xx[..., None] - seeds[:, 1]) ** 2
    return np.argmin(d2, axis=-1).ravel()

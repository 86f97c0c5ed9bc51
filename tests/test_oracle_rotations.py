"""Pins for oracle.rotations (the disorientation equation of section
"SO(3) Spacing" with the 24 proper cubic operators)."""

import os

import numpy as np
import pytest

from oracle import rotations as rot

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = {}
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        k, v, tol = line.split()
        rows[k] = (float(v), float(tol))
    return rows


def _random_matrices(rng, n):
    q = rng.normal(size=(n, 4))
    return rot.quat_to_matrix(rot.quat_normalise(q))


def test_quat_matrix_roundtrip():
    rng = np.random.default_rng(0)
    q = rot.quat_normalise(rng.normal(size=(200, 4)))
    r = rot.quat_to_matrix(q)
    assert np.allclose(r @ np.swapaxes(r, 1, 2), np.eye(3), atol=1e-14)
    assert np.allclose(np.linalg.det(r), 1.0, atol=1e-14)
    assert np.allclose(rot.matrix_to_quat(r), q, atol=1e-14)


def test_quat_matches_axis_angle():
    # q = (cos t/2, n sin t/2) must be the active rotation by t about n
    for axis, ang in (([0, 0, 1], 0.3), ([1, 2, -1], 1.1), ([0, 1, 0], -2.0)):
        n = np.array(axis, float) / np.linalg.norm(axis)
        q = np.concatenate([[np.cos(ang / 2)], np.sin(ang / 2) * n])
        assert np.allclose(rot.quat_to_matrix(rot.quat_normalise(q)), rot.axis_angle_matrix(n, ang), atol=1e-14)
    # rot_z(90 deg) takes +x to +y (right-handed, active)
    assert np.allclose(rot.rot_z(np.pi / 2) @ [1, 0, 0], [0, 1, 0], atol=1e-15)
    assert np.allclose(rot.rot_x(np.pi / 2) @ [0, 1, 0], [0, 0, 1], atol=1e-15)
    assert np.allclose(rot.rot_y(np.pi / 2) @ [0, 0, 1], [1, 0, 0], atol=1e-15)


def test_cubic_group():
    ops = rot.cubic_operators()
    assert ops.shape == (24, 3, 3)
    # integer signed-permutation matrices with det +1: exactly the 24 proper ones
    assert np.allclose(ops, np.round(ops), atol=1e-12)
    assert np.allclose(np.linalg.det(ops), 1.0)
    keys = {tuple(np.round(o).astype(int).ravel()) for o in ops}
    assert len(keys) == 24
    # closed under products
    for a in ops:
        for b in ops:
            assert tuple(np.round(a @ b).astype(int).ravel()) in keys


def test_disorientation_special_values():
    eye = np.eye(3)
    ops = rot.cubic_operators()
    rng = np.random.default_rng(1)
    r = _random_matrices(rng, 5)
    for s in ops:                                       # symmetric equivalents coincide
        assert np.all(rot.disorientation(r, s @ r) < 1e-7)
    d = lambda axis, deg: np.rad2deg(rot.disorientation(eye, rot.axis_angle_matrix(axis, np.deg2rad(deg))))
    assert abs(d([1, 1, 1], 60.0) - 60.0) < 1e-9         # sigma-3 twin
    assert abs(d([0, 0, 1], 45.0) - 45.0) < 1e-9
    assert abs(d([0, 0, 1], 50.0) - 40.0) < 1e-9         # 90 deg operator folds it back
    assert abs(d([1, 1, 1], 120.0)) < 1e-5               # acos near 1: ~1e-8 rad of rounding
    assert abs(d([1, 1, 0], 180.0)) < 1e-5


def test_disorientation_mackenzie():
    g = _golden("disorientation_cubic.txt")
    rng = np.random.default_rng(2)
    a = _random_matrices(rng, 20000)
    b = _random_matrices(rng, 20000)
    w = np.rad2deg(rot.disorientation(a, b))
    assert w.max() <= g["max_deg"][0] + g["max_deg"][1]
    assert w.max() > 58.0
    assert abs(w.mean() - g["mean_deg"][0]) < g["mean_deg"][1]
    # symmetric in its arguments
    assert np.allclose(w[:200], np.rad2deg(rot.disorientation(b[:200], a[:200])), atol=1e-9)


def test_fz_representative_is_minimal():
    rng = np.random.default_rng(3)
    ops = rot.cubic_operators()
    for r in _random_matrices(rng, 50):
        f = rot.fz_representative(r)
        angles = rot.rotation_angle(ops @ r)
        assert abs(rot.rotation_angle(f) - angles.min()) < 1e-12
        assert rot.disorientation(f, r) < 1e-7
        assert rot.rotation_angle(f) <= np.deg2rad(62.81)

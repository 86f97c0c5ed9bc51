"""Pins for oracle.geometry (gnomonic projection with bicubic interpolation,
section "SO(3) Library Generation"; pattern-centre units, footnote 2)."""

import os

import numpy as np

from fixtures import band_intensity, band_master
from oracle import geometry as geo
from oracle import rotations as rot

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_pc_crop_worked_example():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "pc_crop.txt")) if l.strip() and not l.startswith("#")]
    for w, w2, before, after, tol in rows:
        got = geo.crop_pc(float(before), int(w), int(w2))
        assert abs(got - float(after)) <= float(tol)
        assert abs(got - 0.34375) < 1e-15


def test_keys_weights_partition_and_quadratics():
    t = np.linspace(0, 0.999, 37)
    w = geo.keys_weights(t)
    assert np.allclose(w.sum(-1), 1.0, atol=1e-15)
    # Keys (a = -0.5) reproduces polynomials up to degree 2 exactly
    for f in (lambda x: 3 + 0 * x, lambda x: 2 * x - 1, lambda x: x * x - 0.3 * x + 2):
        taps = np.stack([f(-1 - 0 * t), f(0 * t), f(1 + 0 * t), f(2 + 0 * t)], -1)
        assert np.allclose((w * taps).sum(-1), f(t), atol=1e-13)
    assert np.allclose(geo.keys_weights(np.array([0.0])), [[0, 1, 0, 0]])


def _direction(theta, phi):
    return np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])


def test_master_lookup_hits_nodes_and_wraps():
    rng = np.random.default_rng(0)
    m = rng.random((32, 48))
    h, w = m.shape
    for r, q in ((5, 0), (10, 47), (20, 13), (1, 1)):
        c = _direction((r + 0.5) * np.pi / h, 2 * np.pi * q / w)
        assert abs(geo.master_lookup(m, c[None])[0] - m[r, q]) < 1e-12
    # azimuth is periodic: phi and phi + 2 pi and the branch cut agree
    c1 = _direction(1.0, -1e-9)
    c2 = _direction(1.0, 1e-9)
    assert abs(geo.master_lookup(m, c1[None])[0] - geo.master_lookup(m, c2[None])[0]) < 1e-6


def test_master_lookup_reproduces_quadratic_in_grid_coordinates():
    h, w = 64, 64
    rr, qq = np.mgrid[0:h, 0:w].astype(float)
    m = 0.01 * rr ** 2 - 0.2 * rr + 3.0 + 0.0 * qq      # quadratic in row, constant in column
    rng = np.random.default_rng(1)
    v = rng.uniform(3, h - 4, 50)
    u = rng.uniform(0, w, 50)
    c = np.stack([_direction((vv + 0.5) * np.pi / h, uu * 2 * np.pi / w) for vv, uu in zip(v, u)])
    assert np.allclose(geo.master_lookup(m, c), 0.01 * v ** 2 - 0.2 * v + 3.0, atol=1e-9)


def test_gnomonic_angles():
    # the ray through a pixel at distance r px from the pattern centre makes
    # an angle atan(r / (PCz N)) with the screen normal (gnomonic projection)
    n, pc = 64, (0.3, 0.45, 0.7)
    d = geo.pixel_rays(n, pc)
    jj, ii = np.mgrid[0:n, 0:n]
    r = np.hypot(ii + 0.5 - pc[0] * n, jj + 0.5 - pc[1] * n)
    assert np.allclose(np.arccos(d[..., 2]), np.arctan(r / (pc[2] * n)), atol=1e-12)
    # azimuth about the PC: +x toward +row
    az = np.arctan2(d[..., 1], d[..., 0])
    assert np.allclose(np.exp(1j * az), np.exp(1j * np.arctan2(jj + 0.5 - pc[1] * n, ii + 0.5 - pc[0] * n)), atol=1e-12)


def test_great_circles_map_to_lines():
    # a crystal plane n projects onto the screen line {x : (R^T n) . ray(x) = 0}:
    # the sign change of c . n between neighbouring pixels happens along a line
    rng = np.random.default_rng(2)
    r = rot.quat_to_matrix(rot.quat_normalise(rng.normal(size=4)))
    n, pc = 128, (0.5, 0.5, 0.6)
    c = geo.crystal_directions(r, n, pc)
    normal = np.array([1.0, 1.0, 1.0]) / np.sqrt(3)
    f = c @ normal
    # unnormalised ray components are affine in (i, j); so is f * |ray|
    jj, ii = np.mgrid[0:n, 0:n]
    ray = np.stack([(ii + 0.5) / n - pc[0], (jj + 0.5) / n - pc[1], np.full((n, n), pc[2])], -1)
    g = f * np.linalg.norm(ray, axis=-1)
    a = np.stack([ii.ravel(), jj.ravel(), np.ones(n * n)], 1)
    coef, res, *_ = np.linalg.lstsq(a, g.ravel(), rcond=None)
    assert np.max(np.abs(a @ coef - g.ravel())) < 1e-12


def test_pc_offset_is_translation():
    # shifting PC by an integer (dx, dy) px translates the template by (dx, dy)
    m = band_master()
    rng = np.random.default_rng(3)
    r = rot.quat_to_matrix(rot.quat_normalise(rng.normal(size=4)))
    n = 64
    base = geo.project(m, r, n, (0.5, 0.5, 0.6))
    for dx, dy in ((3, -2), (-1, 4)):
        moved = geo.project(m, r, n, (0.5 + dx / n, 0.5 + dy / n, 0.6))
        sl_new = (slice(max(dy, 0), n + min(dy, 0)), slice(max(dx, 0), n + min(dx, 0)))
        sl_old = (slice(max(-dy, 0), n + min(-dy, 0)), slice(max(-dx, 0), n + min(-dx, 0)))
        assert np.allclose(moved[sl_new], base[sl_old], atol=1e-12)


def test_symmetry_invariance_analytic_and_grid():
    # T(S R) = T(R) for every cubic operator: exact with the analytic master,
    # within interpolation error with the 256 x 256 grid
    rng = np.random.default_rng(4)
    r = rot.quat_to_matrix(rot.quat_normalise(rng.normal(size=4)))
    n, pc = 48, (0.5, 0.5, 0.6)
    m = band_master()
    t0 = geo.project_fn(band_intensity, r, n, pc)
    g0 = geo.project(m, r, n, pc)
    assert np.max(np.abs(g0 - t0)) < 0.05 * np.ptp(t0)
    for s in rot.cubic_operators():
        assert np.allclose(geo.project_fn(band_intensity, s @ r, n, pc), t0, atol=1e-12)
        assert np.max(np.abs(geo.project(m, s @ r, n, pc) - g0)) < 0.05 * np.ptp(t0)


def test_rotation_about_screen_normal_rotates_image():
    # with the PC at the screen centre, a crystal rotated by Rz(90 deg) in the
    # detector frame (orientation R Rz^T) gives the template rotated by +90
    # deg in eta = atan2(row - c, col - c)
    rng = np.random.default_rng(5)
    r = rot.quat_to_matrix(rot.quat_normalise(rng.normal(size=4)))
    n, pc = 32, (0.5, 0.5, 0.6)
    t = geo.project_fn(band_intensity, r, n, pc)
    t_rot = geo.project_fn(band_intensity, r @ rot.rot_z(np.pi / 2).T, n, pc)
    # feature at (col, row) offsets (a, b) moves to (-b, a)
    jj, ii = np.mgrid[0:n, 0:n]
    c = (n - 1) / 2
    a, b = ii - c, jj - c
    src_col = (c + b).astype(int)          # inverse map: new (a', b') = (-b, a) -> old (b', -a')
    src_row = (c - a).astype(int)
    assert np.allclose(t_rot, t[src_row, src_col], atol=1e-12)

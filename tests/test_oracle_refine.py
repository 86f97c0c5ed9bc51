"""Pins for oracle.refine (section "Orientation and Pattern Centre
Refinement": Equation 7 for x/y, the log-polar transform for z, iteration)."""

import numpy as np
import pytest

from fixtures import band_intensity, band_master, random_quats, simulate_patterns
from oracle import geometry as geo
from oracle import refine, spectra
from oracle import rotations as rot
from oracle.params import Params


def test_logpolar_samples_affine_images_exactly():
    n = 64
    jj, ii = np.mgrid[0:n, 0:n].astype(float)
    img = 0.3 * ii - 1.7 * jj + 5.0
    lp = refine.logpolar(img, 32, 128)
    r = refine.logpolar_radii(n, 32)
    eta = 2 * np.pi * np.arange(128) / 128
    c = (n - 1) / 2
    want = 0.3 * (c + r[:, None] * np.cos(eta)) - 1.7 * (c + r[:, None] * np.sin(eta)) + 5.0
    assert np.allclose(lp, want, atol=1e-12)
    assert abs(r[0] - 2.0) < 1e-15 and abs(r[-1] - (n / 2 - 2)) < 1e-12
    assert np.allclose(np.diff(np.log(r)), np.log(r[1] / r[0]))


def test_eta_correlation_recovers_cyclic_shift():
    rng = np.random.default_rng(0)
    lt = rng.normal(size=(16, 64))
    for d0 in (0, 5, 63, 32):
        le = np.roll(lt, d0, axis=1)              # Le[m] = Lt[m - d0]
        c = refine.eta_correlation(le, lt)
        assert int(np.argmax(c)) == d0
        assert abs(c[d0] - 1.0) < 1e-12


def test_eta_peak_trigonometric_interpolation():
    # a band-limited periodic sequence peaked at a fractional t0 is located
    # to 0.5 / kappa samples
    n = 64
    m = np.arange(n)
    for t0 in (3.27, -10.5, 0.004):
        c = np.cos(2 * np.pi * (m - t0) / n) + 0.3 * np.cos(4 * np.pi * (m - t0) / n)
        val, t = refine.eta_peak(c, kappa=100)
        assert abs(t - t0) <= 0.005 + 1e-12
        assert abs(val - 1.3) < 1e-6


def _pattern(q, n, pc):
    return simulate_patterns(q[None], n, np.array([pc]), ("none",)).numpy()[0].astype(np.float64)


@pytest.mark.parametrize("axis,deg", [("x", 0.5), ("x", -2.0), ("y", 2.0), ("y", -0.5)])
def test_xy_step_sign_and_magnitude(axis, deg):
    # crystal rotated by Q about detector x or y: one x/y step from the
    # unrotated orientation recovers the angle with the right sign, and the
    # error is second order in the angle
    rng = np.random.default_rng(1)
    master = band_master()
    n, pc = 128, (0.5, 0.5, 0.6)
    r0 = rot.quat_to_matrix(random_quats(rng, 1)[0])
    q = rot.rot_x(np.deg2rad(deg)) if axis == "x" else rot.rot_y(np.deg2rad(deg))
    rt = r0 @ q.T
    pat = _pattern(rot.matrix_to_quat(rt), n, pc)
    t = geo.project(master, r0, n, pc)
    _, s = refine.measure_shift(pat, t, Params())
    dd = pc[2] * n
    if axis == "y":
        assert np.sign(s[1]) == np.sign(deg) and abs(s[1] - dd * np.tan(np.deg2rad(deg))) < 0.1 + 0.05 * abs(deg)
    else:
        assert np.sign(s[0]) == -np.sign(deg) and abs(-s[0] - dd * np.tan(np.deg2rad(deg))) < 0.1 + 0.05 * abs(deg)
    r1 = refine.xy_update(r0, s, pc[2], n)
    before = rot.misorientation_angle(r0, rt)
    after = rot.misorientation_angle(r1, rt)
    assert after < 0.15 * before + np.deg2rad(0.02)


def test_z_step_exact_quarter_turn():
    # PC at the screen centre: Rz(90 deg) is an exact pixel rotation, a
    # shift of N_eta / 4 samples, so gamma = 90 deg to rounding
    rng = np.random.default_rng(2)
    n, pc = 64, (0.5, 0.5, 0.6)
    r0 = rot.quat_to_matrix(random_quats(rng, 1)[0])
    t = geo.project_fn(band_intensity, r0, n, pc)
    pat = geo.project_fn(band_intensity, r0 @ rot.rot_z(np.pi / 2).T, n, pc)
    g = refine.measure_gamma(pat, t, Params())
    assert abs(g - np.pi / 2) < 1e-9


@pytest.mark.parametrize("deg", [2.0, -1.3])
def test_z_step_small_rotation(deg):
    rng = np.random.default_rng(3)
    master = band_master()
    n, pc = 128, (0.5, 0.5, 0.6)
    r0 = rot.quat_to_matrix(random_quats(rng, 1)[0])
    rt = r0 @ rot.rot_z(np.deg2rad(deg)).T
    pat = _pattern(rot.matrix_to_quat(rt), n, pc)
    g = refine.measure_gamma(pat, geo.project(master, r0, n, pc), Params())
    assert abs(np.rad2deg(g) - deg) < 0.03


def test_refinement_converges_noise_free():
    # Figure 7 analogue without noise: start a few degrees away, two
    # iterations land well inside 0.1 deg
    rng = np.random.default_rng(4)
    master = band_master()
    n = 128
    for k in range(3):
        qt = random_quats(rng, 1)[0]
        pc = (0.5 + rng.uniform(-4, 4) / n, 0.5 + rng.uniform(-4, 4) / n, 0.6)
        axis = rng.normal(size=3)
        r_true = rot.quat_to_matrix(qt)
        r0 = r_true @ rot.axis_angle_matrix(axis, np.deg2rad(3.0))
        pat = _pattern(qt, n, pc)
        r, h, s = refine.refine_one(pat, master, r0, pc, Params())
        assert np.rad2deg(rot.disorientation(r, r_true)) < 0.05
        assert h > 0.99

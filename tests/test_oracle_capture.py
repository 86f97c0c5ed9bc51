"""Pins for oracle.capture (section "SO(3) Sampling Frequency", Figures 3
and 4: correlation against detector-frame rotations and its width)."""

import numpy as np
import pytest

from fixtures import band_master, random_quats
from oracle import capture
from oracle import rotations as rot
from oracle.params import Params

T = np.arange(-30.0, 30.0 + 1e-9, 0.5)


@pytest.mark.parametrize("wl,wr", [(4.0, 4.0), (3.3, 7.9), (10.2, 0.8)])
def test_fwhm_of_a_triangle_is_exact(wl, wr):
    # piecewise-linear curve: linear interpolation of the crossing is exact
    h = np.where(T < 0, np.maximum(0.0, 1 + T / wl), np.maximum(0.0, 1 - T / wr))
    assert abs(capture.fwhm(T, h) - 0.5 * (wl + wr)) < 1e-12


def test_fwhm_of_a_gaussian_on_a_floor():
    # level halfway between the peak (1.0) and the floor (0.2): the textbook
    # width 2 sqrt(2 ln 2) sigma of the Gaussian above its baseline
    sigma = 3.0
    h = 0.2 + 0.8 * np.exp(-T ** 2 / (2 * sigma ** 2))
    assert abs(capture.fwhm(T, h) - 2 * sigma * np.sqrt(2 * np.log(2))) < 0.02


def test_fwhm_off_centre_peak_and_open_side():
    h = np.exp(-(T - 7.0) ** 2 / 8.0)
    assert abs(capture.fwhm(T, h) - 2 * 2.0 * np.sqrt(2 * np.log(2))) < 0.02
    # never below half on the right: the width runs to the sampled end
    h2 = np.where(T < 0, np.exp(-T ** 2 / 8.0), 1.0)
    assert h2.min() < 1e-40
    assert abs(capture.fwhm(T, h2) - (30.0 + 2.0 * np.sqrt(2 * np.log(2)))) < 0.02


def test_rotated_orientations_compose_in_the_detector_frame():
    rng = np.random.default_rng(3)
    r = rot.quat_to_matrix(random_quats(rng, 1)[0])
    rs = capture.rotated_orientations(r, "z", [0.0, 90.0])
    assert np.allclose(rs[0], r, atol=1e-15)
    # R Rz^T: crystal direction of the detector direction d is R Rz^T d
    d = np.array([1.0, 0.0, 0.0])
    assert np.allclose(rs[1] @ d, r @ np.array([0.0, -1.0, 0.0]), atol=1e-12)


def test_capture_curve_peaks_at_zero_with_unit_height():
    rng = np.random.default_rng(4)
    master = band_master()
    r = rot.quat_to_matrix(random_quats(rng, 1)[0])
    th = [-6.0, -2.0, 0.0, 2.0, 6.0]
    for axis in ("x", "y", "z"):
        h = capture.capture_curve(master, r, axis, th, 64, (0.5, 0.3, 0.6), (0.5, 0.3, 0.6), Params())
        assert abs(h[2] - 1.0) < 1e-12
        assert np.all(h[[0, 1, 3, 4]] < h[2]) and np.all(h <= 1.0 + 1e-12)
        assert h[1] > h[0] and h[3] > h[4]

"""Parity of ebsd_capture_range (section "SO(3) Sampling Frequency",
Figures 3 and 4) against the FP64 oracle: the integer-peak capture curves to
1e-4 (the peak-height tolerance of the FP32 path) and their FWHM to 0.02 deg
(a 1e-4 height difference moves a crossing on a slope of >= 0.01 per degree
by <= 0.01 deg)."""

import numpy as np
import pytest

import oracle
from fixtures import random_quats
from fixtures import band_master
from oracle import capture
from oracle import rotations as rot

from .gpu_util import banner, dev, host, tm

pytestmark = pytest.mark.gpu

PC = (0.5, 0.3, 0.6)


@pytest.mark.parametrize("n,pc_test", [(64, PC), (128, PC), (128, (0.52, 0.3, 0.6)), (96, (0.5, 0.3, 0.63))])
def test_capture_range_matches_oracle(n, pc_test):
    banner("capture_range n=%d pc_test=%s" % (n, pc_test))
    t = tm()
    rng = np.random.default_rng(40 + n)
    q_ref = random_quats(rng, 2)
    th = np.arange(-10.0, 10.0 + 1e-9, 1.0)
    master = band_master()
    h, w = t.capture_range(dev(master), dev(q_ref), n, PC, pc_test, dev(th))
    h, w = host(h), host(w)
    assert h.shape == (2, 3, len(th)) and w.shape == (2, 3)
    for r in range(2):
        for a, axis in enumerate("xyz"):
            ref = capture.capture_curve(master, rot.quat_to_matrix(q_ref[r]), axis, th, n, PC, pc_test,
                                        oracle.Params())
            assert np.max(np.abs(h[r, a] - ref)) < 1e-4, (r, axis)
            assert abs(w[r, a] - capture.fwhm(th, ref)) < 0.02, (r, axis, w[r, a], capture.fwhm(th, ref))


def test_capture_range_single_angle_and_empty():
    t = tm()
    rng = np.random.default_rng(7)
    q_ref = random_quats(rng, 1)
    master = band_master()
    h, w = t.capture_range(dev(master), dev(q_ref), 64, PC, PC, dev(np.array([0.0])))
    assert np.allclose(host(h), 1.0, atol=1e-5) and np.all(host(w) == 0.0)
    h0, w0 = t.capture_range(dev(master), dev(np.zeros((0, 4))), 64, PC, PC, dev(np.array([0.0, 1.0])))
    assert h0.shape == (0, 3, 2) and w0.shape == (0, 3)

"""Parity of ebsd_so3_library and ebsd_nn_disorientation (section "SO(3)
Spacing", Equation 6, Figure 2) against the FP64 oracle.

Library: the same orientations in the same order (the fundamental-zone
decisions are integer decisions taken in FP64 on both sides with the same
1e-12 tie band), quaternions to 1e-12.  Nearest neighbours: angles to 1e-9
deg; where several neighbours tie, the GPU's index must be one of them
(its oracle disorientation equals the minimum to 1e-9 deg)."""

import numpy as np
import pytest

from fixtures import random_quats
from oracle import rotations as rot
from oracle import so3grid

from .gpu_util import banner, dev, host, tm

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("spacing", [20.0, 15.0, 10.0, 7.5, 5.0])
def test_library_matches_oracle(spacing):
    banner("so3_library %.1f deg" % spacing)
    t = tm()
    got = host(t.so3_library(spacing))
    want = so3grid.library(spacing)
    assert got.shape == want.shape, (got.shape, want.shape)
    assert np.max(np.abs(got - want)) < 1e-12


def test_library_cap_and_query():
    import ctypes
    import torch
    t = tm()
    n = ctypes.c_int64(0)
    assert t.lib().ebsd_so3_library(10.0, None, 0, ctypes.byref(n), None) == 0
    assert n.value == len(so3grid.library(10.0))
    out = torch.full((100, 4), -9.0, dtype=torch.float64, device="cuda:0")
    m = ctypes.c_int64(0)
    assert t.lib().ebsd_so3_library(10.0, ctypes.c_void_p(out.data_ptr()), 50, ctypes.byref(m), None) == 0
    o = host(out)
    assert m.value == n.value
    assert np.max(np.abs(o[:50] - so3grid.library(10.0)[:50])) < 1e-12 and np.all(o[50:] == -9.0)


def _check_nn(q):
    t = tm()
    ang, idx = t.nn_disorientation(dev(q))
    ang, idx = host(ang), host(idx)
    want, _ = so3grid.nn_disorientation(q)
    assert np.max(np.abs(ang - want)) < 1e-9
    r = rot.quat_to_matrix(q)
    assert np.all(idx != np.arange(len(q))) and np.all((idx >= 0) & (idx < len(q)))
    via = np.rad2deg(rot.disorientation(r, r[idx]))
    assert np.max(np.abs(via - want)) < 1e-9


def test_nn_disorientation_on_the_10_deg_library():
    banner("nn_disorientation, 10 deg library")
    _check_nn(so3grid.library(10.0))


@pytest.mark.parametrize("n", [2, 257, 700])
def test_nn_disorientation_random_sets(n):
    banner("nn_disorientation, %d random orientations" % n)
    _check_nn(random_quats(np.random.default_rng(n), n))

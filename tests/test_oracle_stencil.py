"""Pins for oracle.stencil (the 27-point grid of small detector-frame
rotations around a starting orientation, one pass, best by integer peak)."""

import numpy as np
import pytest

from fixtures import band_master, random_quats
from oracle import geometry as geo
from oracle import rotations as rot
from oracle import stencil
from oracle.params import Params

STEP = np.deg2rad(stencil.STEP_DEG)


def test_offsets_are_lexicographic_and_centred():
    off = stencil.stencil_offsets(STEP)
    assert off.shape == (27, 3)
    assert [tuple(o) for o in off] == sorted(tuple(o) for o in off)
    assert np.all(off[13] == 0.0)
    assert set(np.unique(off)) == {-STEP, 0.0, STEP}


def test_single_axis_candidates_rotate_about_detector_axes():
    r0 = rot.quat_to_matrix(random_quats(np.random.default_rng(1), 1)[0])
    cands = stencil.stencil_candidates(r0, STEP)
    assert np.array_equal(cands[13], r0)
    axes = {(2, 1, 1): (0, np.array([1.0, 0, 0])), (1, 2, 1): (1, np.array([0, 1.0, 0])),
            (1, 1, 2): (2, np.array([0, 0, 1.0]))}
    for (ia, ib, ic), (_, e) in axes.items():
        q = r0.T @ cands[9 * ia + 3 * ib + ic]          # = Q^T
        assert abs(np.rad2deg(rot.rotation_angle(q)) - stencil.STEP_DEG) < 1e-9
        assert np.allclose(q @ e, e, atol=1e-15)        # the axis is fixed


def test_rz_candidate_is_an_image_rotation_about_the_centre():
    # with the pattern centre at the screen centre, R Rz(c)^T is the pattern
    # of R turned by c about the screen centre: compare a ray-by-ray lookup
    n = 64
    pc = (0.5, 0.5, 0.6)
    r0 = rot.quat_to_matrix(random_quats(np.random.default_rng(2), 1)[0])
    c = np.deg2rad(10.0)
    rc = r0 @ rot.rot_z(c).T
    d0 = geo.pixel_rays(n, pc).reshape(-1, 3)
    # the ray that Rz(c)^T maps onto d sees, under r0, what d sees under rc
    assert np.allclose((rc @ d0.T).T, (r0 @ (rot.rot_z(c).T @ d0.T)).T, atol=1e-14)
    # and Rz(c)^T turns a detector ray about the normal by -c
    d1 = (rot.rot_z(c).T @ d0.T).T
    ang = np.arctan2(d1[:, 1], d1[:, 0]) - np.arctan2(d0[:, 1], d0[:, 0])
    ang = (ang + np.pi) % (2 * np.pi) - np.pi
    mask = np.hypot(d0[:, 0], d0[:, 1]) > 1e-6
    assert np.allclose(ang[mask], -c, atol=1e-12)


@pytest.mark.parametrize("target", [(2, 1, 1), (0, 1, 1), (1, 2, 1), (1, 0, 1), (1, 1, 2), (1, 1, 0),
                                    (2, 0, 2), (1, 1, 1)])
def test_stencil_finds_the_rotation_that_made_the_pattern(target):
    # noise-free pattern made at R0 Q(a, b, c)^T: the stencil from R0 must pick
    # exactly that candidate with h_int = 1 (identical images); a transposed Q
    # or a flipped axis would pick the mirrored candidate
    n = 64
    pc = (0.5, 0.5, 0.6)
    master = band_master()
    q0 = random_quats(np.random.default_rng(3), 1)
    r0 = rot.quat_to_matrix(q0[0])
    a, b, c = stencil.stencil_offsets(STEP)[9 * target[0] + 3 * target[1] + target[2]]
    rt = r0 @ stencil.stencil_rotation(a, b, c).T
    pat = geo.project(master, rt, n, pc)
    res = stencil.stencil_refine([pat], master, np.array([pc]), q0, Params(max_shift=4))
    want = 9 * target[0] + 3 * target[1] + target[2]
    assert res["idx"][0] == want
    assert abs(res["h_int"][0][want] - 1.0) < 1e-12
    assert np.all(np.delete(res["h_int"][0], want) < 1.0 - 1e-9)
    assert np.allclose(rot.quat_to_matrix(res["q"][0]), rt, atol=1e-12)
    assert abs(res["peak_h"][0] - 1.0) < 1e-9 and np.allclose(res["shift"][0], 0.0, atol=0.01)


def test_stencil_accepts_ragged_sizes():
    master = band_master()
    q0 = random_quats(np.random.default_rng(4), 2)
    rs = rot.quat_to_matrix(q0)
    pcs = np.array([(0.5, 0.5, 0.6), (0.5, 0.5, 0.6)])
    pats = [geo.project(master, rs[0] @ stencil.stencil_rotation(STEP, 0, 0).T, 64, pcs[0]),
            geo.project(master, rs[1] @ stencil.stencil_rotation(0, 0, -STEP).T, 96, pcs[1])]
    res = stencil.stencil_refine(pats, master, pcs, q0, Params())
    assert list(res["idx"]) == [9 * 2 + 3 + 1, 9 + 3 + 0]


def test_stencil_then_refine_fixed_point_and_convergence():
    # The pattern is the gridded master's projection at (R_true, PC_i).
    # Started at R_true Rx(0.5 deg)^T, the stencil's candidate (a = -0.5 deg)
    # is R_true itself (Rx(-a) Rx(a) = I): identical images, shift exactly 0,
    # and the refinement cannot move it.  Started 1.4 deg away about a random
    # axis, the stencil then the refinement land within 0.02 deg.  A first
    # step that used the shift with the wrong axis order or sign would move
    # the fixed point or stall the convergence.
    master = band_master()
    rng = np.random.default_rng(17)
    n = 96
    q_true = random_quats(rng, 2)
    pcs = np.array([[0.5 + 2 / n, 0.5 - 3 / n, 0.6], [0.5 - 1 / n, 0.5 + 4 / n, 0.62]])
    pats = [geo.project(master, rot.quat_to_matrix(q_true[i]), n, pcs[i]) for i in range(2)]
    r_true = rot.quat_to_matrix(q_true)
    q0 = np.stack([rot.matrix_to_quat(r_true[i] @ rot.rot_x(STEP).T) for i in range(2)])
    out = stencil.stencil_then_refine(pats, master, pcs, q0, Params())
    for i in range(2):
        assert out["stencil"]["idx"][i] == 4                      # (a, b, c) = (-d, 0, 0)
        assert np.rad2deg(rot.disorientation_q(out["q"][i], q_true[i])) < 1e-9
        assert abs(out["peak_h"][i] - 1) < 1e-12 and np.allclose(out["shift"][i], 0, atol=1e-12)
    q1 = np.stack([rot.matrix_to_quat(r_true[i] @ rot.axis_angle_matrix(rng.normal(size=3), np.deg2rad(1.4)))
                   for i in range(2)])
    out = stencil.stencil_then_refine(pats, master, pcs, q1, Params())
    for i in range(2):
        d_st = np.rad2deg(rot.disorientation_q(out["stencil"]["q"][i], q_true[i]))
        d = np.rad2deg(rot.disorientation_q(out["q"][i], q_true[i]))
        assert d < 0.02 and d < d_st
        assert out["peak_h"][i] > 0.99

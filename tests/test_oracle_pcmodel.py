"""Pins for oracle.pcmodel and the beam-shift-corrected refinement (section
"Orientation and Pattern Centre Refinement", Figure 6 B: one library at one
PC, the search's shift corrected for the PC move; silicon-map
demonstrations: the PC drifts across the map)."""

import numpy as np
import pytest

from fixtures import band_master, random_quats, simulate_patterns
from oracle import geometry as geo
from oracle import pcmodel, refine
from oracle import rotations as rot
from oracle.params import Params

N = 128
PC0 = (0.5, 0.5, 0.6)


def _pattern(q, pc):
    return simulate_patterns(q[None], N, np.array([pc]), ("none",)).numpy()[0].astype(np.float64)


@pytest.mark.parametrize("dx,dy", [(5, -3), (-12, 7), (0, 9)])
def test_pc_move_translates_pattern_exactly(dx, dy):
    # pixel (i, j) at PC0 + (dx, dy) / n casts the ray of pixel (i - dx,
    # j - dy) at PC0: the image is the nominal one moved by +(dx, dy)
    rng = np.random.default_rng(11)
    master = band_master()
    r = rot.quat_to_matrix(random_quats(rng, 1)[0])
    pc = (PC0[0] + dx / N, PC0[1] + dy / N, PC0[2])
    t = geo.project(master, r, N, PC0)
    e = geo.project(master, r, N, pc)
    jlo, jhi = max(0, dy), N + min(0, dy)
    ilo, ihi = max(0, dx), N + min(0, dx)
    assert np.allclose(e[jlo:jhi, ilo:ihi], t[jlo - dy:jhi - dy, ilo - dx:ihi - dx], atol=1e-9)
    by, bx = pcmodel.beam_shift(pc, PC0, N)
    assert abs(by - dy) < 1e-9 and abs(bx - dx) < 1e-9


def test_search_shift_at_exact_orientation_is_the_beam_shift():
    # the correlation of a pattern at a moved PC with the nominal-PC
    # template of the same orientation peaks at the beam shift; the fixed
    # Hann window pulls the peak a few per cent toward zero
    rng = np.random.default_rng(12)
    master = band_master()
    for _ in range(3):
        q = random_quats(rng, 1)[0]
        dx, dy = rng.uniform(-17, 17), rng.uniform(-10, 10)
        pc = (PC0[0] + dx / N, PC0[1] + dy / N, PC0[2])
        _, s = refine.measure_shift(_pattern(q, pc), geo.project(master, rot.quat_to_matrix(q), N, PC0), Params())
        by, bx = pcmodel.beam_shift(pc, PC0, N)
        assert abs(s[0] - by) < 0.06 * abs(by) + 0.1
        assert abs(s[1] - bx) < 0.06 * abs(bx) + 0.1


@pytest.mark.parametrize("axis", ["x", "y"])
def test_corrected_first_step(axis):
    # crystal rotated 1.5 deg about a detector axis, PC moved by ~(12, -8)
    # px: the corrected first x/y step removes most of the error; the raw
    # search shift would read the PC move as a rotation of several degrees
    rng = np.random.default_rng(13)
    master = band_master()
    r0 = rot.quat_to_matrix(random_quats(rng, 1)[0])
    q = rot.rot_x(np.deg2rad(1.5)) if axis == "x" else rot.rot_y(np.deg2rad(1.5))
    rt = r0 @ q.T
    pc = (PC0[0] + 12.3 / N, PC0[1] - 8.1 / N, PC0[2])
    pat = _pattern(rot.matrix_to_quat(rt), pc)
    _, s = refine.measure_shift(pat, geo.project(master, r0, N, PC0), Params())
    one = Params(n_iter=1)
    trace = []
    refine.refine_one_from_match(pat, master, r0, pc, PC0, s, one, trace=trace)
    r_raw = refine.xy_update(r0, s, pc[2], N)
    before = rot.misorientation_angle(r0, rt)
    after_xy = rot.misorientation_angle(refine.xy_update(r0, trace[0][0], pc[2], N), rt)
    assert after_xy < 0.3 * before
    assert rot.misorientation_angle(r_raw, rt) > 3 * before


def test_from_match_refinement_converges():
    # Figure 7 analogue with one library for a drifting PC: start 2.5 deg
    # away with the PC moved up to 17 x 10 px; two iterations reach < 0.1 deg
    rng = np.random.default_rng(14)
    master = band_master()
    for _ in range(3):
        qt = random_quats(rng, 1)[0]
        r_true = rot.quat_to_matrix(qt)
        pc = (PC0[0] + rng.uniform(-17, 17) / N, PC0[1] + rng.uniform(-10, 10) / N, PC0[2])
        r0 = r_true @ rot.axis_angle_matrix(rng.normal(size=3), np.deg2rad(2.5))
        pat = _pattern(qt, pc)
        _, s = refine.measure_shift(pat, geo.project(master, r0, N, PC0), Params())
        r, h, _ = refine.refine_one_from_match(pat, master, r0, pc, PC0, s, Params())
        assert np.rad2deg(rot.disorientation(r, r_true)) < 0.1
        assert h > 0.99


def test_from_match_without_a_pc_move_takes_the_measured_step():
    # at the nominal PC the corrected shift is the search's own shift, so
    # the first step is the one a re-projection at the start would measure
    rng = np.random.default_rng(15)
    master = band_master()
    qt = random_quats(rng, 1)[0]
    r_true = rot.quat_to_matrix(qt)
    r0 = r_true @ rot.axis_angle_matrix(rng.normal(size=3), np.deg2rad(2.0))
    pat = _pattern(qt, PC0)
    _, s = refine.measure_shift(pat, geo.project(master, r0, N, PC0), Params())
    a = refine.refine_one_from_match(pat, master, r0, PC0, PC0, s, Params())
    b = refine.refine_one(pat, master, r0, PC0, Params())
    assert np.allclose(a[0], b[0], atol=1e-15) and a[1] == b[1]


def test_pc_map_affine_model():
    # the silicon map's drift (pcx 0.39 -> 0.52 across, 0.08 screen widths in
    # y) as an affine model about the map centre
    w, h = 61, 41
    d_col = (0.13 / (w - 1), 0.0, 0.0)
    d_row = (0.0, 0.08 / (h - 1), 0.02 / (h - 1))
    pc0 = (0.455, 0.5, 0.6)
    pcs = pcmodel.pc_map(pc0, d_col, d_row, w, w * h, col0=(w - 1) / 2, row0=(h - 1) / 2)
    assert pcs.shape == (w * h, 3)
    centre = (h - 1) // 2 * w + (w - 1) // 2
    assert np.allclose(pcs[centre], pc0, atol=1e-15)
    assert abs(pcs[0, 0] - 0.39) < 1e-12 and abs(pcs[w - 1, 0] - 0.52) < 1e-12
    assert abs(pcs[-1, 1] - pcs[0, 1] - 0.08) < 1e-12
    grid = pcs.reshape(h, w, 3)
    assert np.allclose(np.diff(grid, axis=1), d_col, atol=1e-15)
    assert np.allclose(np.diff(grid, axis=0), d_row, atol=1e-15)

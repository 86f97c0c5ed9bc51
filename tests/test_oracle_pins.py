"""Known-answer pins for the oracle parts that the stage pins leave open:
the window (section "Fast Fourier Transform": patterns are windowed before
the transform), the band-pass values, the library argmax with its top-2 gap
(section "Method Overview": the best match is the highest coefficient) and
the two composed calls (Figure 1 B-C; section "Orientation and Pattern
Centre Refinement").

Each test names the plausible mistake it catches."""

import numpy as np
import pytest
from scipy.signal import windows

from fixtures import band_master, random_quats
from oracle import geometry as geo
from oracle import pipeline, spectra, xcf
from oracle import rotations as rot
from oracle.params import Params

SIZES = (8, 15, 16, 64, 96, 128, 160, 256)


def _window_1d(n):
    w2 = spectra.hann_window(n)
    w1 = np.sqrt(np.diag(w2))
    return w1, w2


@pytest.mark.parametrize("n", SIZES)
def test_hann_window_is_half_sample_hann(n):
    w1, w2 = _window_1d(n)
    # separable: the 2-D window is the outer product of one 1-D window
    assert np.allclose(w2, np.outer(w1, w1), atol=1e-15, rtol=0)
    # symmetric about the image centre (a window without the half-sample
    # offset, sin^2(pi i / N), is not: w_0 = 0 but w_{N-1} > 0)
    assert np.allclose(w1, w1[::-1], atol=1e-15, rtol=0)
    # strictly positive at both edges (the same mistake gives w_0 = 0)
    assert w1[0] > 0 and w1[-1] > 0
    # tapering, largest at the centre, rising monotonically over the first
    # half (a cos^2 window peaks at the edges instead)
    assert w1[0] < 0.05 * w1[(n - 1) // 2]
    assert np.all(np.diff(w1[: (n + 1) // 2]) > 0)
    assert abs(w1.max() - np.cos(np.pi / (2 * n)) ** 2 * (n % 2 == 0) - (n % 2 == 1)) < 1e-12
    # sum_i sin^2(pi (i + 1/2) / N) = N / 2 for N >= 2 (the cosine terms of
    # the double-angle form cancel over a full period); a plain sine window
    # (no square) sums to 1 / sin(pi / 2N) instead
    assert abs(w1.sum() - n / 2) < 1e-12 * n
    # a raised cosine: its DFT has support {0, +-1} only, with |W(1)| = N/4
    # (a Blackman, Tukey or sine window has wider support)
    wf = np.fft.fft(w1)
    assert abs(wf[0] - n / 2) < 1e-12 * n
    if n > 2:
        assert abs(abs(wf[1]) - n / 4) < 1e-12 * n
        assert np.max(np.abs(wf[2:n - 1])) < 1e-12 * n
    # textbook special case: the periodic Hann window of length 2N sampled
    # at its odd points is exactly this half-sample-offset window
    assert np.allclose(w1, windows.hann(2 * n, sym=False)[1::2], atol=1e-15, rtol=0)


def test_bandpass_is_isotropic():
    # H depends on the radial frequency only: Pythagorean frequency pairs
    # carry identical weights (an |u| + |v| or max(|u|, |v|) radius fails)
    n, prm = 128, Params()
    h = spectra.bandpass(n, prm)
    for (a, b, c) in ((3, 4, 5), (5, 12, 13), (8, 15, 17), (20, 21, 29), (12, 35, 37)):
        vals = [h[a, b], h[b, a], h[-a, b], h[a, -b], h[c, 0], h[0, c], h[-c, 0], h[0, -c]]
        assert np.ptp(vals) < 1e-15, (a, b, c, vals)


def test_bandpass_peak_and_low_pass_slope():
    # Product of a Gaussian high pass and a Gaussian low pass: with
    # x = rho^2 / 2, dH/dx = 0 at x* = s_hp^2 ln(1 + s_lp^2 / s_hp^2)
    # (calculus, not the formula retyped).  On a fine frequency grid (large N,
    # so that the integer frequencies resolve the peak) the maximum along an
    # axis lies at the integer next to rho*.  Far above the high-pass scale
    # the log gain falls as -rho^2 / (2 s_lp^2): a wrong sigma or a missing
    # factor 2 moves either the peak or the slope.
    prm = Params(sigma_hp=6.0, sigma_lp_frac=1.0 / 16, rho_max_frac=0.45)
    n = 512
    h = spectra.bandpass(n, prm)
    s_hp, s_lp = prm.sigma_hp, prm.sigma_lp(n)
    rho_star = np.sqrt(2 * s_hp ** 2 * np.log(1 + s_lp ** 2 / s_hp ** 2))
    axis = h[0, : n // 2]
    k = int(np.argmax(axis))
    assert abs(k - rho_star) <= 0.5 + 1e-9, (k, rho_star)
    r1, r2 = 100, 160
    slope = (np.log(axis[r2]) - np.log(axis[r1])) / (r2 ** 2 - r1 ** 2)
    assert abs(slope + 1 / (2 * s_lp ** 2)) < 1e-6 / (2 * s_lp ** 2) + 1e-12
    # near DC the high pass rises as rho^2 / (2 s_hp^2) (to first order)
    assert abs(axis[1] / (1.0 / (2 * s_hp ** 2)) - 1) < 0.02


def test_library_argmax_gap_known_answers():
    # distinct top two: gap = best - second
    best, h, gap = xcf.library_argmax([0.3, 0.9, 0.5, 0.7])
    assert (best, h) == (1, 0.9) and abs(gap - 0.2) < 1e-15
    # the best after the second-best
    best, h, gap = xcf.library_argmax([0.7, 0.2, 0.95])
    assert (best, h) == (2, 0.95) and abs(gap - 0.25) < 1e-15
    # tie at the top: smallest index, gap exactly 0 (a second-best taken as
    # "the best of the others by value" would skip the tie)
    best, h, gap = xcf.library_argmax([0.4, 0.8, 0.1, 0.8])
    assert (best, h, gap) == (1, 0.8, 0.0)
    # negative scores
    best, h, gap = xcf.library_argmax([-0.5, -0.1, -0.3])
    assert (best, h) == (1, -0.1) and abs(gap - 0.2) < 1e-15
    # one template: no second-best, the gap is unbounded
    assert xcf.library_argmax([0.42]) == (0, 0.42, np.inf)


def test_library_argmax_brute_force():
    rng = np.random.default_rng(11)
    for trial in range(200):
        n = int(rng.integers(2, 40))
        s = np.round(rng.uniform(-1, 1, size=n), int(rng.integers(1, 4)))   # rounding makes ties common
        best, h, gap = xcf.library_argmax(s)
        top = max(s)
        first = min(i for i in range(n) if s[i] == top)
        second = sorted(s)[-2]                           # a multiset: a tied maximum gives gap 0
        assert best == first and h == top and gap == top - second


def _library(rng, master, l, n, pc):
    q = random_quats(rng, l)
    tmpl = np.stack([geo.project(master, r, n, pc) for r in rot.quat_to_matrix(q)])
    return q, tmpl


def test_index_patterns_known_answer_cyclic_shift():
    # Noise-free pattern = library template k cyclically shifted by (dx, dy)
    # px, window off: every step is exact, so the best template is k, its
    # integer and sub-pixel heights are 1, the shift is (dx, dy) in (x, y)
    # order and best_q is library row k.  Catches a swapped (x, y) output, a
    # wrong s_int order, an off-by-one best_q gather and a sign flip of the
    # shift (dx != dy, both signs used).
    rng = np.random.default_rng(21)
    master = band_master()
    n, pc = 64, (0.5, 0.5, 0.6)
    lib_q, tmpl = _library(rng, master, 7, n, pc)
    cases = [(3, 5, -2), (0, -4, 1), (6, 0, 3), (2, 7, 0)]   # (k, dx, dy)
    pats = np.stack([np.roll(tmpl[k], (dy, dx), axis=(0, 1)) for k, dx, dy in cases])
    prm = Params(window=False)
    out = pipeline.index_patterns(pats, master, pc, lib_q, prm)
    for i, (k, dx, dy) in enumerate(cases):
        assert out["best_idx"][i] == k
        assert np.array_equal(out["best_q"][i], lib_q[k])
        assert abs(out["h_int"][i] - 1) < 1e-12 and abs(out["peak_h"][i] - 1) < 1e-12
        assert tuple(out["s_int"][i]) == (dx, dy)
        assert np.allclose(out["shift"][i], (dx, dy), atol=1e-12, rtol=0)
        assert out["gap"][i] > 0.1


def test_index_patterns_known_answer_pc_offset():
    # The same with the physical route: the pattern is projected at the
    # pattern centre moved by (dx, dy) px in the screen plane, which
    # translates it by (dx, dy) (E(x) = T(x - s)); window on (the default).
    # The integer peak is exactly (dx, dy) in (x, y) order, the height just
    # below 1 (new pixels enter at the edges); the fixed window pulls the
    # sub-pixel shift a few per cent toward zero, never past it.
    rng = np.random.default_rng(22)
    master = band_master()
    n, pc = 64, (0.5, 0.5, 0.6)
    lib_q, _ = _library(rng, master, 7, n, pc)
    cases = [(4, 3, -2), (1, -2, 3)]
    pats = np.stack([geo.project(master, rot.quat_to_matrix(lib_q[k]), n, (pc[0] + dx / n, pc[1] + dy / n, pc[2]))
                     for k, dx, dy in cases])
    out = pipeline.index_patterns(pats, master, pc, lib_q, Params())
    for i, (k, dx, dy) in enumerate(cases):
        assert out["best_idx"][i] == k
        assert tuple(out["s_int"][i]) == (dx, dy)
        for got, want in zip(out["shift"][i], (dx, dy)):
            assert 0.9 * abs(want) - 0.01 <= got * np.sign(want) <= abs(want) + 0.01
        assert 0.8 < out["peak_h"][i] < 1.0


def test_refine_orientations_measurement_only():
    # n_iter = 0: the refinement is the final measurement alone.  The
    # orientation is returned unchanged, and the pattern (the template at
    # pattern i's own PC, rolled by (dx, dy)) gives height 1 and shift
    # (dx, dy) in (x, y) order; the per-pattern PCs differ, so reading
    # another pattern's PC fails.
    rng = np.random.default_rng(23)
    master = band_master()
    n = 64
    q = random_quats(rng, 3)
    pcs = np.array([[0.5, 0.5, 0.6], [0.47, 0.53, 0.62], [0.52, 0.46, 0.58]])
    shifts = [(2, -3), (-1, 4), (5, 1)]
    pats = np.stack([np.roll(geo.project(master, rot.quat_to_matrix(q[i]), n, pcs[i]), (dy, dx), axis=(0, 1))
                     for i, (dx, dy) in enumerate(shifts)])
    out = pipeline.refine_orientations(pats, master, pcs, q, Params(window=False, n_iter=0))
    for i, (dx, dy) in enumerate(shifts):
        assert np.allclose(out["q"][i], q[i] * np.sign(q[i][0]), atol=1e-15, rtol=0)
        assert abs(out["peak_h"][i] - 1) < 1e-12
        assert np.allclose(out["shift"][i], (dx, dy), atol=1e-12, rtol=0)


def test_refine_orientations_fixed_point_and_convergence():
    # The pattern is the gridded-master projection at (R_true, PC_i), so the
    # true orientation is a fixed point: started there, both steps measure a
    # zero shift and a zero rotation exactly (identical images) and the
    # orientation does not move.  Started 2 deg away about a random axis,
    # two iterations land within 0.02 deg of the truth with shift ~ 0.
    rng = np.random.default_rng(24)
    master = band_master()
    n = 96
    q_true = random_quats(rng, 3)
    pcs = np.array([[0.5, 0.5, 0.6], [0.5 + 3 / n, 0.5 - 2 / n, 0.6], [0.5 - 4 / n, 0.5 + 1 / n, 0.61]])
    pats = np.stack([geo.project(master, rot.quat_to_matrix(q_true[i]), n, pcs[i]) for i in range(3)])
    out = pipeline.refine_orientations(pats, master, pcs, q_true, Params())
    for i in range(3):
        assert np.rad2deg(rot.disorientation_q(out["q"][i], q_true[i])) < 1e-9
        assert abs(out["peak_h"][i] - 1) < 1e-12
        assert np.allclose(out["shift"][i], 0, atol=1e-12)
    r_true = rot.quat_to_matrix(q_true)
    q0 = np.stack([rot.matrix_to_quat(r_true[i] @ rot.axis_angle_matrix(rng.normal(size=3), np.deg2rad(2.0)))
                   for i in range(3)])
    out = pipeline.refine_orientations(pats, master, pcs, q0, Params())
    for i in range(3):
        assert np.rad2deg(rot.disorientation_q(out["q"][i], q_true[i])) < 0.02
        assert out["peak_h"][i] > 0.99
        assert np.max(np.abs(out["shift"][i])) < 0.05

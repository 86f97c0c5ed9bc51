"""27-point local orientation search in FP64 (oracle; test only).

The closing discussion of the paper names a sampling grid around the best
match as a coarser alternative to the shift / log-polar refinement.  The
reading taken here: one pass of a 3 x 3 x 3 grid of small crystal rotations
about the detector axes around a starting orientation R,

    R' = R Q(a, b, c)^T,   Q = Rz(c) Ry(b) Rx(a),   a, b, c in {-d, 0, +d},

(the same composition as the x / y and z updates of the refinement), with
d = 0.5 deg.  Candidates are numbered 9 i_a + 3 i_b + i_c with i = 0, 1, 2
for -d, 0, +d, so the number order is the lexicographic order of (a, b, c).
Every candidate is projected at the pattern's own pattern centre and scored
by its integer correlation peak h_int (the library score, shift window
max_shift); the largest h_int wins, ties to the smallest number, and the
winner's peak is upsampled as in the search.
"""

import numpy as np

from . import geometry, refine, rotations, spectra, xcf
from .params import Params

STEP_DEG = 0.5


def stencil_offsets(step):
    """[27, 3] angles (a, b, c) in candidate order."""
    v = (-step, 0.0, step)
    return np.array([(a, b, c) for a in v for b in v for c in v], dtype=np.float64)


def stencil_rotation(a, b, c):
    """Q(a, b, c) = Rz(c) Ry(b) Rx(a)."""
    return rotations.rot_z(c) @ rotations.rot_y(b) @ rotations.rot_x(a)


def stencil_candidates(r, step):
    return [r @ stencil_rotation(a, b, c).T for a, b, c in stencil_offsets(step)]


def stencil_one(pattern, master, r0, pc, prm, step):
    """Returns (index, R, h_int [27], gap, h_sub, (s_y, s_x))."""
    n = pattern.shape[0]
    se = spectra.unit_spectrum(pattern, prm)
    cands = stencil_candidates(np.asarray(r0, dtype=np.float64), step)
    specs = [spectra.unit_spectrum(geometry.project(master, rc, n, pc), prm) for rc in cands]
    h = xcf.library_scores(se, specs, prm.max_shift)
    best, _, gap = xcf.library_argmax(h)
    _, s_int = xcf.integer_peak(xcf.xcf_map(se, specs[best]), prm.max_shift)
    h_sub, s_sub = xcf.subpixel_peak(se, specs[best], s_int, prm.upsample)
    return best, cands[best], h, gap, h_sub, s_sub


def stencil_refine(patterns, master, pcs, q_init, prm=None, step_deg=STEP_DEG):
    """patterns: a sequence of square images (sizes may differ); pcs [P, 3].
    Returns dict(idx, q, h_int [P, 27], gap, peak_h, shift (x, y))."""
    prm = prm or Params()
    p = len(patterns)
    step = np.deg2rad(step_deg)
    rs = rotations.quat_to_matrix(np.asarray(q_init, dtype=np.float64).reshape(-1, 4))
    out = dict(idx=np.zeros(p, np.int32), q=np.zeros((p, 4)), h_int=np.zeros((p, 27)), gap=np.zeros(p),
               peak_h=np.zeros(p), shift=np.zeros((p, 2)))
    for i in range(p):
        img = np.asarray(patterns[i], dtype=np.float64)
        best, r, h, gap, h_sub, s_sub = stencil_one(img, master, rs[i], pcs[i], prm, step)
        out["idx"][i] = best
        out["q"][i] = rotations.matrix_to_quat(r)
        out["h_int"][i] = h
        out["gap"][i] = gap
        out["peak_h"][i] = h_sub
        out["shift"][i] = (s_sub[1], s_sub[0])
    return out


def stencil_then_refine(patterns, master, pcs, q_init, prm=None, step_deg=STEP_DEG):
    """The stencil around q_init, then the refinement of section "Orientation
    and Pattern Centre Refinement" from the stencil's pick at each pattern's
    own pattern centre; its first x / y step takes the shift the stencil
    already measured for its winner (projected at that same pattern centre),
    in place of a projection and correlation at the starting orientation.
    Returns dict(stencil (the stencil_refine result), q, peak_h, shift (x, y))."""
    prm = prm or Params()
    st = stencil_refine(patterns, master, pcs, q_init, prm, step_deg)
    p = len(patterns)
    out = dict(stencil=st, q=np.zeros((p, 4)), peak_h=np.zeros(p), shift=np.zeros((p, 2)))
    rs = rotations.quat_to_matrix(st["q"])
    for i in range(p):
        img = np.asarray(patterns[i], dtype=np.float64)
        first = (st["shift"][i][1], st["shift"][i][0])
        r, h, s = refine.refine_one(img, master, rs[i], pcs[i], prm, first_shift=first)
        out["q"][i] = rotations.matrix_to_quat(r)
        out["peak_h"][i] = h
        out["shift"][i] = (s[1], s[0])
    return out

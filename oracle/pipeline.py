"""The two calls of the method, composed from the oracle steps (test only).

``index_patterns``: every pattern against every library template (section
"Method Overview", Figure 1 B-C): templates are projected at the nominal
pattern centre (one library, section "Orientation and Pattern Centre
Refinement"), both sides are filtered into spectra, the integer correlation
peak is the score, the best template wins and its peak is upsampled.

``refine_orientations``: the refinement of section "Orientation and Pattern
Centre Refinement" from a starting orientation, at each pattern's own
pattern centre.

``refine_from_match``: the same refinement whose first x/y step reuses the
search's shift, corrected for the beam-induced PC move (one library for the
whole map).
"""

import numpy as np

from . import geometry, refine, rotations, spectra, xcf
from .params import Params


def library_spectra(master, lib_q, n, pc, prm):
    return [spectra.unit_spectrum(geometry.project(master, r, n, pc), prm)
            for r in rotations.quat_to_matrix(lib_q)]


def index_patterns(patterns, master, pc, lib_q, prm=None, lib_spec=None, return_scores=False):
    """Returns dict(best_idx, best_q, peak_h, shift (x, y) px, h_int, gap[, scores])."""
    prm = prm or Params()
    patterns = np.asarray(patterns, dtype=np.float64)
    p, n, _ = patterns.shape
    lib_q = np.asarray(lib_q, dtype=np.float64)
    if lib_spec is None:
        lib_spec = library_spectra(master, lib_q, n, pc, prm)
    out = dict(best_idx=np.zeros(p, np.int32), best_q=np.zeros((p, 4)), peak_h=np.zeros(p),
               shift=np.zeros((p, 2)), h_int=np.zeros(p), gap=np.zeros(p), s_int=np.zeros((p, 2), np.int64))
    all_scores = []
    for i in range(p):
        se = spectra.unit_spectrum(patterns[i], prm)
        scores = xcf.library_scores(se, lib_spec, prm.max_shift)
        all_scores.append(scores)
        best, h_int, gap = xcf.library_argmax(scores)
        _, s_int = xcf.integer_peak(xcf.xcf_map(se, lib_spec[best]), prm.max_shift)
        h_sub, s_sub = xcf.subpixel_peak(se, lib_spec[best], s_int, prm.upsample)
        out["best_idx"][i] = best
        out["best_q"][i] = lib_q[best]
        out["peak_h"][i] = h_sub
        out["shift"][i] = (s_sub[1], s_sub[0])
        out["h_int"][i] = h_int
        out["gap"][i] = gap
        out["s_int"][i] = (s_int[1], s_int[0])
    if return_scores:
        out["scores"] = np.array(all_scores)
    return out


def refine_orientations(patterns, master, pcs, q_init, prm=None):
    """pcs: [P, 3] per-pattern pattern centres.  Returns dict(q, peak_h, shift (x, y))."""
    prm = prm or Params()
    patterns = np.asarray(patterns, dtype=np.float64)
    p = patterns.shape[0]
    rs = rotations.quat_to_matrix(q_init)
    out = dict(q=np.zeros((p, 4)), peak_h=np.zeros(p), shift=np.zeros((p, 2)))
    for i in range(p):
        r, h, s = refine.refine_one(patterns[i], master, rs[i], pcs[i], prm)
        out["q"][i] = rotations.matrix_to_quat(r)
        out["peak_h"][i] = h
        out["shift"][i] = (s[1], s[0])
    return out


def refine_from_match(patterns, master, pcs, pc_nominal, q_init, match_shift, prm=None):
    """Refinement that starts from the search's own measurement: q_init and
    match_shift [P, 2] (x, y) px are the search's best_q and shift against
    the library projected at pc_nominal; pcs [P, 3] are the points' own
    pattern centres.  Returns dict(q, peak_h, shift (x, y))."""
    prm = prm or Params()
    patterns = np.asarray(patterns, dtype=np.float64)
    p = patterns.shape[0]
    rs = rotations.quat_to_matrix(q_init)
    ms = np.asarray(match_shift, dtype=np.float64)
    out = dict(q=np.zeros((p, 4)), peak_h=np.zeros(p), shift=np.zeros((p, 2)))
    for i in range(p):
        r, h, s = refine.refine_one_from_match(patterns[i], master, rs[i], pcs[i], pc_nominal,
                                               (ms[i, 1], ms[i, 0]), prm)
        out["q"][i] = rotations.matrix_to_quat(r)
        out["peak_h"][i] = h
        out["shift"][i] = (s[1], s[0])
    return out

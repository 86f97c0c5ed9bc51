"""Map-wide pattern-centre model and beam-shift correction (oracle; test only).

Section "Orientation and Pattern Centre Refinement" (Figure 6 B) and the
silicon-map demonstrations: the pattern centre drifts across a map as the
beam moves over the sample.  One library is projected at one nominal PC; the
shift that the search measures against it mixes the orientation error with
the translation that the PC move causes, so that translation is taken off
before Equation 7 turns the shift into a rotation.  Later iterations
re-project the template at the point's own PC.

Readings (the paper imports its PC variation model from the acquisition
software and gives no form):

* the model is affine in the map position: point k of a row-major map
  ``width`` points wide sits at col = k mod width, row = k div width, and
  PC(k) = PC0 + (col - col0) dPC/dcol + (row - row0) dPC/drow, all in
  screen widths;
* a PC move by (dx, dy, 0) screen widths moves every pixel ray by
  (n dx, n dy) pixels, so the pattern is the nominal-PC image translated by
  +n (dx, dy) (shift convention E(x) ~ T(x - s)); a change of PCz scales
  the pattern about the PC instead, which is second order here and is left
  to the re-projected iterations.
"""

import numpy as np


def pc_map(pc0, d_col, d_row, width, p, col0=0.0, row0=0.0):
    """Per-point pattern centres [p, 3] of the affine model."""
    k = np.arange(p, dtype=np.int64)
    col = (k % width).astype(np.float64)
    row = (k // width).astype(np.float64)
    pc0 = np.asarray(pc0, dtype=np.float64)
    d_col = np.asarray(d_col, dtype=np.float64)
    d_row = np.asarray(d_row, dtype=np.float64)
    return pc0[None, :] + (col - col0)[:, None] * d_col[None, :] + (row - row0)[:, None] * d_row[None, :]


def beam_shift(pc_point, pc_nominal, n):
    """(s_y, s_x) px by which the PC move alone translates the pattern."""
    return (n * (pc_point[1] - pc_nominal[1]), n * (pc_point[0] - pc_nominal[0]))

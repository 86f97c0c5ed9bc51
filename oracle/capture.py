"""Capture range of the correlation (oracle; test only).

Section "SO(3) Sampling Frequency", Figures 3 and 4: a reference pattern is
compared with patterns of the same crystal rotated about the detector x, y
or z axis in 0.5 degree steps; the width of the correlation peak as a
function of the rotation angle sets the library spacing, and Figure 4 shows
how that width changes with a pattern-centre error and with the screen size.

Readings (the paper gives no formula for the width):

* the curve is the integer correlation peak h(theta) (the score the library
  search ranks by) of the reference pattern against the pattern rotated by
  theta, a detector-frame rotation Q, orientation R Q^T;
* the full width at half maximum is measured above the curve's floor (the
  correlation of a shifted, unrelated pattern stays well above zero, and
  the paper motivates the width by the contrast of the match over that
  baseline): level = (largest + smallest sample) / 2; from the largest
  sample (the first, on ties) walk outwards on each side to the first
  sample below the level and interpolate linearly between it and its inner
  neighbour; a side that never drops below the level reports the end of
  the sampled range (the width is then a lower bound).
"""

import numpy as np

from . import geometry, rotations, spectra, xcf


def axis_rotation(axis, theta):
    return {"x": rotations.rot_x, "y": rotations.rot_y, "z": rotations.rot_z}[axis](theta)


def rotated_orientations(r_ref, axis, thetas_deg):
    """R Q(theta)^T for each angle (degrees)."""
    return [r_ref @ axis_rotation(axis, np.deg2rad(t)).T for t in thetas_deg]


def capture_curve(master, r_ref, axis, thetas_deg, n, pc_ref, pc_test, prm):
    """h(theta): integer peak of the reference (at pc_ref) against each
    rotated pattern (at pc_test)."""
    ref = spectra.unit_spectrum(geometry.project(master, r_ref, n, pc_ref), prm)
    out = np.empty(len(thetas_deg))
    for k, r in enumerate(rotated_orientations(r_ref, axis, thetas_deg)):
        t = spectra.unit_spectrum(geometry.project(master, r, n, pc_test), prm)
        out[k] = xcf.integer_peak(xcf.xcf_map(ref, t), prm.max_shift)[0]
    return out


def fwhm(thetas_deg, h):
    """Full width at half maximum of a sampled curve (reading above)."""
    t = np.asarray(thetas_deg, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    k0 = int(np.argmax(h))
    level = 0.5 * (h[k0] + np.min(h))

    def edge(step):
        k = k0
        while 0 <= k + step < len(h):
            if h[k + step] < level:
                a, b = h[k], h[k + step]
                return t[k] + (t[k + step] - t[k]) * (a - level) / (a - b)
            k += step
        return t[k]

    return edge(1) - edge(-1)

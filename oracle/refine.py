"""Orientation refinement in FP64 (oracle; test only).

Section "Orientation and Pattern Centre Refinement":

* x / y: a small crystal rotation about the detector x or y axis moves the
  pattern; the shift measured by the correlation gives the angle through
  Equation 7 (angle = shift / detector distance).  Equation 7 is the small
  angle form with unstated units; the reading is beta = atan(s_x / DD),
  alpha = -atan(s_y / DD) with DD = PCz N in pixels, and the update
  R <- R (Ry(beta) Rx(alpha))^T.  (With c = R d, a crystal rotated by Q in
  the detector frame has orientation R Q^T; Ry(beta) moves features near
  the PC by +DD tan(beta) along +x, Rx(alpha) by -DD tan(alpha) along +y.)
* z: the images are resampled in log-polar coordinates about the screen
  centre, where a rotation about the detector normal becomes a shift along
  eta; the shift is measured by correlation and R <- R Rz(gamma)^T with
  gamma = 2 pi d_eta / N_eta.
* the template is re-projected for the updated orientation at the pattern's
  own pattern centre, and the step is iterated (about two iterations; fixed
  at n_iter here).

Unstated details and their readings: the log-polar grid has N_rho radii
log-spaced in [2, N/2 - 2] px and N_eta angles, sampled bilinearly from the
contrast-normalised (unwindowed) image; each radius row has its mean
removed and carries a Hann weight over radius; the eta correlation is the
weighted sum of per-row circular correlations (the rows are the "multiple
windows"); its peak is refined by trigonometric interpolation at 1/kappa
steps over +-0.75 samples; the z step is measured after re-projecting at the
x/y-updated orientation.
"""

import numpy as np

from . import geometry, pcmodel, rotations, spectra, xcf


def xy_update(r, shift, pcz, n):
    """R <- R (Ry(beta) Rx(alpha))^T from a measured shift (s_y, s_x) in px."""
    dd = pcz * n
    beta = np.arctan(shift[1] / dd)
    alpha = -np.arctan(shift[0] / dd)
    q = rotations.rot_y(beta) @ rotations.rot_x(alpha)
    return r @ q.T


def z_update(r, gamma):
    return r @ rotations.rot_z(gamma).T


def logpolar_radii(n, n_rho):
    rmin, rmax = 2.0, n / 2.0 - 2.0
    k = np.arange(n_rho, dtype=np.float64)
    return rmin * (rmax / rmin) ** (k / (n_rho - 1))


def bilinear(img, row, col):
    img = np.asarray(img, dtype=np.float64)
    r0 = np.floor(row).astype(np.int64)
    c0 = np.floor(col).astype(np.int64)
    fr = row - r0
    fc = col - c0
    return ((1 - fr) * (1 - fc) * img[r0, c0] + (1 - fr) * fc * img[r0, c0 + 1]
            + fr * (1 - fc) * img[r0 + 1, c0] + fr * fc * img[r0 + 1, c0 + 1])


def logpolar(img, n_rho, n_eta):
    """L[k, m] sampled at radius r_k and angle eta_m = 2 pi m / n_eta about
    the screen centre; eta = atan2(row - c, col - c)."""
    n = img.shape[0]
    c = (n - 1) / 2.0
    r = logpolar_radii(n, n_rho)
    eta = 2 * np.pi * np.arange(n_eta) / n_eta
    col = c + r[:, None] * np.cos(eta)[None, :]
    row = c + r[:, None] * np.sin(eta)[None, :]
    return bilinear(img, row, col)


def eta_correlation(lp_e, lp_t):
    """c(D) = sum_k w_k sum_m Le[k, m] Lt[k, m - D] (rows mean-removed, Hann
    weights over radius), normalised; D = 0 .. n_eta - 1 (cyclic)."""
    n_rho, n_eta = lp_e.shape
    w = np.sin(np.pi * (np.arange(n_rho) + 0.5) / n_rho) ** 2
    le = lp_e - lp_e.mean(axis=1, keepdims=True)
    lt = lp_t - lp_t.mean(axis=1, keepdims=True)
    c = np.zeros(n_eta)
    for k in range(n_rho):
        for d in range(n_eta):
            c[d] += w[k] * np.dot(le[k], np.roll(lt[k], d))
    norm = np.sqrt(np.sum(w[:, None] * le * le) * np.sum(w[:, None] * lt * lt))
    return c / norm


def eta_value(c, t):
    """Real trigonometric interpolant of the cyclic sequence c at points t
    (the Nyquist term enters as cos(pi t))."""
    n = c.size
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    cf = np.fft.fft(c)
    q = np.arange(1, n // 2)
    return (cf[0].real
            + 2 * np.real(cf[q][None, :] * np.exp(2j * np.pi * np.outer(t, q) / n)).sum(axis=1)
            + cf[n // 2].real * np.cos(np.pi * t)) / n


def eta_peak(c, kappa=100, box=0.75):
    """Integer argmax (ties to the smallest index), then the maximum of the
    trigonometric interpolant of c over D_int + a / kappa, |a| <= ceil(box kappa)
    (ties to the smallest a).  Returns (value, signed shift in samples)."""
    n = c.size
    k = int(np.argmax(c))
    d_int = k - n if k >= n // 2 else k
    m = int(np.ceil(box * kappa))
    t = d_int + np.arange(-m, m + 1) / kappa
    val = eta_value(c, t)
    j = int(np.argmax(val))
    return float(val[j]), float(t[j])


def eta_correlation_of(pattern, template, prm):
    n = pattern.shape[0]
    le = logpolar(spectra.normalise(pattern), prm.nrho(n), prm.neta(n))
    lt = logpolar(spectra.normalise(template), prm.nrho(n), prm.neta(n))
    return eta_correlation(le, lt)


def measure_gamma(pattern, template, prm):
    c = eta_correlation_of(pattern, template, prm)
    _, d = eta_peak(c, prm.upsample)
    return 2 * np.pi * d / c.size


def measure_shift(pattern, template, prm):
    """Sub-pixel (h, (s_y, s_x)) of the pattern against a template."""
    se = spectra.unit_spectrum(pattern, prm)
    st = spectra.unit_spectrum(template, prm)
    h_int, s_int = xcf.integer_peak(xcf.xcf_map(se, st), prm.max_shift)
    return xcf.subpixel_peak(se, st, s_int, prm.upsample)


def refine_one(pattern, master, r0, pc, prm, trace=None, first_shift=None):
    """Refine one pattern from orientation matrix r0 (fixed n_iter iterations),
    then measure the final peak height and shift.  Returns (R, h, (s_y, s_x)).

    first_shift (s_y, s_x), if given, replaces the projection and correlation
    of the first x/y step (the beam-shift-corrected shift of the search)."""
    n = pattern.shape[0]
    r = np.array(r0, dtype=np.float64)
    for it in range(prm.n_iter):
        if it == 0 and first_shift is not None:
            s = (float(first_shift[0]), float(first_shift[1]))
        else:
            t = geometry.project(master, r, n, pc)
            _, s = measure_shift(pattern, t, prm)
        r = xy_update(r, s, pc[2], n)
        t = geometry.project(master, r, n, pc)
        g = measure_gamma(pattern, t, prm)
        r = z_update(r, g)
        if trace is not None:
            trace.append((s, g, r.copy()))
    t = geometry.project(master, r, n, pc)
    h, s = measure_shift(pattern, t, prm)
    return r, h, s


def refine_one_from_match(pattern, master, r0, pc, pc_nominal, match_shift, prm, trace=None):
    """refine_one whose first x/y step uses the shift the search measured
    against the library template (projected at pc_nominal), less the
    translation that the move from pc_nominal to the point's pc causes.
    match_shift is (s_y, s_x) px."""
    n = pattern.shape[0]
    by, bx = pcmodel.beam_shift(pc, pc_nominal, n)
    s0 = (match_shift[0] - by, match_shift[1] - bx)
    return refine_one(pattern, master, r0, pc, prm, trace=trace, first_shift=s0)

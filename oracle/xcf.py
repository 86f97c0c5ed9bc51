"""Cross-correlation, peaks and library search in FP64 (oracle; test only).

Introduction, Equations 2 and 3: the normalised dot product is the zero-shift
value of the cross-correlation image, computed through the FFT.  Section
"Fast Fourier Transform": r_fg(x0) = sum_x f(x) g(x - x0), evaluated in the
Fourier domain, normalised by the autocorrelations so that coefficients lie
in [0, 1], with the peak upsampled for sub-pixel shift.  The printed
Fourier-domain formula is garbled (conjugate missing in Equation 3, F(u,u),
an exponent sign that contradicts its own spatial definition); the reading
used follows the spatial definition with f = experimental pattern and g =
template, so that E(x) ~ T(x - s) peaks at shift s:

    rho(s) = sum_u E'(u) conj(T'(u)) exp(+2 pi i u.s / N) / sqrt(e_E e_T).

Shifts are (s_y, s_x) in rows / columns; the signed range is [-N/2, N/2).
Integer peak: largest value, ties to the smallest unsigned row-major index
((s_y mod N) N + (s_x mod N)).  Library: largest integer peak, ties to the
smallest template index (section "Method Overview": the best match is the
highest coefficient).
"""

import numpy as np

from . import spectra


def xcf_map(spec_e, spec_t):
    """rho(s) on the full N x N cyclic shift grid from two unit-energy spectra."""
    n = spec_e.shape[0]
    z = spec_e * np.conj(spec_t)
    return np.real(np.fft.ifft2(z)) * (n * n)


def xcf_map_direct(img_e, img_t):
    """Direct-space circular correlation sum_x e(x) t(x - s) (brute force)."""
    n = img_e.shape[0]
    out = np.empty((n, n))
    for sy in range(n):
        for sx in range(n):
            out[sy, sx] = np.sum(img_e * np.roll(img_t, (sy, sx), axis=(0, 1)))
    return out


def signed_shift(k, n):
    return k - n if k >= n // 2 else k


def window_mask(n, max_shift):
    if max_shift is None or max_shift < 0:
        return np.ones((n, n), dtype=bool)
    s = np.array([abs(signed_shift(k, n)) for k in range(n)])
    return (s[:, None] <= max_shift) & (s[None, :] <= max_shift)


def integer_peak(rho, max_shift=-1):
    """(h_int, (s_y, s_x) signed) with row-major tie-break inside the window."""
    n = rho.shape[0]
    vals = np.where(window_mask(n, max_shift), rho, -np.inf).ravel()
    k = int(np.argmax(vals))            # first occurrence = smallest index
    sy, sx = divmod(k, n)
    return float(vals[k]), (signed_shift(sy, n), signed_shift(sx, n))


def library_scores(spec_p, spec_lib, max_shift=-1):
    """h_int for one pattern spectrum against every library spectrum."""
    return np.array([integer_peak(xcf_map(spec_p, t), max_shift)[0] for t in spec_lib])


def library_argmax(scores):
    """Best template (ties to the smallest index), its score and the top-2 gap."""
    scores = np.asarray(scores, dtype=np.float64)
    best = int(np.argmax(scores))
    if scores.size > 1:
        second = np.partition(scores, -2)[-2]
        gap = float(scores[best] - second)
    else:
        gap = np.inf
    return best, float(scores[best]), gap


def subpixel_peak(spec_e, spec_t, s_int, kappa=100, box=0.75):
    """Upsampled peak around the integer peak (single-step matrix DFT).

    Section "Fast Fourier Transform" (Equation 5 and the text around it): the
    peak of the correlation is upsampled for sub-pixel resolution.  The
    upsampling method is not given; the reading is the matrix-multiply DFT
    of Guizar-Sicairos, Thurman and Fienup (Opt. Lett. 33, 156, 2008), which
    evaluates the band-limited correlation exactly at s_int + (a, b)/kappa,
    a, b in [-ceil(box kappa), ceil(box kappa)].  Returns (h_sub, (s_y, s_x)).
    The argmax takes the real part; ties go to the smallest (b, a) in
    row-major order.
    """
    n = spec_e.shape[0]
    z = spec_e * np.conj(spec_t)
    m = int(np.ceil(box * kappa))
    off = np.arange(-m, m + 1) / kappa
    f = spectra.signed_freq(n)
    ys = s_int[0] + off
    xs = s_int[1] + off
    ky = np.exp(2j * np.pi * np.outer(ys, f) / n)       # [b, u]
    kx = np.exp(2j * np.pi * np.outer(f, xs) / n)       # [v, a]
    up = np.real(ky @ z @ kx)                           # [b, a]
    k = int(np.argmax(up))
    b, a = divmod(k, up.shape[1])
    return float(up[b, a]), (float(ys[b]), float(xs[a]))


def rho_at(spec_e, spec_t, s):
    """rho at one real-valued shift s = (s_y, s_x) (trigonometric interpolation)."""
    n = spec_e.shape[0]
    f = spectra.signed_freq(n)
    ph = np.exp(2j * np.pi * (f[:, None] * s[0] + f[None, :] * s[1]) / n)
    return float(np.real(np.sum(spec_e * np.conj(spec_t) * ph)))

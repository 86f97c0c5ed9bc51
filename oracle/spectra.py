"""Pattern preprocessing and filtered spectra in FP64 (oracle; test only).

Sections "Fast Fourier Transform" and "SO(3) Sampling Frequency": patterns
and templates are contrast normalised (mean 0, standard deviation 1),
windowed, transformed with the 2-D DFT (Equation 4) and band-pass filtered
(a high pass removes the background, a low pass removes noise); the
correlation is normalised by the autocorrelations.  Window and filter
shapes are not given; see ``oracle.params`` for the readings.

Equation 4 carries a unitary 1/sqrt(MN) factor.  It cancels in the
normalised correlation, so the spectra here are unnormalised DFTs.
"""

import numpy as np


def normalise(img):
    """(x - mean) / std, population std (the choice cancels in the correlation)."""
    x = np.asarray(img, dtype=np.float64)
    return (x - x.mean()) / x.std()


def hann_window(n):
    w1 = np.sin(np.pi * (np.arange(n) + 0.5) / n) ** 2
    return np.outer(w1, w1)


def signed_freq(n):
    k = np.arange(n)
    return np.where(k < n - n // 2, k, k - n).astype(np.float64)


def bandpass(n, prm):
    """H[u, v] on the full n x n DFT grid (u along rows, v along columns)."""
    fu = signed_freq(n)
    rho = np.sqrt(fu[:, None] ** 2 + fu[None, :] ** 2)
    s_hp, s_lp = prm.sigma_hp, prm.sigma_lp(n)
    h = (1.0 - np.exp(-rho ** 2 / (2 * s_hp ** 2))) * np.exp(-rho ** 2 / (2 * s_lp ** 2))
    h[rho > prm.rho_max(n)] = 0.0
    if n % 2 == 0:          # Nyquist row and column carry no weight
        h[n // 2, :] = 0.0
        h[:, n // 2] = 0.0
    return h


def filtered_spectrum(img, prm):
    """X' = H . DFT2(w . normalise(img)) on the full grid, and e = sum |X'|^2."""
    x = normalise(img)
    n = x.shape[0]
    if prm.window:
        x = x * hann_window(n)
    spec = np.fft.fft2(x) * bandpass(n, prm)
    e = float(np.sum(np.abs(spec) ** 2))
    return spec, e


def unit_spectrum(img, prm):
    """Filtered spectrum scaled to unit energy: X' / sqrt(e)."""
    spec, e = filtered_spectrum(img, prm)
    return spec / np.sqrt(e)

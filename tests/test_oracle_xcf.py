"""Pins for oracle.spectra and oracle.xcf (Equations 2-4, the spatial
definition of r_fg, normalisation by the autocorrelations, the upsampled
peak of Equation 5, and the library argmax)."""

import numpy as np

from oracle import spectra, xcf
from oracle.params import Params


def _dft2_brute(x):
    n = x.shape[0]
    k = np.arange(n)
    w = np.exp(-2j * np.pi * np.outer(k, k) / n)
    return w @ x @ w.T          # X[u, v] = sum_{j, i} x[j, i] e^{-2 pi i (u j + v i) / n}


def test_forward_transform_convention():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(8, 8))
    prm = Params(window=False, rho_max_frac=10.0)
    spec, e = spectra.filtered_spectrum(x, prm)
    h = spectra.bandpass(8, prm)
    brute = _dft2_brute(spectra.normalise(x)) * h
    assert np.allclose(spec, brute, atol=1e-12)
    assert abs(e - np.sum(np.abs(brute) ** 2)) < 1e-10
    # u indexes rows: a pure row-wise cosine sits at u = +-1
    img = np.cos(2 * np.pi * np.arange(8) / 8)[:, None] * np.ones((1, 8))
    s = _dft2_brute(img)
    assert abs(s[1, 0] - 32) < 1e-12 and abs(s[0, 1]) < 1e-12


def test_bandpass_shape():
    n, prm = 128, Params()
    h = spectra.bandpass(n, prm)
    assert h[0, 0] == 0.0
    assert np.all(h[n // 2, :] == 0) and np.all(h[:, n // 2] == 0)
    f = spectra.signed_freq(n)
    rho = np.hypot(f[:, None], f[None, :])
    assert np.all(h[rho > 48.0] == 0) and np.all(h[(rho > 0) & (rho <= 48.0)] > 0)
    # symmetric under u -> -u and v -> -v (so filtered spectra stay Hermitian)
    assert np.array_equal(h, np.roll(h[::-1, ::-1], 1, axis=(0, 1)))


def test_parseval_and_energy():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(32, 32))
    spec, e = spectra.filtered_spectrum(x, Params())
    img = np.real(np.fft.ifft2(spec))
    assert abs(np.sum(img ** 2) - e / 32 ** 2) < 1e-10


def _filtered_image(x, prm):
    spec, e = spectra.filtered_spectrum(x, prm)
    return np.real(np.fft.ifft2(spec)), e


def test_xcf_equals_direct_correlation():
    # rho(s) = sum_x e'(x) t'(x - s) / sqrt(sum e'^2 sum t'^2), brute force
    rng = np.random.default_rng(2)
    for n in (8, 16):
        prm = Params(rho_max_frac=0.45)
        a, b = rng.normal(size=(2, n, n))
        ea, _ = _filtered_image(a, prm)
        eb, _ = _filtered_image(b, prm)
        direct = xcf.xcf_map_direct(ea, eb) / np.sqrt(np.sum(ea ** 2) * np.sum(eb ** 2))
        fast = xcf.xcf_map(spectra.unit_spectrum(a, prm), spectra.unit_spectrum(b, prm))
        assert np.allclose(fast, direct, atol=1e-12)


def test_self_correlation_and_bound():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(64, 64))
    y = rng.normal(size=(64, 64))
    sx, sy = spectra.unit_spectrum(x, Params()), spectra.unit_spectrum(y, Params())
    assert abs(xcf.xcf_map(sx, sx)[0, 0] - 1.0) < 1e-12
    assert np.max(np.abs(xcf.xcf_map(sx, sy))) <= 1.0 + 1e-12
    # affine contrast changes do not change rho
    s2 = spectra.unit_spectrum(3.7 * x + 11.0, Params())
    assert np.allclose(xcf.xcf_map(s2, sy), xcf.xcf_map(sx, sy), atol=1e-12)


def test_exact_integer_shift_recovery():
    rng = np.random.default_rng(4)
    n = 32
    t = rng.normal(size=(n, n))
    for window in (False, True):
        prm = Params(window=window)
        st = spectra.unit_spectrum(t, prm)
        # with the window on, the shifted copy must still overlap its template
        shifts = ((0, 0), (3, -5), (-2, 1), (4, 2)) if window else ((0, 0), (3, -5), (-16, 15), (7, 2))
        for s0 in shifts:
            e = np.roll(t, s0, axis=(0, 1))             # E(x) = T(x - s0)
            h, s = xcf.integer_peak(xcf.xcf_map(spectra.unit_spectrum(e, prm), st))
            assert s == s0
            if not window or s0 == (0, 0):
                assert abs(h - 1.0) < 1e-12
            else:
                assert h < 1.0 - 1e-6          # the window is applied after the shift


def test_pearson_special_case():
    # no window and an all-pass filter except DC (odd N has no Nyquist row):
    # rho(0) is the Pearson correlation, i.e. the mean-subtracted normalised
    # dot product of Equation 1
    rng = np.random.default_rng(5)
    n = 15
    prm = Params(window=False, sigma_hp=1e-6, sigma_lp_frac=1e9, rho_max_frac=10.0)
    a, b = rng.normal(size=(2, n, n))
    rho0 = xcf.xcf_map(spectra.unit_spectrum(a, prm), spectra.unit_spectrum(b, prm))[0, 0]
    assert abs(rho0 - np.corrcoef(a.ravel(), b.ravel())[0, 1]) < 1e-12


def test_peak_window_and_tie_break():
    rho = np.zeros((8, 8))
    rho[1, 2] = rho[5, 1] = 0.7                          # tie: smaller row-major index wins
    assert xcf.integer_peak(rho) == (0.7, (1, 2))
    rho[4, 4] = 0.9                                      # outside |s| <= 3 in both axes (signed -4)
    assert xcf.integer_peak(rho)[1] == (-4, -4)
    assert xcf.integer_peak(rho, max_shift=3) == (0.7, (1, 2))
    assert xcf.library_argmax([0.2, 0.5, 0.5, 0.1])[:2] == (1, 0.5)


def test_library_search_brute_force():
    # tiny library: direct-space correlation of every pair, O(L N^4)
    rng = np.random.default_rng(6)
    n, l = 16, 12
    prm = Params(rho_max_frac=0.45)
    lib = rng.normal(size=(l, n, n))
    pat = np.roll(lib[7], (2, -3), axis=(0, 1)) + 0.3 * rng.normal(size=(n, n))
    fp, ep = _filtered_image(pat, prm)
    brute = []
    for t in lib:
        ft, et = _filtered_image(t, prm)
        brute.append(np.max(xcf.xcf_map_direct(fp, ft)) / np.sqrt(np.sum(fp ** 2) * np.sum(ft ** 2)))
    sp = spectra.unit_spectrum(pat, prm)
    scores = xcf.library_scores(sp, [spectra.unit_spectrum(t, prm) for t in lib])
    assert np.allclose(scores, brute, atol=1e-12)
    assert xcf.library_argmax(scores)[0] == 7


def _shifted_spectrum(spec, s):
    n = spec.shape[0]
    f = spectra.signed_freq(n)
    return spec * np.exp(-2j * np.pi * (f[:, None] * s[0] + f[None, :] * s[1]) / n)


def test_subpixel_recovers_band_limited_shift():
    rng = np.random.default_rng(7)
    n = 64
    st = spectra.unit_spectrum(rng.normal(size=(n, n)), Params())
    for s0 in ((0.37, -1.62), (-5.255, 3.5), (2.0, 0.004)):
        se = _shifted_spectrum(st, s0)                  # exact band-limited sub-pixel shift
        h_int, s_int = xcf.integer_peak(xcf.xcf_map(se, st))
        h, s = xcf.subpixel_peak(se, st, s_int, kappa=100)
        assert abs(s[0] - s0[0]) <= 0.005 + 1e-12 and abs(s[1] - s0[1]) <= 0.005 + 1e-12
        assert h >= h_int - 1e-15 and h <= 1.0 + 1e-12
        assert abs(xcf.rho_at(se, st, s) - h) < 1e-12


def test_subpixel_agrees_with_newton_on_analytic_gradient():
    # Equation 5: d|r|^2/dx0 from the spectrum; Newton's method on the
    # analytic gradient and Hessian of rho(s) finds the continuous maximum,
    # which the kappa = 100 grid must bracket to 0.5/kappa
    rng = np.random.default_rng(8)
    n = 64
    prm = Params()
    a = rng.normal(size=(n, n))
    b = np.roll(a, (3, -2), axis=(0, 1)) + 0.8 * rng.normal(size=(n, n))
    se, st = spectra.unit_spectrum(b, prm), spectra.unit_spectrum(a, prm)
    z = se * np.conj(st)
    f = spectra.signed_freq(n)
    fu, fv = np.meshgrid(f, f, indexing="ij")
    h_int, s_int = xcf.integer_peak(xcf.xcf_map(se, st))
    s = np.array(s_int, dtype=float)
    for _ in range(30):
        ph = z * np.exp(2j * np.pi * (fu * s[0] + fv * s[1]) / n)
        k = 2 * np.pi / n
        g = np.real(np.array([np.sum(1j * k * fu * ph), np.sum(1j * k * fv * ph)]))
        hess = np.real(np.array([[np.sum(-(k * fu) ** 2 * ph), np.sum(-(k * k) * fu * fv * ph)],
                                 [np.sum(-(k * k) * fu * fv * ph), np.sum(-(k * fv) ** 2 * ph)]]))
        s = s - np.linalg.solve(hess, g)
    assert np.max(np.abs(g)) < 1e-9
    h, sp = xcf.subpixel_peak(se, st, s_int, kappa=100)
    assert abs(sp[0] - s[0]) <= 0.005 + 1e-9 and abs(sp[1] - s[1]) <= 0.005 + 1e-9
    assert h <= xcf.rho_at(se, st, s) + 1e-12

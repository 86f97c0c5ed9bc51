"""Pins for oracle.split (the emulated split-precision correlation): the
rounding rules against closed forms, the two-product formulation against
the FFT-based windowed correlation of oracle.xcf, and the split error
against its analytic size."""

import numpy as np

from oracle import spectra, split, xcf
from oracle.params import Params


def test_fp16_round_toward_zero():
    one = 1.0
    x = np.array([one + 3 * 2.0 ** -12, -(one + 3 * 2.0 ** -12), 1000.7, 2.0 ** -20 * 1.9])
    h = split.rtz_f16(x)
    assert h[0] == 1.0 and h[1] == -1.0                     # round to nearest would give 1 + 2^-10
    assert h[2] == 1000.5                                      # FP16 step at 1000 is 0.5
    assert np.all(np.abs(h) <= np.abs(x))
    assert np.all(h.astype(np.float16).astype(np.float64) == h)
    assert split.rne_f16(np.array([one + 3 * 2.0 ** -12]))[0] == one + 2.0 ** -10


def test_bf16_round_to_nearest_even():
    x = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20, -(1 + 3 * 2.0 ** -8)])
    r = split.rne_bf16(x)
    assert r[0] == 1.0                                         # tie -> even
    assert r[1] == 1 + 2.0 ** -6                               # tie -> even
    assert r[2] == 1 + 2.0 ** -7                               # above the tie
    assert r[3] == -(1 + 2.0 ** -6)


def test_halves_reconstruct_the_operand():
    rng = np.random.default_rng(0)
    x = rng.normal(size=2000).astype(np.float32).astype(np.float64) * 37.0
    # relative bound, plus the FP16 subnormal spacing 2^-24 for tiny lo halves
    for fmt, rnd, bound, tiny in (("fp16", "rtz", 2.0 ** -20, 2.0 ** -24), ("bf16", "rne", 2.0 ** -16, 0.0)):
        hi, lo = split.split_operand(x, fmt, rnd)
        assert np.all(np.abs(x - (hi + lo)) <= bound * np.abs(x) + tiny), fmt


def _bands(n, k, seed):
    rng = np.random.default_rng(seed)
    b = 3 * n // 8
    rows = np.concatenate([np.arange(0, b + 1), np.arange(n - b, n)])
    full, band = [], []
    for _ in range(k):
        sp = spectra.unit_spectrum(rng.normal(size=(n, n)), Params())
        full.append(sp)
        band.append(sp[rows, :b + 1].T)                        # [v][kk]
    return full, band


def test_unrounded_products_equal_the_windowed_correlation():
    n, s = 64, 9
    full, band = _bands(n, 5, seed=1)
    got = split.emulated_scores(band[0], band[1:], n, s, None)
    ref = xcf.library_scores(full[0], full[1:], max_shift=s)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_split_error_has_the_expected_size():
    n, s = 64, 7
    full, band = _bands(n, 4, seed=2)
    ref = xcf.library_scores(full[0], full[1:], max_shift=s)
    err = {p: np.max(np.abs(split.emulated_scores(band[0], band[1:], n, s, p) - ref))
           for p in ("fp16x2", "bf16x2", "bf16")}
    assert err["fp16x2"] < 2e-6
    assert err["bf16x2"] < 2e-4
    assert 1e-5 < err["bf16"] < 5e-2
    assert err["fp16x2"] < err["bf16x2"] < err["bf16"]

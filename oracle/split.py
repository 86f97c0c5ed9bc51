"""Emulated split-precision correlation (oracle; test only).

The windowed correlation rho(s) = Re sum_{u,v} w_v Z(u, v)
exp(+2 pi i (u s_y + v s_x) / N) (Equations 3 and 6a on the stored
Hermitian half, w_0 = 1, w_v = 2; Z = E conj(T)) written as two products
with phase matrices, evaluated with every operand rounded the way the
split-precision reading rounds it:

* Z is scaled by 2^12 and rounded to FP32; each real operand x is split
  into 16-bit halves x = hi + lo: FP16 halves by rounding toward zero
  (hi = rtz(x), lo = rtz(x - hi)), BF16 halves by round-to-nearest-even;
* the phase matrices W1(u, s_y) = exp(2 pi i u s_y / N) and
  C(v, s_x) = w_v exp(2 pi i v s_x / N) are split with round-to-nearest-even
  in both formats;
* a product of split operands keeps hi*hi + hi*lo + lo*hi (plain BF16: the
  hi halves only, hi*hi);
* stage 1, A(s_y, v) = sum_u Z(u, v) W1(u, s_y), is rounded to FP32 and
  split like Z before stage 2, rho = Re sum_v A C, which is scaled back by
  2^-12.

Sums run in FP64, so the result differs from a kernel that accumulates in
FP32 only by the accumulation rounding, while its difference from the exact
correlation is the error that the split itself causes.  With rounding
switched off (`fmt=None`) it is the exact windowed correlation.
"""

import numpy as np

Z_SCALE = 4096.0


def rtz_f16(x):
    """Round to FP16 toward zero (values assumed inside the FP16 range)."""
    x = np.asarray(x, dtype=np.float64)
    h = x.astype(np.float16).astype(np.float64)
    over = np.abs(h) > np.abs(x)
    h[over] = np.nextafter(h[over].astype(np.float16), np.float16(0)).astype(np.float64)
    return h


def rne_f16(x):
    return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)


def rne_bf16(x):
    """Round FP32 values to BF16, nearest even (no NaN / overflow handling)."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def split_operand(x, fmt, rounding):
    """(hi, lo) halves of FP32 values x; rounding 'rtz' or 'rne'."""
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    if fmt == "fp16":
        r = rtz_f16 if rounding == "rtz" else rne_f16
    else:
        r = rne_bf16
    hi = r(x)
    lo = r((x - hi).astype(np.float32))
    return hi, lo


def split_product(a, b, fmt, two, ra, rb):
    """sum over the contracted index of a b with split operands: a [M][K], b [K][N]."""
    if fmt is None:
        return a @ b
    ah, al = split_operand(a, fmt, ra)
    bh, bl = split_operand(b, fmt, rb)
    out = ah @ bh
    if two:
        out = out + ah @ bl + al @ bh
    return out


def fp32(x, fmt):
    """Round to FP32 when emulating a split format (unchanged when fmt is None)."""
    return x if fmt is None else np.asarray(x).astype(np.float32).astype(np.float64)


def band_freqs(b):
    """Signed row frequencies u of the band rows and the columns v in [0, B]."""
    u = np.concatenate([np.arange(0, b + 1), np.arange(-b, 0)])
    return u, np.arange(0, b + 1)


def emulated_scores(band_e, band_t, n, max_shift, precision):
    """Windowed integer-peak score of pattern band_e against templates.

    band_e: complex [V][K] band spectrum of the pattern (v, kk order as
    returned by the binding's spectra_to_complex), band_t: [L][V][K].
    precision: 'fp16x2', 'bf16x2', 'bf16' or None (no rounding)."""
    b = 3 * n // 8
    u, v = band_freqs(b)
    s = np.arange(-max_shift, max_shift + 1)
    fmt = None if precision is None else ("fp16" if precision == "fp16x2" else "bf16")
    two = precision in ("fp16x2", "bf16x2")
    split_rounding = "rtz" if fmt == "fp16" else "rne"
    ang1 = 2 * np.pi * np.outer(u, s) / n                          # [K][S]
    w1r, w1i = np.cos(ang1), np.sin(ang1)
    wv = np.where(v == 0, 1.0, 2.0)
    ang2 = 2 * np.pi * np.outer(v, s) / n                          # [V][S]
    cr, ci = wv[:, None] * np.cos(ang2), wv[:, None] * np.sin(ang2)
    e = np.asarray(band_e).T                                        # [K][V]
    out = np.empty(len(band_t))
    for j, t in enumerate(band_t):
        z = Z_SCALE * e * np.conj(np.asarray(t).T)                  # [K][V]
        zr, zi = fp32(z.real, fmt), fp32(z.imag, fmt)
        # stage 1: A^T (V x S) = Z^T W1
        ar = (split_product(zr.T, w1r, fmt, two, split_rounding, "rne")
              - split_product(zi.T, w1i, fmt, two, split_rounding, "rne"))
        ai = (split_product(zr.T, w1i, fmt, two, split_rounding, "rne")
              + split_product(zi.T, w1r, fmt, two, split_rounding, "rne"))
        ar, ai = fp32(ar, fmt), fp32(ai, fmt)
        # stage 2: rho (s_y x s_x) = A C_r - A_i C_i
        rho = (split_product(ar.T, cr, fmt, two, split_rounding, "rne")
               - split_product(ai.T, ci, fmt, two, split_rounding, "rne")) / Z_SCALE
        out[j] = rho.max()
    return out

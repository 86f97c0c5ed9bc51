"""Training-data generator of the learned proposal, in FP64 (oracle; test only).

The proposal network is trained on patterns that the projection itself
generates: a random orientation and in-plane pattern-centre offset per
sample, the template projected there, scaled to a mean count level, Poisson
noise (in its normal approximation) plus Gaussian read noise that fixes the
signal-to-noise ratio, binned by block means to 64 x 64 and normalised.

The random numbers come from a counter-based generator, so that the device
and this oracle draw the same numbers without sharing code: Philox4x32-10
(Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2,
3", SC 2011), written here from its definition.  Counter assignment (the
interface both sides follow):

* sample s, orientation and x offset: counters (s_lo, s_hi, 1, 0) and
  (s_lo, s_hi, 2, 0); y offset: (s_lo, s_hi, 3, 0);
* noise of pixel k (row-major in the n x n pattern) of sample s:
  counter c = (s << 20) xor k, words (c_lo, c_hi, 4, 0);
* key = (seed_lo, seed_hi).

Uniforms in (0, 1] take 53 bits from two words, (a << 21) xor (b >> 11),
plus one half, over 2^53 (in double precision the top value rounds to
exactly 1; none is 0); normals come in pairs from the Box-Muller transform (Box and
Muller, 1958); orientations are Shoemake's uniform quaternions (Graphics
Gems III, 1992) from three uniforms.
"""

import numpy as np

from . import cnn, geometry, rotations

_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """ctr: uint64 array [..., 4] of 32-bit words; key: [..., 2].  Ten rounds
    of the Philox S-box (two 32 x 32 -> 64-bit products, their high halves
    xor-ed with the other words and the round key; the key bumped by the Weyl
    constants between rounds).  Returns uint64 [..., 4] of 32-bit words."""
    c = np.array(ctr, dtype=np.uint64) & _MASK32
    k = np.array(key, dtype=np.uint64) & _MASK32
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0, k1 = k[..., 0].copy(), k[..., 1].copy()
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK32
            k1 = (k1 + _W1) & _MASK32
        p0 = c0 * np.uint64(_M0)            # < 2^64: exact in uint64
        p1 = c2 * np.uint64(_M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=-1)


def _draw(counter, stream, seed):
    counter = np.asarray(counter, dtype=np.uint64)
    ctr = np.stack([counter & _MASK32, counter >> np.uint64(32),
                    np.full(counter.shape, stream, np.uint64), np.zeros(counter.shape, np.uint64)], axis=-1)
    key = np.array([seed & _MASK32, (seed >> 32) & _MASK32], dtype=np.uint64)
    return philox4x32_10(ctr, np.broadcast_to(key, counter.shape + (2,)))


def unit(a, b):
    """Uniform in (0, 1] from two 32-bit words: (53 bits + 1/2) / 2^53."""
    x = ((np.asarray(a, np.uint64) << np.uint64(21)) ^ (np.asarray(b, np.uint64) >> np.uint64(11)))
    x = x & np.uint64((1 << 53) - 1)
    return (x.astype(np.float64) + 0.5) / 2.0 ** 53


def box_muller(r):
    """Two standard normals from the four words r[..., 0:4]."""
    u1 = unit(r[..., 0], r[..., 1])
    u2 = unit(r[..., 2], r[..., 3])
    rad = np.sqrt(-2.0 * np.log(u1))
    return rad * np.cos(2 * np.pi * u2), rad * np.sin(2 * np.pi * u2)


def sample_setup(first, count, seed, pc, max_offset_px, n):
    """Orientations q [count, 4] (w >= 0) and pattern centres [count, 3] of
    samples first .. first + count - 1."""
    s = np.arange(first, first + count, dtype=np.uint64)
    r0, r1, r2 = _draw(s, 1, seed), _draw(s, 2, seed), _draw(s, 3, seed)
    u1, u2, u3 = unit(r0[:, 0], r0[:, 1]), unit(r0[:, 2], r0[:, 3]), unit(r1[:, 0], r1[:, 1])
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    q = np.stack([b * np.cos(2 * np.pi * u3), a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                  b * np.sin(2 * np.pi * u3)], axis=1)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    q = np.where(q[:, :1] < 0, -q, q)
    frac = max_offset_px / n
    ox = (2.0 * unit(r1[:, 2], r1[:, 3]) - 1.0) * frac
    oy = (2.0 * unit(r2[:, 0], r2[:, 1]) - 1.0) * frac
    pcs = np.stack([pc[0] + ox, pc[1] + oy, np.full(count, float(pc[2]))], axis=1)
    return q, pcs


def noisy_pattern(clean, s, seed, counts, snr):
    """The clean pattern scaled to `counts` mean counts, with Poisson noise in
    its normal approximation (std sqrt(value)) plus Gaussian noise of the
    variance that makes std(clean signal) / std(noise) = snr; if that
    variance would be negative, the count level is lowered to the one whose
    Poisson noise alone gives the SNR."""
    clean = np.asarray(clean, dtype=np.float64)
    n = clean.shape[0]
    mean = clean.mean()
    ct = clean.std() / mean if mean > 0 else 0.0
    c_eff = counts
    var_g = (counts * ct / snr) ** 2 - counts if ct > 0 else 0.0
    if var_g < 0:
        c_eff = (snr / ct) ** 2
        var_g = 0.0
    v = clean * (c_eff / mean if mean > 0 else 0.0)
    k = np.arange(n * n, dtype=np.uint64)
    z1, z2 = box_muller(_draw((np.uint64(s) << np.uint64(20)) ^ k, 4, seed))
    return v + np.sqrt(np.maximum(v, 0.0)) * z1.reshape(n, n) + np.sqrt(var_g) * z2.reshape(n, n)


def make_batch(master, pc, lib_q, n, count, first, seed, max_offset_px=5.0, counts=1000.0, snr=5.0):
    """Network inputs x [count, 64, 64], labels (nearest library orientation,
    None without a library) and orientations q [count, 4]."""
    q, pcs = sample_setup(first, count, seed, pc, max_offset_px, n)
    rs = rotations.quat_to_matrix(q)
    x = np.stack([cnn.network_input(noisy_pattern(geometry.project(master, rs[j], n, pcs[j]), first + j, seed,
                                                  counts, snr)) for j in range(count)])
    labels = None if lib_q is None else np.array([cnn.nearest_library(q[j], lib_q) for j in range(count)])
    return x, labels, q

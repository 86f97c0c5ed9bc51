"""Pins for oracle.generator (the learned proposal's training-data
generator): Philox4x32-10 against the published known-answer vectors, the
uniform and normal conversions, Shoemake's orientations against the Haar
measure of SO(3), and the noise model against its stated count level and
signal-to-noise ratio."""

import numpy as np

from oracle import generator as gen
from oracle import rotations as rot

# Known-answer vectors distributed with the Random123 library of the paper
# that defines Philox (Salmon et al., SC 2011): (counter, key) -> output.
KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


def test_philox_known_answers():
    for ctr, key, want in KAT:
        got = gen.philox4x32_10(np.array(ctr), np.array(key))
        assert [int(v) for v in got] == list(want)
    # vectorised over a batch of counters: each row as if alone
    ctrs = np.array([k[0] for k in KAT])
    keys = np.array([k[1] for k in KAT])
    assert np.array_equal(gen.philox4x32_10(ctrs, keys), np.array([k[2] for k in KAT], dtype=np.uint64))


def test_unit_range_and_ends():
    # (x + 1/2) / 2^53 for a 53-bit x: never 0 (the Box-Muller logarithm
    # needs u1 > 0); at the top, 2^53 - 1/2 is not a double and rounds to
    # even, 2^53, so the largest value is exactly 1 (harmless: log 1 = 0)
    lo = gen.unit(0, 0)
    hi = gen.unit(0xFFFFFFFF, 0xFFFFFFFF)
    assert lo == 0.5 / 2 ** 53 and hi == 1.0
    assert gen.unit(0xFFFFFFFF, 0xFFFFF000 - (1 << 12)) < 1.0
    # the 53 bits are the 32 of a followed by the top 21 of b
    assert gen.unit(1, 0) == (2 ** 21 + 0.5) / 2 ** 53
    assert gen.unit(0, 1 << 11) == 1.5 / 2 ** 53
    assert gen.unit(0, (1 << 11) - 1) == lo


def test_box_muller_moments():
    r = gen._draw(np.arange(200_000, dtype=np.uint64), 9, 1234)
    u = gen.unit(r[:, 0], r[:, 1])
    assert abs(u.mean() - 0.5) < 3e-3 and abs(u.var() - 1 / 12) < 1e-3
    z1, z2 = gen.box_muller(r)
    for z in (z1, z2):
        assert abs(z.mean()) < 0.01 and abs(z.var() - 1) < 0.015
        assert abs(np.mean(z ** 4) - 3) < 0.06                 # normal kurtosis
    assert abs(np.corrcoef(z1, z2)[0, 1]) < 0.01


def test_orientations_are_haar_uniform():
    # Uniform rotations: each quaternion component squared has mean 1/4, and
    # the rotation angle has density (1 - cos w) / pi on [0, pi], mean
    # pi / 2 + 2 / pi
    q, pcs = gen.sample_setup(0, 100_000, 77, (0.5, 0.5, 0.6), 5.0, 128)
    assert np.allclose(np.linalg.norm(q, axis=1), 1, atol=1e-14) and np.all(q[:, 0] >= 0)
    assert np.all(np.abs((q ** 2).mean(axis=0) - 0.25) < 5e-3)
    w = 2 * np.arccos(np.clip(q[:, 0], -1, 1))
    assert abs(w.mean() - (np.pi / 2 + 2 / np.pi)) < 0.01
    # a rotation and its matrix agree (w >= 0 canonical form)
    r = rot.quat_to_matrix(q[:5])
    assert np.allclose(np.einsum("kij,kil->kjl", r, r), np.eye(3), atol=1e-14)
    # pattern-centre offsets uniform in +-5 px, PCz untouched
    off = (pcs[:, :2] - 0.5) * 128
    assert np.all(np.abs(off) < 5) and np.all(np.abs(off.mean(axis=0)) < 0.05)
    assert np.all(np.abs(off.var(axis=0) - 25 / 3) < 0.1) and np.all(pcs[:, 2] == 0.6)
    # counter-based: a sub-range reproduces the same samples
    q2, pcs2 = gen.sample_setup(500, 10, 77, (0.5, 0.5, 0.6), 5.0, 128)
    assert np.array_equal(q2, q[500:510]) and np.array_equal(pcs2, pcs[500:510])


def test_noise_model_count_level_and_snr():
    # A smooth clean image of contrast c_t = std / mean: after scaling, the
    # mean is the count level, and std(scaled clean) / std(noise) = SNR.
    n = 512
    jj, ii = np.mgrid[0:n, 0:n]
    clean = 2.0 + np.sin(2 * np.pi * ii / 64) * np.cos(2 * np.pi * jj / 96)
    for counts, snr in ((1000.0, 5.0), (1e4, 2.0)):
        noisy = gen.noisy_pattern(clean, 3, 99, counts, snr)
        scaled = clean * counts / clean.mean()
        noise = noisy - scaled
        assert abs(noisy.mean() - counts) < 0.01 * counts
        assert abs(scaled.std() / noise.std() - snr) < 0.02 * snr
        # Poisson part: the noise variance grows with the local count level
        lo, hi = scaled < np.percentile(scaled, 20), scaled > np.percentile(scaled, 80)
        assert noise[hi].var() > noise[lo].var()
    # Poisson alone cannot reach a high SNR at 100 counts: the count level is
    # raised to the one whose Poisson noise gives that SNR
    noisy = gen.noisy_pattern(clean, 4, 99, 100.0, 40.0)
    ct = clean.std() / clean.mean()
    assert abs(noisy.mean() - (40.0 / ct) ** 2) < 0.01 * (40.0 / ct) ** 2

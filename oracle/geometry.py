"""Detector geometry and gnomonic template projection in FP64 (oracle; test only).

Section "SO(3) Library Generation": a template is the gnomonic projection of
a spherical master pattern for a crystal orientation, screen size and
pattern centre, with intensities taken from the master by bicubic
interpolation.  Frame conventions are deferred by the paper to a cited
reference; the readings used here:

* image [row j][col i], pixel centre at (i + 1/2, j + 1/2) px;
* pattern centre (PCx, PCy, PCz) in screen widths (footnote on the PC in
  section "Fast Fourier Transform"): PCx from the left edge, PCy from the
  top edge, PCz = source-to-screen distance over screen width;
* detector frame x = +column, y = +row, z = from the source to the screen;
  pixel ray d = normalise((i + 1/2)/N - PCx, (j + 1/2)/N - PCy, PCz);
* crystal direction c = R d;
* master: H x W equirectangular grid, row r at polar angle (r + 1/2) pi / H
  from crystal +z, column q at azimuth 2 pi q / W from +x toward +y; Keys
  bicubic interpolation (a = -0.5), periodic in azimuth, rows clamped.
  (The paper stores its master stereographically; the equirectangular grid
  is the format of the synthetic master used here.)
"""

import numpy as np


def crop_pc(pcx, width, new_width):
    """PCx after a centred crop from `width` to `new_width` pixels.

    Footnote on the PC (section "Fast Fourier Transform"): PCx is a fraction
    of screen width, so cropping changes it; the worked example crops 200 to
    128 px and moves PCx from 0.4 to about 0.34.
    """
    return (pcx * width - (width - new_width) / 2.0) / new_width


def pixel_rays(n, pc):
    """Unit ray directions d[j, i, :] in the detector frame for an n x n screen."""
    pcx, pcy, pcz = (float(v) for v in pc)
    c = (np.arange(n, dtype=np.float64) + 0.5) / n
    x = np.broadcast_to(c[None, :] - pcx, (n, n))
    y = np.broadcast_to(c[:, None] - pcy, (n, n))
    z = np.full((n, n), pcz)
    d = np.stack([x, y, z], axis=-1)
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


def keys_weights(t, a=-0.5):
    """Keys cubic-convolution weights for taps at offsets -1, 0, 1, 2 from
    floor(x), where t = x - floor(x) in [0, 1)."""
    def w(s):
        s = np.abs(s)
        return np.where(
            s <= 1.0,
            (a + 2) * s ** 3 - (a + 3) * s ** 2 + 1,
            np.where(s < 2.0, a * s ** 3 - 5 * a * s ** 2 + 8 * a * s - 4 * a, 0.0),
        )
    return np.stack([w(1 + t), w(t), w(1 - t), w(2 - t)], axis=-1)


def master_lookup(master, c):
    """Bicubic lookup of the equirectangular master at unit crystal directions c[..., 3]."""
    master = np.asarray(master, dtype=np.float64)
    h, w = master.shape
    theta = np.arccos(np.clip(c[..., 2], -1.0, 1.0))
    phi = np.mod(np.arctan2(c[..., 1], c[..., 0]), 2 * np.pi)
    v = theta * h / np.pi - 0.5
    u = phi * w / (2 * np.pi)
    v = np.clip(v, 0.0, h - 1.0)
    v0 = np.floor(v)
    u0 = np.floor(u)
    wv = keys_weights(v - v0)
    wu = keys_weights(u - u0)
    v0 = v0.astype(np.int64)
    u0 = u0.astype(np.int64)
    out = np.zeros(c.shape[:-1])
    for a in range(4):
        rows = np.clip(v0 + a - 1, 0, h - 1)
        for b in range(4):
            cols = np.mod(u0 + b - 1, w)
            out += wv[..., a] * wu[..., b] * master[rows, cols]
    return out


def crystal_directions(r, n, pc):
    """c = R d for every pixel ray, shape (n, n, 3)."""
    return pixel_rays(n, pc) @ np.asarray(r, dtype=np.float64).T


def project(master, r, n, pc):
    """Template for orientation matrix r (3x3) on an n x n screen at pattern centre pc."""
    return master_lookup(master, crystal_directions(r, n, pc))


def project_fn(fn, r, n, pc):
    """Same geometry with the master given as a function of crystal direction."""
    return fn(crystal_directions(r, n, pc))

"""Synthetic cubic master pattern (input generator).

Kikuchi-band model on the unit sphere of crystal directions c:

    M(c) = 1 + sum_F w_F sum_{n in F/+-} exp(-1/2 (asin(c.n) / sigma_F)^2)

over the plane families F = {111}, {200}, {220}, {311}, with
sigma_F = k_w theta_B,F, theta_B = asin(lambda/(2a) |hkl|) (lambda/a = 0.0244,
a nickel-like lattice at 20 kV), k_w = 1.75, and structure-factor-like weights
1.0, 0.8, 0.55, 0.45.  The grid is equirectangular: row r at polar angle
(r + 1/2) pi / H from +z, column q at azimuth 2 pi q / W from +x toward +y.
"""

import itertools

import numpy as np

FAMILIES = ((1, 1, 1), (2, 0, 0), (2, 2, 0), (3, 1, 1))
WEIGHTS = (1.0, 0.8, 0.55, 0.45)


def family_normals(hkl):
    """Distinct plane normals of a cubic family, one of each +-n pair."""
    out = []
    for perm in set(itertools.permutations(hkl)):
        for signs in itertools.product((1, -1), repeat=3):
            v = np.array(perm, dtype=np.float64) * signs
            if not np.any(v):
                continue
            v = v / np.linalg.norm(v)
            first = v[np.nonzero(np.abs(v) > 1e-12)[0][0]]
            if first < 0:
                v = -v
            if not any(np.allclose(v, u) for u in out):
                out.append(v)
    return np.array(out)


def band_table(lam_over_a=0.0244, k_w=1.75):
    normals, sigmas, weights = [], [], []
    for hkl, w in zip(FAMILIES, WEIGHTS):
        g = np.linalg.norm(hkl)
        theta_b = np.arcsin(0.5 * lam_over_a * g)
        ns = family_normals(hkl)
        normals.append(ns)
        sigmas += [k_w * theta_b] * len(ns)
        weights += [w] * len(ns)
    return np.concatenate(normals), np.array(sigmas), np.array(weights)


def band_intensity(c, lam_over_a=0.0244, k_w=1.75, xp=np):
    """Analytic M(c) for unit directions c[..., 3] (numpy or torch via xp)."""
    normals, sigmas, weights = band_table(lam_over_a, k_w)
    if xp is np:
        c = np.asarray(c, dtype=np.float64)
        dots = np.clip(c @ normals.T, -1.0, 1.0)
        return 1.0 + np.sum(weights * np.exp(-0.5 * (np.arcsin(dots) / sigmas) ** 2), axis=-1)
    import torch
    nt = torch.as_tensor(normals, dtype=c.dtype, device=c.device)
    st = torch.as_tensor(sigmas, dtype=c.dtype, device=c.device)
    wt = torch.as_tensor(weights, dtype=c.dtype, device=c.device)
    dots = torch.clamp(c @ nt.T, -1.0, 1.0)
    return 1.0 + torch.sum(wt * torch.exp(-0.5 * (torch.asin(dots) / st) ** 2), dim=-1)


def band_master(h=256, w=256, lam_over_a=0.0244, k_w=1.75):
    """float32 [h, w] equirectangular master."""
    theta = (np.arange(h) + 0.5) * np.pi / h
    phi = 2 * np.pi * np.arange(w) / w
    st, ct = np.sin(theta)[:, None], np.cos(theta)[:, None]
    c = np.stack([st * np.cos(phi)[None, :], st * np.sin(phi)[None, :], np.broadcast_to(ct, (h, w))], axis=-1)
    return band_intensity(c, lam_over_a, k_w).astype(np.float32)

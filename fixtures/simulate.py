"""Simulated experimental patterns (input generator; torch, CPU or GPU).

Forward model of the experiment: each pixel of an N x N screen sees the
crystal direction c = R d along its ray d (detector frame: x = +column,
y = +row, z = source to screen; pattern centre in screen widths, PCx from
the left, PCy from the top), and records the analytic band intensity M(c)
of ``fixtures.master`` scaled to a mean count level, plus noise.  A per
pattern in-plane pattern-centre offset of (dx, dy) px translates the
pattern by (dx, dy) px.
"""

import numpy as np
import torch

from .master import band_intensity


def quat_matrices(q, dtype, device):
    q = torch.as_tensor(np.asarray(q), dtype=dtype, device=device)
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def clean_patterns(quats, n, pcs, dtype=torch.float64, device="cpu", chunk=64):
    """Noise-free analytic patterns [P, n, n] for orientations `quats` [P, 4]
    and pattern centres `pcs` [P, 3]."""
    p = len(quats)
    rmat = quat_matrices(quats, dtype, device)
    pcs_t = torch.as_tensor(np.asarray(pcs), dtype=dtype, device=device)
    grid = (torch.arange(n, dtype=dtype, device=device) + 0.5) / n
    out = torch.empty((p, n, n), dtype=dtype, device=device)
    for s in range(0, p, chunk):
        e = min(p, s + chunk)
        pc = pcs_t[s:e]
        dx = grid[None, None, :] - pc[:, 0, None, None]
        dy = grid[None, :, None] - pc[:, 1, None, None]
        dz = pc[:, 2, None, None].expand(-1, n, n)
        d = torch.stack([dx.expand(-1, n, n), dy.expand(-1, n, n), dz], dim=-1)
        d = d / torch.linalg.norm(d, dim=-1, keepdim=True)
        c = torch.einsum("pij,pyxj->pyxi", rmat[s:e], d)
        out[s:e] = band_intensity(c, xp=torch)
    return out


def add_noise(clean, model, gen):
    """model: ("none",) | ("poisson", counts) | ("poisson_gauss", counts, snr)."""
    kind = model[0]
    mean = clean.mean(dim=(1, 2), keepdim=True)
    if kind == "none":
        return clean
    if kind == "poisson":
        lam = clean * (model[1] / mean)
        return torch.poisson(lam, generator=gen)
    if kind == "poisson_gauss":
        counts, snr = model[1], model[2]
        ct = clean.std(dim=(1, 2), keepdim=True) / mean           # contrast per pattern
        var_g = (counts * ct / snr) ** 2 - counts
        c_eff = torch.where(var_g < 0, (snr / ct) ** 2, torch.full_like(ct, counts))
        var_g = torch.clamp(var_g, min=0.0)
        lam = clean * (c_eff / mean)
        noisy = torch.poisson(lam, generator=gen)
        g = torch.randn(clean.shape, generator=gen, dtype=clean.dtype, device=clean.device)
        return noisy + g * torch.sqrt(var_g)
    raise ValueError(kind)


def simulate_patterns(quats, n, pcs, noise=("none",), seed=0, device="cpu", dtype=torch.float64):
    """float32 numpy/torch patterns [P, n, n]; returned on `device` as float32."""
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    clean = clean_patterns(quats, n, pcs, dtype=dtype, device=device)
    return add_noise(clean, noise, gen).to(torch.float32)

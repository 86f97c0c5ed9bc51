"""The workloads, as seeded synthetic inputs.

tiny      16 patterns at 64^2, orientations uniform in SO(3), pattern centre
          (0.5, 0.5, 0.6) with a uniform +-3 px in-plane offset per pattern,
          Poisson noise at 100 counts/px; library of 500 orientations uniform
          in the cubic fundamental zone.
map       a 100 x 100 map (10,000 patterns) at 128^2: 20 Voronoi grains with
          uniform orientations and <= 1 deg intragranular spread, +-5 px
          pattern-centre offsets, Poisson (1000 counts) plus Gaussian noise at
          SNR 5; library of 4,000 fundamental-zone orientations.  Its scale
          mirrors the paper's deformed alpha-iron map (9,130 patterns at
          128^2, section "Deformed alpha-Fe Dataset").
map256    the same map at 256^2.
drift     the map with a pattern centre drifting linearly across it (the
          spans of the paper's wide silicon map), one library at the nominal
          PC.
ragged    20,000 patterns with sizes drawn from {64, 96, 128, 160} (25 % each,
          shuffled), otherwise as `map`; library of 8,000.

Every generator takes smaller sizes for tests; `seed` fixes everything.
"""

import numpy as np
import torch

from .master import band_master
from .orient import random_quats, random_fz_quats, perturb_quats, voronoi_map
from .simulate import simulate_patterns

PCZ = 0.6


def _offsets(rng, p, max_px, n, integer=False):
    off = rng.uniform(-max_px, max_px, size=(p, 2))
    if integer:
        off = np.round(off)
    pcs = np.empty((p, 3))
    pcs[:, 0] = 0.5 + off[:, 0] / n
    pcs[:, 1] = 0.5 + off[:, 1] / n
    pcs[:, 2] = PCZ
    return pcs, off


def tiny(seed=1, p=16, n=64, l=500, integer_offsets=False, device="cpu"):
    rng = np.random.default_rng(seed)
    master = band_master()
    true_q = random_quats(rng, p)
    pcs, off = _offsets(rng, p, 3.0, n, integer_offsets)
    lib_q = random_fz_quats(rng, l)
    pats = simulate_patterns(true_q, n, pcs, ("poisson", 100.0), seed=seed + 1000, device=device)
    return dict(master=master, patterns=pats, pcs=pcs, offsets=off, true_q=true_q, lib_q=lib_q,
                n=n, pc=(0.5, 0.5, PCZ))


def map_grid(seed=2, rows=100, cols=100, n=128, l=4000, n_grains=20, device="cpu",
             noise=("poisson_gauss", 1000.0, 5.0), dtype=torch.float64):
    rng = np.random.default_rng(seed)
    master = band_master()
    gid = voronoi_map(rng, rows, cols, n_grains)
    grain_q = random_quats(rng, n_grains)
    true_q = perturb_quats(rng, grain_q[gid], 1.0)
    p = rows * cols
    pcs, off = _offsets(rng, p, 5.0, n)
    lib_q = random_fz_quats(rng, l)
    pats = simulate_patterns(true_q, n, pcs, noise, seed=seed + 1000, device=device, dtype=dtype)
    return dict(master=master, patterns=pats, pcs=pcs, offsets=off, true_q=true_q, lib_q=lib_q,
                n=n, pc=(0.5, 0.5, PCZ), grain=gid)


def drift_map(seed=5, rows=100, cols=100, n=128, l=4000, n_grains=20, span=(0.13, 0.08, 0.02), device="cpu",
              noise=("poisson_gauss", 1000.0, 5.0), dtype=torch.float64):
    """The map workload with a pattern centre that drifts across the map:
    pcx spans 0.13 screen widths along a row and pcy 0.08 down a column
    (the spans of the paper's wide silicon map, 0.39-0.52 and 0.11-0.19),
    pcz 0.02 down a column, linear in the beam position and centred on the
    nominal (0.5, 0.5, 0.6) at the map centre.  `model` holds the affine
    coefficients (pc0, d_col, d_row, col0, row0, width); `pcs` are the true
    per-point centres the patterns were simulated at."""
    rng = np.random.default_rng(seed)
    master = band_master()
    gid = voronoi_map(rng, rows, cols, n_grains)
    grain_q = random_quats(rng, n_grains)
    true_q = perturb_quats(rng, grain_q[gid], 1.0)
    pc0 = (0.5, 0.5, PCZ)
    d_col = (span[0] / max(cols - 1, 1), 0.0, 0.0)
    d_row = (0.0, span[1] / max(rows - 1, 1), span[2] / max(rows - 1, 1))
    col0, row0 = (cols - 1) / 2.0, (rows - 1) / 2.0
    rr, cc = np.meshgrid(np.arange(rows, dtype=np.float64), np.arange(cols, dtype=np.float64), indexing="ij")
    pcs = np.stack([pc0[0] + (cc - col0) * d_col[0], pc0[1] + (rr - row0) * d_row[1],
                    pc0[2] + (rr - row0) * d_row[2]], axis=-1).reshape(-1, 3)
    lib_q = random_fz_quats(rng, l)
    pats = simulate_patterns(true_q, n, pcs, noise, seed=seed + 1000, device=device, dtype=dtype)
    return dict(master=master, patterns=pats, pcs=pcs, true_q=true_q, lib_q=lib_q, n=n, pc=pc0, grain=gid,
                model=dict(pc0=pc0, d_col=d_col, d_row=d_row, col0=col0, row0=row0, width=cols))


def ragged(seed=4, p=20000, l=8000, sizes=(64, 96, 128, 160), device="cpu"):
    rng = np.random.default_rng(seed)
    master = band_master()
    ns = np.repeat(np.array(sizes), int(np.ceil(p / len(sizes))))[:p]
    rng.shuffle(ns)
    true_q = random_quats(rng, p)
    off = rng.uniform(-5.0, 5.0, size=(p, 2))
    pcs = np.stack([0.5 + off[:, 0] / ns, 0.5 + off[:, 1] / ns, np.full(p, PCZ)], axis=1)
    lib_q = random_fz_quats(rng, l)
    pats = []
    for s in sizes:
        idx = np.nonzero(ns == s)[0]
        if idx.size:
            pats.append((idx, simulate_patterns(true_q[idx], int(s), pcs[idx],
                                                ("poisson_gauss", 1000.0, 5.0), seed=seed + s, device=device)))
    return dict(master=master, sizes=ns, pattern_sets=pats, pcs=pcs, true_q=true_q, lib_q=lib_q,
                pc=(0.5, 0.5, PCZ))


def pack_ragged(cfg, device="cpu", dtype=torch.float32):
    """Packs a ragged workload into one flat buffer in pattern order:
    returns (data [sum n_p^2], offsets [P] int64 element offsets, sizes [P])."""
    ns = np.asarray(cfg["sizes"], dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(ns * ns)[:-1]]).astype(np.int64)
    data = torch.empty(int((ns * ns).sum()), dtype=dtype, device=device)
    for idx, pats in cfg["pattern_sets"]:
        s = int(ns[idx[0]])
        flat = pats.to(device=device, dtype=dtype).reshape(len(idx), s * s)
        pos = torch.as_tensor(offsets[idx], device=device)[:, None] + torch.arange(s * s, device=device)[None, :]
        data[pos.reshape(-1)] = flat.reshape(-1)
    return data, offsets, ns.astype(np.int32)


def ragged_pattern(cfg, i):
    """Pattern i of a ragged workload as a host array."""
    for idx, pats in cfg["pattern_sets"]:
        j = np.nonzero(idx == i)[0]
        if j.size:
            return pats[int(j[0])].cpu().numpy()
    raise IndexError(i)

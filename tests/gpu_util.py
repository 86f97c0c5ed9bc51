"""Helpers shared by the GPU tests (loading the built library, moving data)."""

import os

import numpy as np
import torch


def tm():
    import paper_1807_11313_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_1807_11313_amd import build
        build.build()
    pkg.lib()
    return pkg


def dev(x, dtype=None):
    t = torch.as_tensor(np.asarray(x) if not isinstance(x, torch.Tensor) else x)
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0").contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def banner(msg):
    print("[gpu] " + msg, flush=True)


def band_rows(n):
    """Half-width B of the band and the frequency u of each stored band row."""
    b = 3 * n // 8
    return b, np.concatenate([np.arange(0, b + 1), np.arange(-b, 0)]) % n


def oracle_spectra(imgs, n, prm=None):
    """Unit-energy spectra of the given images computed by the oracle, rounded
    once to float32, in three forms holding the same values: the device's band
    input (float32 [K][(2B+1)(B+1)*2]: row kk = frequency u, column v in
    [0, B], re / im interleaved), complex band arrays [K][v][kk] and full-grid
    spectra [K][n][n] (Hermitian completion of the columns v < 0).  Both
    sides of a stage test then start from identical inputs that come from the
    oracle, never from the device."""
    from oracle import spectra as ospec
    from oracle.params import Params
    prm = prm or Params()
    b, u = band_rows(n)
    full = np.stack([ospec.unit_spectrum(np.asarray(x, dtype=np.float64), prm) for x in imgs])
    kkv = full[:, u, :b + 1]
    f32 = np.stack([kkv.real, kkv.imag], axis=-1).astype(np.float32)
    kkv32 = f32[..., 0].astype(np.float64) + 1j * f32[..., 1].astype(np.float64)
    full32 = np.zeros_like(full)
    full32[:, u, :b + 1] = kkv32
    for v in range(1, b + 1):
        full32[:, (-u) % n, n - v] = np.conj(kkv32[:, :, v])
    return dev(f32.reshape(len(imgs), -1)), np.swapaxes(kkv32, 1, 2), full32


def oracle_templates(master, q, n, pc):
    """Templates projected by the oracle (FP64) for orientations q [L, 4]."""
    from oracle import geometry as ogeo
    from oracle import rotations as orot
    return np.stack([ogeo.project(master, r, n, pc) for r in orot.quat_to_matrix(np.asarray(q))])


def fallback_tau(t, val, q_true, pcs, master, pc, lq, percentile=1.0, max_error_deg=1.0):
    """The proposal's fallback threshold: the given percentile of the
    exhaustive search's integer peak height (the score the pruned search
    compares with it) among the correctly indexed validation patterns, those
    whose refined orientation lies within max_error_deg of the truth.
    Returns (tau, fraction correctly indexed)."""
    from oracle import rotations
    ex = t.index_patterns(val, master, pc, lq, scores=True)
    h_int = host(ex.pop("scores").max(dim=1).values)
    rf = t.refine_from_match(val, master, pc, ex["best_q"], ex["shift"], pc_per=dev(pcs))
    q = host(rf["q"])
    err = np.rad2deg([rotations.disorientation_q(q[i], q_true[i]) for i in range(len(q))])
    ok = err < max_error_deg
    return float(np.percentile(h_int[ok], percentile)), float(ok.mean())

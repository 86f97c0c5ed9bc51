"""The map workloads at their full size (10,000 patterns of 128^2 against
4,000 library templates searched over all shifts, and the same map at 256^2
searched by the FP16 hi + lo DFT-GEMM over |s| <= 15 px: the launch
configurations the bench times), checked on sampled patterns that the FP64
oracle indexes and refines one by one from the same inputs.

* Library index: the oracle's, bit-exact outside the near-tie rule
  (tau_tie = 2e-4); inside it the GPU's pick scores within tau_tie of the
  oracle's best.
* Peak height 1e-4, sub-pixel shift 0.02 px (where the picks agree).
* Refinement from the GPU's picks with per-pattern pattern centres: the
  oracle's orientation to 0.05 deg.
"""

import numpy as np
import pytest
import torch

import oracle
from fixtures import configs
from oracle import pipeline, rotations

from .gpu_util import banner, dev, host, tm

pytestmark = pytest.mark.gpu

TAU_TIE = 2e-4
SAMPLE = 8


def test_map_workload_sampled_against_oracle():
    banner("full-size map 10,000 x 4,000 at 128^2, sampled against the oracle")
    t = tm()
    cfg = configs.map_grid(device="cuda:0", dtype=torch.float32)
    pats = cfg["patterns"].contiguous()
    assert tuple(pats.shape) == (10000, 128, 128) and len(cfg["lib_q"]) == 4000
    master, lq = dev(cfg["master"]), dev(cfg["lib_q"])
    res = t.index_patterns(pats, master, cfg["pc"], lq)
    rr = t.refine_orientations(pats, master, cfg["pc"], res["best_q"], pc_per=dev(cfg["pcs"]))
    best_all = host(res["best_idx"])
    h_all, s_all, q_all = host(res["peak_h"]), host(res["shift"]), host(rr["q"])
    assert np.all((best_all >= 0) & (best_all < 4000))

    idx = np.sort(np.random.default_rng(11).choice(len(best_all), SAMPLE, replace=False))
    sample = pats[idx].double().cpu().numpy()
    prm = oracle.Params()
    banner("oracle: 4,000 library spectra and %d full library scans" % SAMPLE)
    lib_spec = pipeline.library_spectra(cfg["master"], cfg["lib_q"], 128, cfg["pc"], prm)
    ref = pipeline.index_patterns(sample, cfg["master"], cfg["pc"], cfg["lib_q"], prm, lib_spec=lib_spec,
                                  return_scores=True)
    best = best_all[idx]
    for a in range(SAMPLE):
        if ref["gap"][a] > TAU_TIE:
            assert best[a] == ref["best_idx"][a], (idx[a], best[a], ref["best_idx"][a])
        else:
            assert ref["scores"][a][best[a]] >= ref["h_int"][a] - TAU_TIE
    same = best == ref["best_idx"]
    assert np.max(np.abs(h_all[idx][same] - ref["peak_h"][same])) < 1e-4
    assert np.max(np.abs(s_all[idx][same] - ref["shift"][same])) <= 0.02 + 1e-6

    banner("oracle: refinement of the sampled patterns")
    rref = pipeline.refine_orientations(sample, cfg["master"], cfg["pcs"][idx], cfg["lib_q"][best], prm)
    d = np.rad2deg([rotations.disorientation_q(a, b) for a, b in zip(q_all[idx], rref["q"])])
    assert np.max(d) < 0.05, d


def test_map256_dftgemm_sampled_against_oracle():
    # the same map at 256^2, searched with the FP16 hi + lo DFT-GEMM over
    # |s| <= 15 px (tolerance of the FP32 path: scores 1e-4, tau = 2e-4)
    banner("full-size map at 256^2, DFT-GEMM FP16x2, sampled against the oracle")
    t = tm()
    s, sample_n = 15, 4
    cfg = configs.map_grid(n=256, device="cuda:0", dtype=torch.float32)
    pats = cfg["patterns"].contiguous()
    assert tuple(pats.shape) == (10000, 256, 256)
    master, lq = dev(cfg["master"]), dev(cfg["lib_q"])
    prm = t.params_default(precision=1, max_shift=s)
    res = t.index_patterns(pats, master, cfg["pc"], lq, prm=prm)
    rr = t.refine_orientations(pats, master, cfg["pc"], res["best_q"], pc_per=dev(cfg["pcs"]), prm=prm)
    best_all = host(res["best_idx"])
    h_all, s_all, q_all = host(res["peak_h"]), host(res["shift"]), host(rr["q"])

    idx = np.sort(np.random.default_rng(12).choice(len(best_all), sample_n, replace=False))
    sample = pats[idx].double().cpu().numpy()
    oprm = oracle.Params(max_shift=s)
    banner("oracle: 4,000 library spectra at 256^2 and %d windowed library scans" % sample_n)
    lib_spec = pipeline.library_spectra(cfg["master"], cfg["lib_q"], 256, cfg["pc"], oprm)
    ref = pipeline.index_patterns(sample, cfg["master"], cfg["pc"], cfg["lib_q"], oprm, lib_spec=lib_spec,
                                  return_scores=True)
    best = best_all[idx]
    for a in range(sample_n):
        if ref["gap"][a] > 2e-4:
            assert best[a] == ref["best_idx"][a], (idx[a], best[a], ref["best_idx"][a])
        else:
            assert ref["scores"][a][best[a]] >= ref["h_int"][a] - 2e-4
    same = best == ref["best_idx"]
    assert np.max(np.abs(h_all[idx][same] - ref["peak_h"][same])) < 1e-4
    assert np.max(np.abs(s_all[idx][same] - ref["shift"][same])) <= 0.02 + 1e-6

    banner("oracle: refinement of the sampled patterns")
    rref = pipeline.refine_orientations(sample, cfg["master"], cfg["pcs"][idx], cfg["lib_q"][best], oprm)
    d = np.rad2deg([rotations.disorientation_q(a, b) for a, b in zip(q_all[idx], rref["q"])])
    assert np.max(d) < 0.05, d

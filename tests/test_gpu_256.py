"""Parity at 256 x 256 (the precision workload's size) against the FP64 oracle.

At this size the spectra run as three passes (rows, columns, scale), the
library search runs only as split-precision DFT-GEMMs on MFMA, and every
integer peak is an exact evaluation over a shift window.  Tolerances are the
ones the smaller sizes use: unit-energy spectra 2e-6 per coefficient;
windowed integer peak bit-exact in position, 5e-6 in height; sub-pixel
height 1e-5 and shift 0.02 px; search scores per precision as in the GEMM
tests (FP16 hi + lo 1e-4, BF16 hi + lo 1e-3, BF16 3e-2); refined
orientation 0.05 deg.
"""

import numpy as np
import pytest

import oracle
from fixtures import band_master, configs, random_quats, simulate_patterns
from oracle import pipeline, rotations
from oracle import spectra as ospec
from oracle import xcf as oxcf
from oracle.params import Params as OParams

from .gpu_util import banner, dev, host, oracle_spectra, oracle_templates, tm

pytestmark = pytest.mark.gpu

N = 256
TOL = {0: 5e-6, 1: 1e-4, 2: 1e-3, 3: 3e-2}


def _pats(k, seed, offsets=5.0):
    rng = np.random.default_rng(seed)
    q = random_quats(rng, k)
    off = rng.uniform(-offsets, offsets, size=(k, 2))
    pcs = np.stack([0.5 + off[:, 0] / N, 0.5 + off[:, 1] / N, np.full(k, 0.6)], 1)
    return simulate_patterns(q, N, pcs, ("poisson", 200.0), seed=seed).numpy()


@pytest.mark.parametrize("window", [1, 0])
def test_spectra256_match_oracle(window):
    banner("spectra n=256 window=%d" % window)
    t = tm()
    pats = _pats(3, seed=5 + window)
    # a constant image has zero variance: its spectrum is all zeros
    pats = np.concatenate([pats, np.full((1, N, N), 7.0, np.float32)])
    spec, en = t.pattern_spectra(dev(pats), t.params_default(window=window), energy=True)
    band = t.spectra_to_complex(spec, N)
    prm = OParams(window=bool(window))
    for k in range(3):
        ref, e = ospec.filtered_spectrum(pats[k].astype(np.float64), prm)
        assert np.max(np.abs(t.band_to_full(band[k], N) - ref / np.sqrt(e))) < 2e-6
        assert abs(host(en)[k] / e - 1.0) < 2e-5
    assert np.all(band[3] == 0)


def test_window_peak256_matches_oracle():
    banner("window peak n=256")
    t = tm()
    pats = _pats(4, seed=11, offsets=7.0)
    spec, _, full = oracle_spectra(pats, N)
    pairs = ((0, 1), (1, 2), (2, 3), (3, 0), (2, 2))
    pi = dev(np.array([a for a, _ in pairs], np.int32))
    li = dev(np.array([b for _, b in pairs], np.int32))
    for s in (0, 5, 15):
        h, sh = t.xcf_peak(spec, spec, pi, li, N, t.params_default(max_shift=s))
        h, sh = host(h), host(sh)
        for k, (a, b) in enumerate(pairs):
            ref = oxcf.xcf_map(full[a], full[b])
            hr, sr = oxcf.integer_peak(ref, max_shift=s)
            assert (sh[k][1], sh[k][0]) == sr, (s, k)
            assert abs(h[k] - hr) < 5e-6


def test_size256_limits():
    t = tm()
    import paper_1807_11313_amd as pkg
    spec = t.pattern_spectra(dev(_pats(1, seed=2)))
    with pytest.raises(pkg.EbsdError):            # no full-map transform at 256
        t.xcf_peak(spec, spec, None, None, N, t.params_default(max_shift=3), want_map=True)
    with pytest.raises(pkg.EbsdError):            # every cyclic shift needs the map
        t.xcf_peak(spec, spec, None, None, N)
    with pytest.raises(pkg.EbsdError):            # the FFT search is not built at 256
        t.xcf_scores(spec, spec, N, t.params_default(max_shift=3, form=1))
    with pytest.raises(pkg.EbsdError):            # the exact DFT form needs a window
        t.xcf_scores(spec, spec, N, t.params_default(form=3))
    with pytest.raises(pkg.EbsdError):            # and runs in FP32 only
        t.xcf_scores(spec, spec, N, t.params_default(form=3, precision=1, max_shift=3))


def test_subpixel256_matches_oracle():
    banner("subpixel n=256")
    t = tm()
    pats = _pats(3, seed=21)
    spec, _, full = oracle_spectra(pats, N)
    pairs = ((0, 1), (1, 2), (2, 0))
    pi = dev(np.array([a for a, _ in pairs], np.int32))
    li = dev(np.array([b for _, b in pairs], np.int32))
    prm = t.params_default(max_shift=15)
    s_ref = [oxcf.integer_peak(oxcf.xcf_map(full[a], full[b]), max_shift=15)[1] for a, b in pairs]
    s_int = dev(np.array([(sx, sy) for sy, sx in s_ref], np.int32))
    h, s = t.xcf_peak(spec, spec, pi, li, N, prm)
    assert np.array_equal(host(s), host(s_int))
    hs, ss = t.xcf_subpixel(spec, spec, pi, li, s_int, N, prm)
    hs, ss = host(hs), host(ss)
    for k, (a, b) in enumerate(pairs):
        hr, sr = oxcf.subpixel_peak(full[a], full[b], s_ref[k], kappa=100)
        assert abs(hs[k] - hr) < 1e-5
        assert abs(ss[k][0] - sr[1]) <= 0.02 + 1e-6 and abs(ss[k][1] - sr[0]) <= 0.02 + 1e-6


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_gemm256_scores_match_oracle(prec):
    # precision 0: the exact FP32 DFT form (AUTO at 256 with a window), the
    # reference the split forms are reported against
    banner("gemm scores n=256 precision=%d" % prec)
    t = tm()
    pats = _pats(2, seed=31 + prec)
    lq = random_quats(np.random.default_rng(prec), 35)
    sp, _, fp = oracle_spectra(pats, N)
    sl, _, fl = oracle_spectra(oracle_templates(band_master(), lq, N, (0.5, 0.5, 0.6)), N)
    for s in (7, 15):
        got = host(t.xcf_scores(sp, sl, N, t.params_default(precision=prec, max_shift=s)))
        err = 0.0
        for i in range(len(pats)):
            ref = oxcf.library_scores(fp[i], fl, max_shift=s)
            err = max(err, float(np.max(np.abs(got[i] - ref))))
        print("[gpu]   n=256 precision=%d S=%d max |dh| = %.3g" % (prec, s, err), flush=True)
        assert err < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_index_and_refine256_match_oracle(prec):
    banner("index + refine n=256 precision=%d" % prec)
    t = tm()
    cfg = configs.tiny(p=4, l=40, n=N, seed=17 + prec)
    s = 12
    prm = t.params_default(precision=prec, max_shift=s)
    res = t.index_patterns(dev(cfg["patterns"]), dev(cfg["master"]), cfg["pc"], dev(cfg["lib_q"]), prm=prm,
                           scores=True)
    oprm = oracle.Params(max_shift=s)
    ref = pipeline.index_patterns(cfg["patterns"].numpy(), cfg["master"], cfg["pc"], cfg["lib_q"], oprm,
                                  return_scores=True)
    assert np.max(np.abs(host(res["scores"]) - ref["scores"])) < TOL[prec] + 1e-5
    best = host(res["best_idx"])
    tau = 2 * TOL[prec]
    for i in range(len(best)):
        if ref["gap"][i] > tau:
            assert best[i] == ref["best_idx"][i]
        else:
            assert ref["scores"][i][best[i]] >= ref["h_int"][i] - tau
    same = best == ref["best_idx"]
    assert np.max(np.abs(host(res["peak_h"])[same] - ref["peak_h"][same])) < 1e-4
    assert np.max(np.abs(host(res["shift"])[same] - ref["shift"][same])) <= 0.02 + 1e-6

    q0 = ref["best_q"]
    rr = t.refine_orientations(dev(cfg["patterns"]), dev(cfg["master"]), cfg["pc"], dev(q0),
                               pc_per=dev(cfg["pcs"]), prm=prm)
    rref = pipeline.refine_orientations(cfg["patterns"].numpy(), cfg["master"], cfg["pcs"], q0, oprm)
    q = host(rr["q"])
    d = np.rad2deg([rotations.disorientation_q(a, b) for a, b in zip(q, rref["q"])])
    print("[gpu]   refined deviation from oracle (deg):", np.round(d, 4), flush=True)
    assert np.max(d) < 0.05, d
    assert np.max(np.abs(host(rr["peak_h"]) - rref["peak_h"])) < 1e-4

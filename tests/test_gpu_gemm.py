"""Parity of the split-precision DFT-GEMM search (MFMA) against the FP64 oracle.

Both sides start from the same float32 band spectra, made by the oracle from
seeded images, so the bound measures only the GEMM arithmetic:
FP16 hi + lo: 1e-4 (the FP32 height tolerance); BF16 hi + lo: 1e-3; plain
BF16 (one product, ~3 significant digits per operand): 3e-2, reported.
"""

import numpy as np
import pytest

import oracle
from fixtures import band_master, configs, random_quats, simulate_patterns
from oracle import pipeline
from oracle import xcf as oxcf

from .gpu_util import banner, dev, host, oracle_spectra, oracle_templates, tm

pytestmark = pytest.mark.gpu

TOL = {1: 1e-4, 2: 1e-3, 3: 3e-2}


def _setup(n, p, l, seed):
    rng = np.random.default_rng(seed)
    q = random_quats(rng, p)
    off = rng.uniform(-4, 4, size=(p, 2))
    pcs = np.stack([0.5 + off[:, 0] / n, 0.5 + off[:, 1] / n, np.full(p, 0.6)], 1)
    pats = simulate_patterns(q, n, pcs, ("poisson", 300.0), seed=seed).numpy()
    lq = random_quats(np.random.default_rng(seed + 1), l)
    return pats, lq


@pytest.mark.parametrize("n", [64, 96, 128, 160])
@pytest.mark.parametrize("prec", [1, 2, 3])
def test_gemm_scores_match_oracle(n, prec):
    banner("gemm scores n=%d precision=%d" % (n, prec))
    t = tm()
    pats, lq = _setup(n, 3, 37, seed=n + 7 * prec)
    master = band_master()
    sp, _, fp = oracle_spectra(pats, n)
    sl, _, fl = oracle_spectra(oracle_templates(master, lq, n, (0.5, 0.5, 0.6)), n)
    for s in (7, 15, 23):
        got = host(t.xcf_scores(sp, sl, n, t.params_default(precision=prec, max_shift=s)))
        err = 0.0
        for i in range(len(pats)):
            ref = oxcf.library_scores(fp[i], fl, max_shift=s)
            err = max(err, float(np.max(np.abs(got[i] - ref))))
        print("[gpu]   n=%d precision=%d S=%d max |dh| = %.3g" % (n, prec, s, err), flush=True)
        assert err < TOL[prec]


def test_gemm_window_limits_and_errors():
    t = tm()
    pats, lq = _setup(128, 1, 3, seed=3)
    sp = t.pattern_spectra(dev(pats))
    import paper_1807_11313_amd as pkg
    with pytest.raises(pkg.EbsdError):            # the GEMM form needs a window
        t.xcf_scores(sp, sp, 128, t.params_default(precision=1))
    with pytest.raises(pkg.EbsdError):            # FFT form is FP32 only
        t.xcf_scores(sp, sp, 128, t.params_default(precision=1, form=1, max_shift=5))
    # a one-shift window (S = 0) is the zero-lag coefficient
    h = host(t.xcf_scores(sp, sp, 128, t.params_default(precision=1, max_shift=0)))
    assert abs(h[0, 0] - 1.0) < 1e-4


@pytest.mark.parametrize("prec", [1, 2])
def test_gemm_index_patterns(prec):
    banner("gemm index_patterns precision=%d" % prec)
    t = tm()
    cfg = configs.tiny(p=8, l=60, n=128, seed=11)
    s = 12
    prm = t.params_default(precision=prec, max_shift=s)
    res = t.index_patterns(dev(cfg["patterns"]), dev(cfg["master"]), cfg["pc"], dev(cfg["lib_q"]), prm=prm,
                           scores=True)
    ref = pipeline.index_patterns(cfg["patterns"].numpy(), cfg["master"], cfg["pc"], cfg["lib_q"],
                                  oracle.Params(max_shift=s), return_scores=True)
    sc = host(res["scores"])
    assert np.max(np.abs(sc - ref["scores"])) < TOL[prec] + 1e-5
    best = host(res["best_idx"])
    tau = 2 * TOL[prec]
    for i in range(len(best)):
        if ref["gap"][i] > tau:
            assert best[i] == ref["best_idx"][i]
        else:
            assert ref["scores"][i][best[i]] >= ref["h_int"][i] - tau
    same = best == ref["best_idx"]
    assert np.max(np.abs(host(res["peak_h"])[same] - ref["peak_h"][same])) < 1e-4


@pytest.mark.parametrize("n", [64, 128, 256])
@pytest.mark.parametrize("prec", [1, 2, 3])
def test_gemm_scores_match_emulated_split(n, prec):
    # against the oracle's emulation of the same split arithmetic in FP64:
    # what remains is the FP32 accumulation, so the bound is far tighter than
    # the split's own error above (which the FP64 comparison measures)
    from oracle import split as osplit
    banner("gemm vs emulated split n=%d precision=%d" % (n, prec))
    t = tm()
    pats, lq = _setup(n, 2, 20, seed=5 * n + prec)
    sp, bp, _ = oracle_spectra(pats, n)
    sl, bl, _ = oracle_spectra(oracle_templates(band_master(), lq, n, (0.5, 0.5, 0.6)), n)
    name = {1: "fp16x2", 2: "bf16x2", 3: "bf16"}[prec]
    for s in (7, 15):
        got = host(t.xcf_scores(sp, sl, n, t.params_default(precision=prec, max_shift=s)))
        err = 0.0
        for i in range(len(pats)):
            emu = osplit.emulated_scores(bp[i], bl, n, s, name)
            err = max(err, float(np.max(np.abs(got[i] - emu))))
        print("[gpu]   n=%d %s S=%d max |gpu - emulated| = %.3g" % (n, name, s, err), flush=True)
        assert err < 3e-6


@pytest.mark.parametrize("n", [64, 96, 128, 160])
def test_exact_dft_form_matches_oracle_and_fft_form(n):
    # the exact FP32 DFT form (form 3) against the oracle at the FP32 bound,
    # and against the FFT form's windowed scores on the same spectra
    banner("exact DFT form n=%d" % n)
    t = tm()
    pats, lq = _setup(n, 3, 29, seed=11 * n)
    sp, _, fp = oracle_spectra(pats, n)
    sl, _, fl = oracle_spectra(oracle_templates(band_master(), lq, n, (0.5, 0.5, 0.6)), n)
    for s in (0, 7, 15):
        got = host(t.xcf_scores(sp, sl, n, t.params_default(form=3, max_shift=s)))
        fft = host(t.xcf_scores(sp, sl, n, t.params_default(form=1, max_shift=s)))
        err = 0.0
        for i in range(len(pats)):
            ref = oxcf.library_scores(fp[i], fl, max_shift=s)
            err = max(err, float(np.max(np.abs(got[i] - ref))))
        print("[gpu]   n=%d S=%d max |dh| = %.3g, vs FFT form %.3g" % (n, s, err, np.max(np.abs(got - fft))),
              flush=True)
        assert err < 5e-6
        assert np.max(np.abs(got - fft)) < 5e-6

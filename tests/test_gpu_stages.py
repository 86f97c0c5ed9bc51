"""Stage-by-stage parity of the HIP kernels against the FP64 oracle.

Tolerances (FP32 path against FP64; derived in the design doc from the
arithmetic): template intensities 2e-5 of the master's range; unit-energy
spectra 2e-6 absolute per coefficient; correlation maps 5e-6 absolute;
integer peaks bit-exact (no near ties in these inputs); sub-pixel shift
0.02 px and height 1e-5; rotation 0.02 deg.
"""

import numpy as np
import pytest
import torch

from fixtures import band_master, random_quats, simulate_patterns
from oracle import geometry as ogeo
from oracle import refine as oref
from oracle import spectra as ospec
from oracle import xcf as oxcf
from oracle.params import Params as OParams

from .gpu_util import banner, dev, host, oracle_spectra, oracle_templates, tm

pytestmark = pytest.mark.gpu

SIZES = (64, 96, 128, 160)


def _pats(n, k, seed, noise=("poisson", 200.0), offsets=3.0):
    rng = np.random.default_rng(seed)
    q = random_quats(rng, k)
    off = rng.uniform(-offsets, offsets, size=(k, 2))
    pcs = np.stack([0.5 + off[:, 0] / n, 0.5 + off[:, 1] / n, np.full(k, 0.6)], 1)
    return q, pcs, simulate_patterns(q, n, pcs, noise, seed=seed).numpy()


@pytest.mark.parametrize("n", SIZES)
def test_projection_matches_oracle(n):
    banner("projection n=%d" % n)
    t = tm()
    master = band_master()
    rng = np.random.default_rng(n)
    q = random_quats(rng, 7)
    pc = (0.45, 0.55, 0.62)
    out = host(t.project_templates(dev(master), dev(q), n, pc))
    rng2 = np.random.default_rng(1)
    pcs = np.stack([rng2.uniform(0.4, 0.6, 7), rng2.uniform(0.4, 0.6, 7), rng2.uniform(0.5, 0.7, 7)], 1)
    out2 = host(t.project_templates(dev(master), dev(q), n, pc, pc_per=dev(pcs)))
    rngv = float(master.max() - master.min())
    from oracle import rotations as orot
    for k in range(7):
        r = orot.quat_to_matrix(q[k])
        assert np.max(np.abs(out[k] - ogeo.project(master, r, n, pc))) < 2e-5 * rngv
        assert np.max(np.abs(out2[k] - ogeo.project(master, r, n, pcs[k]))) < 2e-5 * rngv


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("window", [1, 0])
def test_spectra_match_oracle(n, window):
    banner("spectra n=%d window=%d" % (n, window))
    t = tm()
    _, _, pats = _pats(n, 5, seed=n + window)
    spec, en = t.pattern_spectra(dev(pats), t.params_default(window=window), energy=True)
    band = t.spectra_to_complex(spec, n)
    prm = OParams(window=bool(window))
    for k in range(5):
        ref, e = ospec.filtered_spectrum(pats[k].astype(np.float64), prm)
        full = t.band_to_full(band[k], n)
        assert np.max(np.abs(full - ref / np.sqrt(e))) < 2e-6
        assert abs(host(en)[k] / e - 1.0) < 2e-5


@pytest.mark.parametrize("n", SIZES)
def test_xcf_map_and_integer_peak(n):
    banner("xcf map n=%d" % n)
    t = tm()
    _, _, pats = _pats(n, 6, seed=10 + n)
    spec, _, full = oracle_spectra(pats, n)               # the same float32 spectra on both sides
    pi = dev(np.array([0, 1, 2, 3, 4, 5, 0], np.int32))
    li = dev(np.array([0, 2, 2, 5, 1, 3, 4], np.int32))
    h, s, m = t.xcf_peak(spec, spec, pi, li, n, want_map=True)
    h, s, m = host(h), host(s), host(m)
    for k, (a, b) in enumerate(zip(host(pi), host(li))):
        ref = oxcf.xcf_map(full[a], full[b])
        assert np.max(np.abs(m[k] - ref)) < 5e-6
        hr, sr = oxcf.integer_peak(ref)
        assert (s[k][1], s[k][0]) == sr and abs(h[k] - hr) < 5e-6


@pytest.mark.parametrize("n", SIZES)
def test_xcf_window(n):
    banner("xcf window n=%d" % n)
    t = tm()
    _, _, pats = _pats(n, 3, seed=20 + n, offsets=6.0)
    spec, _, full = oracle_spectra(pats, n)
    pi = dev(np.array([0, 1, 2], np.int32))
    li = dev(np.array([1, 2, 0], np.int32))
    h, s = t.xcf_peak(spec, spec, pi, li, n, t.params_default(max_shift=4))
    h, s = host(h), host(s)
    for k, (a, b) in enumerate(((0, 1), (1, 2), (2, 0))):
        ref = oxcf.xcf_map(full[a], full[b])
        hr, sr = oxcf.integer_peak(ref, max_shift=4)
        assert (s[k][1], s[k][0]) == sr and abs(h[k] - hr) < 5e-6


@pytest.mark.parametrize("n,s", [(64, 0), (64, 9), (96, 5), (128, 0), (128, 15), (128, 40), (160, 7)])
def test_windowed_scores_match_oracle(n, s):
    # the FFT search restricted to |s_x|, |s_y| <= s (s = 0: the origin only;
    # s = 40 at 128: both rows of some packed row pairs inside the window)
    banner("windowed scores n=%d s=%d" % (n, s))
    t = tm()
    p, l = 3, 37
    _, _, pats = _pats(n, p, seed=40 + n + s, offsets=4.0)
    master = band_master()
    lq = random_quats(np.random.default_rng(n + s), l)
    sp, _, fp = oracle_spectra(pats, n)
    sl, _, fl = oracle_spectra(oracle_templates(master, lq, n, (0.5, 0.5, 0.6)), n)
    sc = host(t.xcf_scores(sp, sl, n, t.params_default(max_shift=s)))
    for i in range(p):
        ref = oxcf.library_scores(fp[i], fl, max_shift=s)
        assert np.max(np.abs(sc[i] - ref)) < 5e-6


@pytest.mark.parametrize("s", [-1, 0, 7])
def test_candidate_scores_equal_library_scores(s):
    # each pattern's own candidate list (repeats, out-of-order, K above the
    # 64-template chunk, plus out-of-range indices that clamp to the ends):
    # the same kernel as the library search, so the same bits
    banner("candidate scores s=%d" % s)
    t = tm()
    n, p, l, k = 128, 5, 90, 70
    _, _, pats = _pats(n, p, seed=70 + s, offsets=4.0)
    lq = random_quats(np.random.default_rng(71), l)
    sp, _, fp = oracle_spectra(pats, n)
    sl, _, _ = oracle_spectra(oracle_templates(band_master(), lq, n, (0.5, 0.5, 0.6)), n)
    rng = np.random.default_rng(72)
    cand = rng.integers(0, l, size=(p, k)).astype(np.int32)
    cand[0, :3] = [-5, l, l + 100]
    prm = t.params_default(max_shift=s)
    full = host(t.xcf_scores(sp, sl, n, prm))
    got = host(t.xcf_scores_cand(sp, sl, dev(cand), n, prm))
    idx = np.clip(cand, 0, l - 1)
    assert np.array_equal(got, np.take_along_axis(full, idx, axis=1))
    ref = oxcf.library_scores(fp[1], oracle_spectra(oracle_templates(band_master(), lq[idx[1]], n, (0.5, 0.5, 0.6)),
                                                    n)[2], max_shift=s)
    assert np.max(np.abs(got[1] - ref)) < 5e-6


def test_candidate_scores_argument_errors():
    t = tm()
    import paper_1807_11313_amd as pkg
    f64 = t.spectrum_floats(64)
    sp = torch.zeros((2, f64), device="cuda:0")
    with pytest.raises(pkg.EbsdError):          # built at 128 only
        t.xcf_scores_cand(sp, sp, dev(np.zeros((2, 2), np.int32)), 64)
    f = t.spectrum_floats(128)
    sp = torch.zeros((2, f), device="cuda:0")
    with pytest.raises(pkg.EbsdError):          # K above L
        t.xcf_scores_cand(sp, sp, dev(np.zeros((2, 3), np.int32)), 128)
    with pytest.raises(ValueError):             # one candidate row per pattern
        t.xcf_scores_cand(sp, sp, dev(np.zeros((3, 2), np.int32)), 128)


@pytest.mark.parametrize("n,p,l", [(64, 5, 45), (96, 3, 33), (128, 2, 70), (160, 2, 31)])
def test_scores_match_oracle(n, p, l):
    # L is not a multiple of the 32-template chunk: ragged tail (at 64, where
    # each half-wave takes its own template, an odd tail of 13 leaves the
    # last pair's second half without a template)
    banner("scores n=%d p=%d l=%d" % (n, p, l))
    t = tm()
    _, _, pats = _pats(n, p, seed=30 + n)
    master = band_master()
    lq = random_quats(np.random.default_rng(n), l)
    sp, _, fp = oracle_spectra(pats, n)
    sl, _, fl = oracle_spectra(oracle_templates(master, lq, n, (0.5, 0.5, 0.6)), n)
    sc = host(t.xcf_scores(sp, sl, n))
    for i in range(p):
        ref = oxcf.library_scores(fp[i], fl)
        assert np.max(np.abs(sc[i] - ref)) < 5e-6


@pytest.mark.parametrize("n", SIZES)
def test_subpixel_matches_oracle(n):
    banner("subpixel n=%d" % n)
    t = tm()
    _, _, pats = _pats(n, 4, seed=40 + n)
    spec, _, full = oracle_spectra(pats, n)
    pairs = ((0, 1), (1, 2), (2, 3), (3, 0))
    pi = dev(np.array([a for a, _ in pairs], np.int32))
    li = dev(np.array([b for _, b in pairs], np.int32))
    # the oracle's integer peaks (x, y) start the upsampling on both sides
    s_ref = [oxcf.integer_peak(oxcf.xcf_map(full[a], full[b]))[1] for a, b in pairs]
    s_int = dev(np.array([(sx, sy) for sy, sx in s_ref], np.int32))
    h, s = t.xcf_peak(spec, spec, pi, li, n)
    assert np.array_equal(host(s), host(s_int))
    hs, ss = t.xcf_subpixel(spec, spec, pi, li, s_int, n)
    hs, ss = host(hs), host(ss)
    for k, (a, b) in enumerate(pairs):
        hr, sr = oxcf.subpixel_peak(full[a], full[b], s_ref[k], kappa=100)
        assert abs(hs[k] - hr) < 1e-5
        assert abs(ss[k][0] - sr[1]) <= 0.02 + 1e-6 and abs(ss[k][1] - sr[0]) <= 0.02 + 1e-6


@pytest.mark.parametrize("n", SIZES)
def test_rotation_measurement_matches_oracle(n):
    banner("log-polar n=%d" % n)
    t = tm()
    master = band_master()
    rng = np.random.default_rng(50 + n)
    from oracle import rotations as orot
    q0 = random_quats(rng, 4)
    pc = (0.5, 0.5, 0.6)
    pats, tmpls = [], []
    for k, deg in enumerate((1.5, -2.5, 0.4, 4.0)):
        r0 = orot.quat_to_matrix(q0[k])
        rt = r0 @ orot.rot_z(np.deg2rad(deg)).T
        pats.append(simulate_patterns(orot.matrix_to_quat(rt)[None], n, np.array([pc]), ("poisson", 500.0),
                                      seed=k).numpy()[0])
        tmpls.append(ogeo.project(master, r0, n, pc).astype(np.float32))
    pats, tmpls = np.array(pats), np.array(tmpls)
    g = host(t.measure_rotation(dev(pats), dev(tmpls)))
    prm = OParams()
    n_eta, kappa = prm.neta(n), prm.upsample
    for k in range(4):
        c = oref.eta_correlation_of(pats[k].astype(np.float64), tmpls[k].astype(np.float64), prm)
        v_ref, d_ref = oref.eta_peak(c, kappa)
        d_gpu = g[k] * n_eta / (2 * np.pi)
        # near-tie rule on the flat interpolated peak: the GPU's sample must be
        # within rounding of the oracle's maximum, and at most 3 grid steps away
        assert oref.eta_value(c, d_gpu)[0] >= v_ref - 2e-6
        assert abs(d_gpu - d_ref) <= 3.0 / kappa + 1e-9


@pytest.mark.parametrize("n,n_rho,n_eta", [(128, 64, 384), (128, 44, 512), (96, 50, 192), (64, 20, 320),
                                           (160, 33, 128), (64, 24, 1024)])
def test_rotation_measurement_other_grids(n, n_rho, n_eta):
    # log-polar grids other than the default: the direct eta correlation
    # (n_eta = 384, and 1,024, its largest) and the transform form with row
    # counts that leave the last row group partly empty; the same near-tie
    # rule as above
    banner("log-polar n=%d grid %d x %d" % (n, n_rho, n_eta))
    t = tm()
    master = band_master()
    rng = np.random.default_rng(70 + n_eta)
    from oracle import rotations as orot
    q0 = random_quats(rng, 3)
    pc = (0.5, 0.5, 0.6)
    pats, tmpls = [], []
    for k, deg in enumerate((2.2, -1.1, 3.3)):
        r0 = orot.quat_to_matrix(q0[k])
        rt = r0 @ orot.rot_z(np.deg2rad(deg)).T
        pats.append(simulate_patterns(orot.matrix_to_quat(rt)[None], n, np.array([pc]), ("poisson", 500.0),
                                      seed=k).numpy()[0])
        tmpls.append(ogeo.project(master, r0, n, pc).astype(np.float32))
    pats, tmpls = np.array(pats), np.array(tmpls)
    g = host(t.measure_rotation(dev(pats), dev(tmpls), t.params_default(n_rho=n_rho, n_eta=n_eta)))
    prm = OParams(n_rho=n_rho, n_eta=n_eta)
    kappa = prm.upsample
    for k in range(3):
        c = oref.eta_correlation_of(pats[k].astype(np.float64), tmpls[k].astype(np.float64), prm)
        v_ref, d_ref = oref.eta_peak(c, kappa)
        d_gpu = g[k] * n_eta / (2 * np.pi)
        assert oref.eta_value(c, d_gpu)[0] >= v_ref - 2e-6
        assert abs(d_gpu - d_ref) <= 3.0 / kappa + 1e-9


def test_empty_inputs_are_noops():
    t = tm()
    e = torch.empty((0, 64, 64), dtype=torch.float32, device="cuda:0")
    assert t.pattern_spectra(e).shape[0] == 0
    master = dev(band_master())
    lq = dev(random_quats(np.random.default_rng(0), 3))
    r = t.index_patterns(e, master, (0.5, 0.5, 0.6), lq)
    assert r["best_idx"].numel() == 0


def test_search_larger_than_one_dispatch():
    # 34,000 patterns x 8,000 templates at 128^2 needs more than 2^32
    # work-items as one dispatch of the search kernel: the launcher splits it,
    # and every row must equal the same rows searched on their own
    banner("search split over dispatches")
    t = tm()
    n, p, l = 128, 34000, 8000
    f = t.spectrum_floats(n)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(3)
    sp = torch.randn((p, f), generator=g, device="cuda:0") * 1e-2
    sl = torch.randn((l, f), generator=g, device="cuda:0") * 1e-2
    full = t.xcf_scores(sp, sl, n)
    for rows in (slice(0, 64), slice(p - 64, p), slice(20000, 20064)):
        part = t.xcf_scores(sp[rows].contiguous(), sl, n)
        assert torch.equal(full[rows], part), rows
    del full

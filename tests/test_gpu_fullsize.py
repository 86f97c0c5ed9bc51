"""The map workloads at their full size (10,000 patterns of 128^2 against
4,000 library templates searched over all shifts, and the same map at 256^2
searched by the FP16 hi + lo DFT-GEMM over |s| <= 15 px; the ragged batch of
20,000 patterns against 8,000 templates with its stencil; the learned
proposal trained on 200,000 patterns and run on 50,000; the 3 deg
equispaced library with its nearest neighbours and the capture-range sweep:
the launch configurations the bench times), checked on sampled patterns
that the FP64 oracle indexes and refines one by one from the same inputs
(the proposal against the exhaustive search).

* Library index: the oracle's, bit-exact outside the near-tie rule
  (tau_tie = 2e-4); inside it the GPU's pick scores within tau_tie of the
  oracle's best.
* Peak height 1e-4, sub-pixel shift 0.02 px (where the picks agree).
* Refinement with per-pattern pattern centres (re-projected from the start,
  and from the search's shift as the bench times it), from the oracle's own
  picks and shifts where the picks agree: the oracle's orientation to
  0.05 deg.
"""

import numpy as np
import pytest
import torch

import oracle
from fixtures import configs
from oracle import pipeline, rotations

from .gpu_util import banner, dev, fallback_tau, host, tm

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
    pc_per = dev(cfg["pcs"])
    rr = t.refine_orientations(pats, master, cfg["pc"], res["best_q"], pc_per=pc_per)
    rm = t.refine_from_match(pats, master, cfg["pc"], res["best_q"], res["shift"], pc_per=pc_per)
    best_all = host(res["best_idx"])
    h_all, s_all, q_all, qm_all = host(res["peak_h"]), host(res["shift"]), host(rr["q"]), host(rm["q"])
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

    banner("oracle: refinement of the sampled patterns (both forms)")
    # from the oracle's own picks and shifts; compared where the picks agree
    rref = pipeline.refine_orientations(sample, cfg["master"], cfg["pcs"][idx], ref["best_q"], prm)
    d = np.rad2deg([rotations.disorientation_q(a, b) for a, b in zip(q_all[idx], rref["q"])])
    assert np.max(d[same]) < 0.05, d
    mref = pipeline.refine_from_match(sample, cfg["master"], cfg["pcs"][idx], cfg["pc"], ref["best_q"], ref["shift"],
                                      prm)
    d = np.rad2deg([rotations.disorientation_q(a, b) for a, b in zip(qm_all[idx], mref["q"])])
    assert np.max(d[same]) < 0.05, d


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
    rr = t.refine_from_match(pats, master, cfg["pc"], res["best_q"], res["shift"], pc_per=dev(cfg["pcs"]), prm=prm)
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
    # the bench's refinement (from the search's shift), from the oracle's own
    # picks and shifts, compared where the picks agree
    rref = pipeline.refine_from_match(sample, cfg["master"], cfg["pcs"][idx], cfg["pc"], ref["best_q"], ref["shift"],
                                      oprm)
    d = np.rad2deg([rotations.disorientation_q(a, b) for a, b in zip(q_all[idx], rref["q"])])
    assert np.max(d[same]) < 0.05, d


def test_ragged_batch_sampled_against_oracle():
    # the ragged batch at full size (20,000 patterns of 64 / 96 / 128 / 160,
    # 8,000 templates, 27-point stencil, one graph launch); sampled patterns
    # of the 64 and 96 classes (whose oracle libraries are the cheapest)
    from oracle import stencil
    banner("full-size ragged batch 20,000 x 8,000 + stencil, sampled against the oracle")
    t = tm()
    cfg = configs.ragged(device="cuda:0")
    data, offs, ns = configs.pack_ragged(cfg, device="cuda:0")
    assert len(ns) == 20000 and len(cfg["lib_q"]) == 8000
    plan = t.RaggedPlan(ns, offs, len(cfg["lib_q"]), stencil=True)
    res = plan.run(data, dev(cfg["master"]), cfg["pc"], dev(cfg["lib_q"]), pc_per=dev(cfg["pcs"]))
    best, sidx = host(res["best_idx"]), host(res["stencil_idx"])
    q, h, s = host(res["q"]), host(res["peak_h"]), host(res["shift"])
    plan.close()
    prm = oracle.Params()
    rng = np.random.default_rng(13)
    for n in (64, 96):
        idx = np.sort(rng.choice(np.nonzero(ns == n)[0], 2, replace=False))
        pats = np.stack([configs.ragged_pattern(cfg, i) for i in idx]).astype(np.float64)
        banner("oracle: 8,000 library spectra at %d^2" % n)
        lib_spec = pipeline.library_spectra(cfg["master"], cfg["lib_q"], n, cfg["pc"], prm)
        ref = pipeline.index_patterns(pats, cfg["master"], cfg["pc"], cfg["lib_q"], prm, lib_spec=lib_spec,
                                      return_scores=True)
        for a, i in enumerate(idx):
            if ref["gap"][a] > TAU_TIE:
                assert best[i] == ref["best_idx"][a], (n, i, best[i], ref["best_idx"][a])
            else:
                assert ref["scores"][a][best[i]] >= ref["h_int"][a] - TAU_TIE
        st = stencil.stencil_refine(list(pats), cfg["master"], cfg["pcs"][idx], cfg["lib_q"][best[idx]], prm)
        for a, i in enumerate(idx):
            if st["gap"][a] <= TAU_TIE:
                assert st["h_int"][a][sidx[i]] >= st["h_int"][a].max() - TAU_TIE
                continue
            assert sidx[i] == st["idx"][a], (n, i, sidx[i], st["idx"][a])
            d = np.rad2deg(rotations.misorientation_angle(rotations.quat_to_matrix(q[i]),
                                                          rotations.quat_to_matrix(st["q"][a])))
            assert d < 1e-6, d
            assert abs(h[i] - st["peak_h"][a]) < 1e-4
            assert np.max(np.abs(s[i] - st["shift"][a])) <= 0.02 + 1e-6


def test_learned_proposal_full_size():
    # the proposal workload at full size: the network trained on the GPU on
    # 200,000 projected patterns (2 epochs) for 8,000 classes; 50,000 test
    # patterns at 128^2 searched exhaustively and pruned (top 32 + fallback
    # below tau = 1st percentile of the exhaustive integer peak height among
    # the correctly indexed of 10,000 validation patterns).  The exhaustive search, pinned to the oracle by
    # the tests above, is the reference.
    from fixtures import band_master, random_fz_quats, random_quats, simulate_patterns
    banner("full-size learned proposal: training 200,000 x 2 epochs, 50,000 test patterns")
    t = tm()
    n, L, k, bsz, n_train = 128, 8000, 32, 256, 200000
    lq = dev(random_fz_quats(np.random.default_rng(11), L))
    master = dev(band_master())
    pc = (0.5, 0.5, 0.6)

    def patterns(p, seed, truth=False):
        rng = np.random.default_rng(seed)
        q = random_quats(rng, p)
        off = rng.uniform(-5, 5, size=(p, 2))
        pcs = np.stack([0.5 + off[:, 0] / n, 0.5 + off[:, 1] / n, np.full(p, 0.6)], 1)
        pats = simulate_patterns(q, n, pcs, ("poisson_gauss", 1000.0, 5.0), seed=seed, device="cuda:0",
                                 dtype=torch.float32).contiguous()
        return (q, pcs, pats) if truth else (pcs, pats)

    net = t.Cnn(L, seed=5)
    x = torch.empty((bsz, 64, 64), device="cuda:0")
    y = torch.empty(bsz, dtype=torch.int32, device="cuda:0")
    loss = torch.empty(1, device="cuda:0")
    for s in range(2 * n_train // bsz):
        t.cnn_make_batch(master, pc, lq, n, bsz, (s * bsz) % n_train, 1000 + (s * bsz) // n_train, x=x, labels=y)
        net.train_step(x, y, 1e-3, loss)
    print("[gpu]   final training loss %.3f" % float(loss.item()), flush=True)
    q_val, pcs_val, val = patterns(10000, 31, truth=True)
    tau, ok = fallback_tau(t, val, q_val, pcs_val, master, pc, lq)
    print("[gpu]   validation: %.4f correctly indexed" % ok, flush=True)
    del val
    pcs, test = patterns(50000, 32)
    ex = t.index_patterns(test, master, pc, lq, scores=True)
    top2 = torch.topk(ex.pop("scores"), 2, dim=1).values
    gap = host(top2[:, 0] - top2[:, 1])
    del top2
    pr = t.index_proposed(test, master, pc, lq, net, top_k=k, fallback_tau=tau)
    best_ex, best_pr = host(ex["best_idx"]), host(pr["best_idx"])
    fb = host(pr["fallback"]).astype(bool)
    clear = gap > TAU_TIE
    agree = best_ex == best_pr
    print("[gpu]   agreement %.4f, fallback %.4f, tau %.3f" % (agree.mean(), fb.mean(), tau), flush=True)
    assert np.all(agree[clear & fb])
    assert agree[clear].mean() >= 0.95
    assert np.array_equal(host(pr["peak_h"])[agree], host(ex["peak_h"])[agree])
    assert np.array_equal(host(pr["shift"])[agree], host(ex["shift"])[agree])
    assert len(best_pr) * k + fb.sum() * L < 0.3 * len(best_pr) * L
    # both picks refined the same way
    pc_per = dev(pcs)
    q_ex = host(t.refine_orientations(test, master, pc, ex["best_q"], pc_per=pc_per)["q"])
    q_pr = host(t.refine_orientations(test, master, pc, pr["best_q"], pc_per=pc_per)["q"])
    sub = np.random.default_rng(5).choice(len(q_ex), 2000, replace=False)
    d = np.rad2deg([rotations.disorientation_q(a, b) for a, b in zip(q_ex[sub], q_pr[sub])])
    print("[gpu]   refined pruned vs exhaustive: %.4f within 0.1 deg" % np.mean(d < 0.1), flush=True)
    assert np.mean(d < 0.1) >= 0.99
    net.close()


def test_so3_library_and_neighbours_at_bench_size():
    # the bench's finest library (3 deg, 22,946 orientations): the whole
    # library against the oracle's, and the all-pairs nearest neighbours of
    # 24 sampled members against the oracle's disorientations to every member
    from oracle import so3grid
    banner("so3 library at 3 deg and sampled nearest neighbours")
    t = tm()
    q = t.so3_library(3.0)
    got = host(q)
    want = so3grid.library(3.0)
    assert got.shape == want.shape and np.max(np.abs(got - want)) < 1e-12
    ang, idx = t.nn_disorientation(q)
    ang, idx = host(ang), host(idx)
    r = rotations.quat_to_matrix(want)
    ops = rotations.cubic_operators()
    for a in np.linspace(0, len(want) - 1, 24).astype(int):
        d = np.rad2deg(rotations.disorientation(r[a][None], r, ops))
        d[a] = np.inf
        assert abs(ang[a] - d.min()) < 1e-9 and abs(d[idx[a]] - d.min()) < 1e-9


def test_capture_range_at_bench_size():
    # the bench's sweep shape (8 references x 3 axes x 121 angles over +-30
    # deg at 160^2); one full curve per axis against the oracle
    from fixtures import band_master, random_quats
    from oracle import capture
    banner("capture range 8 x 3 x 121 at 160^2, sampled curves")
    t = tm()
    master = band_master()
    q_ref = random_quats(np.random.default_rng(77), 8)
    th = np.arange(-30.0, 30.0 + 1e-9, 0.5)
    pc = (0.5, 0.3, 0.6)
    h, w = t.capture_range(dev(master), dev(q_ref), 160, pc, pc, dev(th))
    h, w = host(h), host(w)
    for r, a in ((0, 0), (3, 1), (7, 2)):
        ref = capture.capture_curve(master, rotations.quat_to_matrix(q_ref[r]), "xyz"[a], th, 160, pc, pc,
                                    oracle.Params())
        assert np.max(np.abs(h[r, a] - ref)) < 1e-4
        assert abs(w[r, a] - capture.fwhm(th, ref)) < 0.02

"""The pruned search (network top-k, exhaustive fallback below the peak
threshold) against the exhaustive search it replaces, and what the trained
network gains over the same pruning without training.

The exhaustive FP32 search is the reference: where the exhaustive top-2 gap
exceeds tau_tie the pruned search must pick the same template for at least
95 % of the patterns (and for every pattern that fell back), with the same
peak height and shift wherever it picks the same template.  The gain is the number of
(pattern, template) correlations: the trained network resolves most
patterns within its top 32, an untrained one sends most to the fallback.
"""

import numpy as np
import pytest
import torch

from fixtures import band_master, random_fz_quats, random_quats, simulate_patterns

from .gpu_util import banner, dev, fallback_tau, host, tm

pytestmark = pytest.mark.gpu

TAU_TIE = 2e-4


def _patterns(p, seed, n=128, truth=False):
    rng = np.random.default_rng(seed)
    q = random_quats(rng, p)
    off = rng.uniform(-5, 5, size=(p, 2))
    pcs = np.stack([0.5 + off[:, 0] / n, 0.5 + off[:, 1] / n, np.full(p, 0.6)], 1)
    pats = simulate_patterns(q, n, pcs, ("poisson_gauss", 1000.0, 5.0), seed=seed)
    return (q, pcs, pats) if truth else pats


def _train(t, master, lq, steps, seed=3, bsz=256, n=128):
    net = t.Cnn(lq.shape[0], seed=seed)
    x = torch.empty((bsz, 64, 64), device="cuda:0")
    y = torch.empty(bsz, dtype=torch.int32, device="cuda:0")
    loss = torch.empty(1, device="cuda:0")
    for s in range(steps):
        t.cnn_make_batch(master, (0.5, 0.5, 0.6), lq, n, bsz, s * bsz, seed, x=x, labels=y)
        net.train_step(x, y, 1e-3, loss)
    torch.cuda.synchronize()
    return net, float(loss.item())


def test_pruned_search_matches_exhaustive_and_gains_over_untrained():
    banner("proposal: pruned vs exhaustive")
    t = tm()
    L, k = 400, 32
    lib = random_fz_quats(np.random.default_rng(1), L)
    master, lq = dev(band_master()), dev(lib)
    pc = (0.5, 0.5, 0.6)
    net, loss = _train(t, master, lq, 300)
    print("[gpu]   final training loss %.3f" % loss, flush=True)

    # threshold: 1st percentile of the exhaustive integer peak height among
    # the correctly indexed patterns of a validation set
    q_val, pcs_val, val = _patterns(128, seed=20, truth=True)
    tau, ok = fallback_tau(t, dev(val), q_val, pcs_val, master, pc, lq)
    print("[gpu]   validation: %.3f correctly indexed" % ok, flush=True)
    assert ok > 0.9

    test = dev(_patterns(200, seed=21))
    ex = t.index_patterns(test, master, pc, lq, scores=True)
    pr = t.index_proposed(test, master, pc, lq, net, top_k=k, fallback_tau=tau)
    best_ex, best_pr = host(ex["best_idx"]), host(pr["best_idx"])
    sc = host(ex["scores"])
    top2 = np.sort(sc, axis=1)[:, -2:]
    gap = top2[:, 1] - top2[:, 0]
    clear = gap > TAU_TIE
    agree = best_pr == best_ex
    fb = host(pr["fallback"]).astype(bool)
    print("[gpu]   agreement %.3f, fallback %.3f, tau %.3f" % (agree.mean(), fb.mean(), tau), flush=True)
    # the fallback is the exhaustive search itself; without it, the network's
    # candidates must hold the exhaustive winner for nearly every pattern
    assert np.all(agree[clear & fb])
    assert agree[clear].mean() >= 0.95
    same = agree
    assert np.array_equal(host(pr["peak_h"])[same], host(ex["peak_h"])[same])
    assert np.array_equal(host(pr["shift"])[same], host(ex["shift"])[same])
    pairs_pruned = len(best_pr) * k + fb.sum() * L
    print("[gpu]   correlations: pruned %d vs exhaustive %d" % (pairs_pruned, len(best_pr) * L), flush=True)
    assert pairs_pruned < 0.3 * len(best_pr) * L

    # the same pruning with an untrained network falls back far more often
    raw = t.Cnn(L, seed=3)
    pr0 = t.index_proposed(test, master, pc, lq, raw, top_k=k, fallback_tau=tau)
    fb0 = host(pr0["fallback"]).astype(bool)
    print("[gpu]   untrained: fallback %.3f" % fb0.mean(), flush=True)
    assert fb0.mean() > fb.mean() + 0.3
    net.close()
    raw.close()


def test_proposal_argument_errors():
    t = tm()
    import paper_1807_11313_amd as pkg
    lib = dev(random_fz_quats(np.random.default_rng(1), 40))
    net = t.Cnn(40, seed=1)
    pats = dev(_patterns(2, seed=3, n=96))
    with pytest.raises(pkg.EbsdError):          # 96 is not a multiple of 64
        t.index_proposed(pats, dev(band_master()), (0.5, 0.5, 0.6), lib, net)
    pats = dev(_patterns(2, seed=3))
    with pytest.raises(pkg.EbsdError):          # library and network disagree
        t.index_proposed(pats, dev(band_master()), (0.5, 0.5, 0.6), lib[:30].contiguous(), net)
    with pytest.raises(pkg.EbsdError):          # k above L
        t.index_proposed(pats, dev(band_master()), (0.5, 0.5, 0.6), lib, net, top_k=41)
    net.close()

"""Pattern images stored as BF16 (ebsd_params.input = EBSD_INPUT_BF16).

Each pixel is widened to FP32 as it is loaded, so every call on BF16 images
must equal, bit for bit, the same call on FP32 images holding the widened
values; and against the FP64 oracle run on those same (BF16-rounded) images
the FP32 tolerances hold.  The rounding to BF16 happens on the host, as part
of making the input.
"""

import numpy as np
import pytest
import torch

import oracle
from fixtures import band_master, configs, random_fz_quats
from oracle import pipeline, rotations

from .gpu_util import banner, dev, host, tm

pytestmark = pytest.mark.gpu


def _bf16_pair(pats):
    b = torch.as_tensor(np.asarray(pats, dtype=np.float32)).to(torch.bfloat16).to("cuda:0").contiguous()
    return b, b.float().contiguous()


@pytest.mark.parametrize("n", [64, 128, 160])
def test_bf16_images_equal_widened_fp32(n):
    banner("bf16 images n=%d" % n)
    t = tm()
    cfg = configs.tiny(p=5, l=30, n=n, seed=70 + n)
    b, f = _bf16_pair(cfg["patterns"])
    master, lq = dev(cfg["master"]), dev(cfg["lib_q"])
    assert torch.equal(t.pattern_spectra(b), t.pattern_spectra(f))
    rb = t.index_patterns(b, master, cfg["pc"], lq, scores=True)
    rf = t.index_patterns(f, master, cfg["pc"], lq, scores=True)
    for k in rf:
        assert torch.equal(rb[k], rf[k]), k
    pcs = dev(cfg["pcs"])
    qb = t.refine_from_match(b, master, cfg["pc"], rf["best_q"], rf["shift"], pc_per=pcs)
    qf = t.refine_from_match(f, master, cfg["pc"], rf["best_q"], rf["shift"], pc_per=pcs)
    for k in qf:
        assert torch.equal(qb[k], qf[k]), k
    ob = t.refine_orientations(b, master, cfg["pc"], dev(cfg["true_q"]), pc_per=pcs)
    of = t.refine_orientations(f, master, cfg["pc"], dev(cfg["true_q"]), pc_per=pcs)
    for k in of:
        assert torch.equal(ob[k], of[k]), k


def test_bf16_images_match_oracle():
    banner("bf16 images vs oracle")
    t = tm()
    cfg = configs.tiny(p=5, l=40, n=128, seed=77)
    b, f = _bf16_pair(cfg["patterns"])
    pats = host(f).astype(np.float64)                   # the BF16-rounded images the oracle sees
    res = t.index_patterns(b, dev(cfg["master"]), cfg["pc"], dev(cfg["lib_q"]), scores=True)
    ref = pipeline.index_patterns(pats, cfg["master"], cfg["pc"], cfg["lib_q"], oracle.Params(), return_scores=True)
    assert np.max(np.abs(host(res["scores"]) - ref["scores"])) < 1e-4
    best = host(res["best_idx"])
    for i in range(len(best)):
        if ref["gap"][i] > 2e-4:
            assert best[i] == ref["best_idx"][i]
    q0 = ref["best_q"]
    rr = t.refine_orientations(b, dev(cfg["master"]), cfg["pc"], dev(q0), pc_per=dev(cfg["pcs"]))
    rref = pipeline.refine_orientations(pats, cfg["master"], cfg["pcs"], q0, oracle.Params())
    d = np.rad2deg([rotations.disorientation_q(a, c) for a, c in zip(host(rr["q"]), rref["q"])])
    assert np.max(d) < 0.05, d
    assert np.max(np.abs(host(rr["peak_h"]) - rref["peak_h"])) < 1e-4


def test_bf16_images_in_the_pruned_search():
    banner("bf16 images in the pruned search")
    t = tm()
    L = 120
    lq = dev(random_fz_quats(np.random.default_rng(4), L))
    master = dev(band_master())
    net = t.Cnn(L, seed=2)
    cfg = configs.tiny(p=6, l=L, n=128, seed=78)
    b, f = _bf16_pair(cfg["patterns"])
    pb = t.index_proposed(b, master, cfg["pc"], lq, net, top_k=8, fallback_tau=0.3)
    pf = t.index_proposed(f, master, cfg["pc"], lq, net, top_k=8, fallback_tau=0.3)
    for k in pf:
        assert torch.equal(pb[k], pf[k]), k
    net.close()

"""Ragged batches (binnings 64, 96, 128, 160 in one call) and the 27-point
stencil, against the FP64 oracle and against the single-size path.

* Library index per pattern: the oracle's index at the pattern's own size,
  bit-exact unless the oracle's top-2 gap is within tau_tie = 2e-4.
* Stencil candidate: the oracle's (same 27 candidates from the same start),
  bit-exact unless its top-2 gap among the 27 is within tau_tie; the final
  orientation then equals the oracle's to 1e-6 deg, peak height 1e-4,
  sub-pixel shift 0.02 px.
* The persistent search of a class computes exactly what the single-size
  kernels compute, so the library index, peak height and shift equal those
  of ebsd_index_patterns on that class alone, bit for bit.
* Every replay of the captured graph, with unrelated eager work and
  synchronisations between replays, equals the eager enqueue bit for bit.
"""

import numpy as np
import pytest
import torch

import oracle
from fixtures import configs
from oracle import pipeline, rotations, stencil

from .gpu_util import banner, dev, host, tm

pytestmark = pytest.mark.gpu

TAU_TIE = 2e-4


def _workload(p=12, l=40, seed=5, sizes=(64, 96, 128, 160)):
    cfg = configs.ragged(seed=seed, p=p, l=l, sizes=sizes)
    data, offs, ns = configs.pack_ragged(cfg, device="cuda:0")
    return cfg, data, offs, ns


def _run(t, plan, cfg, data, pcs=True):
    return plan.run(data, dev(cfg["master"]), cfg["pc"], dev(cfg["lib_q"]),
                    pc_per=dev(cfg["pcs"]) if pcs else None)


def test_ragged_index_and_stencil_match_oracle():
    banner("ragged index + stencil vs oracle")
    t = tm()
    cfg, data, offs, ns = _workload()
    plan = t.RaggedPlan(ns, offs, len(cfg["lib_q"]), stencil=True)
    print("[gpu]   tiles", plan.tiles(), flush=True)
    res = _run(t, plan, cfg, data)
    best, sidx = host(res["best_idx"]), host(res["stencil_idx"])
    q, h, s = host(res["q"]), host(res["peak_h"]), host(res["shift"])
    prm = oracle.Params()
    for n in (64, 96, 128, 160):
        idx = np.nonzero(ns == n)[0]
        pats = np.stack([configs.ragged_pattern(cfg, i) for i in idx])
        ref = pipeline.index_patterns(pats, cfg["master"], cfg["pc"], cfg["lib_q"], prm)
        for a, i in enumerate(idx):
            if ref["gap"][a] > TAU_TIE:
                assert best[i] == ref["best_idx"][a], (n, i)
        # the stencil from the GPU's library pick
        q0 = cfg["lib_q"][best[idx]]
        st = stencil.stencil_refine(list(pats), cfg["master"], cfg["pcs"][idx], q0, prm)
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
    plan.close()


def test_ragged_search_equals_single_size_path():
    banner("ragged vs single-size index")
    t = tm()
    cfg, data, offs, ns = _workload(p=40, l=70, seed=6)
    plan = t.RaggedPlan(ns, offs, len(cfg["lib_q"]), stencil=False)
    res = _run(t, plan, cfg, data, pcs=False)
    best, h, s, q = host(res["best_idx"]), host(res["peak_h"]), host(res["shift"]), host(res["q"])
    assert np.all(host(res["stencil_idx"]) == -1)
    for n in (64, 96, 128, 160):
        idx = np.nonzero(ns == n)[0]
        pats = dev(np.stack([configs.ragged_pattern(cfg, i) for i in idx]))
        ref = t.index_patterns(pats, dev(cfg["master"]), cfg["pc"], dev(cfg["lib_q"]))
        assert np.array_equal(best[idx], host(ref["best_idx"]))
        assert np.array_equal(h[idx], host(ref["peak_h"]))
        assert np.array_equal(s[idx], host(ref["shift"]))
        assert np.array_equal(q[idx], host(ref["best_q"]))
    plan.close()


def test_graph_replays_equal_eager_enqueue():
    banner("ragged graph replays")
    t = tm()
    cfg, data, offs, ns = _workload(p=16, l=50, seed=7)
    eager = t.RaggedPlan(ns, offs, len(cfg["lib_q"]), stencil=True, eager=True, autotune=False)
    ref = _run(t, eager, cfg, data)
    torch.cuda.synchronize()
    plan = t.RaggedPlan(ns, offs, len(cfg["lib_q"]), stencil=True)
    out = None
    junk = torch.ones(1 << 20, device="cuda:0")
    for rep in range(4):
        if out is None or rep == 2:
            out = _run(t, plan, cfg, data)             # capture (rep 0), new buffers re-capture (rep 2)
        else:
            plan.run_into(data, dev(cfg["master"]), cfg["pc"], dev(cfg["lib_q"]), out, dev(cfg["pcs"]))
        junk.mul_(1.0001)                              # unrelated eager work between replays
        torch.cuda.synchronize()
        for k in ("best_idx", "q", "peak_h", "shift", "stencil_idx"):
            assert torch.equal(out[k], ref[k]), (rep, k)
        for k in out:
            out[k].fill_(0)
    plan.close()
    eager.close()


def test_ragged_with_missing_sizes_and_tiles():
    t = tm()
    cfg, data, offs, ns = _workload(p=6, l=33, seed=8, sizes=(96, 160))
    plan = t.RaggedPlan(ns, offs, len(cfg["lib_q"]), stencil=False)
    tiles = plan.tiles()
    assert sorted(x["n"] for x in tiles) == [96, 160]
    for x in tiles:
        assert x["templates_per_item"] in (8, 16, 32, 64) and x["grid"] >= 1
        assert x["patterns"] == int(np.sum(ns == x["n"]))
    res = _run(t, plan, cfg, data)
    assert np.all(host(res["best_idx"]) >= 0) and np.all(host(res["best_idx"]) < 33)
    plan.close()


def test_ragged_shift_window_equals_single_size_path():
    # the persistent searches' shift-window variants against the single-size path
    banner("ragged with a shift window")
    t = tm()
    cfg, data, offs, ns = _workload(p=24, l=45, seed=9)
    prm = t.params_default(max_shift=6)
    plan = t.RaggedPlan(ns, offs, len(cfg["lib_q"]), prm=prm, stencil=False)
    res = _run(t, plan, cfg, data, pcs=False)
    best, h = host(res["best_idx"]), host(res["peak_h"])
    for n in (64, 96, 128, 160):
        idx = np.nonzero(ns == n)[0]
        pats = dev(np.stack([configs.ragged_pattern(cfg, i) for i in idx]))
        ref = t.index_patterns(pats, dev(cfg["master"]), cfg["pc"], dev(cfg["lib_q"]), prm=prm)
        assert np.array_equal(best[idx], host(ref["best_idx"]))
        assert np.array_equal(h[idx], host(ref["peak_h"]))
    plan.close()

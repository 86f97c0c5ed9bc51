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
* With the refinement in the graph: the final orientation within 0.05 deg of
  the oracle's (stencil then refinement, or the refinement from the search's
  shift without the stencil), peak height 1e-4, shift 0.02 px.
Every oracle computation starts from the oracle's own library pick; patterns
whose device pick differs from it (near ties only) are not compared further.
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


def _oracle_index(cfg, ns, n, prm):
    idx = np.nonzero(ns == n)[0]
    pats = np.stack([configs.ragged_pattern(cfg, i) for i in idx])
    return idx, pats, pipeline.index_patterns(pats, cfg["master"], cfg["pc"], cfg["lib_q"], prm)


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
        idx, pats, ref = _oracle_index(cfg, ns, n, prm)
        for a, i in enumerate(idx):
            if ref["gap"][a] > TAU_TIE:
                assert best[i] == ref["best_idx"][a], (n, i)
        # the stencil from the oracle's own library pick
        q0 = cfg["lib_q"][ref["best_idx"]]
        st = stencil.stencil_refine(list(pats), cfg["master"], cfg["pcs"][idx], q0, prm)
        for a, i in enumerate(idx):
            if best[i] != ref["best_idx"][a]:
                continue
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


@pytest.mark.parametrize("refine", [False, True])
def test_graph_replays_equal_eager_enqueue(refine):
    banner("ragged graph replays refine=%d" % refine)
    t = tm()
    cfg, data, offs, ns = _workload(p=16, l=50, seed=7)
    eager = t.RaggedPlan(ns, offs, len(cfg["lib_q"]), stencil=True, eager=True, autotune=False, refine=refine)
    ref = _run(t, eager, cfg, data)
    torch.cuda.synchronize()
    plan = t.RaggedPlan(ns, offs, len(cfg["lib_q"]), stencil=True, refine=refine)
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


@pytest.mark.parametrize("with_stencil", [True, False])
def test_ragged_refinement_matches_oracle(with_stencil):
    # the refinement inside the graph: after the stencil, its first x / y
    # step from the stencil winner's shift; without it, from the library
    # pick's shift less the PC-move translation
    banner("ragged refinement vs oracle, stencil=%d" % with_stencil)
    t = tm()
    cfg, data, offs, ns = _workload(p=12, l=40, seed=15)
    plan = t.RaggedPlan(ns, offs, len(cfg["lib_q"]), stencil=with_stencil, refine=True)
    res = _run(t, plan, cfg, data)
    best, q, h, s = host(res["best_idx"]), host(res["q"]), host(res["peak_h"]), host(res["shift"])
    sidx = host(res["stencil_idx"])
    prm = oracle.Params()
    compared = 0
    for n in (64, 96, 128, 160):
        idx, pats, ref = _oracle_index(cfg, ns, n, prm)
        q0 = cfg["lib_q"][ref["best_idx"]]
        if with_stencil:
            rr = stencil.stencil_then_refine(list(pats), cfg["master"], cfg["pcs"][idx], q0, prm)
        else:
            rr = pipeline.refine_from_match(pats, cfg["master"], cfg["pcs"][idx], cfg["pc"], q0, ref["shift"], prm)
        for a, i in enumerate(idx):
            if best[i] != ref["best_idx"][a]:
                continue
            if with_stencil and sidx[i] != rr["stencil"]["idx"][a]:
                assert rr["stencil"]["gap"][a] <= TAU_TIE
                continue
            d = np.rad2deg(rotations.disorientation_q(q[i], rr["q"][a]))
            assert d < 0.05, (n, i, d)
            assert abs(h[i] - rr["peak_h"][a]) < 1e-4, (n, i)
            assert np.max(np.abs(s[i] - rr["shift"][a])) <= 0.02 + 1e-6, (n, i)
            compared += 1
    print("[gpu]   compared %d of %d patterns" % (compared, len(ns)), flush=True)
    assert compared >= len(ns) - 2
    plan.close()

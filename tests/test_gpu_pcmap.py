"""Parity of the map-wide pattern-centre model (ebsd_pc_map) and of the
refinement from the search's beam-shift-corrected shift
(ebsd_refine_from_match) against the FP64 oracle.

PC model: bit-exact (both sides round every product and sum separately in
the same order).  Refinement: the tolerances of ebsd_refine_orientations
(0.05 deg disorientation from the oracle's orientation, peak height 1e-4,
final shift 0.02 px), on a map whose PC drifts by the spans of the paper's
wide silicon map.
"""

import numpy as np
import pytest

import oracle
from fixtures import configs
from oracle import pcmodel, pipeline, rotations

from .gpu_util import banner, dev, host, tm

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("width,p,col0,row0", [(1, 5, 0.0, 0.0), (7, 300, 3.0, 1.5), (100, 10000, 49.5, 49.5),
                                               (61, 61 * 41 - 17, 30.0, 20.0)])
def test_pc_map_bit_exact(width, p, col0, row0):
    banner("pc_map width=%d P=%d" % (width, p))
    t = tm()
    pc0 = (0.455, 0.503, 0.61)
    d_col = (0.13 / 60, -1.3e-5, 2.1e-6)
    d_row = (3.7e-6, 0.08 / 40, 0.02 / 40)
    got = host(t.pc_map(pc0, d_col, d_row, width, p, col0, row0))
    want = pcmodel.pc_map(pc0, d_col, d_row, width, p, col0, row0)
    assert got.shape == (p, 3)
    assert np.array_equal(got, want), np.max(np.abs(got - want))


def test_pc_map_empty():
    t = tm()
    assert t.pc_map((0.5, 0.5, 0.6), (0, 0, 0), (0, 0, 0), 4, 0).shape == (0, 3)


def _refine_case(t, cfg, n, pc_per=True, prm=None):
    ref_i = pipeline.index_patterns(cfg["patterns"].numpy(), cfg["master"], cfg["pc"], cfg["lib_q"],
                                    oracle.Params())
    q0 = ref_i["best_q"]
    ms = ref_i["shift"].astype(np.float32)
    pcs = cfg["pcs"] if pc_per else np.tile(np.asarray(cfg["pc"], dtype=np.float64), (len(q0), 1))
    rr = t.refine_from_match(dev(cfg["patterns"]), dev(cfg["master"]), cfg["pc"], dev(q0), dev(ms),
                             pc_per=dev(cfg["pcs"]) if pc_per else None, prm=prm)
    oprm = oracle.Params(n_iter=prm.n_iter) if prm is not None else oracle.Params()
    ref = pipeline.refine_from_match(cfg["patterns"].numpy(), cfg["master"], pcs, cfg["pc"], q0,
                                     ms.astype(np.float64), oprm)
    return rr, ref, q0


@pytest.mark.parametrize("n", [64, 96, 128, 160])
def test_refine_from_match_matches_oracle(n):
    banner("refine_from_match n=%d" % n)
    t = tm()
    cfg = configs.drift_map(seed=20 + n, rows=2, cols=3, n=n, l=200, n_grains=3)
    rr, ref, _ = _refine_case(t, cfg, n)
    q = host(rr["q"])
    d = np.rad2deg([rotations.disorientation_q(a, b) for a, b in zip(q, ref["q"])])
    assert np.max(d) < 0.05, d
    assert np.max(np.abs(host(rr["peak_h"]) - ref["peak_h"])) < 1e-4
    assert np.max(np.abs(host(rr["shift"]) - ref["shift"])) <= 0.02 + 1e-6
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-12) and np.all(q[:, 0] >= 0)


def test_refine_from_match_without_per_point_pc():
    # pc_per NULL: every point at the library's PC, the search's shift is
    # used as measured
    banner("refine_from_match pc_per=NULL")
    t = tm()
    cfg = configs.drift_map(seed=31, rows=1, cols=3, n=64, l=100, n_grains=2, span=(0.0, 0.0, 0.0))
    rr, ref, _ = _refine_case(t, cfg, 64, pc_per=False)
    d = np.rad2deg([rotations.disorientation_q(a, b) for a, b in zip(host(rr["q"]), ref["q"])])
    assert np.max(d) < 0.05, d
    assert np.max(np.abs(host(rr["peak_h"]) - ref["peak_h"])) < 1e-4


def test_refine_from_match_zero_iterations_is_final_measurement():
    t = tm()
    cfg = configs.drift_map(seed=32, rows=1, cols=3, n=64, l=60, n_grains=2)
    rr, ref, q0 = _refine_case(t, cfg, 64, prm=t.params_default(n_iter=0))
    assert np.allclose(host(rr["q"]), q0)
    assert np.max(np.abs(host(rr["peak_h"]) - ref["peak_h"])) < 1e-4

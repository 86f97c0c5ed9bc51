"""Host-side checks of the C-ABI library: it loads without a GPU, exports
every symbol the header declares, and rejects bad arguments before touching
the device (nothing is enqueued, so these run on a CPU-only host)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_1807_11313_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("library not built")
    return pkg, pkg.lib()


def _declared():
    txt = open(os.path.join(ROOT, "include", "ebsd_tm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ebsd_[a-z_0-9]+)\s*\(", txt)))


def test_header_and_binding_agree():
    pkg, _ = _lib()
    assert sorted(pkg.EXPORTS) == _declared()


def test_every_declared_symbol_is_exported():
    _, lib = _lib()
    for name in _declared():
        assert hasattr(lib, name), name


def test_defaults_and_version():
    pkg, lib = _lib()
    p = pkg.params_default()
    assert p.struct_size == ctypes.sizeof(pkg.Params)
    assert (p.window, p.sigma_hp, p.sigma_lp_frac, p.rho_max_frac) == (1, 2.0, 0.125, 0.375)
    assert (p.max_shift, p.upsample, p.n_iter, p.n_rho, p.n_eta) == (-1, 100, 2, 0, 0)
    assert pkg.version() >= 100
    assert pkg.spectrum_floats(128) == 2 * 49 * 97
    assert pkg.spectrum_floats(100) == -1


def _index(pkg, lib, batch, prm, L=10, master=None, geo=None):
    m = master or pkg.Master(0x1000, 256, 256)
    g = geo or pkg.Geometry(0.5, 0.5, 0.6, None)
    return lib.ebsd_index_patterns(ctypes.byref(batch) if batch is not None else None, ctypes.byref(m),
                                   ctypes.byref(g), ctypes.c_void_p(0x2000), L,
                                   ctypes.byref(prm) if prm is not None else None,
                                   ctypes.c_void_p(0x3000), None, ctypes.c_void_p(0x4000),
                                   ctypes.c_void_p(0x5000), None, None)


def test_argument_errors():
    pkg, lib = _lib()
    ok = pkg.Batch(0x6000, 4, 64)
    prm = pkg.params_default()
    assert _index(pkg, lib, None, prm) == -1
    assert _index(pkg, lib, pkg.Batch(0x6000, 4, 100), prm) == -4        # unsupported size
    assert _index(pkg, lib, ok, prm, L=0) == -1                          # empty library
    assert _index(pkg, lib, pkg.Batch(0x6000, -1, 64), prm) == -1
    assert _index(pkg, lib, ok, prm, master=pkg.Master(0, 256, 256)) == -1
    assert _index(pkg, lib, ok, prm, geo=pkg.Geometry(0.5, 0.5, 0.0, None)) == -1
    bad = pkg.params_default()
    bad.struct_size = 8
    assert _index(pkg, lib, ok, bad) == -1
    assert b"struct_size" in lib.ebsd_last_error()
    assert _index(pkg, lib, ok, pkg.params_default(rho_max_frac=0.45)) == -4
    assert _index(pkg, lib, ok, pkg.params_default(upsample=0)) == -1
    assert _index(pkg, lib, ok, pkg.params_default(n_eta=7)) == -1
    assert _index(pkg, lib, ok, pkg.params_default(precision=9)) == -4
    assert _index(pkg, lib, ok, pkg.params_default(max_shift=-3)) == -1
    # an empty batch is a valid no-op
    assert _index(pkg, lib, pkg.Batch(0x6000, 0, 64), prm) == 0


def test_ragged_plan_argument_errors():
    # every rejection below happens before the library touches the device
    pkg, lib = _lib()
    import numpy as np
    sizes = np.array([64, 96, 128, 160], np.int32)
    offs = np.array([0, 4096, 4096 + 9216, 4096 + 9216 + 16384], np.int64)
    h = ctypes.c_void_p()

    def create(sz, off, P=4, L=10, prm=None, step=0.5, flags=1, plan=True):
        return lib.ebsd_ragged_plan_create(None if sz is None else sz.ctypes.data_as(ctypes.c_void_p),
                                           None if off is None else off.ctypes.data_as(ctypes.c_void_p), P, L,
                                           ctypes.byref(prm) if prm is not None else None, step, flags,
                                           ctypes.byref(h) if plan else None)

    assert create(sizes, offs, plan=False) == -1
    assert create(None, offs) == -1
    assert create(sizes, offs, L=0) == -1
    assert create(sizes, offs, P=0) == -1
    assert create(sizes, offs, step=0.0) == -1
    assert create(sizes, offs, flags=64) == -1
    assert create(np.array([64, 96, 128, 256], np.int32), offs) == -4          # 256 is not a ragged size
    assert create(sizes, np.array([0, -1, 5, 6], np.int64)) == -1
    assert create(sizes, offs, prm=pkg.params_default(precision=1, max_shift=5)) == -4
    assert h.value is None
    assert lib.ebsd_ragged_plan_destroy(None) == 0


def test_pc_map_and_refine_from_match_argument_errors():
    pkg, lib = _lib()
    d3 = ctypes.c_double * 3
    good = dict(pc0=d3(0.5, 0.5, 0.6), d_col=d3(1e-3, 0, 0), d_row=d3(0, 1e-3, 0), col0=0.0, row0=0.0, width=10)

    def call(p, out=0x1000, **kw):
        m = pkg.PcModel(**dict(good, **kw))
        return lib.ebsd_pc_map(ctypes.byref(m), p, ctypes.c_void_p(out) if out else None, None)

    assert call(5, width=0) == -1 and b"width" in lib.ebsd_last_error()
    assert call(5, out=0) == -1
    assert call(-1) == -1
    assert call(5, d_col=d3(float("nan"), 0, 0)) == -1 and b"finite" in lib.ebsd_last_error()
    assert call(5, row0=float("inf")) == -1
    assert call(0, out=0) == 0
    assert lib.ebsd_pc_map(None, 5, ctypes.c_void_p(0x1000), None) == -1
    batch = pkg.Batch(0x1000, 4, 128)
    m = pkg.Master(0x2000, 256, 256)
    g = pkg.Geometry(0.5, 0.5, 0.6, None)
    rc = lib.ebsd_refine_from_match(ctypes.byref(batch), ctypes.byref(m), ctypes.byref(g), ctypes.c_void_p(0x3000),
                                    None, None, ctypes.c_void_p(0x4000), ctypes.c_void_p(0x5000),
                                    ctypes.c_void_p(0x6000), None)
    assert rc == -1 and b"match_shift" in lib.ebsd_last_error()
    empty = pkg.Batch(0x1000, 0, 128)
    assert lib.ebsd_refine_from_match(ctypes.byref(empty), ctypes.byref(m), ctypes.byref(g), None, None, None, None,
                                      None, None, None) == 0


def test_capture_range_argument_errors():
    pkg, lib = _lib()
    m = pkg.Master(0x2000, 256, 256)
    g = pkg.Geometry(0.5, 0.3, 0.6, None)
    bad_g = pkg.Geometry(0.5, 0.3, 0.0, None)
    vp = ctypes.c_void_p

    def call(R=2, n=64, T=5, geo_t=g, q=0x3000, out=0x4000):
        return lib.ebsd_capture_range(ctypes.byref(m), vp(q) if q else None, R, n, ctypes.byref(g),
                                      ctypes.byref(geo_t), vp(0x5000), T, None, vp(out) if out else None,
                                      vp(0x6000), None)

    assert call(n=100) == -4
    assert call(T=0) == -1 and b"T must be" in lib.ebsd_last_error()
    assert call(R=-1) == -1
    assert call(geo_t=bad_g) == -1 and b"pcz" in lib.ebsd_last_error()
    assert call(q=0) == -1 and call(out=0) == -1
    assert call(R=1 << 30, T=4) == -1 and b"int32" in lib.ebsd_last_error()
    assert call(R=(1 << 62), T=1000) == -1 and b"int32" in lib.ebsd_last_error()
    assert call(R=0) == 0


def test_so3_library_and_nn_argument_errors():
    _, lib = _lib()
    vp = ctypes.c_void_p
    cnt = ctypes.c_int64(-7)
    assert lib.ebsd_so3_library(0.1, None, 0, ctypes.byref(cnt), None) == -1 and b"spacing" in lib.ebsd_last_error()
    assert lib.ebsd_so3_library(float("nan"), None, 0, ctypes.byref(cnt), None) == -1
    assert lib.ebsd_so3_library(10.0, None, 5, ctypes.byref(cnt), None) == -1 and b"q_out" in lib.ebsd_last_error()
    assert lib.ebsd_so3_library(10.0, None, -1, ctypes.byref(cnt), None) == -1
    assert lib.ebsd_so3_library(10.0, None, 0, None, None) == -1
    assert cnt.value == -7
    assert lib.ebsd_nn_disorientation(vp(0x1000), 1, vp(0x2000), vp(0x3000), None) == -1
    assert lib.ebsd_nn_disorientation(vp(0x1000), 5, None, vp(0x3000), None) == -1
    assert lib.ebsd_nn_disorientation(None, 0, None, None, None) == 0


def test_binding_rejects_mismatched_shapes_before_any_call():
    # Every shape the kernels rely on is checked on the host before a pointer
    # is taken or the library is called (CPU tensors here: a shape error must
    # come before the device-tensor check)
    import numpy as np
    import torch
    pkg, _ = _lib()
    pats = torch.zeros((3, 64, 64))
    master = torch.zeros((32, 32))
    lib_q = torch.zeros((5, 4), dtype=torch.float64)
    q = torch.zeros((3, 4), dtype=torch.float64)
    ms = torch.zeros((3, 2))
    pcs = torch.zeros((3, 3), dtype=torch.float64)
    pc = (0.5, 0.5, 0.6)
    cases = [
        lambda: pkg.index_patterns(torch.zeros((3, 64, 63)), master, pc, lib_q),
        lambda: pkg.index_patterns(torch.zeros((64, 64)), master, pc, lib_q),
        lambda: pkg.index_patterns(pats, master, pc, torch.zeros((5, 3), dtype=torch.float64)),
        lambda: pkg.index_patterns(pats, torch.zeros(32), pc, lib_q),
        lambda: pkg.refine_orientations(pats, master, pc, q[:2]),
        lambda: pkg.refine_orientations(pats, master, pc, q, pc_per=pcs[:2]),
        lambda: pkg.refine_orientations(pats, master, pc, q, pc_per=torch.zeros((3, 2), dtype=torch.float64)),
        lambda: pkg.refine_from_match(pats, master, pc, q, ms[:, :1]),
        lambda: pkg.refine_from_match(pats, master, pc, q, torch.zeros((4, 2))),
        lambda: pkg.refine_from_match(pats, master, pc, q, ms, pc_per=pcs[:1]),
        lambda: pkg.project_templates(master, torch.zeros((3, 3), dtype=torch.float64), 64, pc),
        lambda: pkg.project_templates(master, q, 64, pc, pc_per=pcs[:2]),
        lambda: pkg.pattern_spectra(torch.zeros((2, 64, 32))),
        lambda: pkg.measure_rotation(pats, pats[:2]),
        lambda: pkg.xcf_scores(torch.zeros((2, 7)), torch.zeros((2, 7)), 64),
        lambda: pkg.nn_disorientation(torch.zeros((4, 3), dtype=torch.float64)),
        lambda: pkg.capture_range(master, torch.zeros((2, 3), dtype=torch.float64), 64, pc, pc,
                                  torch.zeros(5, dtype=torch.float64)),
    ]
    for k, f in enumerate(cases):
        with pytest.raises(ValueError):
            f()
    nf = pkg.spectrum_floats(64)
    sp = torch.zeros((4, nf))
    with pytest.raises(ValueError):
        pkg.xcf_subpixel(sp, sp, torch.tensor([0, 4], dtype=torch.int32), torch.tensor([0, 1], dtype=torch.int32),
                         torch.zeros((2, 2), dtype=torch.int32), 64)
    with pytest.raises(ValueError):
        pkg.xcf_peak(sp, sp, torch.tensor([0, 1], dtype=torch.int32), torch.tensor([0], dtype=torch.int32), 64)
    assert np.all(np.isfinite([nf]))


def test_noalloc_refine_rejects_on_the_host():
    # ebsd_refine_orientations_noalloc sizes the call before anything else:
    # argument errors and batches beyond its static scratch return
    # EBSD_E_INVALID (the message stating the bytes needed) without a device
    # call; an empty batch is a no-op
    pkg, lib = _lib()
    m = pkg.Master(0x1000, 256, 256)
    g = pkg.Geometry(0.5, 0.5, 0.6, None)
    prm = pkg.params_default()

    def call(batch, q=0x2000, prm=prm):
        return lib.ebsd_refine_orientations_noalloc(ctypes.byref(batch) if batch is not None else None,
                                                    ctypes.byref(m), ctypes.byref(g), ctypes.c_void_p(q),
                                                    ctypes.byref(prm), ctypes.c_void_p(0x3000),
                                                    ctypes.c_void_p(0x4000), ctypes.c_void_p(0x5000), None)

    assert call(None) == -1
    assert call(pkg.Batch(0x6000, 4, 100)) == -4
    assert call(pkg.Batch(0x6000, 4, 64), q=0) == -1
    assert call(pkg.Batch(0x6000, 4, 256)) == -4             # 256 needs a shift window
    assert call(pkg.Batch(0x6000, 0, 64)) == 0
    for n, p in ((64, 4000), (128, 1000), (160, 700), (256, 210)):
        assert call(pkg.Batch(0x6000, p, n), prm=pkg.params_default(max_shift=12)) == -1
        msg = lib.ebsd_last_error().decode()
        assert "static" in msg and "bytes" in msg, msg


def test_bf16_input_flag_is_validated():
    # the pattern storage flag: unknown values, BF16 at 256 and BF16 given to
    # calls that read no images are rejected before anything is enqueued
    pkg, lib = _lib()
    ok = pkg.Batch(0x6000, 4, 64)
    assert pkg.params_default().input == 0
    assert _index(pkg, lib, ok, pkg.params_default(input=2)) == -4
    assert _index(pkg, lib, pkg.Batch(0x6000, 4, 256), pkg.params_default(input=1, max_shift=5)) == -4
    prm = pkg.params_default(input=1)
    rc = lib.ebsd_xcf_scores(ctypes.c_void_p(0x1000), 2, ctypes.c_void_p(0x2000), 2, 64, ctypes.byref(prm),
                             ctypes.c_void_p(0x3000), None)
    assert rc == -4 and b"FP32 images" in lib.ebsd_last_error()
    # an older caller's parameter block (ending before `input`) reads as FP32
    short = pkg.params_default()
    short.struct_size = ctypes.sizeof(pkg.Params) - 4
    short.input = 7
    assert _index(pkg, lib, pkg.Batch(0x6000, 0, 64), short) == 0


def test_candidate_scores_arguments_are_checked_on_the_host():
    # ebsd_xcf_scores_cand rejects bad arguments before anything is enqueued
    pkg, lib = _lib()
    prm = pkg.params_default()
    vp = ctypes.c_void_p

    def call(n=128, p=2, l=4, k=2, cand=0x3000, prm=prm):
        return lib.ebsd_xcf_scores_cand(vp(0x1000), p, vp(0x2000), l, vp(cand) if cand else None, k, n,
                                        ctypes.byref(prm), vp(0x4000), None)

    assert call(k=5) == -1                        # K above L
    assert call(p=-1) == -1
    assert call(cand=0) == -1                     # null candidate list
    assert call(n=64) == -4                       # built at 128 only
    assert call(n=100) == -4                      # unsupported size
    assert call(prm=pkg.params_default(precision=1, max_shift=15)) == -4
    assert call(p=0) == 0 and call(k=0) == 0      # nothing to do


def test_plan_arguments_are_checked_on_the_host():
    # ebsd_plan_create / ebsd_index_patterns_plan reject bad arguments before
    # any device work; destroying a null plan is a no-op
    pkg, lib = _lib()
    vp = ctypes.c_void_p
    m = pkg.Master(0x1000, 256, 256)
    g = pkg.Geometry(0.5, 0.5, 0.6, None)
    h = vp()

    def create(n=128, L=10, q=0x2000, prm=None, out=True, master=m):
        return lib.ebsd_plan_create(ctypes.byref(master), ctypes.byref(g), vp(q) if q else None, L, n,
                                    ctypes.byref(prm or pkg.params_default()), ctypes.byref(h) if out else None,
                                    None)

    assert create(out=False) == -1
    assert create(L=0) == -1
    assert create(q=0) == -1
    assert create(n=100) == -4
    assert create(n=256) == -4                              # 256 needs a shift window
    assert create(master=pkg.Master(0x1000, 0, 256)) == -1
    b = pkg.Batch(0x3000, 4, 128)
    assert lib.ebsd_index_patterns_plan(None, ctypes.byref(b), vp(1), None, vp(2), vp(3), None, None) == -1
    assert lib.ebsd_plan_destroy(None) == 0


def test_cnn_precision_is_checked_on_the_host():
    import paper_1807_11313_amd as pkg
    lib = pkg.lib()
    assert lib.ebsd_cnn_set_precision(None, pkg.PREC_FP32) == -1
    assert lib.ebsd_cnn_set_precision(None, pkg.PREC_BF16X2) == -1

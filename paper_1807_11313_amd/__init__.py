"""Python binding of libebsd_tm.so, the gfx950 hot path of refined template
matching for EBSD indexing (arXiv 1807.11313).

Argument marshalling only: every step runs in the HIP kernels behind the C
ABI of ``include/ebsd_tm.h``.  Tensors must be contiguous CUDA (HIP) tensors
of the stated dtype; work is enqueued on torch's current stream.  There is no
CPU fallback: if the shared library is missing or fails to load, importing
the binding functions raises.
"""

import ctypes
import os

import numpy as np

__all__ = ["lib", "Params", "index_patterns", "refine_orientations", "project_templates",
           "pattern_spectra", "spectrum_floats", "xcf_peak", "xcf_scores", "xcf_scores_cand", "xcf_subpixel",
           "measure_rotation", "params_default", "version", "RaggedPlan", "Cnn", "cnn_make_batch", "cnn_topk",
           "index_proposed", "refine_from_match", "pc_map", "PcModel", "capture_range", "so3_library",
           "nn_disorientation", "LibraryPlan", "LIB_PATH", "EXPORTS", "PREC_FP32", "PREC_FP16X2", "PREC_BF16X2",
           "PREC_BF16"]

# precision constants of the header (ebsd_params.precision, Cnn.set_precision)
PREC_FP32, PREC_FP16X2, PREC_BF16X2, PREC_BF16 = 0, 1, 2, 3

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libebsd_tm.so")

# Every function the header declares.
EXPORTS = ("ebsd_params_default", "ebsd_version", "ebsd_last_error", "ebsd_index_patterns",
           "ebsd_refine_orientations", "ebsd_refine_orientations_noalloc", "ebsd_project_templates", "ebsd_pattern_spectra",
           "ebsd_spectrum_floats", "ebsd_xcf_peak", "ebsd_xcf_scores", "ebsd_xcf_scores_cand", "ebsd_xcf_subpixel",
           "ebsd_measure_rotation", "ebsd_timing_enable", "ebsd_timing_read", "ebsd_ragged_plan_create",
           "ebsd_ragged_run", "ebsd_ragged_plan_tiles", "ebsd_ragged_plan_destroy", "ebsd_cnn_param_count",
           "ebsd_cnn_create", "ebsd_cnn_destroy", "ebsd_cnn_get_params", "ebsd_cnn_set_params", "ebsd_cnn_input",
           "ebsd_cnn_forward", "ebsd_cnn_set_precision", "ebsd_cnn_gradients", "ebsd_cnn_train_step",
           "ebsd_cnn_apply_gradient", "ebsd_cnn_make_batch", "ebsd_cnn_topk",
           "ebsd_index_proposed", "ebsd_pc_map", "ebsd_refine_from_match", "ebsd_capture_range",
           "ebsd_so3_library", "ebsd_nn_disorientation", "ebsd_plan_create", "ebsd_index_patterns_plan",
           "ebsd_plan_destroy")

RAGGED_STENCIL, RAGGED_EAGER, RAGGED_NO_AUTOTUNE, RAGGED_REFINE = 1, 2, 4, 8

EBSD_OK = 0
ERRORS = {-1: "EBSD_E_INVALID", -2: "EBSD_E_NOMEM", -3: "EBSD_E_DEVICE", -4: "EBSD_E_UNSUPPORTED"}


class Batch(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("P", ctypes.c_int64), ("n", ctypes.c_int32)]


class Master(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32)]


class Geometry(ctypes.Structure):
    _fields_ = [("pcx", ctypes.c_double), ("pcy", ctypes.c_double), ("pcz", ctypes.c_double),
                ("pc_per", ctypes.c_void_p)]


class PcModel(ctypes.Structure):
    _fields_ = [("pc0", ctypes.c_double * 3), ("d_col", ctypes.c_double * 3), ("d_row", ctypes.c_double * 3),
                ("col0", ctypes.c_double), ("row0", ctypes.c_double), ("width", ctypes.c_int64)]


class Params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("window", ctypes.c_int32),
                ("sigma_hp", ctypes.c_double), ("sigma_lp_frac", ctypes.c_double),
                ("rho_max_frac", ctypes.c_double), ("max_shift", ctypes.c_int32),
                ("upsample", ctypes.c_int32), ("n_iter", ctypes.c_int32), ("n_rho", ctypes.c_int32),
                ("n_eta", ctypes.c_int32), ("precision", ctypes.c_int32), ("form", ctypes.c_int32),
                ("input", ctypes.c_int32)]


class EbsdError(RuntimeError):
    def __init__(self, code, func, msg):
        super().__init__("%s failed: %s (%d): %s" % (func, ERRORS.get(code, "?"), code, msg))
        self.code = code


_lib = None


def lib():
    """Loads the shared library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libebsd_tm.so is not built at %s; run paper_1807_11313_amd/build.py" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER
    L.ebsd_params_default.argtypes = [dp(Params)]
    L.ebsd_params_default.restype = None
    L.ebsd_version.restype = ctypes.c_int
    L.ebsd_last_error.restype = ctypes.c_char_p
    L.ebsd_spectrum_floats.argtypes = [i32]
    L.ebsd_spectrum_floats.restype = i64
    L.ebsd_index_patterns.argtypes = [dp(Batch), dp(Master), dp(Geometry), vp, i64, dp(Params), vp, vp, vp, vp,
                                      vp, vp]
    L.ebsd_refine_orientations.argtypes = [dp(Batch), dp(Master), dp(Geometry), vp, dp(Params), vp, vp, vp, vp]
    L.ebsd_plan_create.argtypes = [dp(Master), dp(Geometry), vp, i64, i32, dp(Params), dp(vp), vp]
    L.ebsd_index_patterns_plan.argtypes = [vp, dp(Batch), vp, vp, vp, vp, vp, vp]
    L.ebsd_plan_destroy.argtypes = [vp]
    L.ebsd_refine_orientations_noalloc.argtypes = [dp(Batch), dp(Master), dp(Geometry), vp, dp(Params), vp, vp, vp,
                                                   vp]
    L.ebsd_refine_from_match.argtypes = [dp(Batch), dp(Master), dp(Geometry), vp, vp, dp(Params), vp, vp, vp, vp]
    L.ebsd_pc_map.argtypes = [dp(PcModel), i64, vp, vp]
    L.ebsd_so3_library.argtypes = [ctypes.c_double, vp, i64, dp(i64), vp]
    L.ebsd_nn_disorientation.argtypes = [vp, i64, vp, vp, vp]
    L.ebsd_capture_range.argtypes = [dp(Master), vp, i64, i32, dp(Geometry), dp(Geometry), vp, i32, dp(Params), vp,
                                     vp, vp]
    L.ebsd_project_templates.argtypes = [dp(Master), vp, i64, i32, dp(Geometry), vp, vp]
    L.ebsd_pattern_spectra.argtypes = [vp, i64, i32, dp(Params), vp, vp, vp]
    L.ebsd_xcf_peak.argtypes = [vp, vp, vp, vp, i64, i32, dp(Params), vp, vp, vp, vp]
    L.ebsd_xcf_scores.argtypes = [vp, i64, vp, i64, i32, dp(Params), vp, vp]
    L.ebsd_xcf_scores_cand.argtypes = [vp, i64, vp, i64, vp, i32, i32, dp(Params), vp, vp]
    L.ebsd_xcf_subpixel.argtypes = [vp, vp, vp, vp, i64, i32, vp, dp(Params), vp, vp, vp]
    L.ebsd_measure_rotation.argtypes = [vp, vp, i64, i32, dp(Params), vp, vp]
    L.ebsd_timing_enable.argtypes = [ctypes.c_int]
    L.ebsd_timing_read.argtypes = [dp(ctypes.c_double), dp(ctypes.c_int64)]
    L.ebsd_ragged_plan_create.argtypes = [vp, vp, i64, i64, dp(Params), ctypes.c_double, i32, dp(vp)]
    L.ebsd_ragged_run.argtypes = [vp, vp, dp(Master), dp(Geometry), vp, vp, vp, vp, vp, vp, vp]
    L.ebsd_ragged_plan_tiles.argtypes = [vp, vp, dp(i32)]
    L.ebsd_ragged_plan_destroy.argtypes = [vp]
    u64, f32, f64 = ctypes.c_uint64, ctypes.c_float, ctypes.c_double
    L.ebsd_cnn_param_count.argtypes = [i32]
    L.ebsd_cnn_param_count.restype = i64
    L.ebsd_cnn_create.argtypes = [i32, u64, dp(vp), vp]
    L.ebsd_cnn_destroy.argtypes = [vp]
    L.ebsd_cnn_get_params.argtypes = [vp, vp, vp]
    L.ebsd_cnn_set_params.argtypes = [vp, vp, vp]
    L.ebsd_cnn_input.argtypes = [vp, i64, i32, vp, vp]
    L.ebsd_cnn_forward.argtypes = [vp, vp, i64, vp, vp]
    L.ebsd_cnn_set_precision.argtypes = [vp, i32]
    L.ebsd_cnn_gradients.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.ebsd_cnn_train_step.argtypes = [vp, vp, vp, i64, f32, vp, vp]
    L.ebsd_cnn_apply_gradient.argtypes = [vp, vp, f32, vp]
    L.ebsd_cnn_make_batch.argtypes = [dp(Master), dp(Geometry), vp, i64, i32, i64, i64, u64, f64, f64, f64, vp, vp,
                                      vp, vp]
    L.ebsd_cnn_topk.argtypes = [vp, i64, i32, i32, vp, vp]
    L.ebsd_index_proposed.argtypes = [dp(Batch), dp(Master), dp(Geometry), vp, i64, vp, i32, f32, dp(Params), vp,
                                      vp, vp, vp, vp, vp]
    for name in EXPORTS:
        if name not in ("ebsd_params_default", "ebsd_version", "ebsd_last_error", "ebsd_spectrum_floats",
                        "ebsd_cnn_param_count"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def params_default(**kw):
    p = Params()
    lib().ebsd_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def version():
    return lib().ebsd_version()


def spectrum_floats(n):
    return lib().ebsd_spectrum_floats(n)


def _check(rc, func):
    if rc != EBSD_OK:
        raise EbsdError(rc, func, lib().ebsd_last_error().decode())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    return ctypes.c_void_p(t.data_ptr())


def _shape(t, shape, name):
    """Raises ValueError unless t has the given shape (None = any extent)."""
    if t is None:
        return
    if t.dim() != len(shape) or any(w is not None and g != w for g, w in zip(t.shape, shape)):
        want = "(" + ", ".join("*" if w is None else str(w) for w in shape) + ")"
        raise ValueError("%s must have shape %s, got %s" % (name, want, tuple(t.shape)))


def _patterns(patterns):
    """(P, n) of a [P][n][n] pattern stack."""
    if patterns.dim() != 3 or patterns.shape[1] != patterns.shape[2]:
        raise ValueError("patterns must be [P][n][n], got %s" % (tuple(patterns.shape),))
    return patterns.shape[0], patterns.shape[2]


def _master(master):
    import torch
    _shape(master, (None, None), "master")
    return Master(_ptr(master, torch.float32, "master").value, master.shape[0], master.shape[1])


def _geo(pc, pc_per=None, p=None):
    import torch
    _shape(pc_per, (p, 3), "pc_per")
    return Geometry(float(pc[0]), float(pc[1]), float(pc[2]),
                    None if pc_per is None else _ptr(pc_per, torch.float64, "pc_per").value)


def _params(prm):
    return ctypes.byref(prm) if prm is not None else None


INPUT_F32, INPUT_BF16 = 0, 1


def _images(patterns, prm, name="patterns"):
    """Pointer to float32 or bfloat16 pattern images and the parameter block
    that states their storage (a copy of prm, or the defaults, with input set
    for bfloat16)."""
    import torch
    if patterns.dtype == torch.bfloat16:
        q = Params()
        if prm is None:
            lib().ebsd_params_default(ctypes.byref(q))
        else:
            ctypes.memmove(ctypes.byref(q), ctypes.byref(prm), ctypes.sizeof(Params))
        q.input = INPUT_BF16
        return _ptr(patterns, torch.bfloat16, name), q
    return _ptr(patterns, torch.float32, name), prm


def index_patterns(patterns, master, pc, lib_q, prm=None, scores=False):
    """Returns dict(best_idx, best_q, peak_h, shift[, scores]) as CUDA tensors."""
    import torch
    p, n = _patterns(patterns)
    _shape(lib_q, (None, 4), "lib_q")
    _shape(master, (None, None), "master")
    dev = patterns.device
    out = dict(best_idx=torch.empty(p, dtype=torch.int32, device=dev),
               best_q=torch.empty((p, 4), dtype=torch.float64, device=dev),
               peak_h=torch.empty(p, dtype=torch.float32, device=dev),
               shift=torch.empty((p, 2), dtype=torch.float32, device=dev))
    if scores:
        out["scores"] = torch.empty((p, lib_q.shape[0]), dtype=torch.float32, device=dev)
    data, prm = _images(patterns, prm)
    batch = Batch(data.value, p, n)
    rc = lib().ebsd_index_patterns(ctypes.byref(batch), ctypes.byref(_master(master)), ctypes.byref(_geo(pc)),
                                   _ptr(lib_q, torch.float64, "lib_q"), lib_q.shape[0], _params(prm),
                                   _ptr(out["best_idx"]), _ptr(out["best_q"]), _ptr(out["peak_h"]),
                                   _ptr(out["shift"]), _ptr(out.get("scores")), _stream())
    _check(rc, "ebsd_index_patterns")
    return out


class LibraryPlan:
    """A library whose template spectra are computed once (ebsd_plan_create):
    index(patterns) then searches it like index_patterns."""

    def __init__(self, master, pc, lib_q, n, prm=None, input_bf16=False):
        import torch
        _shape(lib_q, (None, 4), "lib_q")
        _shape(master, (None, None), "master")
        self.n, self.L = int(n), int(lib_q.shape[0])
        self.input_bf16 = bool(input_bf16)
        q = Params()
        if prm is None:
            lib().ebsd_params_default(ctypes.byref(q))
        else:
            ctypes.memmove(ctypes.byref(q), ctypes.byref(prm), ctypes.sizeof(Params))
        if self.input_bf16:
            q.input = INPUT_BF16
        h = ctypes.c_void_p()
        _check(lib().ebsd_plan_create(ctypes.byref(_master(master)), ctypes.byref(_geo(pc)),
                                      _ptr(lib_q, torch.float64, "lib_q"), self.L, self.n, ctypes.byref(q),
                                      ctypes.byref(h), _stream()), "ebsd_plan_create")
        self._h = h

    def index(self, patterns, scores=False):
        import torch
        p, n = _patterns(patterns)
        if n != self.n:
            raise ValueError("patterns are %d x %d, the plan is for %d" % (n, n, self.n))
        if (patterns.dtype == torch.bfloat16) != self.input_bf16:
            raise ValueError("pattern storage differs from the plan's")
        dev = patterns.device
        out = dict(best_idx=torch.empty(p, dtype=torch.int32, device=dev),
                   best_q=torch.empty((p, 4), dtype=torch.float64, device=dev),
                   peak_h=torch.empty(p, dtype=torch.float32, device=dev),
                   shift=torch.empty((p, 2), dtype=torch.float32, device=dev))
        if scores:
            out["scores"] = torch.empty((p, self.L), dtype=torch.float32, device=dev)
        dtype = torch.bfloat16 if self.input_bf16 else torch.float32
        batch = Batch(_ptr(patterns, dtype, "patterns").value, p, n)
        _check(lib().ebsd_index_patterns_plan(self._h, ctypes.byref(batch), _ptr(out["best_idx"]),
                                              _ptr(out["best_q"]), _ptr(out["peak_h"]), _ptr(out["shift"]),
                                              _ptr(out.get("scores")), _stream()), "ebsd_index_patterns_plan")
        return out

    def close(self):
        if getattr(self, "_h", None):
            import torch
            torch.cuda.current_stream().synchronize()  # the plan's calls must have finished
            lib().ebsd_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def refine_orientations(patterns, master, pc, q_init, pc_per=None, prm=None, out=None, noalloc=False):
    """Returns dict(q, peak_h, shift) as CUDA tensors (or fills `out`, a dict
    of such tensors).  noalloc=True calls ebsd_refine_orientations_noalloc,
    which allocates no device memory (the binding allocates none either when
    `out` is given)."""
    import torch
    p, n = _patterns(patterns)
    _shape(q_init, (p, 4), "q_init")
    _shape(pc_per, (p, 3), "pc_per")
    _shape(master, (None, None), "master")
    dev = patterns.device
    if out is None:
        out = dict(q=torch.empty((p, 4), dtype=torch.float64, device=dev),
                   peak_h=torch.empty(p, dtype=torch.float32, device=dev),
                   shift=torch.empty((p, 2), dtype=torch.float32, device=dev))
    for key, shape in (("q", (p, 4)), ("peak_h", (p,)), ("shift", (p, 2))):
        _shape(out[key], shape, key)
    data, prm = _images(patterns, prm)
    batch = Batch(data.value, p, n)
    name = "ebsd_refine_orientations_noalloc" if noalloc else "ebsd_refine_orientations"
    rc = getattr(lib(), name)(ctypes.byref(batch), ctypes.byref(_master(master)), ctypes.byref(_geo(pc, pc_per, p)),
                              _ptr(q_init, torch.float64, "q_init"), _params(prm),
                              _ptr(out["q"], torch.float64, "q"), _ptr(out["peak_h"], torch.float32, "peak_h"),
                              _ptr(out["shift"], torch.float32, "shift"), _stream())
    _check(rc, name)
    return out


def refine_from_match(patterns, master, pc, q_init, match_shift, pc_per=None, prm=None):
    """Refinement whose first x/y step reuses the search's shift (match_shift
    float32 [P, 2] (x, y) px against the library projected at pc), less the
    beam-induced move to pc_per.  Returns dict(q, peak_h, shift) as CUDA
    tensors."""
    import torch
    p, n = _patterns(patterns)
    _shape(q_init, (p, 4), "q_init")
    _shape(pc_per, (p, 3), "pc_per")
    _shape(master, (None, None), "master")
    _shape(match_shift, (p, 2), "match_shift")
    dev = patterns.device
    out = dict(q=torch.empty((p, 4), dtype=torch.float64, device=dev),
               peak_h=torch.empty(p, dtype=torch.float32, device=dev),
               shift=torch.empty((p, 2), dtype=torch.float32, device=dev))
    data, prm = _images(patterns, prm)
    batch = Batch(data.value, p, n)
    rc = lib().ebsd_refine_from_match(ctypes.byref(batch), ctypes.byref(_master(master)),
                                      ctypes.byref(_geo(pc, pc_per, p)), _ptr(q_init, torch.float64, "q_init"),
                                      _ptr(match_shift, torch.float32, "match_shift"), _params(prm),
                                      _ptr(out["q"]), _ptr(out["peak_h"]), _ptr(out["shift"]), _stream())
    _check(rc, "ebsd_refine_from_match")
    return out


def pc_map(pc0, d_col, d_row, width, p, col0=0.0, row0=0.0, device="cuda"):
    """Per-point pattern centres float64 [p, 3] of the affine map model."""
    import torch
    out = torch.empty((p, 3), dtype=torch.float64, device=device)
    m = PcModel((ctypes.c_double * 3)(*map(float, pc0)), (ctypes.c_double * 3)(*map(float, d_col)),
                (ctypes.c_double * 3)(*map(float, d_row)), float(col0), float(row0), int(width))
    rc = lib().ebsd_pc_map(ctypes.byref(m), p, _ptr(out) if p > 0 else None, _stream())
    _check(rc, "ebsd_pc_map")
    return out


def so3_library(spacing_deg, device="cuda"):
    """Equispaced fundamental-zone orientation library float64 [L, 4]."""
    import torch
    count = ctypes.c_int64(0)
    _check(lib().ebsd_so3_library(float(spacing_deg), None, 0, ctypes.byref(count), _stream()), "ebsd_so3_library")
    out = torch.empty((max(count.value, 1), 4), dtype=torch.float64, device=device)
    n = ctypes.c_int64(0)
    _check(lib().ebsd_so3_library(float(spacing_deg), _ptr(out), count.value, ctypes.byref(n), _stream()),
           "ebsd_so3_library")
    return out[:n.value]


def nn_disorientation(q):
    """Nearest-neighbour cubic disorientation (degrees, float64 [L]) and index
    (int32 [L]) within q [L, 4]."""
    import torch
    _shape(q, (None, 4), "q")
    n = q.shape[0]
    ang = torch.empty(n, dtype=torch.float64, device=q.device)
    idx = torch.empty(n, dtype=torch.int32, device=q.device)
    _check(lib().ebsd_nn_disorientation(_ptr(q, torch.float64, "q"), n, _ptr(ang), _ptr(idx), _stream()),
           "ebsd_nn_disorientation")
    return ang, idx


def capture_range(master, q_ref, n, pc_ref, pc_test, theta_deg, prm=None):
    """Capture curves h float32 [R, 3, T] (axes x, y, z) and their FWHM
    float64 [R, 3] (degrees) for reference orientations q_ref [R, 4] and
    ascending angles theta_deg [T] (CUDA float64)."""
    import torch
    _shape(q_ref, (None, 4), "q_ref")
    _shape(theta_deg, (None,), "theta_deg")
    r, t = q_ref.shape[0], theta_deg.shape[0]
    h = torch.empty((r, 3, t), dtype=torch.float32, device=q_ref.device)
    width = torch.empty((r, 3), dtype=torch.float64, device=q_ref.device)
    rc = lib().ebsd_capture_range(ctypes.byref(_master(master)), _ptr(q_ref, torch.float64, "q_ref"), r, n,
                                  ctypes.byref(_geo(pc_ref)), ctypes.byref(_geo(pc_test)),
                                  _ptr(theta_deg, torch.float64, "theta_deg"), t, _params(prm), _ptr(h), _ptr(width),
                                  _stream())
    _check(rc, "ebsd_capture_range")
    return h, width


def project_templates(master, q, n, pc, pc_per=None):
    import torch
    _shape(q, (None, 4), "q")
    _shape(pc_per, (q.shape[0], 3), "pc_per")
    out = torch.empty((q.shape[0], n, n), dtype=torch.float32, device=q.device)
    rc = lib().ebsd_project_templates(ctypes.byref(_master(master)), _ptr(q, torch.float64, "q"), q.shape[0], n,
                                      ctypes.byref(_geo(pc, pc_per, q.shape[0])), _ptr(out), _stream())
    _check(rc, "ebsd_project_templates")
    return out


def pattern_spectra(imgs, prm=None, energy=False):
    """Unit-energy band spectra [K][B+1][2B+1] complex64 (and FP64 energies)."""
    import torch
    k, n = _patterns(imgs)
    nf = spectrum_floats(n)
    if nf < 0:
        raise ValueError("unsupported size %d" % n)
    spec = torch.empty((k, nf), dtype=torch.float32, device=imgs.device)
    en = torch.empty(k, dtype=torch.float64, device=imgs.device) if energy else None
    data, prm = _images(imgs, prm, "imgs")
    rc = lib().ebsd_pattern_spectra(data, k, n, _params(prm), _ptr(spec), _ptr(en), _stream())
    _check(rc, "ebsd_pattern_spectra")
    return (spec, en) if energy else spec


def _spectra_and_pairs(spec_p, spec_l, pi, li, n):
    """Checks band spectra [*][floats(n)] and, for index arrays, that every
    index lies in its stack (a device read: these are test hooks)."""
    nf = spectrum_floats(n)
    if nf < 0:
        raise ValueError("unsupported size %d" % n)
    _shape(spec_p, (None, nf), "spec_p")
    _shape(spec_l, (None, nf), "spec_l")
    if pi is None:
        if spec_l.shape[0] != spec_p.shape[0]:
            raise ValueError("without index arrays spec_p and spec_l pair row by row")
        return spec_p.shape[0]
    _shape(pi, (None,), "pi")
    _shape(li, (pi.shape[0],), "li")
    k = pi.shape[0]
    if k and (int(pi.min()) < 0 or int(pi.max()) >= spec_p.shape[0] or int(li.min()) < 0
              or int(li.max()) >= spec_l.shape[0]):
        raise ValueError("pair index out of range")
    return k


def xcf_peak(spec_p, spec_l, pi, li, n, prm=None, want_map=False):
    import torch
    k = _spectra_and_pairs(spec_p, spec_l, pi, li, n)
    dev = spec_p.device
    h = torch.empty(k, dtype=torch.float32, device=dev)
    s = torch.empty((k, 2), dtype=torch.int32, device=dev)
    mp = torch.empty((k, n, n), dtype=torch.float32, device=dev) if want_map else None
    rc = lib().ebsd_xcf_peak(_ptr(spec_p, torch.float32), _ptr(spec_l, torch.float32),
                             _ptr(pi, torch.int32, "pi"), _ptr(li, torch.int32, "li"), k, n, _params(prm),
                             _ptr(h), _ptr(s), _ptr(mp), _stream())
    _check(rc, "ebsd_xcf_peak")
    return (h, s, mp) if want_map else (h, s)


def xcf_scores(spec_p, spec_l, n, prm=None):
    import torch
    nf = spectrum_floats(n)
    if nf < 0:
        raise ValueError("unsupported size %d" % n)
    _shape(spec_p, (None, nf), "spec_p")
    _shape(spec_l, (None, nf), "spec_l")
    p, l = spec_p.shape[0], spec_l.shape[0]
    out = torch.empty((p, l), dtype=torch.float32, device=spec_p.device)
    rc = lib().ebsd_xcf_scores(_ptr(spec_p, torch.float32), p, _ptr(spec_l, torch.float32), l, n, _params(prm),
                               _ptr(out), _stream())
    _check(rc, "ebsd_xcf_scores")
    return out


def xcf_scores_cand(spec_p, spec_l, cand, n, prm=None):
    """scores[p][j] of pattern p against template cand[p][j] (n = 128)."""
    import torch
    nf = spectrum_floats(n)
    if nf < 0:
        raise ValueError("unsupported size %d" % n)
    _shape(spec_p, (None, nf), "spec_p")
    _shape(spec_l, (None, nf), "spec_l")
    p, l = spec_p.shape[0], spec_l.shape[0]
    _shape(cand, (p, None), "cand")
    k = cand.shape[1]
    out = torch.empty((p, k), dtype=torch.float32, device=spec_p.device)
    rc = lib().ebsd_xcf_scores_cand(_ptr(spec_p, torch.float32), p, _ptr(spec_l, torch.float32), l,
                                    _ptr(cand, torch.int32, "cand"), k, n, _params(prm), _ptr(out), _stream())
    _check(rc, "ebsd_xcf_scores_cand")
    return out


def xcf_subpixel(spec_p, spec_l, pi, li, s_int, n, prm=None):
    import torch
    k = _spectra_and_pairs(spec_p, spec_l, pi, li, n)
    _shape(s_int, (k, 2), "s_int")
    h = torch.empty(k, dtype=torch.float32, device=spec_p.device)
    s = torch.empty((k, 2), dtype=torch.float32, device=spec_p.device)
    rc = lib().ebsd_xcf_subpixel(_ptr(spec_p, torch.float32), _ptr(spec_l, torch.float32),
                                 _ptr(pi, torch.int32, "pi"), _ptr(li, torch.int32, "li"), k, n,
                                 _ptr(s_int, torch.int32, "s_int"), _params(prm), _ptr(h), _ptr(s), _stream())
    _check(rc, "ebsd_xcf_subpixel")
    return h, s


def measure_rotation(pats, tmpls, prm=None):
    import torch
    k, n = _patterns(pats)
    _shape(tmpls, (k, n, n), "tmpls")
    g = torch.empty(k, dtype=torch.float64, device=pats.device)
    rc = lib().ebsd_measure_rotation(_ptr(pats, torch.float32, "pats"), _ptr(tmpls, torch.float32, "tmpls"), k, n,
                                     _params(prm), _ptr(g), _stream())
    _check(rc, "ebsd_measure_rotation")
    return g


def timing_enable(on=True):
    lib().ebsd_timing_enable(1 if on else 0)


def timing_read():
    """(total ms, launches) of the search kernel since the last read."""
    ms, cnt = ctypes.c_double(), ctypes.c_int64()
    _check(lib().ebsd_timing_read(ctypes.byref(ms), ctypes.byref(cnt)), "ebsd_timing_read")
    return ms.value, cnt.value


def spectra_to_complex(spec, n):
    """Host copy of a [K][floats] spectrum tensor (stored [kk][v]) as complex [K][v][kk]."""
    b = 3 * n // 8
    a = spec.detach().cpu().numpy().reshape(spec.shape[0], 2 * b + 1, b + 1, 2)
    return np.swapaxes(a[..., 0] + 1j * a[..., 1], 1, 2)


def band_to_full(band, n):
    """Place a [.., B+1, 2B+1] band spectrum onto the full n x n grid X[u, v]
    (Hermitian completion for v < 0); used to compare with full-grid spectra."""
    b = 3 * n // 8
    full = np.zeros(band.shape[:-2] + (n, n), dtype=np.complex128)
    u = np.concatenate([np.arange(0, b + 1), np.arange(-b, 0)]) % n
    for v in range(b + 1):
        full[..., u, v] = band[..., v, :]
        if v > 0:
            full[..., (-u) % n, n - v] = np.conj(band[..., v, :])
    return full


class RaggedPlan:
    """A ragged batch layout (ebsd_ragged_plan_create): pattern p of side
    sizes[p] at element offset offsets[p] of one packed float32 buffer
    (host arrays), a library of L orientations and the parameters."""

    def __init__(self, sizes, offsets, L, prm=None, stencil=True, step_deg=0.5, eager=False, autotune=True,
                 refine=False):
        sizes = np.ascontiguousarray(sizes, dtype=np.int32)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        if sizes.shape != offsets.shape or sizes.ndim != 1:
            raise ValueError("sizes and offsets must be 1-D arrays of equal length")
        self.P, self.L = int(sizes.shape[0]), int(L)
        self.min_floats = int(np.max(offsets + sizes.astype(np.int64) ** 2)) if self.P else 0
        flags = (RAGGED_STENCIL if stencil else 0) | (RAGGED_EAGER if eager else 0) | \
            (0 if autotune else RAGGED_NO_AUTOTUNE) | (RAGGED_REFINE if refine else 0)
        h = ctypes.c_void_p()
        _check(lib().ebsd_ragged_plan_create(sizes.ctypes.data_as(ctypes.c_void_p),
                                             offsets.ctypes.data_as(ctypes.c_void_p), self.P, self.L,
                                             _params(prm), float(step_deg), flags, ctypes.byref(h)),
               "ebsd_ragged_plan_create")
        self._h = h

    def run(self, data, master, pc, lib_q, pc_per=None, stencil_idx=True):
        import torch
        dev = data.device
        p = self.P
        out = dict(best_idx=torch.empty(p, dtype=torch.int32, device=dev),
                   q=torch.empty((p, 4), dtype=torch.float64, device=dev),
                   peak_h=torch.empty(p, dtype=torch.float32, device=dev),
                   shift=torch.empty((p, 2), dtype=torch.float32, device=dev))
        if stencil_idx:
            out["stencil_idx"] = torch.empty(p, dtype=torch.int32, device=dev)
        self.run_into(data, master, pc, lib_q, out, pc_per)
        return out

    def run_into(self, data, master, pc, lib_q, out, pc_per=None):
        import torch
        if lib_q.shape[0] != self.L:
            raise ValueError("library size differs from the plan's")
        _shape(lib_q, (self.L, 4), "lib_q")
        _shape(data, (None,), "data")
        if data.shape[0] < self.min_floats:
            raise ValueError("data holds %d floats, the layout needs %d" % (data.shape[0], self.min_floats))
        for key, shape in (("best_idx", (self.P,)), ("q", (self.P, 4)), ("peak_h", (self.P,)),
                           ("shift", (self.P, 2)), ("stencil_idx", (self.P,))):
            _shape(out.get(key), shape, key)
        m, g = _master(master), _geo(pc, pc_per, self.P)
        _check(lib().ebsd_ragged_run(self._h, _ptr(data, torch.float32, "data"), ctypes.byref(m), ctypes.byref(g),
                                     _ptr(lib_q, torch.float64, "lib_q"), _ptr(out.get("best_idx")),
                                     _ptr(out["q"]), _ptr(out["peak_h"]), _ptr(out["shift"]),
                                     _ptr(out.get("stencil_idx")), _stream()),
               "ebsd_ragged_run")
        return out

    def tiles(self):
        t = (ctypes.c_int32 * 16)()
        c = ctypes.c_int32()
        _check(lib().ebsd_ragged_plan_tiles(self._h, t, ctypes.byref(c)), "ebsd_ragged_plan_tiles")
        return [dict(n=t[4 * k], patterns=t[4 * k + 1], templates_per_item=t[4 * k + 2], grid=t[4 * k + 3])
                for k in range(c.value)]

    def close(self):
        if getattr(self, "_h", None):
            lib().ebsd_ragged_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Cnn:
    """The proposal network (ebsd_cnn_*): parameters, Adam state and
    workspace on the current device."""

    def __init__(self, n_classes, seed=0):
        self.n_classes = int(n_classes)
        h = ctypes.c_void_p()
        _check(lib().ebsd_cnn_create(self.n_classes, int(seed), ctypes.byref(h), _stream()), "ebsd_cnn_create")
        self._h = h

    @property
    def param_count(self):
        return lib().ebsd_cnn_param_count(self.n_classes)

    def get_params(self):
        import torch
        out = torch.empty(self.param_count, dtype=torch.float32, device="cuda")
        _check(lib().ebsd_cnn_get_params(self._h, _ptr(out), _stream()), "ebsd_cnn_get_params")
        return out

    def set_params(self, t):
        import torch
        if t.numel() != self.param_count:
            raise ValueError("expected %d parameters" % self.param_count)
        _check(lib().ebsd_cnn_set_params(self._h, _ptr(t, torch.float32, "params"), _stream()),
               "ebsd_cnn_set_params")

    @staticmethod
    def input(patterns):
        import torch
        p, n = _patterns(patterns)
        x = torch.empty((p, 64, 64), dtype=torch.float32, device=patterns.device)
        _check(lib().ebsd_cnn_input(_ptr(patterns, torch.float32, "patterns"), p, n, _ptr(x), _stream()),
               "ebsd_cnn_input")
        return x

    def forward(self, x):
        import torch
        _shape(x, (None, 64, 64), "x")
        out = torch.empty((x.shape[0], self.n_classes), dtype=torch.float32, device=x.device)
        _check(lib().ebsd_cnn_forward(self._h, _ptr(x, torch.float32, "x"), x.shape[0], _ptr(out), _stream()),
               "ebsd_cnn_forward")
        return out

    def set_precision(self, precision):
        """Precision of the inference, training fc and backward products: PREC_BF16X2 (default) or PREC_FP32."""
        _check(lib().ebsd_cnn_set_precision(self._h, int(precision)), "ebsd_cnn_set_precision")

    def gradients(self, x, labels):
        import torch
        _shape(x, (None, 64, 64), "x")
        _shape(labels, (x.shape[0],), "labels")
        g = torch.empty(self.param_count, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(lib().ebsd_cnn_gradients(self._h, _ptr(x, torch.float32, "x"), _ptr(labels, torch.int32, "labels"),
                                        x.shape[0], _ptr(g), _ptr(loss), _stream()), "ebsd_cnn_gradients")
        return g, loss

    def train_step(self, x, labels, lr, loss=None):
        import torch
        _shape(x, (None, 64, 64), "x")
        _shape(labels, (x.shape[0],), "labels")
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(lib().ebsd_cnn_train_step(self._h, _ptr(x, torch.float32, "x"), _ptr(labels, torch.int32, "labels"),
                                         x.shape[0], float(lr), _ptr(loss), _stream()), "ebsd_cnn_train_step")
        return loss

    def apply_gradient(self, grad, lr):
        """One Adam step from a given gradient (float32 [param_count])."""
        import torch
        if grad.numel() != self.param_count:
            raise ValueError("expected %d gradient values" % self.param_count)
        _check(lib().ebsd_cnn_apply_gradient(self._h, _ptr(grad, torch.float32, "grad"), float(lr), _stream()),
               "ebsd_cnn_apply_gradient")

    def close(self):
        if getattr(self, "_h", None):
            lib().ebsd_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cnn_make_batch(master, pc, lib_q, n, batch, first, seed, max_offset_px=5.0, counts=1000.0, snr=5.0,
                   x=None, labels=None, q_true=None):
    import torch
    dev = master.device
    x = x if x is not None else torch.empty((batch, 64, 64), dtype=torch.float32, device=dev)
    _shape(x, (batch, 64, 64), "x")
    _shape(labels, (batch,), "labels")
    _shape(q_true, (batch, 4), "q_true")
    _shape(lib_q, (None, 4), "lib_q")
    m, g = _master(master), _geo(pc)
    L = lib_q.shape[0] if lib_q is not None else 0
    _check(lib().ebsd_cnn_make_batch(ctypes.byref(m), ctypes.byref(g), _ptr(lib_q, torch.float64, "lib_q"), L, n,
                                     batch, first, int(seed), float(max_offset_px), float(counts), float(snr),
                                     _ptr(x), _ptr(labels, torch.int32, "labels"),
                                     _ptr(q_true, torch.float64, "q_true"), _stream()),
           "ebsd_cnn_make_batch")
    return x


def cnn_topk(logits, k):
    import torch
    _shape(logits, (None, None), "logits")
    idx = torch.empty((logits.shape[0], k), dtype=torch.int32, device=logits.device)
    _check(lib().ebsd_cnn_topk(_ptr(logits, torch.float32, "logits"), logits.shape[0], logits.shape[1], k, _ptr(idx),
                               _stream()), "ebsd_cnn_topk")
    return idx


def index_proposed(patterns, master, pc, lib_q, cnn, top_k=32, fallback_tau=0.0, prm=None):
    import torch
    p, n = _patterns(patterns)
    _shape(lib_q, (None, 4), "lib_q")
    _shape(master, (None, None), "master")
    dev = patterns.device
    out = dict(best_idx=torch.empty(p, dtype=torch.int32, device=dev),
               best_q=torch.empty((p, 4), dtype=torch.float64, device=dev),
               peak_h=torch.empty(p, dtype=torch.float32, device=dev),
               shift=torch.empty((p, 2), dtype=torch.float32, device=dev),
               fallback=torch.empty(p, dtype=torch.int32, device=dev))
    data, prm = _images(patterns, prm)
    b = Batch(data.value, p, n)
    m, g = _master(master), _geo(pc)
    _check(lib().ebsd_index_proposed(ctypes.byref(b), ctypes.byref(m), ctypes.byref(g),
                                     _ptr(lib_q, torch.float64, "lib_q"), lib_q.shape[0], cnn._h, top_k,
                                     float(fallback_tau), _params(prm), _ptr(out["best_idx"]), _ptr(out["best_q"]),
                                     _ptr(out["peak_h"]), _ptr(out["shift"]), _ptr(out["fallback"]), _stream()),
           "ebsd_index_proposed")
    return out

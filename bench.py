"""Benchmark of the template-matching hot path on one MI355X.

One step = ebsd_index_patterns (exhaustive FP32 correlation of every
pattern against every library template, library projection included) +
ebsd_refine_from_match (two x/y + log-polar z iterations, the first x/y step
from the search's own shift less each point's pattern-centre offset, and the
final correlation) over the map workload: 10,000 synthetic 128 x 128 patterns
(a 100 x 100 map of 20 grains) against 4,000 fundamental-zone templates,
inputs already resident in HBM.

Prints one JSON line: patterns/s (value) plus XCF pairs/s, the roofline of
the dominant kernel (the correlation search, timed with HIP events on the
stream it runs on) and the FP64 CPU oracle timed on a bounded sample.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Nominal flop count per (pattern, template) pair at N = 128: cross-power
# spectrum 6 N (N/2 + 1), inverse real 2-D FFT 2.5 N^2 log2(N^2), peak search N^2.
def pair_flops(n):
    import math
    return 6 * n * (n // 2 + 1) + 2.5 * n * n * math.log2(n * n) + n * n


PEAK_FP32_VALU = 157.3e12   # MI355X fp32 vector, FLOP/s (published)
PEAK_MFMA_FP32 = 157.3e12   # dense FP32 matrix (v_mfma_f32_*), published
PEAK_MFMA_16BIT = 2.5e15    # MI355X dense FP16 / BF16 matrix, FLOP/s (published)


# Algorithmic matrix flops per pair of the windowed DFT-GEMM search with
# |s_x|, |s_y| <= S: stage 1 a complex product over the band (2B + 1 rows,
# B + 1 columns, 2S + 1 shifts, 8 flops per complex multiply-add), stage 2
# the real part of a complex product (4 flops per term) over B + 1 columns
# and (2S + 1)^2 shifts; times 3 for the hi*hi + hi*lo + lo*hi products of
# the split forms.
def gemm_pair_flops(n, s, precision):
    b = 3 * n // 8
    w = 2 * s + 1
    one = 8 * (2 * b + 1) * (b + 1) * w + 4 * (b + 1) * w * w
    return one * (1 if precision == 3 else 3)


def kernel_source_hash(prof):
    """sha256 prefix of the profiled kernel's definition and of its launcher
    (each from its marker to the closing brace at column 0; the launcher
    sets the template chunk, which sets the traffic) and of the headers it
    includes: the byte counters are used only while these are unchanged."""
    import hashlib
    src = open(os.path.join(ROOT, prof["source"])).read()
    h = hashlib.sha256()
    for marker in [prof["kernel_marker"]] + ([prof["launcher_marker"]] if "launcher_marker" in prof else []):
        i = src.index(marker)
        j = src.index("\n}\n", i) + 3
        h.update(src[i:j].encode())
    for hdr in prof["headers"]:
        h.update(open(os.path.join(ROOT, hdr), "rb").read())
    return h.hexdigest()[:16]


def _cpu_threads():
    """Host threads this process may use (the GPU machine's CPU share is 16)."""
    try:
        c = len(os.sched_getaffinity(0))
    except AttributeError:
        c = os.cpu_count() or 1
    return max(1, min(c, 16))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_templates(job):
    import oracle
    from oracle import pipeline
    master, qs, n, pc = job
    return pipeline.library_spectra(master, qs, n, pc, oracle.Params())


def _oracle_pairs(job):
    import oracle
    from oracle import spectra, xcf
    pats, lib_spec = job
    prm = oracle.Params()
    for p in pats:
        xcf.library_scores(spectra.unit_spectrum(p, prm), lib_spec)
    return len(pats)


def _oracle_refine(job):
    import oracle
    from oracle import pipeline
    pats, master, pcs, pc, q0, ms = job
    pipeline.refine_from_match(pats, master, pcs, pc, q0, ms, oracle.Params())
    return len(pats)


def cpu_baseline(sample, n, l_full, p_full):
    """The FP64 oracle as it stands, run by a pool of worker processes over
    all host threads the process may use, on a stratified sample of the map
    workload: the projection and spectra of every 100th library template,
    the correlation of 1,000 patterns (every 10th map point) against those
    templates, and the refinement of 64 map points.  Each phase is timed by
    the wall clock; the per-unit times are extrapolated to the full workload
    (L templates, P x L pairs, P refinements)."""
    import multiprocessing as mp
    import numpy as np

    workers = _cpu_threads()
    ctx = mp.get_context("spawn")          # fresh interpreters: nothing of the GPU process is inherited
    pats, lib_q = sample["patterns"], sample["lib_q"]
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_pairs, [(pats[:1], [])] * workers)           # start-up outside the timings
        t0 = time.perf_counter()
        parts = pool.map(_oracle_templates, [(sample["master"], q, n, sample["pc"])
                                             for q in np.array_split(lib_q, min(workers, len(lib_q)))])
        t_tmpl = time.perf_counter() - t0
        lib_spec = [s for part in parts for s in part]
        t0 = time.perf_counter()
        pool.map(_oracle_pairs, [(c, lib_spec) for c in np.array_split(pats, workers * 4)])
        t_pairs = time.perf_counter() - t0
        r = sample["refine"]
        jobs = [(r["patterns"][k], sample["master"], r["pcs"][k], sample["pc"], r["q0"][k], r["shift"][k])
                for k in np.array_split(np.arange(len(r["q0"])), workers)]
        t0 = time.perf_counter()
        pool.map(_oracle_refine, jobs)
        t_ref = time.perf_counter() - t0
    n_pairs = len(pats) * len(lib_q)
    total = l_full * t_tmpl / len(lib_q) + p_full * l_full * t_pairs / n_pairs + p_full * t_ref / len(r["q0"])
    return {"value": p_full / total, "unit": "patterns/s", "cores": workers, "kind": "oracle",
            "cpu_model": _cpu_model(),
            "sample": "FP64 oracle in %d worker processes: %d templates (every %dth of the library) projected and "
                      "transformed, %d patterns (every %dth map point) x those templates correlated, %d map points "
                      "refined; per-unit wall times extrapolated to %d x %d (extrapolated, not a full run)"
                      % (workers, len(lib_q), l_full // len(lib_q), len(pats), p_full // len(pats), len(r["q0"]),
                         p_full, l_full),
            "pairs_per_s": n_pairs / t_pairs, "s_per_template": t_tmpl / len(lib_q),
            "s_per_refine": t_ref / len(r["q0"]),
            "phase_wall_s": {"templates": t_tmpl, "pairs": t_pairs, "refine": t_ref}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--patterns", type=int, default=10000, help="map size (must be a square)")
    ap.add_argument("--library", type=int, default=4000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the windowed / split-precision comparison")
    ap.add_argument("--search-precision", type=int, default=0,
                    help="precision of the timed step's search (0 FP32 FFT, 1 FP16x2, 2 BF16x2, 3 BF16)")
    ap.add_argument("--search-max-shift", type=int, default=-1, help="shift window of the timed step (-1: all)")
    ap.add_argument("--form-steps", type=int, default=3)
    ap.add_argument("--no-drift", action="store_true",
                    help="skip the drifting-pattern-centre map (beam-shift-corrected refinement)")
    ap.add_argument("--drift-steps", type=int, default=3)
    ap.add_argument("--no-capture", action="store_true", help="skip the capture-range (FWHM) sweep")
    ap.add_argument("--no-search-kernels", action="store_true",
                    help="skip timing each size's search kernel alone (4,096 x 4,096 random spectra)")
    ap.add_argument("--no-so3", action="store_true",
                    help="skip the equispaced-library sweep (sizes, nearest-neighbour statistics, map at 7 deg)")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the split-precision search on the same map at 256^2")
    ap.add_argument("--precision-patterns", type=int, default=10000)
    ap.add_argument("--precision-steps", type=int, default=2)
    ap.add_argument("--precision-fp32-steps", type=int, default=1)
    ap.add_argument("--no-ragged", action="store_true",
                    help="skip the ragged batch (binnings 64-160, 27-point stencil, one graph launch)")
    ap.add_argument("--ragged-patterns", type=int, default=20000)
    ap.add_argument("--ragged-library", type=int, default=8000)
    ap.add_argument("--ragged-steps", type=int, default=2)
    ap.add_argument("--no-proposal", action="store_true",
                    help="skip the learned proposal (CNN trained on the GPU, top-32 search with fallback)")
    ap.add_argument("--proposal-library", type=int, default=8000)
    ap.add_argument("--proposal-train", type=int, default=200000, help="distinct training patterns")
    ap.add_argument("--proposal-epochs", type=float, default=2.0)
    ap.add_argument("--proposal-test", type=int, default=50000)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one elementwise copy of this many MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU form "
              "(patterns would be split across GPUs with the library replicated)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1807_11313_amd as tm
    if not os.path.exists(tm.LIB_PATH):
        from paper_1807_11313_amd import build
        build.build()
    tm.lib()
    from fixtures import configs

    side = int(round(args.patterns ** 0.5))
    n = 128
    dev = torch.device("cuda:0")
    if args.copy_calibration_mib > 0:
        # one read and one write of exactly this many bytes, as a single kernel
        src = torch.ones(args.copy_calibration_mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    print("[bench] generating map workload %dx%d patterns at %d^2, library %d" % (side, side, n, args.library),
          file=sys.stderr, flush=True)
    cfg = configs.map_grid(rows=side, cols=side, n=n, l=args.library, device=dev, dtype=torch.float32)
    pats = cfg["patterns"].contiguous()
    master = torch.as_tensor(cfg["master"], device=dev).contiguous()
    lib_q = torch.as_tensor(cfg["lib_q"], device=dev).contiguous()
    pc_per = torch.as_tensor(cfg["pcs"], device=dev).contiguous()
    P, L = pats.shape[0], lib_q.shape[0]
    torch.cuda.synchronize()

    main_prm = tm.params_default(precision=args.search_precision, max_shift=args.search_max_shift)

    def step():
        r = tm.index_patterns(pats, master, cfg["pc"], lib_q, prm=main_prm)
        return tm.refine_from_match(pats, master, cfg["pc"], r["best_q"], r["shift"], pc_per=pc_per), r

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)
    tm.timing_read()
    tm.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ev = []
    for i in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        out, idx = step()
        e1.record()
        step_ev.append((e0, e1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm.timing_enable(False)
    xcf_ms, launches = tm.timing_read()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    step_ms = sorted(a.elapsed_time(b) for a, b in step_ev)
    median_ms = step_ms[len(step_ms) // 2] if len(step_ms) % 2 else 0.5 * (step_ms[len(step_ms) // 2 - 1] +
                                                                           step_ms[len(step_ms) // 2])

    # the same patterns copied from pinned host memory first (reported, not the value)
    host_pats = torch.empty(pats.shape, dtype=pats.dtype, pin_memory=True)
    host_pats.copy_(pats)
    dev_copy = torch.empty_like(pats)
    torch.cuda.synchronize()
    h0 = torch.cuda.Event(enable_timing=True)
    h1 = torch.cuda.Event(enable_timing=True)
    h0.record()
    dev_copy.copy_(host_pats, non_blocking=True)
    h1.record()
    torch.cuda.synchronize()
    h2d_ms = h0.elapsed_time(h1)
    del host_pats, dev_copy
    value = P / (ms_per_step / 1e3)
    xcf_avg_s = xcf_ms / 1e3 / max(launches, 1)
    flops_launch = P * L * pair_flops(n)
    achieved = flops_launch / xcf_avg_s

    # HBM traffic of the search kernel, from the committed counter profile,
    # only while the kernel source is the one the counters were taken on
    traffic = None
    try:
        prof = json.load(open(os.path.join(ROOT, "profiles", "xcf_search_128_map.json")))
        if kernel_source_hash(prof) == prof["kernel_sha256_prefix"] and (P, L, n) == (10000, 4000, 128):
            traffic = prof["fetch_bytes_per_launch"] + prof["write_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        traffic = None

    # accuracy of the last step against the simulated truth (context, not parity)
    from oracle import rotations
    q = out["q"].cpu().numpy()
    sample = np.linspace(0, P - 1, 200).astype(int)
    mis = np.rad2deg([rotations.disorientation_q(q[i], cfg["true_q"][i]) for i in sample])

    line = {
        "metric": "patterns indexed/s and XCF pairs/s at 128² (exhaustive vs pruned), 1 MI355X",
        "value": value, "unit": "patterns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32", "data": "synthetic",
        "config": {"workload": "map: %d patterns (%dx%d grid, 20 grains) at %dx%d fp32 vs %d-orientation cubic "
                               "library, exhaustive FFT XCF + 2-iteration refinement from the search's "
                               "shift" % (P, side, side, n, n, L),
                   "patterns": P, "library": L, "pattern_size": n, "form": "fft", "precision": "fp32",
                   "parallelism": "single GPU"},
        "median_ms_per_step": median_ms,
        "h2d": {"ms": h2d_ms, "bytes": pats.numel() * 4, "GB_per_s": pats.numel() * 4 / h2d_ms / 1e6,
                "patterns_per_s_including_copy": P / ((ms_per_step + h2d_ms) / 1e3),
                "note": "pinned host -> HBM copy of the step's patterns, timed with HIP events; not in value"},
        "xcf_pairs_per_s": P * L / xcf_avg_s,
        "xcf_pairs_per_s_whole_step": P * L / (ms_per_step / 1e3),
        "roofline": {"bound": "alu", "kernel": "k_xcf_scores<128>", "achieved": achieved / 1e12,
                     "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU,
                     "traffic": traffic, "traffic_unit": "bytes per launch (HBM, counters)",
                     "algorithmic_bytes": (P + L) * 2 * 49 * 97 * 4 + P * L * 4,
                     "avg_launch_ms": xcf_avg_s * 1e3,
                     "flops_per_launch": flops_launch, "flops_per_pair": pair_flops(n)},
        "accuracy": {"refined_misorientation_deg_median": float(np.median(mis)),
                     "refined_misorientation_deg_p95": float(np.percentile(mis, 95)),
                     "sample": "200 map points vs simulated truth"},
    }
    if not args.no_forms:
        line["forms"] = compare_forms(tm, pats, master, cfg, lib_q, pc_per, idx["best_idx"], out["q"], args.form_steps)
    # the oracle's stratified sample, on the host, before the 128^2 map is
    # released: every 10th map point, every 100th template, 64 refinements
    # started at the simulated truth (the refinement's cost does not depend
    # on its start)
    ref_idx = np.linspace(0, P - 1, 64).astype(int)
    cpu_sample = {"patterns": cfg["patterns"][::max(1, P // 1000)][:1000].cpu().numpy().astype(np.float64),
                  "lib_q": cfg["lib_q"][::max(1, L // 40)][:40], "master": cfg["master"], "pc": cfg["pc"],
                  "refine": {"patterns": cfg["patterns"][torch.as_tensor(ref_idx, device=dev)].cpu().numpy()
                             .astype(np.float64), "pcs": cfg["pcs"][ref_idx], "q0": cfg["true_q"][ref_idx],
                             "shift": np.zeros((len(ref_idx), 2))}}
    if not args.no_search_kernels:
        line["search_kernels"] = search_kernels(tm)
    if not args.no_so3:
        line["so3"] = so3_sweep(tm, pats, master, cfg, pc_per)
    if not args.no_capture:
        line["capture"] = capture_sweep(tm)
    if not args.no_drift:
        line["drift"] = drift_map(tm, args.patterns, args.library, args.drift_steps)
        torch.cuda.empty_cache()
    if not args.no_precision:
        del pats, cfg, out, idx
        torch.cuda.empty_cache()
        line["precision256"] = precision_256(tm, args.precision_patterns, args.library, args.precision_steps,
                                             fp32_steps=args.precision_fp32_steps)
    if not args.no_ragged:
        torch.cuda.empty_cache()
        line["ragged"] = ragged_batch(tm, args.ragged_patterns, args.ragged_library, args.ragged_steps)
    if not args.no_proposal:
        torch.cuda.empty_cache()
        line["proposal"] = learned_proposal(tm, args.proposal_library, args.proposal_train, args.proposal_epochs,
                                            args.proposal_test)
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a bounded sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(cpu_sample, n, L, P)
    print(json.dumps(line), flush=True)


def compare_forms(tm, pats, master, cfg, lib_q, pc_per, best_ref, q_ref, steps):
    """The same step with the search in other forms: the FP32 FFT form and the
    split-precision DFT-GEMM forms with a +-15 px shift window (the map's
    pattern-centre offsets are within +-5 px and a library step moves the
    pattern by <= ~6 px).  Indexing accuracy is compared with the exhaustive
    FP32 step: agreement of the best template, and the refined orientation's
    misorientation from the exhaustive one and from the simulated truth."""
    import numpy as np
    import torch
    from oracle import rotations

    P, L = pats.shape[0], lib_q.shape[0]
    best_ref = best_ref.cpu().numpy()
    q_ref = q_ref.cpu().numpy()
    sample = np.linspace(0, P - 1, 200).astype(int)
    res = {}
    for name, kw in (("fft_fp32_window15", dict(precision=0, max_shift=15)),
                     ("dftgemm_fp16x2_window15", dict(precision=1, max_shift=15)),
                     ("dftgemm_bf16x2_window15", dict(precision=2, max_shift=15)),
                     ("dftgemm_bf16_window15", dict(precision=3, max_shift=15))):
        prm = tm.params_default(**kw)

        def step():
            r = tm.index_patterns(pats, master, cfg["pc"], lib_q, prm=prm)
            return tm.refine_from_match(pats, master, cfg["pc"], r["best_q"], r["shift"], pc_per=pc_per), r

        step()
        torch.cuda.synchronize()
        tm.timing_read()
        tm.timing_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            out, idx = step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tm.timing_enable(False)
        ms, cnt = tm.timing_read()
        q = out["q"].cpu().numpy()
        best = idx["best_idx"].cpu().numpy()
        vs_ref = np.rad2deg([rotations.disorientation_q(q[i], q_ref[i]) for i in sample])
        vs_true = np.rad2deg([rotations.disorientation_q(q[i], cfg["true_q"][i]) for i in sample])
        res[name] = {"patterns_per_s": P * steps / (t1 - t0),
                     "xcf_pairs_per_s": P * L / (ms / 1e3 / max(cnt, 1)),
                     "search_ms": ms / max(cnt, 1),
                     "best_index_agreement_with_exhaustive_fp32": float(np.mean(best == best_ref)),
                     "refined_vs_exhaustive_deg_p99": float(np.percentile(vs_ref, 99)),
                     "refined_vs_truth_deg_median": float(np.median(vs_true)),
                     "refined_vs_truth_deg_p95": float(np.percentile(vs_true, 95))}
        print("[bench] form %s: %.0f patterns/s" % (name, res[name]["patterns_per_s"]), file=sys.stderr, flush=True)
    return res


def drift_map(tm, patterns, library, steps, sample=1000):
    """The map with a pattern centre drifting across it (pcx over 0.13 and pcy
    over 0.08 screen widths, pcz over 0.02), one library at the nominal PC.
    A step evaluates the affine PC model on the device, runs the exhaustive
    FP32 search and refines either from the search's beam-shift-corrected
    shift (ebsd_refine_from_match) or by re-projecting at each point's PC
    from the start (ebsd_refine_orientations); without any PC correction
    (every point refined at the nominal PC) the drift reads as rotation."""
    import numpy as np
    import torch
    from fixtures import configs
    from oracle import rotations

    dev = torch.device("cuda:0")
    side = int(round(patterns ** 0.5))
    print("[bench] generating drifting-PC map %dx%d at 128^2, library %d" % (side, side, library),
          file=sys.stderr, flush=True)
    cfg = configs.drift_map(rows=side, cols=side, n=128, l=library, device=dev, dtype=torch.float32)
    pats = cfg["patterns"].contiguous()
    master = torch.as_tensor(cfg["master"], device=dev).contiguous()
    lib_q = torch.as_tensor(cfg["lib_q"], device=dev).contiguous()
    m = cfg["model"]
    P = pats.shape[0]
    pick = np.linspace(0, P - 1, min(sample, P)).astype(int)

    def pcs():
        return tm.pc_map(m["pc0"], m["d_col"], m["d_row"], m["width"], P, m["col0"], m["row0"])

    variants = {
        "from_match": lambda r, pc: tm.refine_from_match(pats, master, cfg["pc"], r["best_q"], r["shift"], pc_per=pc),
        "reproject": lambda r, pc: tm.refine_orientations(pats, master, cfg["pc"], r["best_q"], pc_per=pc),
        "no_pc_correction": lambda r, pc: tm.refine_orientations(pats, master, cfg["pc"], r["best_q"]),
    }
    res = {"workload": "drifting PC: %d patterns (%dx%d, 20 grains) at 128x128 fp32, %d-orientation library at the "
                       "nominal PC, pcx/pcy/pcz drift 0.13/0.08/0.02 screen widths across the map, SNR 5"
                       % (P, side, side, lib_q.shape[0])}
    for name, refine in variants.items():
        def step():
            pc = pcs()
            r = tm.index_patterns(pats, master, cfg["pc"], lib_q)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            out = refine(r, pc)
            e1.record()
            return out, (e0, e1)

        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs = []
        for _ in range(steps):
            out, ev = step()
            evs.append(ev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        q = out["q"].cpu().numpy()
        mis = np.rad2deg([rotations.disorientation_q(q[i], cfg["true_q"][i]) for i in pick])
        res[name] = {"patterns_per_s": P * steps / (t1 - t0),
                     "refine_ms": float(np.mean([a.elapsed_time(b) for a, b in evs])),
                     "refined_vs_truth_deg_median": float(np.median(mis)),
                     "refined_vs_truth_deg_p95": float(np.percentile(mis, 95)),
                     "within_0.2_deg": float(np.mean(mis < 0.2))}
        print("[bench] drift %s: %.0f patterns/s, refine %.1f ms, median %.3f deg, within 0.2 deg %.4f"
              % (name, res[name]["patterns_per_s"], res[name]["refine_ms"], res[name]["refined_vs_truth_deg_median"],
                 res[name]["within_0.2_deg"]), file=sys.stderr, flush=True)
    res["accuracy_sample"] = "%d map points vs simulated truth" % len(pick)
    return res


def search_kernels(tm, sizes=(64, 96, 128, 160), count=4096, reps=2):
    """The FFT-form search kernel of each size alone: count x count random
    band spectra, every cyclic shift, HIP-event timing of the kernel
    (pairs/s and nominal TFLOP/s against the FP32 vector peak)."""
    import torch

    g = torch.Generator(device="cuda:0")
    g.manual_seed(1)
    res = {"workload": "%d x %d random band spectra per size, all shifts" % (count, count)}
    for n in sizes:
        f = tm.spectrum_floats(n)
        sp = torch.randn((count, f), generator=g, device="cuda:0") * 1e-2
        sl = torch.randn((count, f), generator=g, device="cuda:0") * 1e-2
        tm.xcf_scores(sp, sl, n)
        torch.cuda.synchronize()
        tm.timing_read()
        tm.timing_enable(True)
        for _ in range(reps):
            tm.xcf_scores(sp, sl, n)
        torch.cuda.synchronize()
        tm.timing_enable(False)
        ms, c = tm.timing_read()
        ms /= max(c, 1)
        pairs = count * count / (ms / 1e3)
        res[str(n)] = {"ms": ms, "pairs_per_s": pairs, "tflops_nominal": pairs * pair_flops(n) / 1e12,
                       "frac_of_fp32_vector_peak": pairs * pair_flops(n) / PEAK_FP32_VALU}
        del sp, sl
    print("[bench] search kernels alone: " + ", ".join("%s: %.3g pairs/s" % (n, res[str(n)]["pairs_per_s"])
                                                        for n in sizes), file=sys.stderr, flush=True)
    return res


def so3_sweep(tm, pats, master, cfg, pc_per, spacings=(10.0, 7.0, 5.0, 3.0), index_spacing=7.0):
    """Equispaced fundamental-zone libraries (Figure 2 analogue): size,
    generation time and nearest-neighbour disorientation statistics per
    spacing; then the map step with the library at the paper's 7 deg in
    place of the random one."""
    import numpy as np
    import torch
    from oracle import rotations

    res = {"libraries": {}}
    for sp in spacings:
        tm.so3_library(sp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q = tm.so3_library(sp)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ang, _ = tm.nn_disorientation(q)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        a = ang.cpu().numpy()
        hist, edges = np.histogram(a, bins=np.arange(0.0, a.max() + 0.2, 0.1))
        res["libraries"]["%g" % sp] = {
            "orientations": int(q.shape[0]), "generate_ms": (t1 - t0) * 1e3, "nn_ms": (t2 - t1) * 1e3,
            "nn_pairs_per_s": q.shape[0] ** 2 / (t2 - t1),
            "nn_deg_max": float(a.max()), "nn_deg_mean": float(a.mean()), "nn_deg_median": float(np.median(a)),
            "nn_deg_mode": float(edges[int(np.argmax(hist))] + 0.05),
            "nn_below_0.9_spacing": float(np.mean(a < 0.9 * sp))}
        print("[bench] so3 %g deg: %d orientations, nn max %.3f mean %.3f deg" % (sp, q.shape[0], a.max(), a.mean()),
              file=sys.stderr, flush=True)
    lib = tm.so3_library(index_spacing)
    P = pats.shape[0]

    def step():
        r = tm.index_patterns(pats, master, cfg["pc"], lib)
        return tm.refine_from_match(pats, master, cfg["pc"], r["best_q"], r["shift"], pc_per=pc_per)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    q = out["q"].cpu().numpy()
    pick = np.linspace(0, P - 1, 500).astype(int)
    mis = np.rad2deg([rotations.disorientation_q(q[i], cfg["true_q"][i]) for i in pick])
    res["map_with_library"] = {"spacing_deg": index_spacing, "library": int(lib.shape[0]),
                               "patterns_per_s": P / dt, "refined_vs_truth_deg_median": float(np.median(mis)),
                               "refined_vs_truth_deg_p95": float(np.percentile(mis, 95)),
                               "within_0.2_deg": float(np.mean(mis < 0.2)), "accuracy_sample": "500 map points"}
    print("[bench] map with the %g deg library (%d): %.0f patterns/s, median %.3f deg, within 0.2 deg %.3f"
          % (index_spacing, lib.shape[0], P / dt, np.median(mis), np.mean(mis < 0.2)), file=sys.stderr, flush=True)
    return res


def capture_sweep(tm, n_ref=8, span=30.0, step=0.5):
    """Capture range of the correlation (Figures 3 and 4 analogues): the
    integer peak of a reference pattern against the crystal rotated about
    the detector x, y and z axes in 0.5 deg steps over +-30 deg, at the PC
    (0.5, 0.3, 0.6); FWHM per axis averaged over n_ref random reference
    orientations, per screen size, and at 128^2 per pattern-centre error of
    the rotated patterns."""
    import numpy as np
    import torch
    from fixtures import band_master, random_quats

    dev = torch.device("cuda:0")
    pc = (0.5, 0.3, 0.6)
    master = torch.as_tensor(band_master(), device=dev).contiguous()
    q_ref = torch.as_tensor(random_quats(np.random.default_rng(77), n_ref), device=dev).contiguous()
    th_h = np.arange(-span, span + 1e-9, step)
    th = torch.as_tensor(th_h, device=dev).contiguous()

    def run(n, pc_test):
        tm.capture_range(master, q_ref, n, pc, pc_test, th)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, w = tm.capture_range(master, q_ref, n, pc, pc_test, th)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        w = w.cpu().numpy()
        return {"fwhm_deg_mean_xyz": [float(v) for v in w.mean(axis=0)],
                "fwhm_deg_min_xyz": [float(v) for v in w.min(axis=0)],
                "rotated_patterns_per_s": n_ref * 3 * len(th_h) / dt}

    res = {"workload": "capture range: %d reference orientations x 3 detector axes x %d angles (%.1f deg steps "
                       "over +-%.0f deg), PC (0.5, 0.3, 0.6), integer correlation peak" % (n_ref, len(th_h), step, span),
           "screen": {}, "pc_error_128": {}}
    for n in (64, 96, 128, 160):
        res["screen"][str(n)] = run(n, pc)
    for axis, k in (("x", 0), ("y", 1), ("z", 2)):
        for d in (0.01, 0.03, 0.05):
            pt = list(pc)
            pt[k] += d
            res["pc_error_128"]["%s+%.2f" % (axis, d)] = run(128, tuple(pt))
    s = res["screen"]
    print("[bench] capture FWHM (x, y, z) deg: " + ", ".join(
        "%s: %s" % (n, "/".join("%.1f" % v for v in s[n]["fwhm_deg_mean_xyz"])) for n in s), file=sys.stderr, flush=True)
    return res


def precision_256(tm, patterns, library, steps, window=15, sample=3, n_sub=96, fp32_steps=1):
    """The map at 256 x 256 with the search over a +-15 px window, followed by
    the same refinement: first in FP32 (the exact windowed DFT on the vector
    ALUs; the FFT form is not built at this size), then as split-precision
    DFT-GEMMs on MFMA.  Per precision: patterns/s, pairs/s and the roofline of
    the search kernel, agreement of the best template with the FP32 search,
    accuracy against the simulated truth, and the error against the FP64
    oracle on a sample of patterns: scores over a random subset of the
    library, and where the device picked the oracle's start (its nearest
    library orientation to the truth) the winner's sub-pixel peak height and
    shift and the refined orientation."""
    import numpy as np
    import torch
    import oracle
    from fixtures import configs
    from oracle import geometry, pipeline, rotations, spectra, xcf

    n = 256
    side = int(round(patterns ** 0.5))
    dev = torch.device("cuda:0")
    print("[bench] generating map workload %dx%d patterns at %d^2, library %d" % (side, side, n, library),
          file=sys.stderr, flush=True)
    cfg = configs.map_grid(rows=side, cols=side, n=n, l=library, device=dev, dtype=torch.float32)
    pats = cfg["patterns"].contiguous()
    master = torch.as_tensor(cfg["master"], device=dev).contiguous()
    lib_q = torch.as_tensor(cfg["lib_q"], device=dev).contiguous()
    pc_per = torch.as_tensor(cfg["pcs"], device=dev).contiguous()
    P, L = pats.shape[0], lib_q.shape[0]
    pts = np.linspace(0, P - 1, 200).astype(int)
    smp = np.linspace(0, P - 1, sample + 2).astype(int)[1:-1]
    rng = np.random.default_rng(7)
    sub = np.sort(rng.choice(L, size=min(n_sub, L), replace=False))

    # oracle side of the error sample (independent of the precision)
    oprm = oracle.Params(max_shift=window)
    pats_h = cfg["patterns"][smp].cpu().numpy().astype(np.float64)
    o_pat = [spectra.unit_spectrum(pats_h[i], oprm) for i in range(len(smp))]
    o_lib = {}

    from oracle import cnn as ocnn
    o_start = [ocnn.nearest_library(cfg["true_q"][i], cfg["lib_q"]) for i in smp]

    def o_spec(j):
        if j not in o_lib:
            img = geometry.project(cfg["master"], rotations.quat_to_matrix(cfg["lib_q"][j]), n, cfg["pc"])
            o_lib[j] = spectra.unit_spectrum(img, oprm)
        return o_lib[j]

    res = {"workload": "map: %d patterns (%dx%d grid, 20 grains) at %dx%d fp32 vs %d-orientation cubic library, "
                       "DFT-GEMM search |s| <= %d px + 2-iteration refinement" % (P, side, side, n, n, L, window),
           "error_sample": "%d patterns x %d random templates against the FP64 oracle; the winner's peak and "
                           "the refinement where the device's pick is the oracle's start (its nearest library "
                           "orientation to the truth)" % (len(smp), len(sub))}
    ref_best = None
    for name, prec in (("fp32", 0), ("fp16x2", 1), ("bf16x2", 2), ("bf16", 3)):
        prm = tm.params_default(precision=prec, max_shift=window)
        n_steps = fp32_steps if prec == 0 else steps

        def step():
            r = tm.index_patterns(pats, master, cfg["pc"], lib_q, prm=prm)
            return tm.refine_from_match(pats, master, cfg["pc"], r["best_q"], r["shift"], pc_per=pc_per,
                                        prm=prm), r

        step()
        torch.cuda.synchronize()
        tm.timing_read()
        tm.timing_enable(True)
        t0 = time.perf_counter()
        for _ in range(n_steps):
            out, idx = step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tm.timing_enable(False)
        ms, cnt = tm.timing_read()
        search_s = ms / 1e3 / max(cnt, 1)
        flops = P * L * gemm_pair_flops(n, window, 3 if prec == 0 else prec)
        best = idx["best_idx"].cpu().numpy()
        if ref_best is None:
            ref_best = best
        q = out["q"].cpu().numpy()
        vs_true = np.rad2deg([rotations.disorientation_q(q[i], cfg["true_q"][i]) for i in pts])

        # error against the FP64 oracle on the sample: scores over the random
        # library subset; the winner's peak and the refinement where the
        # device picked the oracle's start (its nearest library orientation
        # to the truth), which the oracle then indexes and refines itself
        sc = tm.index_patterns(pats[smp], master, cfg["pc"], lib_q, prm=prm, scores=True)
        sc_h = sc["scores"].cpu().numpy()
        d_score = d_h = d_s = d_q = 0.0
        n_cmp = 0
        for a in range(len(smp)):
            ref = xcf.library_scores(o_pat[a], [o_spec(j) for j in sub], max_shift=window)
            d_score = max(d_score, float(np.max(np.abs(sc_h[a, sub] - ref))))
            b = o_start[a]
            if int(sc["best_idx"][a]) != b:
                continue
            n_cmp += 1
            ho, so = xcf.subpixel_peak(o_pat[a], o_spec(b),
                                       xcf.integer_peak(xcf.xcf_map(o_pat[a], o_spec(b)), window)[1], oprm.upsample)
            d_h = max(d_h, abs(float(sc["peak_h"][a]) - ho))
            sg = sc["shift"][a].cpu().numpy()
            d_s = max(d_s, abs(sg[0] - so[1]), abs(sg[1] - so[0]))
            rr = pipeline.refine_from_match(pats_h[a:a + 1], cfg["master"], cfg["pcs"][smp[a]:smp[a] + 1], cfg["pc"],
                                            cfg["lib_q"][b][None], np.array([[so[1], so[0]]]), oprm)
            d_q = max(d_q, float(np.rad2deg(rotations.disorientation_q(q[smp[a]], rr["q"][0]))))
        if prec == 0:
            roof = {"bound": "alu", "kernel": "k_grid_peak (library mode)", "achieved": flops / search_s / 1e12,
                    "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s", "frac": flops / search_s / PEAK_FP32_VALU,
                    "flops_per_pair": gemm_pair_flops(n, window, 3)}
        else:
            roof = {"bound": "mfma", "kernel": "k_xcf_gemm<256>", "achieved": flops / search_s / 1e12,
                    "peak": PEAK_MFMA_16BIT / 1e12, "unit": "TFLOP/s", "frac": flops / search_s / PEAK_MFMA_16BIT,
                    "flops_per_pair": gemm_pair_flops(n, window, prec)}
        res[name] = {"patterns_per_s": P * n_steps / (t1 - t0), "xcf_pairs_per_s": P * L / search_s,
                     "search_ms": search_s * 1e3, "roofline": roof,
                     "best_index_agreement_with_fp32": float(np.mean(best == ref_best)),
                     "refined_vs_truth_deg_median": float(np.median(vs_true)),
                     "refined_vs_truth_deg_p95": float(np.percentile(vs_true, 95)),
                     "vs_oracle": {"max_abs_score": d_score, "max_abs_peak_h": d_h, "max_abs_shift_px": float(d_s),
                                   "max_refined_misorientation_deg": float(d_q), "picks_compared": n_cmp}}
        print("[bench] 256 %s: %.0f patterns/s, %.3g pairs/s, oracle |dh| %.2g"
              % (name, res[name]["patterns_per_s"], res[name]["xcf_pairs_per_s"], d_score),
              file=sys.stderr, flush=True)
    return res


def ragged_batch(tm, patterns, library, steps, sample_per_size=1):
    """Patterns of binnings 64, 96, 128 and 160 (25 % each, shuffled) against
    one library, followed by the 27-point +-0.5 deg stencil and the 2-iteration
    refinement (its first x/y step from the stencil winner's shift), as one
    graph launch per step (plan built once, tiles autotuned at plan
    creation).  Reports patterns/s and library pairs/s of the whole step, the
    chosen tiles, accuracy against the simulated truth, and, on a sample, the
    final orientation against the FP64 oracle's stencil and refinement started
    from the oracle's own nearest library orientation (compared where the
    device's library pick is that same orientation)."""
    import numpy as np
    import torch
    import oracle
    from fixtures import configs
    from oracle import cnn as ocnn
    from oracle import rotations, stencil

    dev = torch.device("cuda:0")
    print("[bench] generating ragged workload: %d patterns, library %d" % (patterns, library),
          file=sys.stderr, flush=True)
    cfg = configs.ragged(p=patterns, l=library, device=dev)
    data, offs, ns = configs.pack_ragged(cfg, device=dev)
    cfg["pattern_sets"] = [(idx, pats.cpu()) for idx, pats in cfg["pattern_sets"]]
    master = torch.as_tensor(cfg["master"], device=dev).contiguous()
    lib_q = torch.as_tensor(cfg["lib_q"], device=dev).contiguous()
    pc_per = torch.as_tensor(cfg["pcs"], device=dev).contiguous()
    P, L = len(ns), len(cfg["lib_q"])
    t0 = time.perf_counter()
    plan = tm.RaggedPlan(ns, offs, L, stencil=True, refine=True)
    t_plan = time.perf_counter() - t0
    out = plan.run(data, master, cfg["pc"], lib_q, pc_per=pc_per)       # capture + first run
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.run_into(data, master, cfg["pc"], lib_q, out, pc_per)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    q = out["q"].cpu().numpy()
    best = out["best_idx"].cpu().numpy()
    sidx = out["stencil_idx"].cpu().numpy()
    pts = np.linspace(0, P - 1, 200).astype(int)
    vs_true = np.rad2deg([rotations.disorientation_q(q[i], cfg["true_q"][i]) for i in pts])
    lib_true = np.rad2deg([rotations.disorientation_q(cfg["lib_q"][best[i]], cfg["true_q"][i]) for i in pts])
    # the oracle's stencil + refinement from its own start on a sample
    agree, dq, dh, total = 0, 0.0, 0.0, 0
    prm = oracle.Params()
    for n in (64, 96, 128, 160):
        found = 0
        for i in np.nonzero(ns == n)[0][:20]:
            j = ocnn.nearest_library(cfg["true_q"][i], cfg["lib_q"])
            if j != best[i]:
                continue
            rr = stencil.stencil_then_refine([configs.ragged_pattern(cfg, i)], cfg["master"], cfg["pcs"][i:i + 1],
                                             cfg["lib_q"][j][None], prm)
            total += 1
            if rr["stencil"]["idx"][0] == sidx[i]:
                agree += 1
                dq = max(dq, float(np.rad2deg(rotations.disorientation_q(q[i], rr["q"][0]))))
                dh = max(dh, abs(float(out["peak_h"][i]) - rr["peak_h"][0]))
            found += 1
            if found >= sample_per_size:
                break
    res = {"workload": "ragged: %d patterns, binnings 64/96/128/160 (25%% each, shuffled), %d-orientation cubic "
                       "library, exhaustive FFT XCF + 27-point +-0.5 deg stencil + 2-iteration refinement, one "
                       "graph launch per step" % (P, L),
           "patterns_per_s": P / dt, "ms_per_step": dt * 1e3, "library_pairs_per_s_whole_step": P * L / dt,
           "stencil_candidates_per_step": 27 * P, "plan_create_s_incl_autotune": t_plan,
           "tiles": plan.tiles(), "steps": steps,
           "library_pick_vs_truth_deg_median": float(np.median(lib_true)),
           "refined_vs_truth_deg_median": float(np.median(vs_true)),
           "refined_vs_truth_deg_p95": float(np.percentile(vs_true, 95)),
           "refined_within_0.1_deg": float(np.mean(vs_true < 0.1)),
           "vs_oracle": {"stencil_agreement": agree / max(total, 1), "sample": total,
                         "max_refined_misorientation_deg": dq, "max_abs_peak_h": dh,
                         "start": "the oracle's nearest library orientation to the truth, where the device "
                                  "picked the same one"}}
    print("[bench] ragged: %.0f patterns/s, %.3g library pairs/s, refined median %.3f deg"
          % (res["patterns_per_s"], res["library_pairs_per_s_whole_step"], res["refined_vs_truth_deg_median"]),
          file=sys.stderr, flush=True)
    plan.close()
    return res


def cnn_flops_per_sample(n_classes):
    """Multiply-adds x 2 of one forward pass (four 3 x 3 convolutions, the
    fully connected layer); a training step is counted as 3 forward passes."""
    macs, ci, w = 0, 1, 64
    for co in (32, 64, 128, 128):
        macs += w * w * co * ci * 9
        ci, w = co, w // 2
    return 2 * (macs + 2048 * n_classes)


def learned_proposal(tm, library, n_train, epochs, n_test, k=32, bsz=256, n=128):
    """The network trained on the GPU on projected noisy patterns (fixed set
    of n_train sample counters, fresh noise per epoch), then the pruned search
    (top-k correlation + exhaustive fallback below tau) against the
    exhaustive FP32 search on n_test simulated 128 x 128 patterns.  tau is the
    1st percentile of the exhaustive integer peak height among the correctly
    indexed patterns of a validation set."""
    import numpy as np
    import torch
    from fixtures import band_master, random_fz_quats, random_quats, simulate_patterns
    from oracle import rotations

    dev = torch.device("cuda:0")
    lib = random_fz_quats(np.random.default_rng(11), library)
    master = torch.as_tensor(band_master(), device=dev).contiguous()
    lq = torch.as_tensor(lib, device=dev).contiguous()
    pc = (0.5, 0.5, 0.6)

    def patterns(p, seed):
        rng = np.random.default_rng(seed)
        q = random_quats(rng, p)
        off = rng.uniform(-5, 5, size=(p, 2))
        pcs = np.stack([0.5 + off[:, 0] / n, 0.5 + off[:, 1] / n, np.full(p, 0.6)], 1)
        return q, pcs, simulate_patterns(q, n, pcs, ("poisson_gauss", 1000.0, 5.0), seed=seed, device=dev,
                                         dtype=torch.float32).contiguous()

    print("[bench] proposal: training on %d patterns x %.1f epochs, library %d" % (n_train, epochs, library),
          file=sys.stderr, flush=True)
    net = tm.Cnn(library, seed=5)
    x = torch.empty((bsz, 64, 64), device=dev)
    y = torch.empty(bsz, dtype=torch.int32, device=dev)
    loss = torch.empty(1, device=dev)
    steps = int(epochs * n_train / bsz)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        first = (s * bsz) % n_train
        tm.cnn_make_batch(master, pc, lq, n, bsz, first, 1000 + (s * bsz) // n_train, x=x, labels=y)
        net.train_step(x, y, 1e-3, loss)
        if s % 500 == 0:
            print("[bench]   step %d/%d loss %.3f" % (s, steps, float(loss.item())), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    final_loss = float(loss.item())
    # network throughput alone (forward + backward + Adam) on one batch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        net.train_step(x, y, 1e-3, loss)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / 20
    train_flops = 3 * cnn_flops_per_sample(library) * bsz

    # tau: 1st percentile of the exhaustive integer peak height (the score the
    # pruned search compares with it) among the correctly indexed validation
    # patterns (refined within 1 deg of the truth)
    q_val, pcs_val, val = patterns(10000, 31)
    ex_val = tm.index_patterns(val, master, pc, lq, scores=True)
    h_val = ex_val.pop("scores").max(dim=1).values.cpu().numpy()
    rf_val = tm.refine_from_match(val, master, pc, ex_val["best_q"], ex_val["shift"],
                                  pc_per=torch.as_tensor(pcs_val, device=dev).contiguous())
    qv = rf_val["q"].cpu().numpy()
    ok_val = np.rad2deg([rotations.disorientation_q(qv[i], q_val[i]) for i in range(len(qv))]) < 1.0
    tau = float(np.percentile(h_val[ok_val], 1.0))
    tau_all = float(np.percentile(h_val, 1.0))
    del val, ex_val, rf_val
    q_test, pcs_test, test = patterns(n_test, 32)
    pc_per = torch.as_tensor(pcs_test, device=dev).contiguous()

    def timed(fn, reps=2):
        fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t1) / reps

    ex, t_ex = timed(lambda: tm.index_patterns(test, master, pc, lq))
    pr, t_pr = timed(lambda: tm.index_proposed(test, master, pc, lq, net, top_k=k, fallback_tau=tau))
    x_test = tm.Cnn.input(test[:bsz * 8])
    _, t_fwd = timed(lambda: net.forward(x_test), reps=5)  # default inference precision: BF16 split halves
    net.set_precision(tm.PREC_FP32)
    _, t_fwd32 = timed(lambda: net.forward(x_test), reps=5)
    net.set_precision(tm.PREC_BF16X2)
    # both picks refined the same way (the library pick is only the start)
    rf_ex, t_rf = timed(lambda: tm.refine_from_match(test, master, pc, ex["best_q"], ex["shift"], pc_per=pc_per),
                        reps=1)
    rf_pr, _ = timed(lambda: tm.refine_from_match(test, master, pc, pr["best_q"], pr["shift"], pc_per=pc_per), reps=1)
    b_ex, b_pr = ex["best_idx"].cpu().numpy(), pr["best_idx"].cpu().numpy()
    fb = pr["fallback"].cpu().numpy().astype(bool)
    q_ex, q_pr = rf_ex["q"].cpu().numpy(), rf_pr["q"].cpu().numpy()
    pts = np.linspace(0, n_test - 1, 500).astype(int)
    mis_ex = np.rad2deg([rotations.disorientation_q(lib[b_ex[i]], q_test[i]) for i in pts])
    mis_pr = np.rad2deg([rotations.disorientation_q(lib[b_pr[i]], q_test[i]) for i in pts])
    rex = np.rad2deg([rotations.disorientation_q(q_ex[i], q_test[i]) for i in pts])
    rpr = np.rad2deg([rotations.disorientation_q(q_pr[i], q_test[i]) for i in pts])
    rpe = np.rad2deg([rotations.disorientation_q(q_pr[i], q_ex[i]) for i in pts])
    pairs_pr = n_test * k + int(fb.sum()) * library
    res = {"workload": "proposal: CNN (4 conv 32-128 ch on 64x64 binned input, fc to %d) trained on the GPU "
                       "(convolutions FP32, fc and backward products on BF16 split halves) on %d projected noisy patterns x %.1f epochs; inference products on BF16 split halves "
                       "(hi*hi + hi*lo + lo*hi, FP32 sums); %d test patterns at 128x128 fp32, top-%d "
                       "correlation with exhaustive fallback below tau" % (library, n_train, epochs, n_test, k),
           "train_s": t_train, "train_steps": steps, "batch": bsz, "final_loss": final_loss,
           "train_samples_per_s": steps * bsz / t_train,
           "train_step_roofline": {"bound": "mfma", "achieved": train_flops / t_step / 1e12,
                                   "peak": PEAK_MFMA_FP32 / 1e12, "unit": "TFLOP/s",
                                   "frac": train_flops / t_step / PEAK_MFMA_FP32,
                                   "flops_per_sample_forward": cnn_flops_per_sample(library),
                                   "note": "network flops (one product per multiply-add) against the FP32 "
                                           "matrix peak; the fc and backward products run as three BF16 "
                                           "products on split halves"},
           "forward_patterns_per_s": bsz * 8 / t_fwd,
           "forward_patterns_per_s_fp32": bsz * 8 / t_fwd32,
           "forward_tflops_network": cnn_flops_per_sample(library) * bsz * 8 / t_fwd / 1e12,
           "tau": tau, "tau_rule": "1st percentile of the exhaustive integer peak height among the correctly "
                                   "indexed of 10,000 validation patterns (refined within 1 deg of the truth)",
           "validation_correctly_indexed": float(ok_val.mean()), "tau_over_all_validation": tau_all,
           "refine_s": t_rf,
           "exhaustive": {"search_patterns_per_s": n_test / t_ex, "patterns_per_s_with_refinement":
                          n_test / (t_ex + t_rf), "pairs": n_test * library,
                          "pick_vs_truth_deg_median": float(np.median(mis_ex)),
                          "refined_vs_truth_deg_median": float(np.median(rex)),
                          "refined_vs_truth_deg_p95": float(np.percentile(rex, 95))},
           "pruned": {"search_patterns_per_s": n_test / t_pr, "patterns_per_s_with_refinement":
                      n_test / (t_pr + t_rf), "pairs": pairs_pr, "fallback_fraction": float(fb.mean()),
                      "pick_agreement_with_exhaustive": float(np.mean(b_pr == b_ex)),
                      "pick_vs_truth_deg_median": float(np.median(mis_pr)),
                      "refined_vs_truth_deg_median": float(np.median(rpr)),
                      "refined_vs_truth_deg_p95": float(np.percentile(rpr, 95)),
                      "refined_vs_exhaustive_refined_deg_median": float(np.median(rpe)),
                      "refined_within_0.1deg_of_exhaustive": float(np.mean(rpe <= 0.1))},
           "accuracy_sample": "500 test patterns",
           "search_speedup": t_ex / t_pr}
    # the same test patterns stored as BF16 (half the bytes; each pixel widened
    # to FP32 as it is loaded), against the exhaustive FP32 search above
    test_b = test.to(torch.bfloat16).contiguous()
    del test
    exb, t_exb = timed(lambda: tm.index_patterns(test_b, master, pc, lq))
    prb, t_prb = timed(lambda: tm.index_proposed(test_b, master, pc, lq, net, top_k=k, fallback_tau=tau))
    rf_prb, t_rfb = timed(lambda: tm.refine_from_match(test_b, master, pc, prb["best_q"], prb["shift"], pc_per=pc_per),
                          reps=1)
    b_exb, b_prb = exb["best_idx"].cpu().numpy(), prb["best_idx"].cpu().numpy()
    q_prb = rf_prb["q"].cpu().numpy()
    rpb = np.rad2deg([rotations.disorientation_q(q_prb[i], q_test[i]) for i in pts])
    rpbe = np.rad2deg([rotations.disorientation_q(q_prb[i], q_ex[i]) for i in pts])
    res["bf16_input"] = {
        "exhaustive": {"search_patterns_per_s": n_test / t_exb,
                       "pick_agreement_with_exhaustive_fp32": float(np.mean(b_exb == b_ex))},
        "pruned": {"search_patterns_per_s": n_test / t_prb,
                   "patterns_per_s_with_refinement": n_test / (t_prb + t_rfb),
                   "fallback_fraction": float(prb["fallback"].cpu().numpy().astype(bool).mean()),
                   "pick_agreement_with_exhaustive_fp32": float(np.mean(b_prb == b_ex)),
                   "refined_vs_truth_deg_median": float(np.median(rpb)),
                   "refined_within_0.1deg_of_exhaustive_fp32": float(np.mean(rpbe <= 0.1))},
        "pattern_bytes": int(test_b.numel() * 2)}
    print("[bench] proposal: exhaustive %.0f patterns/s, pruned %.0f patterns/s (search), refined within 0.1 deg "
          "%.4f, fallback %.3f" % (res["exhaustive"]["search_patterns_per_s"], res["pruned"]["search_patterns_per_s"],
                                   res["pruned"]["refined_within_0.1deg_of_exhaustive"],
                                   res["pruned"]["fallback_fraction"]),
          file=sys.stderr, flush=True)
    net.close()
    return res


if __name__ == "__main__":
    main()

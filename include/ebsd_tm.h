/*
 * ebsd_tm.h -- C ABI of the MI355X (gfx950) hot path of refined template
 * matching for EBSD indexing (Foden, Collins, Wilkinson & Britton, arXiv
 * 1807.11313).
 *
 * The problem (Introduction and section "Method Overview"): experimental
 * patterns are compared with a library of templates, each a gnomonic
 * projection of a spherical master pattern for one crystal orientation; the
 * comparison is the normalised cross-correlation of filtered images,
 * evaluated for every relative shift through the Fourier domain (Equations
 * 2-4); the best match is the template with the highest correlation peak,
 * and its peak position gives the pattern shift.  One library is projected
 * at one nominal pattern centre.  Section "Orientation and Pattern Centre
 * Refinement" then refines each best match: the measured shift gives the
 * rotation about the detector x and y axes (Equation 7, angle = shift /
 * detector distance), a log-polar resampling gives the rotation about the
 * detector normal, and the template is re-projected at the pattern's own
 * pattern centre, about two iterations.  The correlation peak height is the
 * per-pattern quality output (section "Demonstrations").
 *
 * Conventions (the paper defers these to a reference it cites):
 *   image      row-major [row j][col i], float32, square n x n;
 *   PC         (pcx, pcy, pcz) in screen widths: pcx from the left edge,
 *              pcy from the top edge, pcz = source-to-screen distance /
 *              screen width (footnote 2 of section "Fast Fourier Transform");
 *   frame      detector x = +column, y = +row, z = source to screen; pixel
 *              ray d = normalise((i+1/2)/n - pcx, (j+1/2)/n - pcy, pcz);
 *   orientation unit quaternion (w, x, y, z), w >= 0, float64, of the
 *              rotation R with crystal direction c = R d;
 *   master     equirectangular float32 [H][W]: row r at polar angle
 *              (r + 1/2) pi / H from crystal +z, column q at azimuth
 *              2 pi q / W from +x toward +y;
 *   shift      (s_x, s_y) px with E(x) ~ T(x - s): the pattern is the
 *              template moved by +s;
 *   peak h     normalised correlation in [-1, 1].
 *
 * Memory: every array pointer is a DEVICE pointer (hipMalloc / torch CUDA
 * tensors), contiguous, at least 16-byte aligned; structs are host memory.
 * The caller owns all buffers.  The library keeps no caller pointer after a
 * call returns; its scratch is allocated and freed stream-ordered on the
 * caller's stream (hipMallocAsync / hipFreeAsync).
 *
 * Execution: asynchronous on `stream` (a hipStream_t; NULL = null stream).
 * Outputs are valid once the stream has been synchronised.
 *
 * Errors: every function returns EBSD_OK (0) or a negative code; on an
 * argument error nothing is enqueued and no output is written.
 * ebsd_last_error() returns a thread-local description of the last error.
 *
 * Supported pattern sizes: n in {64, 96, 128, 160, 256}.  At n = 256 the
 * FFT form of the search and the full correlation map are not built: the
 * search runs in the DFT-GEMM or the exact FP32 DFT form and every integer
 * peak needs a shift window (max_shift >= 0); other calls return
 * EBSD_E_UNSUPPORTED.
 */
#ifndef EBSD_TM_H
#define EBSD_TM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EBSD_OK 0
#define EBSD_E_INVALID (-1)     /* null pointer, bad size or parameter      */
#define EBSD_E_NOMEM (-2)       /* device allocation failed                 */
#define EBSD_E_DEVICE (-3)      /* HIP runtime or launch error              */
#define EBSD_E_UNSUPPORTED (-4) /* valid request the library does not serve */

/* Arithmetic of the correlation search (the library ranking):
 *   FP32    FP32 FFT form (every cyclic shift, or a window), or the exact
 *           FP32 DFT form over a window
 *   FP16X2  DFT-GEMMs on MFMA, operands split into FP16 hi + lo halves,
 *           products hi*hi + hi*lo + lo*hi accumulated in FP32
 *   BF16X2  the same with BF16 halves
 *   BF16    BF16 operands, one product (reported, not parity-bound)
 * The winner's integer peak, sub-pixel peak and the refinement always run
 * in FP32. */
#define EBSD_PREC_FP32 0
#define EBSD_PREC_FP16X2 1
#define EBSD_PREC_BF16X2 2
#define EBSD_PREC_BF16 3

/* Form of the search: AUTO picks FFT for FP32 (DFT at n = 256, where the
 * FFT form is not built, when max_shift >= 0) and DFTGEMM otherwise.
 * DFTGEMM evaluates only the shift window |s_x|, |s_y| <= max_shift
 * (max_shift >= 0 required; the window's 2 max_shift + 1 shifts are padded
 * to a multiple of 16 and must fit the on-chip constant operands).
 * DFT is the same windowed evaluation in FP32 on the vector ALUs, exactly
 * the two products of the band-limited correlation (Equations 3 and 6a at
 * the window's shifts, no split): the FP32 reference of the split forms,
 * at every supported size (max_shift >= 0, 2 max_shift + 1 <= 208). */
#define EBSD_FORM_AUTO 0
#define EBSD_FORM_FFT 1
#define EBSD_FORM_DFTGEMM 2
#define EBSD_FORM_DFT 3

/* Storage of the caller's pattern images (ebsd_params.input): FP32, or BF16
 * (the bit pattern of bfloat16 values, 2 bytes per pixel, passed through the
 * same float pointer) widened to FP32 as each pixel is loaded.  BF16 images
 * are read by ebsd_pattern_spectra, ebsd_index_patterns, the refinements and
 * ebsd_index_proposed at n <= 160; every other call, and n = 256, returns
 * EBSD_E_UNSUPPORTED for them. */
#define EBSD_INPUT_F32 0
#define EBSD_INPUT_BF16 1

/* A batch of P square patterns of side n, pattern p at data + p n n. */
typedef struct {
  const float* data;
  int64_t P;
  int32_t n;
} ebsd_batch;

/* Equirectangular master pattern, H rows x W columns. */
typedef struct {
  const float* data;
  int32_t H, W;
} ebsd_master;

/* Nominal pattern centre, and optionally one per pattern (device [P][3]). */
typedef struct {
  double pcx, pcy, pcz;
  const double* pc_per;
} ebsd_geometry;

/*
 * Method parameters.  The paper leaves window, filter, upsampling and the
 * log-polar grid unspecified; the defaults (ebsd_params_default) are:
 *   window        1: separable Hann w_i = sin^2(pi (i + 1/2) / n); 0: none
 *   sigma_hp      2.0 cycles/image: high pass 1 - exp(-rho^2 / 2 sigma_hp^2)
 *   sigma_lp_frac 0.125: low pass exp(-rho^2 / 2 (frac n)^2)
 *   rho_max_frac  0.375: filter is zero for rho > frac n (must be <= 0.375)
 *   max_shift     -1: every cyclic shift; k >= 0: |s_x|, |s_y| <= k
 *   upsample      100: sub-pixel step 1/upsample over +-0.75 px
 *   n_iter        2 refinement iterations (fixed, no early exit)
 *   n_rho, n_eta  0, 0: log-polar grid n/2 radii x 2n angles
 *   precision     EBSD_PREC_FP32 (see above)
 *   form          EBSD_FORM_AUTO
 *   input         EBSD_INPUT_F32 (pattern image storage; a caller whose
 *                 struct_size ends before this field gets FP32)
 */
typedef struct {
  uint32_t struct_size; /* sizeof(ebsd_params) */
  int32_t window;
  double sigma_hp, sigma_lp_frac, rho_max_frac;
  int32_t max_shift;
  int32_t upsample;
  int32_t n_iter;
  int32_t n_rho, n_eta;
  int32_t precision;
  int32_t form;
  int32_t input;
} ebsd_params;

/* Fills *p with the defaults above. */
void ebsd_params_default(ebsd_params* p);

/* Library version (major * 10000 + minor * 100 + patch). */
int ebsd_version(void);

/* Thread-local text of the last error ("" if none). */
const char* ebsd_last_error(void);

/*
 * Index every pattern against every library orientation (section "Method
 * Overview", Figure 1 B-C; Equations 2-5).
 *   pats      P patterns of side n (device float32 [P][n][n])
 *   mp        master pattern (device float32 [H][W])
 *   geo       nominal pattern centre; geo->pc_per is ignored (one library)
 *   lib_q     L library orientations (device float64 [L][4], unit, w >= 0)
 *   prm       parameters (NULL: defaults)
 * Outputs (device):
 *   best_idx  int32 [P]   template with the largest integer correlation
 *                         peak, ties to the smallest index
 *   best_q    float64 [P][4]  lib_q[best_idx]        (may be NULL)
 *   peak_h    float32 [P] upsampled peak height of the winner
 *   shift     float32 [P][2] upsampled (s_x, s_y) px of the winner
 *   scores    float32 [P][L] integer peak of every pair (may be NULL)
 */
int ebsd_index_patterns(const ebsd_batch* pats, const ebsd_master* mp, const ebsd_geometry* geo,
                        const double* lib_q, int64_t L, const ebsd_params* prm, int32_t* best_idx,
                        double* best_q, float* peak_h, float* shift, float* scores, void* stream);

/*
 * Library plan: the paper generates its library once and matches every
 * pattern of a map against it (sections "Method Overview" and "Orientation
 * and Pattern Centre Refinement", one library at the nominal pattern
 * centre).  ebsd_plan_create projects the L templates at geo's nominal
 * pattern centre and keeps their filtered band spectra, with a copy of
 * lib_q, in device memory the plan owns (L x 38 KB at n = 128); the
 * parameters are fixed with it.  It first checks on the device that every
 * lib_q row is a unit quaternion (| |q| - 1 | <= 1e-6; EBSD_E_INVALID
 * otherwise, nothing kept) and therefore waits for `stream` once.  The
 * spectra are ready in stream order: calls on the same stream may follow at
 * once, calls on another stream after it has been synchronised.
 *
 * ebsd_index_patterns_plan is ebsd_index_patterns against the plan's library
 * (pats->n must equal the plan's n; outputs as there, best_q from the plan's
 * copy of lib_q).  The results equal those of ebsd_index_patterns with the
 * same library and parameters.  A plan may serve calls on several streams;
 * destroy it only after every such call has finished (synchronise those
 * streams first).
 */
typedef struct ebsd_plan_s* ebsd_plan;
int ebsd_plan_create(const ebsd_master* mp, const ebsd_geometry* geo, const double* lib_q, int64_t L, int32_t n,
                     const ebsd_params* prm, ebsd_plan* plan, void* stream);
int ebsd_index_patterns_plan(ebsd_plan plan, const ebsd_batch* pats, int32_t* best_idx, double* best_q,
                             float* peak_h, float* shift, float* scores, void* stream);
int ebsd_plan_destroy(ebsd_plan plan);

/*
 * Refine starting orientations (section "Orientation and Pattern Centre
 * Refinement"): n_iter times { project the template at (R, PC_p); measure
 * the upsampled shift s; R <- R (Ry(beta) Rx(alpha))^T with beta =
 * atan(s_x / DD), alpha = -atan(s_y / DD), DD = pcz n px; re-project; measure
 * the log-polar eta shift d; R <- R Rz(gamma)^T, gamma = 2 pi d / n_eta };
 * then a final projection and correlation give peak_h and shift.
 *   geo->pc_per  per-pattern pattern centres (device [P][3]) or NULL for
 *                the nominal one
 *   q_init       device float64 [P][4]
 * Outputs (device): q_out float64 [P][4] (may alias q_init), peak_h float32
 * [P], shift float32 [P][2].
 */
int ebsd_refine_orientations(const ebsd_batch* pats, const ebsd_master* mp, const ebsd_geometry* geo,
                             const double* q_init, const ebsd_params* prm, double* q_out, float* peak_h,
                             float* shift, void* stream);

/*
 * Map-wide pattern-centre model (section "Orientation and Pattern Centre
 * Refinement", Figure 6 B, and the silicon-map demonstrations: the PC drifts
 * as the beam scans the map; the paper imports its model and states no
 * form).  Affine in the map position: point k of a row-major map `width`
 * points wide sits at col = k mod width, row = k / width (integer division)
 * and has
 *   pc(k) = pc0 + (col - col0) d_col + (row - row0) d_row,
 * each a (pcx, pcy, pcz) triple in screen widths.
 */
typedef struct {
  double pc0[3];
  double d_col[3];
  double d_row[3];
  double col0, row0;
  int64_t width;
} ebsd_pc_model;

/*
 * Evaluates the model for points 0 .. P-1 into pc_out (device float64
 * [P][3], the layout of ebsd_geometry.pc_per).  width >= 1; P = 0 is a
 * no-op.
 */
int ebsd_pc_map(const ebsd_pc_model* model, int64_t P, double* pc_out, void* stream);

/*
 * ebsd_refine_orientations without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * ebsd_refine_orientations (bit for bit); its scratch is one static device
 * array of 256 MiB per GPU, held from the library's first use on that GPU
 * until the process ends.  A batch needs per pattern
 * 4 n^2 + 16 (2B+1)(B+1) + 8 n_rho n_eta + 32 bytes (B = 3n/8), at n = 256
 * another 198,768 bytes of transform scratch, plus tables of a few KB and
 * 256-byte alignment of each buffer: at the default parameters at most
 * about 980 patterns of 128 x 128, or 200 of 256 x 256, per call.
 * Larger batches return EBSD_E_INVALID (the message states the bytes needed)
 * before anything is enqueued.  Nothing in the scratch needs to start at
 * zero: every buffer is written before it is read.  All calls on one GPU
 * share its array, which keeps the last call's contents: calls that overlap
 * in time on one GPU (different streams or threads) race and must be
 * serialised by the caller.
 */
int ebsd_refine_orientations_noalloc(const ebsd_batch* pats, const ebsd_master* mp, const ebsd_geometry* geo,
                                     const double* q_init, const ebsd_params* prm, double* q_out, float* peak_h,
                                     float* shift, void* stream);

/*
 * Refinement that starts from the search's own measurement (section
 * "Orientation and Pattern Centre Refinement": one library at one pattern
 * centre; the shift measured against it is corrected for the beam-induced
 * PC move before Equation 7 turns it into a rotation).  The first x/y step
 * takes
 *   s = match_shift - n (pc_per[p].x - pcx, pc_per[p].y - pcy)
 * (a PC move by (dx, dy) screen widths translates the pattern by +n (dx, dy)
 * px) in place of a projection and correlation at the starting
 * orientation; the z step, the further iterations and the final
 * measurement are those of ebsd_refine_orientations at each point's own PC.
 * With n_iter = 0 it is the final measurement alone.
 *   geo          pcx, pcy, pcz: the PC the library was projected at;
 *                pc_per: per-point PCs (device [P][3]) or NULL (every point
 *                at the library's PC: no correction)
 *   q_init       device float64 [P][4]: the search's best_q
 *   match_shift  device float32 [P][2] (s_x, s_y) px: the search's shift
 *                for the same patterns and orientations
 * Outputs as ebsd_refine_orientations (q_out may alias q_init).
 */
int ebsd_refine_from_match(const ebsd_batch* pats, const ebsd_master* mp, const ebsd_geometry* geo,
                           const double* q_init, const float* match_shift, const ebsd_params* prm, double* q_out,
                           float* peak_h, float* shift, void* stream);

/*
 * Capture range of the correlation (section "SO(3) Sampling Frequency",
 * Figures 3 and 4): for each reference orientation r and each detector axis
 * a = x, y, z, the integer correlation peak of the reference pattern
 * (projected at geo_ref's PC) against the pattern of the crystal rotated by
 * theta_k about that axis (orientation R Q^T, projected at geo_test's PC, so
 * that a PC error can be studied), and the full width at half maximum of
 * that curve above its floor: the level is halfway between its largest and
 * smallest samples (the correlation of a shifted, unrelated pattern stays
 * well above zero); from the largest sample the width runs outwards to the
 * first sample below the level on each side, interpolated linearly (a side
 * that never drops reports the end of the sampled range).
 *   q_ref      device float64 [R][4]
 *   theta_deg  device float64 [T], ascending, degrees
 *   geo_ref, geo_test  pattern centres (pc_per ignored)
 *   h          out: device float32 [R][3][T]
 *   width      out: device float64 [R][3], degrees
 * Scratch holds the 3 R T rotated images and spectra.
 */
int ebsd_capture_range(const ebsd_master* mp, const double* q_ref, int64_t R, int32_t n,
                       const ebsd_geometry* geo_ref, const ebsd_geometry* geo_test, const double* theta_deg,
                       int32_t T, const ebsd_params* prm, float* h, double* width, void* stream);

/*
 * Equispaced orientation library (section "SO(3) Spacing", Figure 2): an
 * S^2 x S^1 sampling of SO(3) reduced to the cubic fundamental zone.  For a
 * spacing d: m = round(pi / d) polar rings theta_i = pi i / m, ring i with
 * n_i = max(1, round(2 m sin theta_i)) azimuths phi_j = 2 pi j / n_i; the
 * circle with n_psi = round(2 pi / d) angles psi_k = 2 pi k / n_psi (rounding
 * half to even); grid point (theta, phi, psi) is the orientation
 * Rz(phi) Ry(theta) Rz(psi - phi).  A point is kept if no cubic equivalent
 * has a larger |w| by more than 1e-12; among equivalents tied within 1e-12
 * only the one whose canonical quaternion (w >= 0; at w = 0 the first
 * non-zero component positive) is lexicographically smallest is kept.  The
 * full grid over SO(3) holds 24 x 618.0 points at 10 deg and 24 x 4956 at
 * 5 deg (the paper's library sizes, 618 and 4958).
 *   spacing_deg  in [0.5, 90]
 *   q_out        device float64 [cap][4], the kept points in grid order
 *                (w >= 0); only the first cap are written (cap = 0 and
 *                q_out = NULL query the size)
 *   count        HOST int64: the number of library orientations
 * Synchronises `stream` (the count is read back); scratch holds the full
 * grid (32 B per point, 8 pi^2 / d^3 points).
 */
int ebsd_so3_library(double spacing_deg, double* q_out, int64_t cap, int64_t* count, void* stream);

/*
 * Nearest-neighbour disorientation within a set of orientations (Equation 6
 * with the 24 proper cubic operators; Figure 2): for each orientation, the
 * smallest disorientation angle to any other member and that member's
 * index (ties to the smaller index).
 *   q       device float64 [L][4] unit quaternions; L = 0 or L >= 2
 *   nn_deg  out: device float64 [L], degrees
 *   nn_idx  out: device int32 [L]
 * All pairs are compared (L^2 work).
 */
int ebsd_nn_disorientation(const double* q, int64_t L, double* nn_deg, int32_t* nn_idx, void* stream);

/* ---- stage entry points (the same kernels, exposed for stage-by-stage checks) ---- */

/*
 * Gnomonic projection (section "SO(3) Library Generation"): K templates of
 * side n for orientations q (device float64 [K][4]) at geo's pattern centre
 * (or geo->pc_per[k]); out: device float32 [K][n][n], raw master intensities.
 */
int ebsd_project_templates(const ebsd_master* mp, const double* q, int64_t K, int32_t n,
                           const ebsd_geometry* geo, float* out, void* stream);

/*
 * Filtered unit-energy spectra of K images of side n (device float32
 * [K][n][n]): contrast normalised, windowed, 2-D DFT (Equation 4 without
 * the unitary factor), band-passed, scaled to unit energy.
 * spec: device complex64 (interleaved float32 pairs) [K][2B+1][B+1],
 * B = 3n/8, element [kk][v] = X(u, v) with u = kk (kk <= B) or kk - 2B - 1;
 * energy: device float64 [K], the pre-scaling energy sum |X'|^2 over the
 * full spectrum (may be NULL).
 */
int ebsd_pattern_spectra(const float* imgs, int64_t K, int32_t n, const ebsd_params* prm, float* spec,
                         double* energy, void* stream);

/* Number of float32 values (2 per complex) of one stored spectrum of side n, or -1. */
int64_t ebsd_spectrum_floats(int32_t n);

/*
 * Integer correlation peak of K (pattern, template) spectrum pairs
 * (spec_p[pi[k]], spec_l[li[k]]): h_int float32 [K], s_int int32 [K][2]
 * (s_x, s_y signed in [-n/2, n/2)), and optionally the full map float32
 * [K][n][n] indexed [s_y mod n][s_x mod n] (map may be NULL).
 */
int ebsd_xcf_peak(const float* spec_p, const float* spec_l, const int32_t* pi, const int32_t* li,
                  int64_t K, int32_t n, const ebsd_params* prm, float* h_int, int32_t* s_int, float* map,
                  void* stream);

/* Score matrix h_int[p][l] of P pattern spectra against L template spectra. */
int ebsd_xcf_scores(const float* spec_p, int64_t P, const float* spec_l, int64_t L, int32_t n,
                    const ebsd_params* prm, float* scores, void* stream);

/*
 * Scores of each pattern against its own K candidate templates (the pruned
 * search of the learned proposal): scores float32 [P][K], scores[p][j] =
 * h_int of pattern p against template cand[p][j] (cand int32 [P][K], device;
 * an index outside [0, L) is clamped to the nearest template).  The values
 * equal those ebsd_xcf_scores gives the same pairs (same kernel).  FP32 FFT
 * form at n = 128 only (EBSD_E_UNSUPPORTED otherwise); K <= L.
 */
int ebsd_xcf_scores_cand(const float* spec_p, int64_t P, const float* spec_l, int64_t L,
                         const int32_t* cand, int32_t K, int32_t n, const ebsd_params* prm,
                         float* scores, void* stream);

/* Upsampled peak around s_int for K pairs: h_sub float32 [K], s_sub float32 [K][2] (x, y). */
int ebsd_xcf_subpixel(const float* spec_p, const float* spec_l, const int32_t* pi, const int32_t* li,
                      int64_t K, int32_t n, const int32_t* s_int, const ebsd_params* prm, float* h_sub,
                      float* s_sub, void* stream);

/*
 * Log-polar rotation measurement: gamma float64 [K] (radians) of pattern k
 * relative to template k (both device float32 [K][n][n]); positive gamma
 * means the pattern is the template rotated by +gamma in
 * eta = atan2(row - c, col - c).
 */
int ebsd_measure_rotation(const float* pats, const float* tmpls, int64_t K, int32_t n,
                          const ebsd_params* prm, double* gamma, void* stream);

/*
 * Instrumentation.  While enabled, every launch of the correlation search
 * kernel (the dominant kernel of ebsd_index_patterns and ebsd_xcf_scores)
 * is bracketed by a pair of HIP events recorded on the caller's stream.
 * ebsd_timing_read (after the stream has been synchronised) returns the
 * summed elapsed time in ms and the number of launches, and clears the
 * record.  Not for concurrent use from several threads.
 */
int ebsd_timing_enable(int enable);
int ebsd_timing_read(double* total_ms, int64_t* launches);

/*
 * Ragged batches (patterns of several detector binnings in one call).
 *
 * A plan fixes the batch layout: P patterns, pattern p of side n_per[p]
 * (64, 96, 128 or 160) stored row-major at element offset offset[p] of one
 * packed float32 buffer; both arrays are HOST memory, read during the call.
 * It also fixes the library size L and the parameters (the FP32 FFT form;
 * max_shift, filter and upsampling as in ebsd_params).  Creating a plan
 * allocates all device memory the runs need, and times candidate tiles of
 * the persistent search kernel for every size present (the number of
 * templates each work item correlates and the persistent grid), keeping the
 * fastest (EBSD_RAGGED_NO_AUTOTUNE keeps 16 templates and the resident
 * capacity).  The chosen tiles are kept for the life of the process, keyed by
 * the device architecture, compute-unit count, size and shift window, and
 * reused by later plans.
 *
 * ebsd_ragged_run indexes the batch against the library (method of
 * ebsd_index_patterns, each pattern against templates projected at its own
 * size and the nominal pattern centre) and, with EBSD_RAGGED_STENCIL, then
 * evaluates around each pattern's best template the 27 orientations
 * R Q(a, b, c)^T, Q = Rz(c) Ry(b) Rx(a), a, b, c in {-d, 0, +d} with
 * d = stencil_step_deg (numbered 9 i_a + 3 i_b + i_c, i = 0, 1, 2 for -d,
 * 0, +d), each projected at the pattern's own pattern centre (geo->pc_per
 * [P][3] device, or the nominal one), keeps the candidate with the largest
 * integer correlation peak (ties: smaller number) and upsamples its peak;
 * this grid search is the coarse alternative to the refinement that the
 * paper's closing discussion mentions.  With EBSD_RAGGED_REFINE the
 * orientation is then refined as by ebsd_refine_orientations (n_iter x / y
 * and z steps at each pattern's own pattern centre, section "Orientation
 * and Pattern Centre Refinement"), the first x / y step taken from the shift
 * already measured: the stencil winner's, or without the stencil the
 * library pick's less the PC-move translation (as ebsd_refine_from_match);
 * peak_h and shift are then the final measurement's.
 * Outputs in pattern order (device): best_idx [P] library index (may be
 * NULL), q_out [P][4] final orientation, peak_h [P], shift [P][2] (x, y) of
 * the final template, stencil_idx [P] chosen candidate number (-1 without
 * the stencil; may be NULL).  The first run captures the whole sequence into
 * one HIP graph; later runs with the same pointers and geometry replay it
 * (EBSD_RAGGED_EAGER enqueues the kernels directly instead).  A plan serves
 * one run at a time: runs of one plan on different streams race.
 */
typedef struct ebsd_ragged_plan_s* ebsd_ragged_plan;
#define EBSD_RAGGED_STENCIL 1
#define EBSD_RAGGED_EAGER 2
#define EBSD_RAGGED_NO_AUTOTUNE 4
#define EBSD_RAGGED_REFINE 8

int ebsd_ragged_plan_create(const int32_t* n_per, const int64_t* offset, int64_t P, int64_t L,
                            const ebsd_params* prm, double stencil_step_deg, int32_t flags,
                            ebsd_ragged_plan* plan);
int ebsd_ragged_run(ebsd_ragged_plan plan, const float* data, const ebsd_master* mp, const ebsd_geometry* geo,
                    const double* lib_q, int32_t* best_idx, double* q_out, float* peak_h, float* shift,
                    int32_t* stencil_idx, void* stream);
/* Chosen tiles: for each size present, tiles[4 k ..] = (n, patterns,
 * templates per work item, persistent grid blocks); *count sizes (<= 4). */
int ebsd_ragged_plan_tiles(ebsd_ragged_plan plan, int32_t* tiles, int32_t* count);
/* Waits for the plan's last run (on the caller's stream it was given) and
 * its own streams, then frees the plan; other work on the device is not
 * waited for. */
int ebsd_ragged_plan_destroy(ebsd_ragged_plan plan);

/*
 * Learned proposal.  The paper ranks every template by correlation; here a
 * small convolutional network ranks the library orientations first and the
 * correlation runs only on its top k, with the exhaustive search as the
 * fallback for every pattern whose best peak height stays below a threshold
 * (the peak height is the paper's quality measure, section "Deformed
 * alpha-Fe Dataset").  Network: the pattern binned by block means to
 * 64 x 64 and normalised to zero mean, unit variance; four 3 x 3
 * convolutions (zero padding, bias, ReLU) with 32, 64, 128, 128 channels,
 * each followed by a 2 x 2 max pool; a fully connected layer from the
 * 128 x 4 x 4 features to the L library orientations; softmax
 * cross-entropy against the library orientation nearest (cubic
 * disorientation) to the true one.  The convolutions of the training
 * forward pass (ebsd_cnn_gradients, ebsd_cnn_train_step) run in FP32; its
 * fc product, the backward products and inference (ebsd_cnn_forward,
 * ebsd_index_proposed) in the precision ebsd_cnn_set_precision chose.  Parameters are one
 * flat float vector: conv_i.w [co][ci][3][3], conv_i.b [co] for i = 1..4,
 * fc.w [L][2048], fc.b [L].  A network object owns its parameters, Adam
 * state and workspace on the device it was created on.
 */
typedef struct ebsd_cnn_s* ebsd_cnn;

/* Number of parameters for L classes (-1 for L < 1). */
int64_t ebsd_cnn_param_count(int32_t n_classes);
/* He-normal weights from a Philox4x32-10 stream keyed by seed, zero biases. */
int ebsd_cnn_create(int32_t n_classes, uint64_t seed, ebsd_cnn* out, void* stream);
int ebsd_cnn_destroy(ebsd_cnn cnn);
/* Copy the parameter vector out of / into the network (device [count]);
 * setting parameters also resets the Adam state. */
int ebsd_cnn_get_params(ebsd_cnn cnn, float* out, void* stream);
int ebsd_cnn_set_params(ebsd_cnn cnn, const float* in, void* stream);
/* Network inputs x [P][64][64] from patterns [P][n][n], n a multiple of 64. */
int ebsd_cnn_input(const float* pats, int64_t P, int32_t n, float* x, void* stream);
/* Scores over the library, logits [B][L]. */
int ebsd_cnn_forward(ebsd_cnn cnn, const float* x, int64_t B, float* logits, void* stream);
/* Precision of the inference products and of the training's backward
 * products: EBSD_PREC_BF16X2 (the default) splits every FP32 operand into
 * BF16 hi + lo halves and accumulates hi*hi + hi*lo + lo*hi in FP32 on the
 * BF16 matrix cores (scores within about 1e-5 of the largest, gradients
 * about 1e-5, relative); EBSD_PREC_FP32 uses FP32 operands throughout.
 * EBSD_E_UNSUPPORTED for FP16X2 and BF16, EBSD_E_INVALID for other values.
 * The convolutions of the training forward are FP32 either way: they decide
 * which ReLU and pooling inputs carry the gradient, and split rounding would
 * move that choice for near ties. */
int ebsd_cnn_set_precision(ebsd_cnn cnn, int32_t precision);
/* Mean cross-entropy of the batch (device float *loss) and its gradient
 * (device [count], parameter order); B in [1, 4096]. */
int ebsd_cnn_gradients(ebsd_cnn cnn, const float* x, const int32_t* labels, int64_t B, float* grad, float* loss,
                       void* stream);
/* One Adam step (beta 0.9, 0.999, eps 1e-8) on the batch's gradient. */
int ebsd_cnn_train_step(ebsd_cnn cnn, const float* x, const int32_t* labels, int64_t B, float lr, float* loss,
                        void* stream);
/* One Adam step (Kingma and Ba, Algorithm 1: beta 0.9, 0.999, eps 1e-8,
 * bias-corrected moments; step count t = 1, 2, ... since creation or the last
 * ebsd_cnn_set_params) from a caller-supplied gradient grad (device [count],
 * parameter order), with step size lr > 0.  ebsd_cnn_train_step is
 * ebsd_cnn_gradients followed by this step. */
int ebsd_cnn_apply_gradient(ebsd_cnn cnn, const float* grad, float lr, void* stream);
/* Training data made on the device: sample s in [first, first + B) gets a
 * uniform random orientation and an in-plane pattern-centre offset of up to
 * +-max_offset_px (Philox4x32-10 keyed by seed, counter s), is projected at
 * n x n from the master, scaled to `counts` mean counts with Poisson noise
 * (normal approximation) plus Gaussian noise for the given SNR, and binned
 * into x [B][64][64]; labels [B] (optional) is its nearest library
 * orientation, q_true [B][4] (optional) its orientation. */
int ebsd_cnn_make_batch(const ebsd_master* mp, const ebsd_geometry* geo, const double* lib_q, int64_t L, int32_t n,
                        int64_t B, int64_t first, uint64_t seed, double max_offset_px, double counts, double snr,
                        float* x, int32_t* labels, double* q_true, void* stream);
/* The k best library indices per row of logits [rows][L], best first (ties:
 * smaller index). */
int ebsd_cnn_topk(const float* logits, int64_t rows, int32_t L, int32_t k, int32_t* idx, void* stream);
/* ebsd_index_patterns with the search pruned to the network's top_k
 * orientations per pattern (n = 64 or 128, FP32 FFT form): the best
 * candidate by integer peak height (ties: smaller library index); patterns
 * whose best stays below fallback_tau are searched exhaustively, and
 * fallback [P] (optional) marks them.  Outputs as ebsd_index_patterns.  The
 * call waits for the stream once, to learn how many patterns fall back. */
int ebsd_index_proposed(const ebsd_batch* pats, const ebsd_master* mp, const ebsd_geometry* geo,
                        const double* lib_q, int64_t L, ebsd_cnn cnn, int32_t top_k, float fallback_tau,
                        const ebsd_params* prm, int32_t* best_idx, double* best_q, float* peak_h, float* shift,
                        int32_t* fallback, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* EBSD_TM_H */

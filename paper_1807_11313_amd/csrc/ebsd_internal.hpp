// Internal launch interface between the C-ABI layer and the kernels.
// Every launcher enqueues on `stream` and returns the hipError_t of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ebsd {

struct FilterParams {
  int window;
  float sigma_hp, sigma_lp, rho_max;
};

// Band half-width of the stored spectra for a supported size (3N/8), or -1.
// Sizes 64, 96, 128, 160 run every stage; 256 runs the spectra, the
// DFT-GEMM search and the shift-window peaks (its full-map FFT does not fit
// one block's LDS).
int band_of(int n);
bool size_supported(int n);
bool fft_supported(int n);

// Spectra at 256 x 256 (three passes through a scratch of
// spectra256_scratch_bytes(k) bytes); images contiguous.
size_t spectra256_scratch_bytes(int64_t k);
hipError_t launch_spectra256(const float* imgs, int64_t k, const FilterParams& fp, float2* spec, double* energy,
                             void* scratch, hipStream_t stream);

// Integer peak inside the shift window |s_x|, |s_y| <= max_shift, evaluated
// exactly in FP32 on the band (any supported size); tables of
// window_table_size complex elements built by launch_window_tables.
bool window_peak_supported(int n, int max_shift);
int window_table_size(int n, int max_shift);
hipError_t launch_window_tables(int n, int max_shift, float2* tab, hipStream_t stream);
hipError_t launch_window_peak(int n, const float2* spec_p, const float2* spec_l, const int32_t* pi,
                              const int32_t* li, int64_t k, int max_shift, const float2* tab, float* h_int,
                              int32_t* s_int, hipStream_t stream);
// The same exact FP32 evaluation as a library search: scores[p][l] = the
// window's largest value for every pattern x template.
hipError_t launch_window_scores(int n, const float2* spec_p, int64_t p, const float2* spec_l, int64_t l,
                                int max_shift, const float2* tab, float* scores, hipStream_t stream);

// Contrast-normalise, window, forward 2-D DFT, band-pass, FP64 energy and
// unit-energy scaling of K n x n images (image k at imgs + k * img_stride).
// Output: spec[k][kk][v] complex64 (kk in [0, 2B + 1), v in [0, B]), energy[k].
hipError_t launch_spectra(int n, const float* imgs, int64_t img_stride, int64_t k,
                          const FilterParams& fp, float2* spec, double* energy,
                          hipStream_t stream);
// The same from BF16 pixels (each widened to FP32 on load; n <= 160).
hipError_t launch_spectra(int n, const __bf16* imgs, int64_t img_stride, int64_t k,
                          const FilterParams& fp, float2* spec, double* energy,
                          hipStream_t stream);

// Spectra of K images at element offsets img_off[k] of imgs.
hipError_t launch_spectra_gather(int n, const float* imgs, const int64_t* img_off, int64_t k,
                                 const FilterParams& fp, float2* spec, double* energy, hipStream_t stream);

// Persistent form of the search (sizes 64 to 160): `grid` blocks take
// (pattern, chunk of lchunk templates) items from the device counter *queue,
// which must be zero when the kernel starts.  Block size and the resident
// blocks per CU of the kernel that serves size n.
hipError_t xcf_persistent_occupancy(int n, int max_shift, int* blocks_per_cu);
hipError_t launch_xcf_scores_persistent(int n, const float2* spec_p, int64_t p, const float2* spec_l, int64_t l,
                                        int max_shift, float* scores, int lchunk, int grid, int* queue,
                                        hipStream_t stream);

// Integer-peak scores h[p][l] = max_s rho(p, l; s) for every pattern x template.
hipError_t launch_xcf_scores(int n, const float2* spec_p, int64_t p, const float2* spec_l,
                             int64_t l, int max_shift, float* scores, hipStream_t stream);
// The same for each pattern's own k candidates among l templates: scores[p][j]
// for template cand[p][j], clamped to [0, l) (n = 128; hipErrorInvalidValue for
// other sizes).
hipError_t launch_xcf_scores_cand(int n, const float2* spec_p, int64_t p, const float2* spec_l, int64_t l,
                                  const int32_t* cand, int k, int max_shift, float* scores, hipStream_t stream);

// Integer peak (value, signed shift) for K explicit pairs (pi[k], li[k]),
// and optionally the full correlation map [K][n][n] (row = s_y mod n).
hipError_t launch_xcf_peak(int n, const float2* spec_p, const float2* spec_l,
                           const int32_t* pi, const int32_t* li, int64_t k, int max_shift,
                           float* h_int, int32_t* s_int, float* map, hipStream_t stream);

// Phase tables of the upsampled peak for (n, kappa): size in complex
// elements, their construction, and the LDS one block of the kernel needs.
int subpixel_table_size(int n, int kappa);
size_t subpixel_lds_bytes(int n, int kappa);
hipError_t launch_subpixel_tables(int n, int kappa, float2* tab, hipStream_t stream);

// Upsampled peak around s_int: h_sub[k], s_sub[k] = (s_x, s_y) px.
hipError_t launch_subpixel(int n, const float2* spec_p, const float2* spec_l,
                           const int32_t* pi, const int32_t* li, int64_t k,
                           const int32_t* s_int, int kappa, const float2* tab,
                           float* h_sub, float* s_sub, hipStream_t stream);

// exp(2 pi i k / m) for k in [0, m), computed in FP64 and rounded.
hipError_t launch_roots(int m, float2* out, hipStream_t stream);

// Gnomonic projection of the master for K orientations (FP64 quaternions),
// at one pattern centre or one per orientation.
hipError_t launch_project(int n, const float* master, int mh, int mw, const double* q,
                          int64_t k, const double* pc_per, double pcx, double pcy, double pcz,
                          float* out, hipStream_t stream);

// Windowed search as split-precision DFT-GEMMs on MFMA (precision 0: FP16
// hi + lo, 1: BF16 hi + lo, 2: BF16), |s_x|, |s_y| <= max_shift.  `frag` is
// scratch of gemm_frag_bytes(n, max_shift) bytes for the constant operands.
bool gemm_supported(int n, int max_shift);
size_t gemm_frag_bytes(int n, int max_shift);
hipError_t launch_xcf_gemm(int n, int precision, const float2* spec_p, int64_t p, const float2* spec_l,
                           int64_t l, int max_shift, unsigned short* frag, float* scores, hipStream_t stream);

// Best template per pattern from the score matrix (ties: smallest index).
hipError_t launch_library_argmax(const float* scores, int64_t p, int64_t l, int32_t* best,
                                 float* best_h, hipStream_t stream);

// best_q[p] = lib_q[best[p]]
hipError_t launch_gather_q(const double* lib_q, const int32_t* best, int64_t p, double* best_q,
                           hipStream_t stream);

// Log-polar resampling of contrast-normalised images, rows mean-removed.
hipError_t launch_logpolar(int n, const float* imgs, int64_t k, int n_rho, int n_eta,
                           float* out, hipStream_t stream);
hipError_t launch_logpolar(int n, const __bf16* imgs, int64_t k, int n_rho, int n_eta,
                           float* out, hipStream_t stream);

// eta correlation of pattern / template log-polar images, peak refined by
// trigonometric interpolation: gamma[k] (radians).
hipError_t launch_eta_peak(const float* lp_e, const float* lp_t, int64_t k, int n_rho,
                           int n_eta, int kappa, double* gamma, hipStream_t stream);

// FP64 orientation updates: R <- R (Ry(beta) Rx(alpha))^T from s_sub, and
// R <- R Rz(gamma)^T.  beam_pc0 (x, y), if given with pc_per, is the PC the
// shift was measured at: the PC-move translation is subtracted first.
hipError_t launch_update_xy(double* q, const float* s_sub, int64_t k, const double* pc_per,
                            double pcz, int n, hipStream_t stream, const double* beam_pc0 = nullptr);

// Affine map-wide pattern-centre model: pc(k) = pc0 + (col - col0) d_col +
// (row - row0) d_row, col = k mod width, row = k / width.
struct PcModel {
  double pc0[3], d_col[3], d_row[3];
  double col0, row0;
  int64_t width;
};
hipError_t launch_pc_map(const PcModel& m, int64_t k, double* out, hipStream_t stream);

// Capture range: rotated test orientations q[(r*3 + a)*nt + k] = q_ref[r] (x)
// conj(q_a(theta_k)) with ref_of = r, and the FWHM of nc sampled curves.
hipError_t launch_capture_orient(const double* q_ref, int64_t nr, const double* theta_deg, int nt, double* q,
                                 int32_t* ref_of, hipStream_t stream);
hipError_t launch_fwhm(const float* h, int64_t nc, const double* t, int nt, double* width, hipStream_t stream);

// Equispaced orientation library: the S^2 x S^1 grid (ring_off[m + 2]: first
// azimuth index of each of the m + 1 polar rings, then the total), reduced
// to the cubic fundamental zone and compacted in grid order into q_out (at
// most cap entries); *count (device) receives the full count.
hipError_t launch_so3_library(const int64_t* ring_off, int m, int n_psi, int64_t n_all, double* q_all,
                              unsigned char* keep, double* q_out, int64_t cap, int64_t* count, hipStream_t stream);
// Nearest-neighbour cubic disorientation (degrees) and index of each of n
// orientations.
hipError_t launch_nn_disorientation(const double* q, int64_t n, double* nn_deg, int32_t* nn_idx,
                                    hipStream_t stream);
hipError_t launch_update_z(double* q, const double* gamma, int64_t k, hipStream_t stream);

}  // namespace ebsd

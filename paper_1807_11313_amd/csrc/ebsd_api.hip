// C-ABI layer: argument validation, stream-ordered scratch, and the kernel
// sequence of each entry point (declared and documented in include/ebsd_tm.h).
#include "../../include/ebsd_tm.h"
#include "ebsd_internal.hpp"
#include "api_util.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace ebsd;

namespace ebsd {
namespace api {

thread_local std::string g_last_error;

int fail(int code, const char* msg) {
  g_last_error = msg;
  return code;
}

int fail_hip(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return EBSD_E_DEVICE;
}

#define EBSD_TRY(expr, where)                      \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return fail_hip(e_, where); \
  } while (0)

// Where an entry point's device scratch comes from.
class Arena {
 public:
  virtual ~Arena() = default;
  virtual void* raw(size_t bytes, hipError_t* err) = 0;
  template <class T>
  T* get(size_t count, hipError_t* err) {
    return static_cast<T*>(raw((count ? count : 1) * sizeof(T), err));
  }
};

// Scratch allocated in stream order on the caller's stream and released in
// stream order when the call returns; the device memory pool keeps it for
// the next call, so repeated calls do not reach the kernel-mode allocator.
class Scratch : public Arena {
 public:
  explicit Scratch(hipStream_t s) : stream_(s) {}
  ~Scratch() override {
    for (void* p : ptrs_) (void)hipFreeAsync(p, stream_);
  }
  void* raw(size_t bytes, hipError_t* err) override {
    void* p = nullptr;
    *err = hipMallocAsync(&p, bytes, stream_);
    if (*err != hipSuccess) return nullptr;
    ptrs_.push_back(p);
    return p;
  }

 private:
  hipStream_t stream_;
  std::vector<void*> ptrs_;
};

// Consecutive 256-byte aligned pieces of one caller-given device buffer
// (base may be null: the arena then only adds up the bytes it would hand
// out, to size a call before anything is enqueued).
class FixedArena : public Arena {
 public:
  FixedArena(void* base, size_t cap) : base_(static_cast<char*>(base)), cap_(cap) {}
  void* raw(size_t bytes, hipError_t* err) override {
    const size_t at = (used_ + 255) & ~size_t(255);
    if (at + bytes > cap_ || at + bytes < at) {
      *err = hipErrorOutOfMemory;
      return nullptr;
    }
    used_ = at + bytes;
    *err = hipSuccess;
    return base_ ? base_ + at : reinterpret_cast<void*>(at + 256);
  }
  size_t used() const { return used_; }

 private:
  char* base_;
  size_t cap_;
  size_t used_ = 0;
};

#define EBSD_ALLOC(var, T, count, scratch)                                   \
  T* var = nullptr;                                                          \
  do {                                                                       \
    hipError_t e_ = hipSuccess;                                              \
    var = (scratch).template get<T>((size_t)(count), &e_);                   \
    if (e_ != hipSuccess) return fail(EBSD_E_NOMEM, "device allocation failed: " #var); \
  } while (0)

constexpr size_t kParamsV1 = offsetof(ebsd_params, form) + sizeof(int32_t);

// Copies the caller's parameter block (of any size >= the first version)
// over the defaults and validates it.
int resolve_params(const ebsd_params* in, int n, ebsd_params* out) {
  ebsd_params_default(out);
  if (in) {
    if (in->struct_size < kParamsV1) return fail(EBSD_E_INVALID, "ebsd_params.struct_size too small");
    const size_t sz = in->struct_size < sizeof(ebsd_params) ? in->struct_size : sizeof(ebsd_params);
    std::memcpy(out, in, sz);
    out->struct_size = sizeof(ebsd_params);
  }
  if (!(out->sigma_hp > 0.0) || !(out->sigma_lp_frac > 0.0) || !(out->rho_max_frac > 0.0))
    return fail(EBSD_E_INVALID, "filter parameters must be positive");
  if (out->rho_max_frac > 0.375 + 1e-12)
    return fail(EBSD_E_UNSUPPORTED, "rho_max_frac above 3/8 is outside the stored band");
  if (out->upsample < 1 || out->upsample > 128) return fail(EBSD_E_INVALID, "upsample must be in [1, 128]");
  if (size_supported(n) && subpixel_lds_bytes(n, out->upsample) > 160 * 1024)
    return fail(EBSD_E_UNSUPPORTED, "upsample too large for this pattern size");
  if (out->n_iter < 0 || out->n_iter > 64) return fail(EBSD_E_INVALID, "n_iter must be in [0, 64]");
  if (out->n_rho == 0) out->n_rho = n / 2;
  if (out->n_eta == 0) out->n_eta = 2 * n;
  if (out->n_rho < 2 || out->n_rho > 4096) return fail(EBSD_E_INVALID, "n_rho must be in [2, 4096]");
  if (out->n_eta < 4 || out->n_eta > 1024 || (out->n_eta & 1))
    return fail(EBSD_E_INVALID, "n_eta must be even and in [4, 1024]");
  if (out->precision < EBSD_PREC_FP32 || out->precision > EBSD_PREC_BF16)
    return fail(EBSD_E_UNSUPPORTED, "unknown precision");
  if (out->form < EBSD_FORM_AUTO || out->form > EBSD_FORM_DFT) return fail(EBSD_E_UNSUPPORTED, "unknown form");
  if (out->max_shift < -1) return fail(EBSD_E_INVALID, "max_shift must be >= -1");
  if (out->input != EBSD_INPUT_F32 && out->input != EBSD_INPUT_BF16)
    return fail(EBSD_E_UNSUPPORTED, "unknown pattern input type");
  if (out->input == EBSD_INPUT_BF16 && n > 160)
    return fail(EBSD_E_UNSUPPORTED, "BF16 pattern images are read at n <= 160 only");
  if (out->form == EBSD_FORM_AUTO) {
    if (out->precision != EBSD_PREC_FP32) out->form = EBSD_FORM_DFTGEMM;
    else if (size_supported(n) && !fft_supported(n) && out->max_shift >= 0) out->form = EBSD_FORM_DFT;
    else out->form = EBSD_FORM_FFT;
  }
  if (out->form == EBSD_FORM_FFT && out->precision != EBSD_PREC_FP32)
    return fail(EBSD_E_UNSUPPORTED, "the FFT form runs in FP32 only");
  if (out->form == EBSD_FORM_DFT) {
    if (out->precision != EBSD_PREC_FP32) return fail(EBSD_E_UNSUPPORTED, "the exact DFT form runs in FP32 only");
    if (out->max_shift < 0) return fail(EBSD_E_INVALID, "the exact DFT form needs a shift window (max_shift >= 0)");
    if (size_supported(n) && !window_peak_supported(n, out->max_shift))
      return fail(EBSD_E_UNSUPPORTED, "shift window too large for the exact DFT form at this size");
  }
  if (out->form == EBSD_FORM_DFTGEMM) {
    if (out->precision == EBSD_PREC_FP32) return fail(EBSD_E_UNSUPPORTED, "the DFT-GEMM form runs in 16-bit halves");
    if (out->max_shift < 0) return fail(EBSD_E_INVALID, "the DFT-GEMM form needs a shift window (max_shift >= 0)");
    if (size_supported(n) && !gemm_supported(n, out->max_shift))
      return fail(EBSD_E_UNSUPPORTED, "shift window too large for the DFT-GEMM form at this size");
  }
  return EBSD_OK;
}

FilterParams filter_of(const ebsd_params& p, int n) {
  FilterParams f;
  f.window = p.window;
  f.sigma_hp = (float)p.sigma_hp;
  f.sigma_lp = (float)(p.sigma_lp_frac * n);
  f.rho_max = (float)(p.rho_max_frac * n);
  return f;
}

// Spectra of K contiguous images: one kernel up to 160, three passes through
// scratch at 256 (s256: spectra256_scratch_bytes(k) bytes, or taken from ws
// when null).
int do_spectra(int n, const float* imgs, int64_t k, const FilterParams& fp, float2* spec, double* energy,
               Arena& ws, hipStream_t st, void* s256 = nullptr) {
  if (n == 256) {
    if (!s256) {
      EBSD_ALLOC(buf, unsigned char, spectra256_scratch_bytes(k), ws);
      s256 = buf;
    }
    EBSD_TRY(launch_spectra256(imgs, k, fp, spec, energy, s256, st), "spectra256");
    return EBSD_OK;
  }
  EBSD_TRY(launch_spectra(n, imgs, (int64_t)n * n, k, fp, spec, energy, st), "spectra");
  return EBSD_OK;
}

// Integer peak of explicit pairs: the full-map FFT form where it exists,
// otherwise the exact shift-window evaluation (needs max_shift >= 0) with
// the phase tables tab (built here into ws when null).
int do_peak(int n, const ebsd_params& p, const float2* sp, const float2* sl, const int32_t* pi, const int32_t* li,
            int64_t k, float* h, int32_t* s, Arena& ws, hipStream_t st, const float2* tab = nullptr) {
  if (fft_supported(n)) {
    EBSD_TRY(launch_xcf_peak(n, sp, sl, pi, li, k, p.max_shift, h, s, nullptr, st), "xcf_peak");
    return EBSD_OK;
  }
  if (!window_peak_supported(n, p.max_shift))
    return fail(EBSD_E_UNSUPPORTED, "this size needs a shift window (max_shift >= 0) for the integer peak");
  if (!tab) {
    EBSD_ALLOC(t, float2, window_table_size(n, p.max_shift), ws);
    EBSD_TRY(launch_window_tables(n, p.max_shift, t, st), "window tables");
    tab = t;
  }
  EBSD_TRY(launch_window_peak(n, sp, sl, pi, li, k, p.max_shift, tab, h, s, st), "window peak");
  return EBSD_OK;
}

// Calls that never read the caller's pattern images reject a BF16 input flag.
int f32_images_only(const ebsd_params& p) {
  if (p.input != EBSD_INPUT_F32) return fail(EBSD_E_UNSUPPORTED, "this call reads FP32 images only");
  return EBSD_OK;
}

// Spectra and log-polar images of the caller's patterns (FP32, or BF16 as
// p.input says).
int pattern_spectra(int n, const ebsd_params& p, const float* imgs, int64_t k, const FilterParams& fp, float2* spec,
                    double* energy, Arena& ws, hipStream_t st, void* s256 = nullptr) {
  if (p.input == EBSD_INPUT_BF16) {
    EBSD_TRY(launch_spectra(n, reinterpret_cast<const __bf16*>(imgs), (int64_t)n * n, k, fp, spec, energy, st),
             "spectra(bf16)");
    return EBSD_OK;
  }
  return do_spectra(n, imgs, k, fp, spec, energy, ws, st, s256);
}

hipError_t pattern_logpolar(int n, const ebsd_params& p, const float* imgs, int64_t k, float* out, hipStream_t st) {
  if (p.input == EBSD_INPUT_BF16)
    return launch_logpolar(n, reinterpret_cast<const __bf16*>(imgs), k, p.n_rho, p.n_eta, out, st);
  return launch_logpolar(n, imgs, k, p.n_rho, p.n_eta, out, st);
}

int64_t spec_complex(int n) {
  const int b = band_of(n);
  return b < 0 ? -1 : (int64_t)(b + 1) * (2 * b + 1);
}

int check_size(int n) {
  if (!size_supported(n)) return fail(EBSD_E_UNSUPPORTED, "pattern size not supported (64, 96, 128, 160, 256)");
  return EBSD_OK;
}

int check_master(const ebsd_master* mp) {
  if (!mp || !mp->data) return fail(EBSD_E_INVALID, "null master");
  if (mp->H < 4 || mp->W < 4) return fail(EBSD_E_INVALID, "master must be at least 4 x 4");
  return EBSD_OK;
}

int check_geometry(const ebsd_geometry* geo) {
  if (!geo) return fail(EBSD_E_INVALID, "null geometry");
  if (!(geo->pcz > 0.0) || !std::isfinite(geo->pcx) || !std::isfinite(geo->pcy))
    return fail(EBSD_E_INVALID, "pattern centre must be finite with pcz > 0");
  return EBSD_OK;
}

// Event pairs around the search kernel while timing is enabled.
bool g_timing = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;

// Constant operands of the search form: the split DFT-GEMM fragments, or the
// phase tables of the exact FP32 DFT form (built here); none for the FFT form.
struct SearchConsts {
  unsigned short* frag = nullptr;
  float2* wtab = nullptr;
};

int search_consts(int n, const ebsd_params& p, Arena& ws, hipStream_t st, SearchConsts* c) {
  if (p.form == EBSD_FORM_DFTGEMM) {
    EBSD_ALLOC(f, unsigned short, gemm_frag_bytes(n, p.max_shift) / 2, ws);
    c->frag = f;
  } else if (p.form == EBSD_FORM_DFT) {
    EBSD_ALLOC(t, float2, window_table_size(n, p.max_shift), ws);
    EBSD_TRY(launch_window_tables(n, p.max_shift, t, st), "window tables");
    c->wtab = t;
  }
  return EBSD_OK;
}

// The search in the requested form: FFT (FP32), split-precision DFT-GEMM, or
// the exact FP32 DFT over the shift window.
hipError_t launch_search(int n, const ebsd_params& prm, const float2* sp, int64_t p, const float2* sl, int64_t l,
                         const SearchConsts& c, float* out, hipStream_t st) {
  if (prm.form == EBSD_FORM_DFTGEMM)
    return launch_xcf_gemm(n, prm.precision - 1, sp, p, sl, l, prm.max_shift, c.frag, out, st);
  if (prm.form == EBSD_FORM_DFT) return launch_window_scores(n, sp, p, sl, l, prm.max_shift, c.wtab, out, st);
  return launch_xcf_scores(n, sp, p, sl, l, prm.max_shift, out, st);
}

hipError_t timed_scores(int n, const ebsd_params& prm, const float2* sp, int64_t p, const float2* sl, int64_t l,
                        const SearchConsts& frag, float* out, hipStream_t st) {
  if (!g_timing) return launch_search(n, prm, sp, p, sl, l, frag, out, st);
  hipEvent_t a, b;
  hipError_t e;
  if ((e = hipEventCreate(&a)) != hipSuccess) return e;
  if ((e = hipEventCreate(&b)) != hipSuccess) return e;
  if ((e = hipEventRecord(a, st)) != hipSuccess) return e;
  if ((e = launch_search(n, prm, sp, p, sl, l, frag, out, st)) != hipSuccess) return e;
  if ((e = hipEventRecord(b, st)) != hipSuccess) return e;
  g_events.emplace_back(a, b);
  return hipSuccess;
}

// Steps A2-A8 of ebsd_index_patterns against library spectra already in
// spec_l (L templates, orientations lib_q): pattern spectra, search, library
// argmax, the winner's integer and sub-pixel peaks.
int index_against(int n, const ebsd_params& p, const float* pats, int64_t P, const float2* spec_l,
                  const double* lib_q, int64_t L, int32_t* best_idx, double* best_q, float* peak_h, float* shift,
                  float* scores, Arena& ws, hipStream_t st) {
  int rc;
  const int64_t sc = spec_complex(n);
  const FilterParams fp = filter_of(p, n);
  EBSD_ALLOC(spec_p, float2, sc * P, ws);
  float* sc_out = scores;
  if (!sc_out) {
    EBSD_ALLOC(tmp_scores, float, P * L, ws);
    sc_out = tmp_scores;
  }
  EBSD_ALLOC(h_int, float, P, ws);
  EBSD_ALLOC(s_int, int32_t, 2 * P, ws);
  EBSD_ALLOC(h_tmp, float, P, ws);
  EBSD_ALLOC(roots, float2, subpixel_table_size(n, p.upsample), ws);
  if (int e = pattern_spectra(n, p, pats, P, fp, spec_p, nullptr, ws, st)) return e;
  SearchConsts consts;
  if ((rc = search_consts(n, p, ws, st, &consts))) return rc;
  EBSD_TRY(timed_scores(n, p, spec_p, P, spec_l, L, consts, sc_out, st), "xcf_scores");
  EBSD_TRY(launch_library_argmax(sc_out, P, L, best_idx, h_int, st), "library_argmax");
  if (int e = do_peak(n, p, spec_p, spec_l, nullptr, best_idx, P, h_tmp, s_int, ws, st)) return e;
  EBSD_TRY(launch_subpixel_tables(n, p.upsample, roots, st), "subpixel tables");
  EBSD_TRY(launch_subpixel(n, spec_p, spec_l, nullptr, best_idx, P, s_int, p.upsample, roots, peak_h, shift, st),
           "subpixel");
  if (best_q) EBSD_TRY(launch_gather_q(lib_q, best_idx, P, best_q, st), "gather_q");
  return EBSD_OK;
}

// Arguments of a library search at size n common to the direct call and the plan.
int check_search(int n, const ebsd_params& p) {
  if (p.form == EBSD_FORM_FFT && !fft_supported(n))
    return fail(EBSD_E_UNSUPPORTED, "the FFT search is not built at this size; use the DFT-GEMM form");
  if (!fft_supported(n) && !window_peak_supported(n, p.max_shift))
    return fail(EBSD_E_UNSUPPORTED, "at this size the peak needs a shift window (max_shift >= 0)");
  return EBSD_OK;
}

// Largest | |q| - 1 | over L quaternions, as the bits of a non-negative float
// (NaN counts as infinite), into *worst (zeroed by the caller).
__global__ void k_unit_check(const double* __restrict__ q, int64_t L, unsigned* __restrict__ worst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= L) return;
  const double a = q[4 * i], b = q[4 * i + 1], c = q[4 * i + 2], d = q[4 * i + 3];
  float dev = (float)fabs(sqrt(a * a + b * b + c * c + d * d) - 1.0);
  if (!(dev <= 3.0e38f)) dev = INFINITY;
  atomicMax(worst, __float_as_uint(dev));
}

}  // namespace api
}  // namespace ebsd

using namespace ebsd::api;

extern "C" {

int ebsd_timing_enable(int enable) {
  g_timing = enable != 0;
  return EBSD_OK;
}

int ebsd_timing_read(double* total_ms, int64_t* launches) {
  double tot = 0.0;
  int64_t cnt = 0;
  int rc = EBSD_OK;
  for (auto& ev : g_events) {
    float ms = 0.0f;
    hipError_t e = hipEventElapsedTime(&ms, ev.first, ev.second);
    if (e != hipSuccess) rc = fail_hip(e, "timing_read");
    tot += ms;
    ++cnt;
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  g_events.clear();
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  return rc;
}

void ebsd_params_default(ebsd_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(ebsd_params);
  p->window = 1;
  p->sigma_hp = 2.0;
  p->sigma_lp_frac = 0.125;
  p->rho_max_frac = 0.375;
  p->max_shift = -1;
  p->upsample = 100;
  p->n_iter = 2;
  p->n_rho = 0;
  p->n_eta = 0;
  p->precision = EBSD_PREC_FP32;
  p->form = EBSD_FORM_AUTO;
}

int ebsd_version(void) { return 100; }

const char* ebsd_last_error(void) { return g_last_error.c_str(); }

int64_t ebsd_spectrum_floats(int32_t n) {
  const int64_t c = spec_complex(n);
  return c < 0 ? -1 : 2 * c;
}

int ebsd_project_templates(const ebsd_master* mp, const double* q, int64_t K, int32_t n,
                           const ebsd_geometry* geo, float* out, void* stream) {
  g_last_error.clear();
  int rc;
  if ((rc = check_master(mp)) || (rc = check_geometry(geo))) return rc;
  if (n < 4 || n > 4096) return fail(EBSD_E_INVALID, "n must be in [4, 4096]");
  if (K < 0) return fail(EBSD_E_INVALID, "K must be >= 0");
  if (K == 0) return EBSD_OK;
  if (!q || !out) return fail(EBSD_E_INVALID, "null pointer");
  EBSD_TRY(launch_project(n, mp->data, mp->H, mp->W, q, K, geo->pc_per, geo->pcx, geo->pcy, geo->pcz, out,
                          (hipStream_t)stream),
           "project");
  return EBSD_OK;
}

int ebsd_pattern_spectra(const float* imgs, int64_t K, int32_t n, const ebsd_params* prm, float* spec,
                         double* energy, void* stream) {
  g_last_error.clear();
  int rc;
  ebsd_params p;
  if ((rc = check_size(n)) || (rc = resolve_params(prm, n, &p))) return rc;
  if (K < 0) return fail(EBSD_E_INVALID, "K must be >= 0");
  if (K == 0) return EBSD_OK;
  if (!imgs || !spec) return fail(EBSD_E_INVALID, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  Scratch ws(st);
  return pattern_spectra(n, p, imgs, K, filter_of(p, n), (float2*)spec, energy, ws, st);
}

int ebsd_xcf_peak(const float* spec_p, const float* spec_l, const int32_t* pi, const int32_t* li, int64_t K,
                  int32_t n, const ebsd_params* prm, float* h_int, int32_t* s_int, float* map, void* stream) {
  g_last_error.clear();
  int rc;
  ebsd_params p;
  if ((rc = check_size(n)) || (rc = resolve_params(prm, n, &p)) || (rc = f32_images_only(p))) return rc;
  if (K < 0) return fail(EBSD_E_INVALID, "K must be >= 0");
  if (K == 0) return EBSD_OK;
  if (!spec_p || !spec_l || !h_int || !s_int) return fail(EBSD_E_INVALID, "null pointer");
  if (K > 0x7fffffffLL) return fail(EBSD_E_INVALID, "K too large");
  if (map) {
    if (!fft_supported(n)) return fail(EBSD_E_UNSUPPORTED, "the full correlation map is not built at this size");
    EBSD_TRY(launch_xcf_peak(n, (const float2*)spec_p, (const float2*)spec_l, pi, li, K, p.max_shift, h_int, s_int,
                             map, (hipStream_t)stream),
             "xcf_peak");
    return EBSD_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  Scratch ws(st);
  return do_peak(n, p, (const float2*)spec_p, (const float2*)spec_l, pi, li, K, h_int, s_int, ws, st);
}

int ebsd_xcf_scores(const float* spec_p, int64_t P, const float* spec_l, int64_t L, int32_t n,
                    const ebsd_params* prm, float* scores, void* stream) {
  g_last_error.clear();
  int rc;
  ebsd_params p;
  if ((rc = check_size(n)) || (rc = resolve_params(prm, n, &p)) || (rc = f32_images_only(p))) return rc;
  if (P < 0 || L < 0) return fail(EBSD_E_INVALID, "P and L must be >= 0");
  if (P == 0 || L == 0) return EBSD_OK;
  if (!spec_p || !spec_l || !scores) return fail(EBSD_E_INVALID, "null pointer");
  if (p.form == EBSD_FORM_FFT && !fft_supported(n))
    return fail(EBSD_E_UNSUPPORTED, "the FFT search is not built at this size; use the DFT-GEMM form");
  hipStream_t st = (hipStream_t)stream;
  Scratch ws(st);
  SearchConsts consts;
  if ((rc = search_consts(n, p, ws, st, &consts))) return rc;
  EBSD_TRY(timed_scores(n, p, (const float2*)spec_p, P, (const float2*)spec_l, L, consts, scores, st), "xcf_scores");
  return EBSD_OK;
}

int ebsd_xcf_scores_cand(const float* spec_p, int64_t P, const float* spec_l, int64_t L, const int32_t* cand,
                         int32_t K, int32_t n, const ebsd_params* prm, float* scores, void* stream) {
  g_last_error.clear();
  int rc;
  ebsd_params p;
  if ((rc = check_size(n)) || (rc = resolve_params(prm, n, &p)) || (rc = f32_images_only(p))) return rc;
  if (P < 0 || L < 0 || K < 0) return fail(EBSD_E_INVALID, "P, L and K must be >= 0");
  if (K > L) return fail(EBSD_E_INVALID, "K must not exceed L");
  if (P == 0 || K == 0) return EBSD_OK;
  if (!spec_p || !spec_l || !cand || !scores) return fail(EBSD_E_INVALID, "null pointer");
  if (n != 128 || p.form == EBSD_FORM_DFTGEMM || p.form == EBSD_FORM_DFT || p.precision != EBSD_PREC_FP32)
    return fail(EBSD_E_UNSUPPORTED, "candidate-list scores are built for the FP32 FFT search at n = 128");
  hipStream_t st = (hipStream_t)stream;
  EBSD_TRY(launch_xcf_scores_cand(n, (const float2*)spec_p, P, (const float2*)spec_l, L, cand, K, p.max_shift, scores,
                                  st),
           "xcf_scores_cand");
  return EBSD_OK;
}

int ebsd_xcf_subpixel(const float* spec_p, const float* spec_l, const int32_t* pi, const int32_t* li, int64_t K,
                      int32_t n, const int32_t* s_int, const ebsd_params* prm, float* h_sub, float* s_sub,
                      void* stream) {
  g_last_error.clear();
  int rc;
  ebsd_params p;
  if ((rc = check_size(n)) || (rc = resolve_params(prm, n, &p)) || (rc = f32_images_only(p))) return rc;
  if (K < 0) return fail(EBSD_E_INVALID, "K must be >= 0");
  if (K == 0) return EBSD_OK;
  if (!spec_p || !spec_l || !s_int || !h_sub || !s_sub) return fail(EBSD_E_INVALID, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  Scratch ws(st);
  EBSD_ALLOC(roots, float2, subpixel_table_size(n, p.upsample), ws);
  EBSD_TRY(launch_subpixel_tables(n, p.upsample, roots, st), "subpixel tables");
  EBSD_TRY(launch_subpixel(n, (const float2*)spec_p, (const float2*)spec_l, pi, li, K, s_int, p.upsample, roots,
                           h_sub, s_sub, st),
           "subpixel");
  return EBSD_OK;
}

int ebsd_measure_rotation(const float* pats, const float* tmpls, int64_t K, int32_t n, const ebsd_params* prm,
                          double* gamma, void* stream) {
  g_last_error.clear();
  int rc;
  ebsd_params p;
  if ((rc = check_size(n)) || (rc = resolve_params(prm, n, &p)) || (rc = f32_images_only(p))) return rc;
  if (K < 0) return fail(EBSD_E_INVALID, "K must be >= 0");
  if (K == 0) return EBSD_OK;
  if (!pats || !tmpls || !gamma) return fail(EBSD_E_INVALID, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  Scratch ws(st);
  const size_t lp = (size_t)p.n_rho * p.n_eta;
  EBSD_ALLOC(lp_e, float, lp * K, ws);
  EBSD_ALLOC(lp_t, float, lp * K, ws);
  EBSD_TRY(launch_logpolar(n, pats, K, p.n_rho, p.n_eta, lp_e, st), "logpolar");
  EBSD_TRY(launch_logpolar(n, tmpls, K, p.n_rho, p.n_eta, lp_t, st), "logpolar");
  EBSD_TRY(launch_eta_peak(lp_e, lp_t, K, p.n_rho, p.n_eta, p.upsample, gamma, st), "eta_peak");
  return EBSD_OK;
}

int ebsd_index_patterns(const ebsd_batch* pats, const ebsd_master* mp, const ebsd_geometry* geo,
                        const double* lib_q, int64_t L, const ebsd_params* prm, int32_t* best_idx, double* best_q,
                        float* peak_h, float* shift, float* scores, void* stream) {
  g_last_error.clear();
  int rc;
  if (!pats) return fail(EBSD_E_INVALID, "null batch");
  const int n = pats->n;
  ebsd_params p;
  if ((rc = check_size(n)) || (rc = resolve_params(prm, n, &p)) || (rc = check_master(mp)) ||
      (rc = check_geometry(geo)))
    return rc;
  const int64_t P = pats->P;
  if (P < 0) return fail(EBSD_E_INVALID, "P must be >= 0");
  if (L < 1) return fail(EBSD_E_INVALID, "library must hold at least one orientation");
  if (L > 0x7fffffffLL || P > 0x7fffffffLL) return fail(EBSD_E_INVALID, "P and L must fit in int32");
  if (!lib_q) return fail(EBSD_E_INVALID, "null library");
  if (P == 0) return EBSD_OK;
  if (!pats->data || !best_idx || !peak_h || !shift) return fail(EBSD_E_INVALID, "null pointer");
  if ((rc = check_search(n, p))) return rc;

  hipStream_t st = (hipStream_t)stream;
  Scratch ws(st);
  const int64_t sc = spec_complex(n);
  const int64_t npix = (int64_t)n * n;
  const FilterParams fp = filter_of(p, n);
  EBSD_ALLOC(tmpl, float, npix * L, ws);
  EBSD_ALLOC(spec_l, float2, sc * L, ws);
  EBSD_TRY(launch_project(n, mp->data, mp->H, mp->W, lib_q, L, nullptr, geo->pcx, geo->pcy, geo->pcz, tmpl, st),
           "project");
  if (int e = do_spectra(n, tmpl, L, fp, spec_l, nullptr, ws, st)) return e;
  return index_against(n, p, pats->data, P, spec_l, lib_q, L, best_idx, best_q, peak_h, shift, scores, ws, st);
}


// ---------------------------------------------------------------------------
// Library plans: the templates' band spectra computed once and reused.
struct ebsd_plan_s {
  int n;
  ebsd_params p;
  int64_t L;
  float2* spec_l;
  double* lib_q;
};

int ebsd_plan_create(const ebsd_master* mp, const ebsd_geometry* geo, const double* lib_q, int64_t L, int32_t n,
                     const ebsd_params* prm, ebsd_plan* out, void* stream) {
  g_last_error.clear();
  int rc;
  if (!out) return fail(EBSD_E_INVALID, "null output");
  *out = nullptr;
  ebsd_params p;
  if ((rc = check_size(n)) || (rc = resolve_params(prm, n, &p)) || (rc = check_master(mp)) ||
      (rc = check_geometry(geo)) || (rc = check_search(n, p)))
    return rc;
  if (L < 1 || L > 0x7fffffffLL) return fail(EBSD_E_INVALID, "L must be in [1, 2^31)");
  if (!lib_q) return fail(EBSD_E_INVALID, "null library");
  hipStream_t st = (hipStream_t)stream;
  // every library orientation must be a unit quaternion (checked on the
  // device, then read back: plan creation waits for the stream)
  {
    Scratch ws(st);
    EBSD_ALLOC(worst, unsigned, 1, ws);
    EBSD_TRY(hipMemsetAsync(worst, 0, sizeof(unsigned), st), "unit check");
    hipLaunchKernelGGL(k_unit_check, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, st, lib_q, L, worst);
    EBSD_TRY(hipGetLastError(), "unit check");
    unsigned bits = 0;
    EBSD_TRY(hipMemcpyAsync(&bits, worst, sizeof(unsigned), hipMemcpyDeviceToHost, st), "unit check");
    EBSD_TRY(hipStreamSynchronize(st), "unit check");
    float dev;
    memcpy(&dev, &bits, sizeof(float));
    if (!(dev <= 1e-6f)) return fail(EBSD_E_INVALID, "library orientations must be unit quaternions");
  }
  auto* pl = new (std::nothrow) ebsd_plan_s{n, p, L, nullptr, nullptr};
  if (!pl) return fail(EBSD_E_NOMEM, "plan allocation failed");
  const int64_t sc = spec_complex(n);
  if (hipMalloc(&pl->spec_l, sizeof(float2) * sc * L) != hipSuccess ||
      hipMalloc(&pl->lib_q, sizeof(double) * 4 * L) != hipSuccess) {
    ebsd_plan_destroy(pl);
    return fail(EBSD_E_NOMEM, "plan device allocation failed");
  }
  rc = [&]() -> int {
    Scratch ws(st);
    EBSD_TRY(hipMemcpyAsync(pl->lib_q, lib_q, sizeof(double) * 4 * L, hipMemcpyDeviceToDevice, st), "plan copy");
    EBSD_ALLOC(tmpl, float, (int64_t)n * n * L, ws);
    EBSD_TRY(launch_project(n, mp->data, mp->H, mp->W, lib_q, L, nullptr, geo->pcx, geo->pcy, geo->pcz, tmpl, st),
             "project");
    return do_spectra(n, tmpl, L, filter_of(p, n), pl->spec_l, nullptr, ws, st);
  }();
  if (rc) {
    (void)hipStreamSynchronize(st);
    ebsd_plan_destroy(pl);
    return rc;
  }
  *out = pl;
  return EBSD_OK;
}

int ebsd_index_patterns_plan(ebsd_plan plan, const ebsd_batch* pats, int32_t* best_idx, double* best_q,
                             float* peak_h, float* shift, float* scores, void* stream) {
  g_last_error.clear();
  if (!plan) return fail(EBSD_E_INVALID, "null plan");
  if (!pats) return fail(EBSD_E_INVALID, "null batch");
  if (pats->n != plan->n) return fail(EBSD_E_INVALID, "pattern size differs from the plan's");
  const int64_t P = pats->P;
  if (P < 0 || P > 0x7fffffffLL) return fail(EBSD_E_INVALID, "P must be in [0, 2^31)");
  if (P == 0) return EBSD_OK;
  if (!pats->data || !best_idx || !peak_h || !shift) return fail(EBSD_E_INVALID, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  Scratch ws(st);
  return index_against(plan->n, plan->p, pats->data, P, plan->spec_l, plan->lib_q, plan->L, best_idx, best_q,
                       peak_h, shift, scores, ws, st);
}

int ebsd_plan_destroy(ebsd_plan plan) {
  if (!plan) return EBSD_OK;
  if (plan->spec_l) (void)hipFree(plan->spec_l);
  if (plan->lib_q) (void)hipFree(plan->lib_q);
  delete plan;
  return EBSD_OK;
}

}  // extern "C"

// Scratch of the allocation-free refinement: one file-scope device array,
// which each GPU the library runs on holds until the process ends.  In host
// code its name is not a device address; the address of each device's copy
// comes from hipGetSymbolAddress on the first call on that device.
constexpr size_t kNoAllocBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

// Every device buffer of one refinement call, taken from one arena before
// anything is enqueued.
struct RefineBufs {
  float* tmpl;
  float2* spec_p;
  float2* spec_t;
  float* lp_e;
  float* lp_t;
  float* h_int;
  float* h_sub;
  int32_t* s_int;
  float* s_sub;
  double* gam;
  float2* roots;
  void* s256;     // spectra scratch at 256 (null below)
  float2* wtab;   // shift-window phase tables (null where the FFT form runs)
};

int alloc_refine(Arena& ws, int n, int64_t P, const ebsd_params& p, RefineBufs* b) {
  const int64_t sc = spec_complex(n);
  const int64_t npix = (int64_t)n * n;
  const int64_t lp = (int64_t)p.n_rho * p.n_eta;
  EBSD_ALLOC(tmpl, float, npix * P, ws);
  EBSD_ALLOC(spec_p, float2, sc * P, ws);
  EBSD_ALLOC(spec_t, float2, sc * P, ws);
  EBSD_ALLOC(lp_e, float, lp * P, ws);
  EBSD_ALLOC(lp_t, float, lp * P, ws);
  EBSD_ALLOC(h_int, float, P, ws);
  EBSD_ALLOC(h_sub, float, P, ws);
  EBSD_ALLOC(s_int, int32_t, 2 * P, ws);
  EBSD_ALLOC(s_sub, float, 2 * P, ws);
  EBSD_ALLOC(gam, double, P, ws);
  EBSD_ALLOC(roots, float2, subpixel_table_size(n, p.upsample), ws);
  *b = RefineBufs{tmpl, spec_p, spec_t, lp_e, lp_t, h_int, h_sub, s_int, s_sub, gam, roots, nullptr, nullptr};
  if (n == 256) {
    EBSD_ALLOC(s256, unsigned char, spectra256_scratch_bytes(P), ws);
    b->s256 = s256;
  }
  if (!fft_supported(n)) {
    EBSD_ALLOC(wtab, float2, window_table_size(n, p.max_shift), ws);
    b->wtab = wtab;
  }
  return EBSD_OK;
}

// Validates the arguments of a refinement call; P = 0 leaves *n = 0.
int check_refine(const ebsd_batch* pats, const ebsd_master* mp, const ebsd_geometry* geo, const double* q_init,
                 const ebsd_params* prm, double* q_out, float* peak_h, float* shift, ebsd_params* p, int* n_out) {
  int rc;
  *n_out = 0;
  if (!pats) return fail(EBSD_E_INVALID, "null batch");
  const int n = pats->n;
  if ((rc = check_size(n)) || (rc = resolve_params(prm, n, p)) || (rc = check_master(mp)) ||
      (rc = check_geometry(geo)))
    return rc;
  const int64_t P = pats->P;
  if (P < 0) return fail(EBSD_E_INVALID, "P must be >= 0");
  if (P > 0x7fffffffLL) return fail(EBSD_E_INVALID, "P must fit in int32");
  if (P == 0) return EBSD_OK;
  if (!pats->data || !q_init || !q_out || !peak_h || !shift) return fail(EBSD_E_INVALID, "null pointer");
  if (!fft_supported(n) && !window_peak_supported(n, p->max_shift))
    return fail(EBSD_E_UNSUPPORTED, "at this size the peak needs a shift window (max_shift >= 0)");
  *n_out = n;
  return EBSD_OK;
}

// The kernel sequence of the refinement on buffers b; match_shift (may be
// NULL) replaces the first iteration's projection and correlation by the
// search's shift less the beam-induced PC translation.
int refine_run(const ebsd_batch* pats, const ebsd_master* mp, const ebsd_geometry* geo, const double* q_init,
               const float* match_shift, const ebsd_params& p, const RefineBufs& b, double* q_out, float* peak_h,
               float* shift, hipStream_t st) {
  int rc;
  const int n = pats->n;
  const int64_t P = pats->P;
  const FilterParams fp = filter_of(p, n);
  FixedArena none(nullptr, 0);   // every buffer is in b: nothing more may be taken
  if (q_out != q_init) EBSD_TRY(hipMemcpyAsync(q_out, q_init, sizeof(double) * 4 * P, hipMemcpyDeviceToDevice, st), "copy q");
  EBSD_TRY(launch_subpixel_tables(n, p.upsample, b.roots, st), "subpixel tables");
  if (b.wtab) EBSD_TRY(launch_window_tables(n, p.max_shift, b.wtab, st), "window tables");
  if ((rc = pattern_spectra(n, p, pats->data, P, fp, b.spec_p, nullptr, none, st, b.s256))) return rc;
  EBSD_TRY(pattern_logpolar(n, p, pats->data, P, b.lp_e, st), "logpolar(patterns)");
  const double* pcp = geo->pc_per;
  auto measure_shift = [&](float* h_out, float* s_out) -> int {
    EBSD_TRY(launch_project(n, mp->data, mp->H, mp->W, q_out, P, pcp, geo->pcx, geo->pcy, geo->pcz, b.tmpl, st),
             "project");
    if (int e = do_spectra(n, b.tmpl, P, fp, b.spec_t, nullptr, none, st, b.s256)) return e;
    if (int e = do_peak(n, p, b.spec_p, b.spec_t, nullptr, nullptr, P, b.h_int, b.s_int, none, st, b.wtab)) return e;
    EBSD_TRY(launch_subpixel(n, b.spec_p, b.spec_t, nullptr, nullptr, P, b.s_int, p.upsample, b.roots, h_out, s_out,
                             st),
             "subpixel");
    return EBSD_OK;
  };
  const double pc0[2] = {geo->pcx, geo->pcy};
  for (int it = 0; it < p.n_iter; ++it) {
    if (it == 0 && match_shift) {
      EBSD_TRY(launch_update_xy(q_out, match_shift, P, pcp, geo->pcz, n, st, pc0), "update_xy(match)");
    } else {
      if ((rc = measure_shift(b.h_sub, b.s_sub))) return rc;
      EBSD_TRY(launch_update_xy(q_out, b.s_sub, P, pcp, geo->pcz, n, st), "update_xy");
    }
    EBSD_TRY(launch_project(n, mp->data, mp->H, mp->W, q_out, P, pcp, geo->pcx, geo->pcy, geo->pcz, b.tmpl, st),
             "project");
    EBSD_TRY(launch_logpolar(n, b.tmpl, P, p.n_rho, p.n_eta, b.lp_t, st), "logpolar(templates)");
    EBSD_TRY(launch_eta_peak(b.lp_e, b.lp_t, P, p.n_rho, p.n_eta, p.upsample, b.gam, st), "eta_peak");
    EBSD_TRY(launch_update_z(q_out, b.gam, P, st), "update_z");
  }
  if ((rc = measure_shift(peak_h, shift))) return rc;
  return EBSD_OK;
}

// The refinement of both pool-backed entry points.
int refine_impl(const ebsd_batch* pats, const ebsd_master* mp, const ebsd_geometry* geo, const double* q_init,
                const float* match_shift, const ebsd_params* prm, double* q_out, float* peak_h, float* shift,
                void* stream) {
  int rc, n;
  ebsd_params p;
  if ((rc = check_refine(pats, mp, geo, q_init, prm, q_out, peak_h, shift, &p, &n))) return rc;
  if (n == 0) return EBSD_OK;
  hipStream_t st = (hipStream_t)stream;
  Scratch ws(st);
  RefineBufs b;
  if ((rc = alloc_refine(ws, n, pats->P, p, &b))) return rc;
  return refine_run(pats, mp, geo, q_init, match_shift, p, b, q_out, peak_h, shift, st);
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(void** out) {
  int dev = -1;
  EBSD_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(EBSD_E_UNSUPPORTED, "device ordinal beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    EBSD_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(EBSD_E_DEVICE, "hipGetSymbolAddress(scratch) returned null");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return EBSD_OK;
}

}  // namespace

extern "C" {

int ebsd_refine_orientations(const ebsd_batch* pats, const ebsd_master* mp, const ebsd_geometry* geo,
                             const double* q_init, const ebsd_params* prm, double* q_out, float* peak_h,
                             float* shift, void* stream) {
  g_last_error.clear();
  return refine_impl(pats, mp, geo, q_init, nullptr, prm, q_out, peak_h, shift, stream);
}

int ebsd_refine_orientations_noalloc(const ebsd_batch* pats, const ebsd_master* mp, const ebsd_geometry* geo,
                                     const double* q_init, const ebsd_params* prm, double* q_out, float* peak_h,
                                     float* shift, void* stream) {
  g_last_error.clear();
  int rc, n;
  ebsd_params p;
  if ((rc = check_refine(pats, mp, geo, q_init, prm, q_out, peak_h, shift, &p, &n))) return rc;
  if (n == 0) return EBSD_OK;
  // size the call first: nothing is enqueued if it does not fit
  FixedArena sizing(nullptr, kNoAllocBytes);
  RefineBufs b;
  if (alloc_refine(sizing, n, pats->P, p, &b) != EBSD_OK) {
    FixedArena need(nullptr, ~size_t(0));
    (void)alloc_refine(need, n, pats->P, p, &b);
    char msg[200];
    std::snprintf(msg, sizeof(msg),
                  "batch needs %zu bytes of scratch, above the static %zu (%lld patterns of %d x %d)", need.used(),
                  kNoAllocBytes, (long long)pats->P, n, n);
    return fail(EBSD_E_INVALID, msg);
  }
  void* base = nullptr;
  if ((rc = scratch_of_current_device(&base))) return rc;
  FixedArena arena(base, kNoAllocBytes);
  if ((rc = alloc_refine(arena, n, pats->P, p, &b))) return rc;
  return refine_run(pats, mp, geo, q_init, nullptr, p, b, q_out, peak_h, shift, (hipStream_t)stream);
}

int ebsd_refine_from_match(const ebsd_batch* pats, const ebsd_master* mp, const ebsd_geometry* geo,
                           const double* q_init, const float* match_shift, const ebsd_params* prm, double* q_out,
                           float* peak_h, float* shift, void* stream) {
  g_last_error.clear();
  if (pats && pats->P > 0 && !match_shift) return fail(EBSD_E_INVALID, "null match_shift");
  return refine_impl(pats, mp, geo, q_init, match_shift, prm, q_out, peak_h, shift, stream);
}

int ebsd_capture_range(const ebsd_master* mp, const double* q_ref, int64_t R, int32_t n,
                       const ebsd_geometry* geo_ref, const ebsd_geometry* geo_test, const double* theta_deg,
                       int32_t T, const ebsd_params* prm, float* h, double* width, void* stream) {
  g_last_error.clear();
  int rc;
  ebsd_params p;
  if ((rc = check_size(n)) || (rc = resolve_params(prm, n, &p)) || (rc = check_master(mp)) ||
      (rc = check_geometry(geo_ref)) || (rc = check_geometry(geo_test)) || (rc = f32_images_only(p)))
    return rc;
  if (R < 0) return fail(EBSD_E_INVALID, "R must be >= 0");
  if (T < 1) return fail(EBSD_E_INVALID, "T must be >= 1");
  if (R > 0x7fffffffLL / (3 * (int64_t)T)) return fail(EBSD_E_INVALID, "R x 3 x T must fit in int32");
  if (R == 0) return EBSD_OK;
  if (!q_ref || !theta_deg || !h || !width) return fail(EBSD_E_INVALID, "null pointer");
  if (!fft_supported(n) && !window_peak_supported(n, p.max_shift))
    return fail(EBSD_E_UNSUPPORTED, "at this size the peak needs a shift window (max_shift >= 0)");

  hipStream_t st = (hipStream_t)stream;
  Scratch ws(st);
  const int64_t K = R * 3 * (int64_t)T;
  const int64_t sc = spec_complex(n);
  const int64_t npix = (int64_t)n * n;
  const FilterParams fp = filter_of(p, n);
  EBSD_ALLOC(qt, double, 4 * K, ws);
  EBSD_ALLOC(ref_of, int32_t, K, ws);
  EBSD_ALLOC(img_r, float, npix * R, ws);
  EBSD_ALLOC(img_t, float, npix * K, ws);
  EBSD_ALLOC(spec_r, float2, sc * R, ws);
  EBSD_ALLOC(spec_t, float2, sc * K, ws);
  EBSD_ALLOC(s_int, int32_t, 2 * K, ws);
  EBSD_TRY(launch_capture_orient(q_ref, R, theta_deg, T, qt, ref_of, st), "capture orientations");
  EBSD_TRY(launch_project(n, mp->data, mp->H, mp->W, q_ref, R, nullptr, geo_ref->pcx, geo_ref->pcy, geo_ref->pcz,
                          img_r, st),
           "project(references)");
  EBSD_TRY(launch_project(n, mp->data, mp->H, mp->W, qt, K, nullptr, geo_test->pcx, geo_test->pcy, geo_test->pcz,
                          img_t, st),
           "project(rotated)");
  if ((rc = do_spectra(n, img_r, R, fp, spec_r, nullptr, ws, st))) return rc;
  if ((rc = do_spectra(n, img_t, K, fp, spec_t, nullptr, ws, st))) return rc;
  if ((rc = do_peak(n, p, spec_r, spec_t, ref_of, nullptr, K, h, s_int, ws, st))) return rc;
  EBSD_TRY(launch_fwhm(h, R * 3, theta_deg, T, width, st), "fwhm");
  return EBSD_OK;
}

int ebsd_so3_library(double spacing_deg, double* q_out, int64_t cap, int64_t* count, void* stream) {
  g_last_error.clear();
  if (!count) return fail(EBSD_E_INVALID, "null count");
  if (!(spacing_deg >= 0.5 && spacing_deg <= 90.0)) return fail(EBSD_E_INVALID, "spacing must be in [0.5, 90] deg");
  if (cap < 0) return fail(EBSD_E_INVALID, "cap must be >= 0");
  if (cap > 0 && !q_out) return fail(EBSD_E_INVALID, "null q_out");
  // ring and circle counts (round half to even, as the grid is defined)
  const double d = spacing_deg * (M_PI / 180.0);
  const int m = std::max(1, (int)std::nearbyint(M_PI / d));
  const int n_psi = std::max(1, (int)std::nearbyint(2.0 * M_PI / d));
  std::vector<int64_t> off((size_t)m + 2, 0);
  for (int i = 0; i <= m; ++i) {
    const double theta = M_PI * i / m;
    off[(size_t)i + 1] = off[(size_t)i] + std::max<int64_t>(1, (int64_t)std::nearbyint((2.0 * m) * std::sin(theta)));
  }
  const int64_t n_all = off[(size_t)m + 1] * n_psi;
  hipStream_t st = (hipStream_t)stream;
  {
    Scratch ws(st);
    EBSD_ALLOC(ring_off, int64_t, m + 2, ws);
    EBSD_ALLOC(q_all, double, 4 * n_all, ws);
    EBSD_ALLOC(keep, unsigned char, n_all, ws);
    EBSD_ALLOC(dcount, int64_t, 1, ws);
    EBSD_TRY(hipMemcpyAsync(ring_off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice, st),
             "ring table");
    EBSD_TRY(launch_so3_library(ring_off, m, n_psi, n_all, q_all, keep, q_out, cap, dcount, st), "so3 library");
    EBSD_TRY(hipMemcpyAsync(count, dcount, sizeof(int64_t), hipMemcpyDeviceToHost, st), "count");
    EBSD_TRY(hipStreamSynchronize(st), "synchronise");
  }
  return EBSD_OK;
}

int ebsd_nn_disorientation(const double* q, int64_t L, double* nn_deg, int32_t* nn_idx, void* stream) {
  g_last_error.clear();
  if (L < 0 || L == 1) return fail(EBSD_E_INVALID, "L must be 0 or at least 2");
  if (L > 0x7fffffffLL) return fail(EBSD_E_INVALID, "L must fit in int32");
  if (L == 0) return EBSD_OK;
  if (!q || !nn_deg || !nn_idx) return fail(EBSD_E_INVALID, "null pointer");
  EBSD_TRY(launch_nn_disorientation(q, L, nn_deg, nn_idx, (hipStream_t)stream), "nn disorientation");
  return EBSD_OK;
}

int ebsd_pc_map(const ebsd_pc_model* model, int64_t P, double* pc_out, void* stream) {
  g_last_error.clear();
  if (!model) return fail(EBSD_E_INVALID, "null model");
  if (P < 0) return fail(EBSD_E_INVALID, "P must be >= 0");
  if (model->width < 1) return fail(EBSD_E_INVALID, "width must be >= 1");
  for (int c = 0; c < 3; ++c)
    if (!std::isfinite(model->pc0[c]) || !std::isfinite(model->d_col[c]) || !std::isfinite(model->d_row[c]))
      return fail(EBSD_E_INVALID, "model coefficients must be finite");
  if (!std::isfinite(model->col0) || !std::isfinite(model->row0)) return fail(EBSD_E_INVALID, "col0, row0 must be finite");
  if (P > 0x7fffffffLL) return fail(EBSD_E_INVALID, "P must fit in int32");
  if (P == 0) return EBSD_OK;
  if (!pc_out) return fail(EBSD_E_INVALID, "null pc_out");
  PcModel m;
  for (int c = 0; c < 3; ++c) {
    m.pc0[c] = model->pc0[c];
    m.d_col[c] = model->d_col[c];
    m.d_row[c] = model->d_row[c];
  }
  m.col0 = model->col0;
  m.row0 = model->row0;
  m.width = model->width;
  EBSD_TRY(launch_pc_map(m, P, pc_out, (hipStream_t)stream), "pc_map");
  return EBSD_OK;
}

}  // extern "C"

// C-ABI of the learned proposal: the network object (parameters, Adam
// state, workspace), its training on patterns generated on the device by
// the projection, and the pruned search (correlation on the network's top-k
// library orientations, with the exhaustive search as fallback whenever the
// best peak height stays below a threshold).
#include "api_util.hpp"
#include "cnn_internal.hpp"
#include "ebsd_common.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

using namespace ebsd;
using namespace ebsd::api;

#define CN_TRY(expr, where)                            \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return fail_hip(e_, where);  \
  } while (0)

namespace {

// patterns per network pass of inference: 2,048 fill the chip in the small
// late layers and the fc product (50,000 patterns: 111 ms against 127 ms in
// passes of 256; 4,096: 110 ms for twice the workspace); the logits do not
// depend on it (no K split in the forward products)
#ifndef EBSD_CNN_CHUNK
#define EBSD_CNN_CHUNK 2048
#endif
constexpr int64_t kChunk = EBSD_CNN_CHUNK;

inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

// pairs (p, cand[p][j]) of the pruned search
__global__ void k_pairs(const int32_t* __restrict__ cand, int64_t p, int k, int32_t* __restrict__ pi) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= p * k) return;
  pi[i] = (int32_t)(i / k);
}

// best candidate per pattern by integer peak (ties: smaller library index);
// flag[p] = 1 when the best stays below tau
__global__ void k_pick_candidate(const float* __restrict__ h, const int32_t* __restrict__ cand, int64_t p, int k,
                                 float tau, int32_t* __restrict__ best, float* __restrict__ h_best,
                                 int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= p) return;
  float bv = -INFINITY;
  int bi = 0x7fffffff;
  for (int j = 0; j < k; ++j) {
    const float v = h[i * k + j];
    const int l = cand[i * k + j];
    if (v > bv || (v == bv && l < bi)) {
      bv = v;
      bi = l;
    }
  }
  if (bi == 0x7fffffff) bi = cand[i * k];
  best[i] = bi;
  h_best[i] = bv;
  flag[i] = !(bv >= tau);
}

// list of flagged patterns in increasing order and its length (one block)
__global__ __launch_bounds__(1024) void k_compact(const int32_t* __restrict__ flag, int64_t p,
                                                  int32_t* __restrict__ list, int32_t* __restrict__ count) {
  __shared__ int32_t part[1024];
  __shared__ int32_t base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int64_t s = 0; s < p; s += 1024) {
    const int64_t i = s + threadIdx.x;
    const int32_t f = i < p ? flag[i] : 0;
    part[threadIdx.x] = f;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan
      const int32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
      __syncthreads();
      part[threadIdx.x] += v;
      __syncthreads();
    }
    if (f) list[base + part[threadIdx.x] - 1] = (int32_t)i;
    __syncthreads();
    if (threadIdx.x == 1023) base += part[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = base;
}

__global__ void k_gather_rows(const float2* __restrict__ src, const int32_t* __restrict__ list, int64_t f,
                              int64_t row, float2* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= f * row) return;
  const int64_t r = i / row, c = i - r * row;
  dst[i] = src[(int64_t)list[r] * row + c];
}

__global__ void k_scatter_best(const int32_t* __restrict__ list, int64_t f, const int32_t* __restrict__ b,
                               const float* __restrict__ h, int32_t* __restrict__ best, float* __restrict__ h_best) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= f) return;
  best[list[i]] = b[i];
  h_best[list[i]] = h[i];
}

}  // namespace

struct ebsd_cnn_s {
  int device = 0;
  int32_t prec = EBSD_PREC_BF16X2;  // precision of the inference and backward products
  cnn::Layout lay{};
  float* params = nullptr;
  float* grad = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  int64_t step = 0;
  int64_t ws_batch = 0;
  void* ws = nullptr;
  cnn::Acts act{};
  float* part = nullptr;
  size_t part_floats = 0;
  double* loss_row = nullptr;
};

namespace {

constexpr size_t kPartFloats = size_t(8) << 20;

// Workspace for batches of up to bsz patterns (grown on demand; the caller's
// stream is synchronised before a reallocation).
int ensure_ws(ebsd_cnn_s* c, int64_t bsz, hipStream_t st) {
  if (bsz <= c->ws_batch) return EBSD_OK;
  CN_TRY(hipStreamSynchronize(st), "cnn workspace sync");
  if (c->ws) (void)hipFree(c->ws);
  c->ws = nullptr;
  c->ws_batch = 0;
  // offsets in floats, each region rounded up to 64 floats
  size_t off = 0;
  auto take = [&off](size_t floats) {
    const size_t o = off;
    off += (floats + 63) & ~size_t(63);
    return o;
  };
  size_t o_arg[4], o_g[4], o_p[4], o_dp[4];
  int w = cnn::kInSize;
  for (int i = 0; i < 4; ++i) {
    const size_t full = (size_t)bsz * cnn::kChannels[i] * w * w;
    const size_t half = full / 4;
    o_arg[i] = take((half + 3) / 4);  // one byte per pooled output
    o_g[i] = i ? take(full) : 0;  // the first layer's gradient map is never formed
    o_p[i] = take(half);
    o_dp[i] = take(half);
    w /= 2;
  }
  const size_t o_logits = take((size_t)bsz * c->lay.classes);
  const size_t o_dz = take((size_t)bsz * c->lay.classes);
  const size_t o_part = take(kPartFloats);
  const size_t o_wt = take((size_t)cnn::kTapWeights);
  // BF16 hi and lo halves (one float slot each) of the tap-major and the fc weights
  const size_t o_wts = take((size_t)cnn::kTapWeights);
  const size_t o_fcs = take((size_t)c->lay.classes * cnn::kFeatures);
  const size_t loss_bytes = sizeof(double) * (size_t)bsz;
  if (hipMalloc(&c->ws, off * sizeof(float) + loss_bytes) != hipSuccess)
    return fail(EBSD_E_NOMEM, "cnn workspace allocation failed");
  float* base = (float*)c->ws;
  for (int i = 0; i < 4; ++i) {
    c->act.arg[i] = reinterpret_cast<uint8_t*>(base + o_arg[i]);
    c->act.g[i] = i ? base + o_g[i] : nullptr;
    c->act.p[i] = base + o_p[i];
    c->act.dp[i] = base + o_dp[i];
  }
  c->act.logits = base + o_logits;
  c->act.dz = base + o_dz;
  c->part = base + o_part;
  c->act.wt = base + o_wt;
  c->act.wts = reinterpret_cast<unsigned short*>(base + o_wts);
  c->act.fcs = reinterpret_cast<unsigned short*>(base + o_fcs);
  c->part_floats = kPartFloats;
  c->loss_row = (double*)(base + off);
  c->ws_batch = bsz;
  return EBSD_OK;
}

int check_cnn(ebsd_cnn_s* c) {
  if (!c) return fail(EBSD_E_INVALID, "null network");
  int dev = -1;
  CN_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev != c->device) return fail(EBSD_E_INVALID, "the network was created on another device");
  return EBSD_OK;
}

int forward_chunks(ebsd_cnn_s* c, const float* x, int64_t bsz, float* logits, hipStream_t st) {
  int rc;
  if ((rc = ensure_ws(c, std::min(bsz, kChunk), st))) return rc;
  const int L = c->lay.classes;
  const bool split = c->prec == EBSD_PREC_BF16X2;
  CN_TRY(cnn::prepare(c->params, c->lay, c->act, split, st), "cnn weights");
  for (int64_t s = 0; s < bsz; s += kChunk) {
    const int64_t b = std::min(kChunk, bsz - s);
    cnn::Acts a = c->act;
    a.logits = logits + s * L;
    CN_TRY(cnn::forward(c->params, c->lay, x + s * cnn::kInSize * cnn::kInSize, b, a, st, false, split),
           "cnn forward");
  }
  return EBSD_OK;
}

int grads(ebsd_cnn_s* c, const float* x, const int32_t* labels, int64_t bsz, float* loss, hipStream_t st) {
  int rc;
  if ((rc = ensure_ws(c, bsz, st))) return rc;
  CN_TRY(cnn::prepare(c->params, c->lay, c->act, false, st), "cnn weights");
  CN_TRY(cnn::forward(c->params, c->lay, x, bsz, c->act, st, true, c->prec == EBSD_PREC_BF16X2), "cnn forward");
  CN_TRY(cnn::backward(c->params, c->lay, x, labels, bsz, c->act, c->grad, c->part, c->part_floats, c->loss_row,
                       loss, st, c->prec == EBSD_PREC_BF16X2),
         "cnn backward");
  return EBSD_OK;
}

}  // namespace

extern "C" {

int64_t ebsd_cnn_param_count(int32_t n_classes) {
  if (n_classes < 1) return -1;
  return cnn::layout_of(n_classes).total;
}

int ebsd_cnn_create(int32_t n_classes, uint64_t seed, ebsd_cnn* out, void* stream) {
  g_last_error.clear();
  if (!out) return fail(EBSD_E_INVALID, "null output");
  *out = nullptr;
  if (n_classes < 1 || n_classes > 40000) return fail(EBSD_E_INVALID, "n_classes must be in [1, 40000]");
  auto* c = new ebsd_cnn_s();
  c->lay = cnn::layout_of(n_classes);
  hipStream_t st = (hipStream_t)stream;
  const size_t bytes = sizeof(float) * (size_t)c->lay.total;
  hipError_t e;
  if ((e = hipGetDevice(&c->device)) || (e = hipMalloc(&c->params, bytes)) || (e = hipMalloc(&c->grad, bytes)) ||
      (e = hipMalloc(&c->m, bytes)) || (e = hipMalloc(&c->v, bytes))) {
    ebsd_cnn_destroy(c);
    return fail(EBSD_E_NOMEM, "network allocation failed");
  }
  if ((e = cnn::init_params(c->params, c->lay, seed, st)) || (e = hipMemsetAsync(c->m, 0, bytes, st)) ||
      (e = hipMemsetAsync(c->v, 0, bytes, st))) {
    ebsd_cnn_destroy(c);
    return fail_hip(e, "network init");
  }
  *out = c;
  return EBSD_OK;
}

int ebsd_cnn_destroy(ebsd_cnn c) {
  if (!c) return EBSD_OK;
  (void)hipDeviceSynchronize();
  if (c->params) (void)hipFree(c->params);
  if (c->grad) (void)hipFree(c->grad);
  if (c->m) (void)hipFree(c->m);
  if (c->v) (void)hipFree(c->v);
  if (c->ws) (void)hipFree(c->ws);
  delete c;
  return EBSD_OK;
}

int ebsd_cnn_get_params(ebsd_cnn c, float* out, void* stream) {
  g_last_error.clear();
  int rc;
  if ((rc = check_cnn(c))) return rc;
  if (!out) return fail(EBSD_E_INVALID, "null pointer");
  CN_TRY(hipMemcpyAsync(out, c->params, sizeof(float) * c->lay.total, hipMemcpyDeviceToDevice,
                        (hipStream_t)stream),
         "get params");
  return EBSD_OK;
}

int ebsd_cnn_set_params(ebsd_cnn c, const float* in, void* stream) {
  g_last_error.clear();
  int rc;
  if ((rc = check_cnn(c))) return rc;
  if (!in) return fail(EBSD_E_INVALID, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  const size_t bytes = sizeof(float) * c->lay.total;
  CN_TRY(hipMemcpyAsync(c->params, in, bytes, hipMemcpyDeviceToDevice, st), "set params");
  CN_TRY(hipMemsetAsync(c->m, 0, bytes, st), "reset optimiser");
  CN_TRY(hipMemsetAsync(c->v, 0, bytes, st), "reset optimiser");
  c->step = 0;
  return EBSD_OK;
}

int ebsd_cnn_input(const float* pats, int64_t P, int32_t n, float* x, void* stream) {
  g_last_error.clear();
  if (P < 0) return fail(EBSD_E_INVALID, "P must be >= 0");
  if (n < cnn::kInSize || n % cnn::kInSize || n > 1024)
    return fail(EBSD_E_UNSUPPORTED, "pattern side must be a multiple of 64 (at most 1024)");
  if (P == 0) return EBSD_OK;
  if (!pats || !x) return fail(EBSD_E_INVALID, "null pointer");
  if (P > 0x7fffffffLL) return fail(EBSD_E_INVALID, "P must fit in int32");
  CN_TRY(cnn::noise_bin(pats, n, P, 0, 0, 0.0f, 1.0f, 0, x, (hipStream_t)stream), "cnn input");
  return EBSD_OK;
}

int ebsd_cnn_forward(ebsd_cnn c, const float* x, int64_t B, float* logits, void* stream) {
  g_last_error.clear();
  int rc;
  if ((rc = check_cnn(c))) return rc;
  if (B < 0) return fail(EBSD_E_INVALID, "B must be >= 0");
  if (B == 0) return EBSD_OK;
  if (!x || !logits) return fail(EBSD_E_INVALID, "null pointer");
  return forward_chunks(c, x, B, logits, (hipStream_t)stream);
}

int ebsd_cnn_set_precision(ebsd_cnn c, int32_t precision) {
  g_last_error.clear();
  if (!c) return fail(EBSD_E_INVALID, "null network");
  if (precision == EBSD_PREC_FP16X2 || precision == EBSD_PREC_BF16)
    return fail(EBSD_E_UNSUPPORTED, "the network's products run in FP32 or BF16X2");
  if (precision != EBSD_PREC_FP32 && precision != EBSD_PREC_BF16X2) return fail(EBSD_E_INVALID, "unknown precision");
  c->prec = precision;
  return EBSD_OK;
}

int ebsd_cnn_gradients(ebsd_cnn c, const float* x, const int32_t* labels, int64_t B, float* grad, float* loss,
                       void* stream) {
  g_last_error.clear();
  int rc;
  if ((rc = check_cnn(c))) return rc;
  if (B < 1 || B > 4096) return fail(EBSD_E_INVALID, "B must be in [1, 4096]");
  if (!x || !labels || !grad || !loss) return fail(EBSD_E_INVALID, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  if ((rc = grads(c, x, labels, B, loss, st))) return rc;
  CN_TRY(hipMemcpyAsync(grad, c->grad, sizeof(float) * c->lay.total, hipMemcpyDeviceToDevice, st), "gradients");
  return EBSD_OK;
}

int ebsd_cnn_train_step(ebsd_cnn c, const float* x, const int32_t* labels, int64_t B, float lr, float* loss,
                        void* stream) {
  g_last_error.clear();
  int rc;
  if ((rc = check_cnn(c))) return rc;
  if (B < 1 || B > 4096) return fail(EBSD_E_INVALID, "B must be in [1, 4096]");
  if (!(lr > 0.0f)) return fail(EBSD_E_INVALID, "lr must be > 0");
  if (!x || !labels || !loss) return fail(EBSD_E_INVALID, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  if ((rc = grads(c, x, labels, B, loss, st))) return rc;
  c->step += 1;
  CN_TRY(cnn::adam(c->params, c->grad, c->m, c->v, c->lay.total, c->step, lr, st), "adam");
  return EBSD_OK;
}

int ebsd_cnn_apply_gradient(ebsd_cnn c, const float* grad, float lr, void* stream) {
  g_last_error.clear();
  int rc;
  if ((rc = check_cnn(c))) return rc;
  if (!(lr > 0.0f)) return fail(EBSD_E_INVALID, "lr must be > 0");
  if (!grad) return fail(EBSD_E_INVALID, "null pointer");
  c->step += 1;
  CN_TRY(cnn::adam(c->params, grad, c->m, c->v, c->lay.total, c->step, lr, (hipStream_t)stream), "adam");
  return EBSD_OK;
}

int ebsd_cnn_make_batch(const ebsd_master* mp, const ebsd_geometry* geo, const double* lib_q, int64_t L, int32_t n,
                        int64_t B, int64_t first, uint64_t seed, double max_offset_px, double counts, double snr,
                        float* x, int32_t* labels, double* q_true, void* stream) {
  g_last_error.clear();
  int rc;
  if ((rc = check_master(mp)) || (rc = check_geometry(geo))) return rc;
  if (n < cnn::kInSize || n % cnn::kInSize || n > 1024)
    return fail(EBSD_E_UNSUPPORTED, "pattern side must be a multiple of 64 (at most 1024)");
  if (B < 0 || first < 0 || L < 0 || L > 0x7fffffffLL) return fail(EBSD_E_INVALID, "bad sizes");
  if (!(counts > 0.0) || !(snr > 0.0) || !(max_offset_px >= 0.0))
    return fail(EBSD_E_INVALID, "counts and snr must be > 0, max_offset_px >= 0");
  if (B == 0) return EBSD_OK;
  if (!x) return fail(EBSD_E_INVALID, "null pointer");
  if (labels && (!lib_q || L < 1)) return fail(EBSD_E_INVALID, "labels need a library");
  hipStream_t st = (hipStream_t)stream;
  double* q = nullptr;
  double* pc = nullptr;
  float* img = nullptr;
  hipError_t e;
  if ((e = hipMallocAsync(&q, sizeof(double) * 4 * B, st)) || (e = hipMallocAsync(&pc, sizeof(double) * 3 * B, st)) ||
      (e = hipMallocAsync(&img, sizeof(float) * B * n * n, st)))
    return fail(EBSD_E_NOMEM, "batch scratch allocation failed");
  rc = EBSD_OK;
  if ((e = cnn::sample_setup(first, B, seed, geo->pcx, geo->pcy, geo->pcz, max_offset_px / n, q, pc, st)) ||
      (e = launch_project(n, mp->data, mp->H, mp->W, q, B, pc, geo->pcx, geo->pcy, geo->pcz, img, st)) ||
      (e = cnn::noise_bin(img, n, B, first, seed, (float)counts, (float)snr, 1, x, st)) ||
      (labels && (e = cnn::nearest_library(q, B, lib_q, (int)L, labels, st))) ||
      (q_true && (e = hipMemcpyAsync(q_true, q, sizeof(double) * 4 * B, hipMemcpyDeviceToDevice, st))))
    rc = fail_hip(e, "make batch");
  (void)hipFreeAsync(q, st);
  (void)hipFreeAsync(pc, st);
  (void)hipFreeAsync(img, st);
  return rc;
}

int ebsd_cnn_topk(const float* logits, int64_t rows, int32_t L, int32_t k, int32_t* idx, void* stream) {
  g_last_error.clear();
  if (rows < 0 || L < 1 || k < 1 || k > L) return fail(EBSD_E_INVALID, "need rows >= 0 and 1 <= k <= L");
  if (rows == 0) return EBSD_OK;
  if (!logits || !idx) return fail(EBSD_E_INVALID, "null pointer");
  if ((size_t)L * 4 > 160 * 1024) return fail(EBSD_E_UNSUPPORTED, "L too large for one block's LDS");
  CN_TRY(cnn::topk(logits, rows, L, k, idx, (hipStream_t)stream), "topk");
  return EBSD_OK;
}

int ebsd_index_proposed(const ebsd_batch* pats, const ebsd_master* mp, const ebsd_geometry* geo,
                        const double* lib_q, int64_t L, ebsd_cnn c, int32_t top_k, float fallback_tau,
                        const ebsd_params* prm, int32_t* best_idx, double* best_q, float* peak_h, float* shift,
                        int32_t* fallback, void* stream) {
  g_last_error.clear();
  int rc;
  if (!pats) return fail(EBSD_E_INVALID, "null batch");
  const int n = pats->n;
  ebsd_params p;
  if (n != 64 && n != 128) return fail(EBSD_E_UNSUPPORTED, "the proposal path serves 64 and 128 pixel patterns");
  if ((rc = resolve_params(prm, n, &p)) || (rc = check_master(mp)) || (rc = check_geometry(geo))) return rc;
  if ((rc = check_cnn(c))) return rc;
  if (p.form != EBSD_FORM_FFT) return fail(EBSD_E_UNSUPPORTED, "the proposal path runs the FP32 FFT form");
  if (L != c->lay.classes) return fail(EBSD_E_INVALID, "library size differs from the network's classes");
  if (top_k < 1 || top_k > L) return fail(EBSD_E_INVALID, "top_k must be in [1, L]");
  const int64_t P = pats->P;
  if (P < 0 || P > 0x7fffffffLL / top_k) return fail(EBSD_E_INVALID, "bad P");
  if (P == 0) return EBSD_OK;
  if (!pats->data || !lib_q || !best_idx || !peak_h || !shift) return fail(EBSD_E_INVALID, "null pointer");
  hipStream_t st = (hipStream_t)stream;
  const int64_t sc = spec_complex(n);
  const int64_t npix = (int64_t)n * n;
  const FilterParams fp = filter_of(p, n);
  const int64_t PK = P * top_k;
  // scratch (stream ordered)
  std::vector<void*> held;
  auto get = [&](size_t bytes) -> void* {
    void* ptr = nullptr;
    if (hipMallocAsync(&ptr, bytes ? bytes : 1, st) != hipSuccess) return nullptr;
    held.push_back(ptr);
    return ptr;
  };
  auto release = [&]() {
    for (void* ptr : held) (void)hipFreeAsync(ptr, st);
  };
  float* x = (float*)get(sizeof(float) * P * cnn::kInSize * cnn::kInSize);
  float* logits = (float*)get(sizeof(float) * std::min<int64_t>(P, kChunk) * L);
  int32_t* cand = (int32_t*)get(sizeof(int32_t) * PK);
  int32_t* pi = (int32_t*)get(sizeof(int32_t) * PK);
  float* hk = (float*)get(sizeof(float) * PK);
  int32_t* sk = (int32_t*)get(sizeof(int32_t) * 2 * PK);
  float* tmpl = (float*)get(sizeof(float) * npix * L);
  float2* spec_l = (float2*)get(sizeof(float2) * sc * L);
  float2* spec_p = (float2*)get(sizeof(float2) * sc * P);
  float* h_best = (float*)get(sizeof(float) * P);
  int32_t* flag = (int32_t*)get(sizeof(int32_t) * P);
  int32_t* list = (int32_t*)get(sizeof(int32_t) * P);
  int32_t* count = (int32_t*)get(sizeof(int32_t));
  int32_t* s_int = (int32_t*)get(sizeof(int32_t) * 2 * P);
  float* h_tmp = (float*)get(sizeof(float) * P);
  float2* roots = (float2*)get(sizeof(float2) * subpixel_table_size(n, p.upsample));
  for (void* ptr : held)
    if (!ptr) {
      release();
      return fail(EBSD_E_NOMEM, "proposal scratch allocation failed");
    }
  auto run = [&]() -> int {
    int r;
    // network: top-k library orientations per pattern
    const bool bf16 = p.input == EBSD_INPUT_BF16;
    const __bf16* pats_bf16 = reinterpret_cast<const __bf16*>(pats->data);
    if (bf16) CN_TRY(cnn::noise_bin(pats_bf16, n, P, 0, 0, 0.0f, 1.0f, 0, x, st), "cnn input");
    else CN_TRY(cnn::noise_bin(pats->data, n, P, 0, 0, 0.0f, 1.0f, 0, x, st), "cnn input");
    for (int64_t s = 0; s < P; s += kChunk) {
      const int64_t b = std::min(kChunk, P - s);
      if ((r = forward_chunks(c, x + s * cnn::kInSize * cnn::kInSize, b, logits, st))) return r;
      CN_TRY(cnn::topk(logits, b, (int)L, top_k, cand + s * top_k, st), "topk");
    }
    // spectra of the library and the patterns
    CN_TRY(launch_project(n, mp->data, mp->H, mp->W, lib_q, L, nullptr, geo->pcx, geo->pcy, geo->pcz, tmpl, st),
           "project");
    CN_TRY(launch_spectra(n, tmpl, npix, L, fp, spec_l, nullptr, st), "spectra(templates)");
    if (bf16) CN_TRY(launch_spectra(n, pats_bf16, npix, P, fp, spec_p, nullptr, st), "spectra(patterns)");
    else CN_TRY(launch_spectra(n, pats->data, npix, P, fp, spec_p, nullptr, st), "spectra(patterns)");
    // correlation on the candidates only
    // (at 128 by the library search kernel over each pattern's candidate list,
    // the scores the exhaustive search gives the same pairs; elsewhere pair by pair)
    if (n == 128) {
      CN_TRY(launch_xcf_scores_cand(n, spec_p, P, spec_l, L, cand, top_k, p.max_shift, hk, st), "xcf(candidates)");
    } else {
      hipLaunchKernelGGL(k_pairs, dim3(nb(PK)), dim3(256), 0, st, cand, P, top_k, pi);
      CN_TRY(launch_xcf_peak(n, spec_p, spec_l, pi, cand, PK, p.max_shift, hk, sk, nullptr, st), "xcf(candidates)");
    }
    hipLaunchKernelGGL(k_pick_candidate, dim3(nb(P)), dim3(256), 0, st, hk, cand, P, top_k, fallback_tau, best_idx,
                       h_best, flag);
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, st, flag, P, list, count);
    CN_TRY(hipGetLastError(), "pick");
    // exhaustive search for the patterns below the threshold
    int32_t nf = 0;
    CN_TRY(hipMemcpyAsync(&nf, count, sizeof(int32_t), hipMemcpyDeviceToHost, st), "fallback count");
    CN_TRY(hipStreamSynchronize(st), "fallback count");
    if (nf > 0) {
      float2* spec_f = (float2*)get(sizeof(float2) * sc * nf);
      float* sc_f = (float*)get(sizeof(float) * (size_t)nf * L);
      int32_t* b_f = (int32_t*)get(sizeof(int32_t) * nf);
      float* h_f = (float*)get(sizeof(float) * nf);
      if (!spec_f || !sc_f || !b_f || !h_f) return fail(EBSD_E_NOMEM, "fallback scratch allocation failed");
      hipLaunchKernelGGL(k_gather_rows, dim3(nb((int64_t)nf * sc)), dim3(256), 0, st, spec_p, list, (int64_t)nf, sc,
                         spec_f);
      CN_TRY(launch_xcf_scores(n, spec_f, nf, spec_l, L, p.max_shift, sc_f, st), "xcf(fallback)");
      CN_TRY(launch_library_argmax(sc_f, nf, L, b_f, h_f, st), "argmax(fallback)");
      hipLaunchKernelGGL(k_scatter_best, dim3(nb(nf)), dim3(256), 0, st, list, (int64_t)nf, b_f, h_f, best_idx,
                         h_best);
      CN_TRY(hipGetLastError(), "fallback scatter");
    }
    // the winner's peaks
    CN_TRY(launch_xcf_peak(n, spec_p, spec_l, nullptr, best_idx, P, p.max_shift, h_tmp, s_int, nullptr, st),
           "xcf_peak");
    CN_TRY(launch_subpixel_tables(n, p.upsample, roots, st), "subpixel tables");
    CN_TRY(launch_subpixel(n, spec_p, spec_l, nullptr, best_idx, P, s_int, p.upsample, roots, peak_h, shift, st),
           "subpixel");
    if (best_q) CN_TRY(launch_gather_q(lib_q, best_idx, P, best_q, st), "gather_q");
    if (fallback) CN_TRY(hipMemcpyAsync(fallback, flag, sizeof(int32_t) * P, hipMemcpyDeviceToDevice, st), "flags");
    return EBSD_OK;
  };
  rc = run();
  release();
  return rc;
}

}  // extern "C"

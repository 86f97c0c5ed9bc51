// Ragged batches: patterns of several binnings (64, 96, 128, 160) indexed
// against one orientation library and, optionally, refined by the 27-point
// stencil of small detector-frame rotations, all replayed as one captured
// HIP graph per call.
//
// Inside the graph, patterns are grouped by size (class-major rows, heaviest
// size first).  Each class projects the library at its own size, takes the
// spectra of its patterns (gathered from the caller's packed buffer), and
// runs the correlation search as a persistent kernel that drains a device
// work queue of (pattern, template chunk) items; the four searches are forked
// onto separate streams of the capture, so one class's tail overlaps the
// next class's work.  The template chunk and the persistent grid of every
// class are chosen by timing candidates on the device when the plan is built.
// The winner's integer and sub-pixel peaks, the stencil (27 candidates per
// pattern, projected at the pattern's own pattern centre, scored by the
// integer peak, best by score with ties to the smaller candidate number), the
// refinement (x / y shift steps and log-polar z steps at each pattern's own
// pattern centre, the first x / y step taken from the stencil's or the
// search's own shift) and the scatter back to pattern order follow on the
// capture stream.
#include "api_util.hpp"
#include "ebsd_common.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

using namespace ebsd;
using namespace ebsd::api;

#define RG_TRY(expr, where)                               \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return fail_hip(e_, where);     \
  } while (0)

namespace ebsd {
namespace {

constexpr int kNumClasses = 4;
constexpr int kClassN[kNumClasses] = {160, 128, 96, 64};
constexpr int kStencil = 27;
constexpr size_t kStencilBudget = size_t(4) << 30;  // bytes of candidate images + spectra per chunk
constexpr size_t kRefineBudget = size_t(4) << 30;   // bytes of refinement buffers per chunk

// Pattern images k = 0 .. cc - 1 at element offsets img_off[k] of the packed
// buffer, copied contiguous (the log-polar resampling reads whole images).
// One block per image.
__global__ void k_gather_imgs(const float* __restrict__ data, const int64_t* __restrict__ img_off, int64_t cc,
                              int npix, float* __restrict__ out) {
  const int64_t k = blockIdx.x;
  if (k >= cc) return;
  const float* src = data + img_off[k];
  float* dst = out + k * (int64_t)npix;
  for (int i = threadIdx.x; i < npix; i += 256) dst[i] = src[i];
}

__global__ void k_fill_i32(int* __restrict__ p, int n, int v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// Synthetic band spectra for the tile timing (values only shape the timing).
__global__ void k_fill_spec(float2* __restrict__ s, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t h = (uint32_t)(i * 2654435761u) ^ (uint32_t)(i >> 32);
  s[i] = make_float2((float)(h & 0xffff) * 1.5e-5f - 0.5f, (float)(h >> 16) * 1.5e-5f - 0.5f);
}

__global__ void k_rows_pc(const double* __restrict__ pc_per, const int32_t* __restrict__ row_pat, int64_t p,
                          double pcx, double pcy, double pcz, double* __restrict__ pc_row) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= p) return;
  if (pc_per) {
    const int64_t i = row_pat[r];
    pc_row[3 * r] = pc_per[3 * i];
    pc_row[3 * r + 1] = pc_per[3 * i + 1];
    pc_row[3 * r + 2] = pc_per[3 * i + 2];
  } else {
    pc_row[3 * r] = pcx;
    pc_row[3 * r + 1] = pcy;
    pc_row[3 * r + 2] = pcz;
  }
}

// Candidate k = 27 i + j of pattern i0 + i (class-local index), row row0 + i0 + i:
// q_row (x) conj(q_x(a)) (x) conj(q_y(b)) (x) conj(q_z(c)), i.e. R Q^T with
// Q = Rz(c) Ry(b) Rx(a), (a, b, c) = step * (j / 9 - 1, (j / 3) % 3 - 1, j % 3 - 1).
__global__ void k_stencil_prep(const double* __restrict__ q_row, const double* __restrict__ pc_row, int64_t row0,
                               int64_t i0, int64_t cc, double step, double* __restrict__ cand_q,
                               double* __restrict__ cand_pc, int32_t* __restrict__ cand_pat) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= cc * kStencil) return;
  const int64_t i = i0 + k / kStencil;
  const int j = (int)(k % kStencil);
  const int64_t r = row0 + i;
  const double a = step * (double)(j / 9 - 1), b = step * (double)((j / 3) % 3 - 1), c = step * (double)(j % 3 - 1);
  const double cx[4] = {cos(0.5 * a), -sin(0.5 * a), 0.0, 0.0};
  const double cy[4] = {cos(0.5 * b), 0.0, -sin(0.5 * b), 0.0};
  const double cz[4] = {cos(0.5 * c), 0.0, 0.0, -sin(0.5 * c)};
  double t1[4], t2[4], o[4];
  qmul(q_row + 4 * r, cx, t1);
  qmul(t1, cy, t2);
  qmul(t2, cz, o);
  qstore(cand_q + 4 * k, o);
  cand_pc[3 * k] = pc_row[3 * r];
  cand_pc[3 * k + 1] = pc_row[3 * r + 1];
  cand_pc[3 * k + 2] = pc_row[3 * r + 2];
  cand_pat[k] = (int32_t)i;
}

// Best of the 27 integer-peak scores per pattern (largest, ties to the
// smaller candidate number), committed to the pattern's row.
__global__ void k_stencil_pick(const float* __restrict__ h27, const int32_t* __restrict__ s27,
                               const double* __restrict__ cand_q, int64_t row0, int64_t i0, int64_t cc,
                               int32_t* __restrict__ pick_k, int32_t* __restrict__ pick_pat,
                               int32_t* __restrict__ s_best, double* __restrict__ q_row,
                               int32_t* __restrict__ sidx_row) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= cc) return;
  float best = -INFINITY;
  int bj = 0;
  for (int j = 0; j < kStencil; ++j) {
    const float h = h27[i * kStencil + j];
    if (h > best) {
      best = h;
      bj = j;
    }
  }
  const int64_t k = i * kStencil + bj;
  const int64_t r = row0 + i0 + i;
  pick_k[i] = (int32_t)k;
  pick_pat[i] = (int32_t)(i0 + i);
  s_best[2 * i] = s27[2 * k];
  s_best[2 * i + 1] = s27[2 * k + 1];
#pragma unroll
  for (int c = 0; c < 4; ++c) q_row[4 * r + c] = cand_q[4 * k + c];
  sidx_row[r] = bj;
}

__global__ void k_scatter(const int32_t* __restrict__ row_pat, int64_t p, const int32_t* __restrict__ best_row,
                          const double* __restrict__ q_row, const float* __restrict__ h_row,
                          const float* __restrict__ s_row, const int32_t* __restrict__ sidx_row,
                          int32_t* __restrict__ best_idx, double* __restrict__ q_out, float* __restrict__ peak_h,
                          float* __restrict__ shift, int32_t* __restrict__ stencil_idx) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= p) return;
  const int64_t i = row_pat[r];
  if (best_idx) best_idx[i] = best_row[r];
#pragma unroll
  for (int c = 0; c < 4; ++c) q_out[4 * i + c] = q_row[4 * r + c];
  peak_h[i] = h_row[r];
  shift[2 * i] = s_row[2 * r];
  shift[2 * i + 1] = s_row[2 * r + 1];
  if (stencil_idx) stencil_idx[i] = sidx_row ? sidx_row[r] : -1;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// Bump allocator over one device allocation.
struct Arena {
  size_t off = 0;
  char* base = nullptr;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? (T*)(base + off) : nullptr;
    off += (count ? count : 1) * sizeof(T);
    return p;
  }
};

struct ClassPlan {
  int n = 0;
  int64_t count = 0, row0 = 0;
  int lchunk = 16, grid = 0;
  int64_t chunk = 0;   // stencil patterns per chunk
  int64_t rchunk = 0;  // refinement patterns per chunk
  ebsd_params prm{};   // the parameters resolved at this size (log-polar grid)
  float2* lib_spec = nullptr;
  float2* pat_spec = nullptr;
  float2* sub_tab = nullptr;
  int64_t* img_off = nullptr;
  int* queue = nullptr;
  hipStream_t branch = nullptr;
  hipEvent_t done = nullptr;
};

}  // namespace
}  // namespace ebsd

struct ebsd_ragged_plan_s {
  int device = 0;
  int64_t P = 0, L = 0;
  ebsd_params prm{};
  double step = 0.0;
  int flags = 0;
  int cus = 0;
  std::vector<int32_t> row_pat_h;
  std::vector<std::vector<int64_t>> off_h;
  ClassPlan cls[kNumClasses];
  void* mem = nullptr;
  // rows (class-major)
  int32_t* row_pat = nullptr;
  float* scores = nullptr;
  int32_t* best_row = nullptr;
  float* hint_row = nullptr;
  int32_t* sint_row = nullptr;
  float* h_row = nullptr;
  float* s_row = nullptr;
  double* q_row = nullptr;
  double* pc_row = nullptr;
  int32_t* sidx_row = nullptr;
  // images (library projection, then stencil candidates) and stencil buffers
  float* img = nullptr;
  double* cand_q = nullptr;
  double* cand_pc = nullptr;
  int32_t* cand_pat = nullptr;
  float2* cand_spec = nullptr;
  float* h27 = nullptr;
  int32_t* s27 = nullptr;
  int32_t* pick_k = nullptr;
  int32_t* pick_pat = nullptr;
  int32_t* s_best = nullptr;
  // refinement buffers (one chunk)
  float* r_img = nullptr;
  float* r_tmpl = nullptr;
  float2* r_spec = nullptr;
  float* r_lpe = nullptr;
  float* r_lpt = nullptr;
  float* r_hint = nullptr;
  int32_t* r_sint = nullptr;
  float* r_hsub = nullptr;
  float* r_ssub = nullptr;
  double* r_gam = nullptr;
  int* queues = nullptr;
  hipStream_t cap = nullptr;
  hipEvent_t fork = nullptr;
  hipEvent_t ran = nullptr;    // recorded on the caller's stream after each run
  bool ran_recorded = false;
  hipGraphExec_t exec = nullptr;
  std::vector<uintptr_t> key;
};

namespace {

int plan_layout(ebsd_ragged_plan_s* pl, Arena& a) {
  const int64_t P = pl->P, L = pl->L;
  size_t img_floats = 0, cand = 0, cand_spec = 0;
  size_t r_pix = 0, r_spec = 0, r_lp = 0, r_rows = 0;
  for (auto& c : pl->cls) {
    if (!c.count) continue;
    const int64_t sc = spec_complex(c.n);
    if (pl->flags & EBSD_RAGGED_REFINE) {
      const size_t lp = (size_t)c.prm.n_rho * c.prm.n_eta;
      const size_t per = (size_t)c.n * c.n * 8 + (size_t)sc * 8 + lp * 8 + 40;
      c.rchunk = std::max<int64_t>(1, std::min<int64_t>(c.count, (int64_t)(kRefineBudget / per)));
      r_pix = std::max(r_pix, (size_t)(c.rchunk * c.n * c.n));
      r_spec = std::max(r_spec, (size_t)(c.rchunk * sc));
      r_lp = std::max(r_lp, (size_t)c.rchunk * lp);
      r_rows = std::max(r_rows, (size_t)c.rchunk);
    }
    c.lib_spec = a.take<float2>((size_t)(L * sc));
    c.pat_spec = a.take<float2>((size_t)(c.count * sc));
    c.sub_tab = a.take<float2>((size_t)subpixel_table_size(c.n, pl->prm.upsample));
    c.img_off = a.take<int64_t>((size_t)c.count);
    img_floats = std::max(img_floats, (size_t)(L * c.n * c.n));
    if (pl->flags & EBSD_RAGGED_STENCIL) {
      const size_t per = (size_t)kStencil * ((size_t)c.n * c.n * 4 + (size_t)sc * 8);
      c.chunk = std::max<int64_t>(1, std::min<int64_t>(c.count, (int64_t)(kStencilBudget / per)));
      img_floats = std::max(img_floats, (size_t)(kStencil * c.chunk * c.n * c.n));
      cand = std::max(cand, (size_t)(kStencil * c.chunk));
      cand_spec = std::max(cand_spec, (size_t)(kStencil * c.chunk * sc));
    }
  }
  pl->row_pat = a.take<int32_t>((size_t)P);
  pl->scores = a.take<float>((size_t)(P * L));
  pl->best_row = a.take<int32_t>((size_t)P);
  pl->hint_row = a.take<float>((size_t)P);
  pl->sint_row = a.take<int32_t>((size_t)(2 * P));
  pl->h_row = a.take<float>((size_t)P);
  pl->s_row = a.take<float>((size_t)(2 * P));
  pl->q_row = a.take<double>((size_t)(4 * P));
  pl->pc_row = a.take<double>((size_t)(3 * P));
  pl->sidx_row = a.take<int32_t>((size_t)P);
  pl->img = a.take<float>(img_floats);
  pl->cand_q = a.take<double>(4 * cand);
  pl->cand_pc = a.take<double>(3 * cand);
  pl->cand_pat = a.take<int32_t>(cand);
  pl->cand_spec = a.take<float2>(cand_spec);
  pl->h27 = a.take<float>(cand);
  pl->s27 = a.take<int32_t>(2 * cand);
  const size_t pc = cand / kStencil + 1;
  pl->pick_k = a.take<int32_t>(pc);
  pl->pick_pat = a.take<int32_t>(pc);
  pl->s_best = a.take<int32_t>(2 * pc);
  pl->r_img = a.take<float>(r_pix);
  pl->r_tmpl = a.take<float>(r_pix);
  pl->r_spec = a.take<float2>(r_spec);
  pl->r_lpe = a.take<float>(r_lp);
  pl->r_lpt = a.take<float>(r_lp);
  pl->r_hint = a.take<float>(r_rows);
  pl->r_sint = a.take<int32_t>(2 * r_rows);
  pl->r_hsub = a.take<float>(r_rows);
  pl->r_ssub = a.take<float>(2 * r_rows);
  pl->r_gam = a.take<double>(r_rows);
  pl->queues = a.take<int>(kNumClasses);
  for (int i = 0; i < kNumClasses; ++i) pl->cls[i].queue = pl->queues ? pl->queues + i : nullptr;
  return EBSD_OK;
}

// Tiles chosen by timing, kept for the life of the process: keyed by the
// device's architecture and compute-unit count, the size, the shift window
// and the FP32 FFT form (the only form of the ragged searches).
using TuneKey = std::tuple<std::string, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune_cache;

TuneKey tune_key(const ebsd_ragged_plan_s* pl, const ClassPlan& c) {
  hipDeviceProp_t prop;
  std::string arch = "?";
  if (hipGetDeviceProperties(&prop, pl->device) == hipSuccess) arch = prop.gcnArchName;
  return TuneKey(arch, pl->cus, c.n, pl->prm.max_shift);
}

// Times the persistent search of one class for candidate template chunks and
// grids on synthetic spectra of the class's size; keeps the fastest (once per
// process for each key).
int autotune_class(ebsd_ragged_plan_s* pl, ClassPlan& c) {
  int occ = 0;
  RG_TRY(xcf_persistent_occupancy(c.n, pl->prm.max_shift, &occ), "occupancy");
  occ = std::max(1, std::min(occ, 4));
  c.lchunk = 16;
  c.grid = occ * pl->cus;
  if (pl->flags & EBSD_RAGGED_NO_AUTOTUNE) return EBSD_OK;
  const TuneKey key = tune_key(pl, c);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      c.lchunk = it->second.first;
      c.grid = it->second.second;
      return EBSD_OK;
    }
  }
  const int64_t ps = std::min<int64_t>(c.count, 1024), ls = std::min<int64_t>(pl->L, 512);
  const int64_t sc = spec_complex(c.n);
  float2 *sp = nullptr, *sl = nullptr;
  float* out = nullptr;
  int* q = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipStream_t st = pl->cap;
  int rc = EBSD_OK;
  auto cleanup = [&]() {
    if (sp) (void)hipFree(sp);
    if (sl) (void)hipFree(sl);
    if (out) (void)hipFree(out);
    if (q) (void)hipFree(q);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  do {
    hipError_t e;
    if ((e = hipMalloc(&sp, sizeof(float2) * ps * sc)) || (e = hipMalloc(&sl, sizeof(float2) * ls * sc)) ||
        (e = hipMalloc(&out, sizeof(float) * ps * ls)) || (e = hipMalloc(&q, sizeof(int))) ||
        (e = hipEventCreate(&e0)) || (e = hipEventCreate(&e1))) {
      rc = fail_hip(e, "autotune setup");
      break;
    }
    hipLaunchKernelGGL(k_fill_spec, dim3(blocks_for(ps * sc)), dim3(256), 0, st, sp, ps * sc);
    hipLaunchKernelGGL(k_fill_spec, dim3(blocks_for(ls * sc)), dim3(256), 0, st, sl, ls * sc);
    float best_ms = INFINITY;
    const int chunks[] = {8, 16, 32, 64};
    for (int lc : chunks) {
      for (int bpc = 1; bpc <= occ; ++bpc) {
        const int grid = bpc * pl->cus;
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && rc == EBSD_OK; ++rep) {
          hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, st, q, 1, 0);
          if ((e = hipEventRecord(e0, st)) ||
              (e = launch_xcf_scores_persistent(c.n, sp, ps, sl, ls, pl->prm.max_shift, out, lc, grid, q, st)) ||
              (e = hipEventRecord(e1, st)) || (e = hipEventSynchronize(e1)) ||
              (e = hipEventElapsedTime(&ms, e0, e1)))
            rc = fail_hip(e, "autotune run");
        }
        if (rc != EBSD_OK) break;
        if (ms < best_ms) {
          best_ms = ms;
          c.lchunk = lc;
          c.grid = grid;
        }
      }
      if (rc != EBSD_OK) break;
    }
  } while (0);
  cleanup();
  if (rc == EBSD_OK) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache[key] = std::make_pair(c.lchunk, c.grid);
  }
  return rc;
}

// The whole ragged pipeline on stream st (the capture stream, or the
// caller's stream in eager mode).
int enqueue(ebsd_ragged_plan_s* pl, const float* data, const ebsd_master* mp, const ebsd_geometry* geo,
            const double* lib_q, int32_t* best_idx, double* q_out, float* peak_h, float* shift,
            int32_t* stencil_idx, hipStream_t st) {
  const ebsd_params& p = pl->prm;
  const int64_t P = pl->P, L = pl->L;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, st, pl->queues, kNumClasses, 0);
  hipLaunchKernelGGL(k_rows_pc, dim3(blocks_for(P)), dim3(256), 0, st, geo->pc_per, pl->row_pat, P, geo->pcx,
                     geo->pcy, geo->pcz, pl->pc_row);
  RG_TRY(hipGetLastError(), "ragged setup");
  for (auto& c : pl->cls) {
    if (!c.count) continue;
    const FilterParams fp = filter_of(p, c.n);
    RG_TRY(launch_project(c.n, mp->data, mp->H, mp->W, lib_q, L, nullptr, geo->pcx, geo->pcy, geo->pcz, pl->img,
                          st),
           "ragged project(library)");
    RG_TRY(launch_spectra(c.n, pl->img, (int64_t)c.n * c.n, L, fp, c.lib_spec, nullptr, st),
           "ragged spectra(library)");
    RG_TRY(launch_spectra_gather(c.n, data, c.img_off, c.count, fp, c.pat_spec, nullptr, st),
           "ragged spectra(patterns)");
    RG_TRY(launch_subpixel_tables(c.n, p.upsample, c.sub_tab, st), "ragged subpixel tables");
  }
  // the searches of the classes run concurrently
  RG_TRY(hipEventRecord(pl->fork, st), "fork");
  for (auto& c : pl->cls) {
    if (!c.count) continue;
    RG_TRY(hipStreamWaitEvent(c.branch, pl->fork, 0), "fork wait");
    RG_TRY(launch_xcf_scores_persistent(c.n, c.pat_spec, c.count, c.lib_spec, L, p.max_shift,
                                        pl->scores + c.row0 * L, c.lchunk, c.grid, c.queue, c.branch),
           "ragged search");
    RG_TRY(hipEventRecord(c.done, c.branch), "join record");
  }
  for (auto& c : pl->cls)
    if (c.count) RG_TRY(hipStreamWaitEvent(st, c.done, 0), "join wait");
  RG_TRY(launch_library_argmax(pl->scores, P, L, pl->best_row, pl->hint_row, st), "ragged argmax");
  RG_TRY(launch_gather_q(lib_q, pl->best_row, P, pl->q_row, st), "ragged gather q");
  for (auto& c : pl->cls) {
    if (!c.count) continue;
    RG_TRY(launch_xcf_peak(c.n, c.pat_spec, c.lib_spec, nullptr, pl->best_row + c.row0, c.count, p.max_shift,
                           pl->hint_row + c.row0, pl->sint_row + 2 * c.row0, nullptr, st),
           "ragged peak");
    RG_TRY(launch_subpixel(c.n, c.pat_spec, c.lib_spec, nullptr, pl->best_row + c.row0, c.count,
                           pl->sint_row + 2 * c.row0, p.upsample, c.sub_tab, pl->h_row + c.row0,
                           pl->s_row + 2 * c.row0, st),
           "ragged subpixel");
  }
  if (pl->flags & EBSD_RAGGED_STENCIL) {
    for (auto& c : pl->cls) {
      if (!c.count) continue;
      const FilterParams fp = filter_of(p, c.n);
      for (int64_t i0 = 0; i0 < c.count; i0 += c.chunk) {
        const int64_t cc = std::min<int64_t>(c.chunk, c.count - i0);
        const int64_t k = cc * kStencil;
        hipLaunchKernelGGL(k_stencil_prep, dim3(blocks_for(k)), dim3(256), 0, st, pl->q_row, pl->pc_row, c.row0,
                           i0, cc, pl->step, pl->cand_q, pl->cand_pc, pl->cand_pat);
        RG_TRY(hipGetLastError(), "stencil prep");
        RG_TRY(launch_project(c.n, mp->data, mp->H, mp->W, pl->cand_q, k, pl->cand_pc, geo->pcx, geo->pcy,
                              geo->pcz, pl->img, st),
               "stencil project");
        RG_TRY(launch_spectra(c.n, pl->img, (int64_t)c.n * c.n, k, fp, pl->cand_spec, nullptr, st),
               "stencil spectra");
        RG_TRY(launch_xcf_peak(c.n, c.pat_spec, pl->cand_spec, pl->cand_pat, nullptr, k, p.max_shift, pl->h27,
                               pl->s27, nullptr, st),
               "stencil peak");
        hipLaunchKernelGGL(k_stencil_pick, dim3(blocks_for(cc)), dim3(256), 0, st, pl->h27, pl->s27, pl->cand_q,
                           c.row0, i0, cc, pl->pick_k, pl->pick_pat, pl->s_best, pl->q_row, pl->sidx_row);
        RG_TRY(hipGetLastError(), "stencil pick");
        RG_TRY(launch_subpixel(c.n, c.pat_spec, pl->cand_spec, pl->pick_pat, pl->pick_k, cc, pl->s_best,
                               p.upsample, c.sub_tab, pl->h_row + c.row0 + i0, pl->s_row + 2 * (c.row0 + i0), st),
               "stencil subpixel");
      }
    }
  }
  const bool sten = (pl->flags & EBSD_RAGGED_STENCIL) != 0;
  if (pl->flags & EBSD_RAGGED_REFINE) {
    // x / y steps from the correlation shift, z steps from the log-polar eta
    // correlation, at each pattern's own pattern centre; the first x / y step
    // takes the shift already measured: the stencil winner's (projected at
    // the pattern's PC) or the library pick's (projected at the nominal PC,
    // so the PC-move translation is subtracted first)
    const double pc0[2] = {geo->pcx, geo->pcy};
    for (auto& c : pl->cls) {
      if (!c.count) continue;
      const ebsd_params& cp = c.prm;
      const FilterParams fp = filter_of(cp, c.n);
      const int64_t sc = spec_complex(c.n);
      const int npix = c.n * c.n;
      for (int64_t i0 = 0; i0 < c.count; i0 += c.rchunk) {
        const int64_t cc = std::min<int64_t>(c.rchunk, c.count - i0);
        const int64_t r0 = c.row0 + i0;
        double* q = pl->q_row + 4 * r0;
        const double* pcp = pl->pc_row + 3 * r0;
        const float2* sp = c.pat_spec + sc * i0;
        hipLaunchKernelGGL(k_gather_imgs, dim3((unsigned)cc), dim3(256), 0, st, data, c.img_off + i0, cc, npix,
                           pl->r_img);
        RG_TRY(hipGetLastError(), "refine gather");
        RG_TRY(launch_logpolar(c.n, pl->r_img, cc, cp.n_rho, cp.n_eta, pl->r_lpe, st), "refine logpolar(patterns)");
        auto measure = [&](float* hh, float* ss) -> int {
          RG_TRY(launch_project(c.n, mp->data, mp->H, mp->W, q, cc, pcp, geo->pcx, geo->pcy, geo->pcz, pl->r_tmpl,
                                st),
                 "refine project");
          RG_TRY(launch_spectra(c.n, pl->r_tmpl, npix, cc, fp, pl->r_spec, nullptr, st), "refine spectra");
          RG_TRY(launch_xcf_peak(c.n, sp, pl->r_spec, nullptr, nullptr, cc, cp.max_shift, pl->r_hint, pl->r_sint,
                                 nullptr, st),
                 "refine peak");
          RG_TRY(launch_subpixel(c.n, sp, pl->r_spec, nullptr, nullptr, cc, pl->r_sint, cp.upsample, c.sub_tab, hh,
                                 ss, st),
                 "refine subpixel");
          return EBSD_OK;
        };
        for (int it = 0; it < cp.n_iter; ++it) {
          if (it == 0) {
            RG_TRY(launch_update_xy(q, pl->s_row + 2 * r0, cc, pcp, geo->pcz, c.n, st, sten ? nullptr : pc0),
                   "refine update_xy(first)");
          } else {
            if (int rc = measure(pl->r_hsub, pl->r_ssub)) return rc;
            RG_TRY(launch_update_xy(q, pl->r_ssub, cc, pcp, geo->pcz, c.n, st), "refine update_xy");
          }
          RG_TRY(launch_project(c.n, mp->data, mp->H, mp->W, q, cc, pcp, geo->pcx, geo->pcy, geo->pcz, pl->r_tmpl,
                                st),
                 "refine project");
          RG_TRY(launch_logpolar(c.n, pl->r_tmpl, cc, cp.n_rho, cp.n_eta, pl->r_lpt, st), "refine logpolar");
          RG_TRY(launch_eta_peak(pl->r_lpe, pl->r_lpt, cc, cp.n_rho, cp.n_eta, cp.upsample, pl->r_gam, st),
                 "refine eta");
          RG_TRY(launch_update_z(q, pl->r_gam, cc, st), "refine update_z");
        }
        if (int rc = measure(pl->h_row + r0, pl->s_row + 2 * r0)) return rc;
      }
    }
  }
  hipLaunchKernelGGL(k_scatter, dim3(blocks_for(P)), dim3(256), 0, st, pl->row_pat, P, pl->best_row, pl->q_row,
                     pl->h_row, pl->s_row, sten ? pl->sidx_row : nullptr, best_idx, q_out, peak_h, shift,
                     stencil_idx);
  RG_TRY(hipGetLastError(), "ragged scatter");
  return EBSD_OK;
}

void plan_free(ebsd_ragged_plan_s* pl) {
  if (!pl) return;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  for (auto& c : pl->cls) {
    if (c.branch) (void)hipStreamDestroy(c.branch);
    if (c.done) (void)hipEventDestroy(c.done);
  }
  if (pl->fork) (void)hipEventDestroy(pl->fork);
  if (pl->ran) (void)hipEventDestroy(pl->ran);
  if (pl->cap) (void)hipStreamDestroy(pl->cap);
  if (pl->mem) (void)hipFree(pl->mem);
  delete pl;
}

}  // namespace

extern "C" {

int ebsd_ragged_plan_create(const int32_t* n_per, const int64_t* offset, int64_t P, int64_t L,
                            const ebsd_params* prm, double stencil_step_deg, int32_t flags,
                            ebsd_ragged_plan* plan) {
  g_last_error.clear();
  if (!plan) return fail(EBSD_E_INVALID, "null plan");
  *plan = nullptr;
  if (P < 1 || L < 1) return fail(EBSD_E_INVALID, "P and L must be >= 1");
  if (P > 0x7fffffffLL || L > 0x7fffffffLL) return fail(EBSD_E_INVALID, "P and L must fit in int32");
  if (!n_per || !offset) return fail(EBSD_E_INVALID, "null size or offset array");
  if (flags & ~(EBSD_RAGGED_STENCIL | EBSD_RAGGED_EAGER | EBSD_RAGGED_NO_AUTOTUNE | EBSD_RAGGED_REFINE))
    return fail(EBSD_E_INVALID, "unknown flags");
  if (!(stencil_step_deg > 0.0) || stencil_step_deg > 10.0)
    return fail(EBSD_E_INVALID, "stencil step must be in (0, 10] degrees");
  ebsd_params p;
  int rc;
  if ((rc = resolve_params(prm, 128, &p)) || (rc = f32_images_only(p))) return rc;
  if (p.form != EBSD_FORM_FFT) return fail(EBSD_E_UNSUPPORTED, "ragged batches run the FP32 FFT form");
  auto* pl = new ebsd_ragged_plan_s();
  pl->P = P;
  pl->L = L;
  pl->prm = p;
  pl->step = stencil_step_deg * 3.14159265358979323846 / 180.0;
  pl->flags = flags;
  // rows: class-major, pattern order within a class
  pl->off_h.resize(kNumClasses);
  int64_t row = 0;
  for (int ci = 0; ci < kNumClasses; ++ci) {
    ClassPlan& c = pl->cls[ci];
    c.n = kClassN[ci];
    c.row0 = row;
    for (int64_t i = 0; i < P; ++i) {
      if (n_per[i] == c.n) {
        if (offset[i] < 0) {
          delete pl;
          return fail(EBSD_E_INVALID, "negative pattern offset");
        }
        pl->row_pat_h.push_back((int32_t)i);
        pl->off_h[ci].push_back(offset[i]);
      }
    }
    c.count = (int64_t)pl->off_h[ci].size();
    row += c.count;
  }
  if (row != P) {
    delete pl;
    return fail(EBSD_E_UNSUPPORTED, "ragged pattern sizes must be 64, 96, 128 or 160");
  }
  for (auto& c : pl->cls) {
    if (c.count && (rc = resolve_params(prm, c.n, &c.prm))) {
      delete pl;
      return rc;
    }
  }
  hipError_t e;
  if ((e = hipGetDevice(&pl->device))) {
    delete pl;
    return fail_hip(e, "hipGetDevice");
  }
  if ((e = hipDeviceGetAttribute(&pl->cus, hipDeviceAttributeMultiprocessorCount, pl->device))) {
    delete pl;
    return fail_hip(e, "device attribute");
  }
  Arena a;
  plan_layout(pl, a);
  if ((e = hipMalloc(&pl->mem, a.off))) {
    plan_free(pl);
    return fail(EBSD_E_NOMEM, "ragged plan: device allocation failed");
  }
  a.base = (char*)pl->mem;
  a.off = 0;
  plan_layout(pl, a);
  if ((e = hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking)) ||
      (e = hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming)) ||
      (e = hipEventCreateWithFlags(&pl->ran, hipEventDisableTiming))) {
    plan_free(pl);
    return fail_hip(e, "ragged plan streams");
  }
  for (auto& c : pl->cls) {
    if ((e = hipStreamCreateWithFlags(&c.branch, hipStreamNonBlocking)) ||
        (e = hipEventCreateWithFlags(&c.done, hipEventDisableTiming))) {
      plan_free(pl);
      return fail_hip(e, "ragged plan streams");
    }
  }
  int ci = 0;
  for (auto& c : pl->cls) {
    if (c.count &&
        (e = hipMemcpyAsync(c.img_off, pl->off_h[ci].data(), sizeof(int64_t) * c.count, hipMemcpyHostToDevice,
                            pl->cap))) {
      plan_free(pl);
      return fail_hip(e, "ragged plan upload");
    }
    ++ci;
  }
  if ((e = hipMemcpyAsync(pl->row_pat, pl->row_pat_h.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice,
                          pl->cap))) {
    plan_free(pl);
    return fail_hip(e, "ragged plan upload");
  }
  for (auto& c : pl->cls) {
    if (c.count && (rc = autotune_class(pl, c))) {
      plan_free(pl);
      return rc;
    }
  }
  if ((e = hipStreamSynchronize(pl->cap))) {
    plan_free(pl);
    return fail_hip(e, "ragged plan setup");
  }
  *plan = pl;
  return EBSD_OK;
}

int ebsd_ragged_plan_destroy(ebsd_ragged_plan plan) {
  if (!plan) return EBSD_OK;
  // runs go to callers' streams: wait for the last one (each run records
  // plan->ran after its work on its stream, and a plan serves one run at a
  // time), then for the plan's own streams
  if (plan->ran_recorded) (void)hipEventSynchronize(plan->ran);
  if (plan->cap) (void)hipStreamSynchronize(plan->cap);
  plan_free(plan);
  return EBSD_OK;
}

int ebsd_ragged_plan_tiles(ebsd_ragged_plan plan, int32_t* tiles, int32_t* count) {
  g_last_error.clear();
  if (!plan || !tiles || !count) return fail(EBSD_E_INVALID, "null pointer");
  int k = 0;
  for (auto& c : plan->cls) {
    if (!c.count) continue;
    tiles[4 * k] = c.n;
    tiles[4 * k + 1] = (int32_t)c.count;
    tiles[4 * k + 2] = c.lchunk;
    tiles[4 * k + 3] = c.grid;
    ++k;
  }
  *count = k;
  return EBSD_OK;
}

int ebsd_ragged_run(ebsd_ragged_plan plan, const float* data, const ebsd_master* mp, const ebsd_geometry* geo,
                    const double* lib_q, int32_t* best_idx, double* q_out, float* peak_h, float* shift,
                    int32_t* stencil_idx, void* stream) {
  g_last_error.clear();
  int rc;
  if (!plan) return fail(EBSD_E_INVALID, "null plan");
  if ((rc = check_master(mp)) || (rc = check_geometry(geo))) return rc;
  if (!data || !lib_q || !q_out || !peak_h || !shift) return fail(EBSD_E_INVALID, "null pointer");
  int dev = -1;
  hipError_t e;
  if ((e = hipGetDevice(&dev))) return fail_hip(e, "hipGetDevice");
  if (dev != plan->device) return fail(EBSD_E_INVALID, "the plan was built on another device");
  hipStream_t st = (hipStream_t)stream;
  if (plan->flags & EBSD_RAGGED_EAGER) {
    if ((rc = enqueue(plan, data, mp, geo, lib_q, best_idx, q_out, peak_h, shift, stencil_idx, st))) return rc;
    RG_TRY(hipEventRecord(plan->ran, st), "ragged record");
    plan->ran_recorded = true;
    return EBSD_OK;
  }
  double pcs[3] = {geo->pcx, geo->pcy, geo->pcz};
  uintptr_t pcbits[3];
  std::memcpy(pcbits, pcs, sizeof(pcs));
  const std::vector<uintptr_t> key = {(uintptr_t)data, (uintptr_t)mp->data, (uintptr_t)mp->H, (uintptr_t)mp->W,
                                      pcbits[0], pcbits[1], pcbits[2], (uintptr_t)geo->pc_per,
                                      (uintptr_t)lib_q, (uintptr_t)best_idx, (uintptr_t)q_out,
                                      (uintptr_t)peak_h, (uintptr_t)shift, (uintptr_t)stencil_idx};
  if (!plan->exec || key != plan->key) {
    // the previous replay may still be reading the plan's buffers
    if (plan->exec) {
      if ((e = hipStreamSynchronize(st))) return fail_hip(e, "ragged sync");
      (void)hipGraphExecDestroy(plan->exec);
      plan->exec = nullptr;
    }
    if ((e = hipStreamBeginCapture(plan->cap, hipStreamCaptureModeRelaxed))) return fail_hip(e, "begin capture");
    rc = enqueue(plan, data, mp, geo, lib_q, best_idx, q_out, peak_h, shift, stencil_idx, plan->cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(plan->cap, &graph);
    if (rc != EBSD_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail_hip(e, "end capture");
    e = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      plan->exec = nullptr;
      return fail_hip(e, "graph instantiate");
    }
    plan->key = key;
  }
  RG_TRY(hipGraphLaunch(plan->exec, st), "graph launch");
  RG_TRY(hipEventRecord(plan->ran, st), "ragged record");
  plan->ran_recorded = true;
  return EBSD_OK;
}

}  // extern "C"

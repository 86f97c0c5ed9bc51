// Peak of the correlation on a local grid of shifts (gfx950):
//   rho(c + (a - m, b - m) / kappa),  a, b in [0, 2m + 1),
// evaluated exactly as a matrix DFT over the band (Equation 5 and the peak
// upsampling of section "Fast Fourier Transform"; the integer-shift window
// is the same evaluation with kappa = 1).
//
// With the integer centre c = (x0, y0) applied as exact n-th-root phase ramps,
//   Z'(u, v)  = E(u, v) conj(T(u, v)) exp(2 pi i u y0 / n)
//   G(b, v)   = sum_u F1(u, b) Z'(u, v),     F1(u, b) = exp(2 pi i u (b - m) / (kappa n))
//   G'(b, v)  = G(b, v) exp(2 pi i v x0 / n) w_v   (w_0 = 1, w_v = 2: Hermitian half)
//   rho(b, a) = Re sum_v G'(b, v) F2(v, a),  F2(v, a) = exp(2 pi i v (a - m) / (kappa n))
// Both stages are products with pattern-independent phase matrices (built in
// FP64 once per call); Z' and F1 / F2 are streamed through LDS in 16-row
// chunks, G stays in LDS.  One block evaluates one pair: explicit pairs
// (pi[k], li[k]), or, as the exact FP32 library search over a shift window,
// every pair of P patterns x L templates (block k0 + blockIdx.x is pattern
// (k0 + blockIdx.x) / L, template ... % L; its score goes to h_out at that
// same row-major index).  The largest real value wins; ties go to the
// smallest (b, a) for the sub-pixel grid, and to the smallest unsigned
// row-major shift index ((s_y mod n) n + (s_x mod n)) for the integer window.
#include "ebsd_common.hpp"
#include "ebsd_internal.hpp"

#include <math.h>

namespace ebsd {

namespace {
constexpr int UC = 16;  // rows of Z' / F1 / F2 staged per step
}

int grid_table_size(int n, int kappa, int m) {
  const int b = band_of(n);
  return (3 * b + 2) * (2 * m + 1) + n;
}

size_t grid_lds_bytes(int n, int m) {
  const int bnd = band_of(n);
  const int msz = 2 * m + 1, nv = bnd + 1;
  return sizeof(cf) * ((size_t)UC * nv + (size_t)UC * msz + (size_t)msz * nv);
}

// F1 [2B+1][M], F2 [B+1][M], roots_n [n] in FP64, rounded
__global__ void k_grid_tables(int n, int bnd, int kappa, int m, float2* tab) {
  const int msz = 2 * m + 1;
  const int nk = 2 * bnd + 1, nv = bnd + 1;
  const long kn = (long)kappa * n;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int total = (nk + nv) * msz + n;
  if (i >= total) return;
  long idx, den;
  if (i < nk * msz) {
    const int kk = i / msz, b = i - kk * msz;
    const int u = kk <= bnd ? kk : kk - nk;
    idx = (long)u * (b - m);
    den = kn;
  } else if (i < (nk + nv) * msz) {
    const int j = i - nk * msz;
    const int v = j / msz, a = j - v * msz;
    idx = (long)v * (a - m);
    den = kn;
  } else {
    idx = i - (nk + nv) * msz;
    den = n;
  }
  idx %= den;
  if (idx < 0) idx += den;
  double s, c;
  sincospi(2.0 * (double)idx / (double)den, &s, &c);
  tab[i] = make_float2((float)c, (float)s);
}

// TB x TB threads: thread (ty, tx) holds rows b = ty + TB i and columns
// v (or a) = tx + TB j.  TB = 32 (16 waves) where the LDS of one block leaves
// no room for a second on the CU, so the CU still has 4 waves per SIMD.
template <int VJ, int MB, int TB>
__global__ __launch_bounds__(TB * TB) void k_grid_peak(int n, int bnd, const cf* __restrict__ spec_p,
                                                   const cf* __restrict__ spec_l, const int32_t* __restrict__ pi,
                                                   const int32_t* __restrict__ li, const int32_t* __restrict__ centre,
                                                   int kappa, int m, int int_keys, const cf* __restrict__ tab,
                                                   float* __restrict__ h_out, float* __restrict__ s_out,
                                                   int32_t* __restrict__ s_int_out, int64_t k0, int64_t lib_l) {
  extern __shared__ cf sm[];
  const int nv = bnd + 1, nk = 2 * bnd + 1, spec = nv * nk;
  const int msz = 2 * m + 1;
  cf* zc = sm;                 // Z' rows [UC][nv]
  cf* fc = zc + UC * nv;       // phase-matrix rows [UC][msz]
  cf* g = fc + UC * msz;       // G [msz][nv]
  const cf* F1 = tab;
  const cf* F2 = tab + nk * msz;
  const cf* rn = tab + (nk + nv) * msz;
  constexpr int NT = TB * TB;
  const int tid = threadIdx.x;
  const int tx = tid % TB, ty = tid / TB;
  const int64_t k = k0 + blockIdx.x;
  const int64_t kp = lib_l > 0 ? k / lib_l : (pi ? (int64_t)pi[k] : k);
  const int64_t kl = lib_l > 0 ? k - (k / lib_l) * lib_l : (li ? (int64_t)li[k] : k);
  const cf* E = spec_p + kp * spec;
  const cf* T = spec_l + kl * spec;
  const int x0 = centre ? centre[2 * k] : 0, y0 = centre ? centre[2 * k + 1] : 0;

  // stage 1: thread (ty, tx) accumulates G(b = ty + 16 i, v = tx + 16 j)
  cf acc[MB][VJ];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < VJ; ++j) acc[i][j] = cf{0.f, 0.f};
  for (int u0 = 0; u0 < nk; u0 += UC) {
    const int uc = min(UC, nk - u0);
    __syncthreads();
    for (int t = tid; t < uc * nv; t += NT) {
      const int kk = u0 + t / nv;
      const int u = kk <= bnd ? kk : kk - nk;
      int r = (u * y0) % n;
      if (r < 0) r += n;
      const int e = u0 * nv + t;
      zc[t] = cmul(cmulc(E[e], T[e]), rn[r]);
    }
    for (int t = tid; t < uc * msz; t += NT) fc[t] = F1[u0 * msz + t];
    __syncthreads();
    for (int uu = 0; uu < uc; ++uu) {
      cf zv[VJ];
#pragma unroll
      for (int j = 0; j < VJ; ++j) {
        const int v = tx + TB * j;
        zv[j] = v < nv ? zc[uu * nv + v] : cf{0.f, 0.f};
      }
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        const int b = ty + TB * i;
        const cf f = b < msz ? fc[uu * msz + b] : cf{0.f, 0.f};
#pragma unroll
        for (int j = 0; j < VJ; ++j) {
          acc[i][j].x = __fmaf_rn(f.x, zv[j].x, __fmaf_rn(-f.y, zv[j].y, acc[i][j].x));
          acc[i][j].y = __fmaf_rn(f.x, zv[j].y, __fmaf_rn(f.y, zv[j].x, acc[i][j].y));
        }
      }
    }
  }
  // G'(b, v) = G(b, v) exp(2 pi i v x0 / n) w_v
#pragma unroll
  for (int j = 0; j < VJ; ++j) {
    const int v = tx + TB * j;
    if (v < nv) {
      int r = (v * x0) % n;
      if (r < 0) r += n;
      const cf w = cscale(rn[r], v == 0 ? 1.0f : 2.0f);
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        const int b = ty + TB * i;
        if (b < msz) g[b * nv + v] = cmul(acc[i][j], w);
      }
    }
  }
  // stage 2: thread (ty, tx) accumulates rho(b = ty + 16 i, a = tx + 16 j)
  float rho[MB][MB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < MB; ++j) rho[i][j] = 0.0f;
  for (int v0 = 0; v0 < nv; v0 += UC) {
    const int vc = min(UC, nv - v0);
    __syncthreads();
    for (int t = tid; t < vc * msz; t += NT) fc[t] = F2[v0 * msz + t];
    __syncthreads();
    for (int vv = 0; vv < vc; ++vv) {
      cf gv[MB], fv[MB];
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        const int b = ty + TB * i;
        gv[i] = b < msz ? g[b * nv + v0 + vv] : cf{0.f, 0.f};
        const int a = tx + TB * i;
        fv[i] = a < msz ? fc[vv * msz + a] : cf{0.f, 0.f};
      }
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < MB; ++j)
          rho[i][j] = __fmaf_rn(gv[i].x, fv[j].x, __fmaf_rn(-gv[i].y, fv[j].y, rho[i][j]));
    }
  }
  float best = -INFINITY;
  int bi = 0x7fffffff;
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = ty + TB * i;
#pragma unroll
    for (int j = 0; j < MB; ++j) {
      const int a = tx + TB * j;
      if (b < msz && a < msz) {
        int key = b * msz + a;
        if (int_keys) {
          int sy = (y0 + b - m) % n, sx = (x0 + a - m) % n;
          if (sy < 0) sy += n;
          if (sx < 0) sx += n;
          key = sy * n + sx;
        }
        argmax_merge(best, bi, rho[i][j], key);
      }
    }
  }
  wave_argmax(best, bi);
  __shared__ float rv[NT / 64];
  __shared__ int ri[NT / 64];
  if ((tid & 63) == 0) {
    rv[tid >> 6] = best;
    ri[tid >> 6] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < NT / 64; ++w) argmax_merge(best, bi, rv[w], ri[w]);
    int da, db;  // grid offsets of the winner
    if (int_keys) {
      const int limit = n * n;
      if (bi < 0 || bi >= limit) bi = 0;
      int sy = bi / n, sx = bi - sy * n;
      sy = sy >= n / 2 ? sy - n : sy;
      sx = sx >= n / 2 ? sx - n : sx;
      db = sy - y0;
      da = sx - x0;
    } else {
      if (bi < 0 || bi >= msz * msz) bi = m * msz + m;
      db = bi / msz - m;
      da = bi - (bi / msz) * msz - m;
    }
    h_out[k] = best;
    if (s_out) {
      s_out[2 * k] = (float)x0 + (float)da / (float)kappa;
      s_out[2 * k + 1] = (float)y0 + (float)db / (float)kappa;
    }
    if (s_int_out) {
      s_int_out[2 * k] = x0 + da;
      s_int_out[2 * k + 1] = y0 + db;
    }
  }
}

hipError_t launch_grid_tables(int n, int kappa, int m, float2* tab, hipStream_t stream) {
  const int bnd = band_of(n);
  if (bnd < 0) return hipErrorInvalidValue;
  const int total = grid_table_size(n, kappa, m);
  hipLaunchKernelGGL(k_grid_tables, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, n, bnd, kappa, m,
                     tab);
  return hipGetLastError();
}

template <int VJ, int TB>
static hipError_t grid_vj(int n, int bnd, const float2* spec_p, const float2* spec_l, const int32_t* pi,
                          const int32_t* li, int64_t k, const int32_t* centre, int kappa, int m, int int_keys,
                          const float2* tab, float* h, float* s, int32_t* si, hipStream_t stream, int64_t k0 = 0,
                          int64_t lib_l = 0) {
  const int msz = 2 * m + 1;
  const size_t shm = grid_lds_bytes(n, m);
  const int mb = (msz + TB - 1) / TB;
#define EBSD_GRID(MBV)                                                                                              \
  do {                                                                                                              \
    (void)hipFuncSetAttribute((const void*)k_grid_peak<VJ, MBV, TB>, hipFuncAttributeMaxDynamicSharedMemorySize,  \
                              (int)shm);                                                                          \
    hipLaunchKernelGGL((k_grid_peak<VJ, MBV, TB>), dim3((unsigned)k), dim3(TB * TB), shm, stream, n, bnd,             \
                       (const cf*)spec_p, (const cf*)spec_l, pi, li, centre, kappa, m, int_keys,                    \
                       (const cf*)tab, h, s, si, k0, lib_l);                                                        \
  } while (0)
  // rows per thread rounded up as little as possible: every extra row is a
  // full set of FMAs on zeros (the sub-pixel grid, 151 rows at kappa = 100,
  // takes 5 on 32 x 32 threads)
  if (mb <= 1) EBSD_GRID(1);
  else if (mb <= 2) EBSD_GRID(2);
  else if (mb <= 3) EBSD_GRID(3);
  else if (mb <= 4) EBSD_GRID(4);
  else if (mb <= 5) EBSD_GRID(5);
  else if (mb <= 6) EBSD_GRID(6);
  else if (mb <= 7) EBSD_GRID(7);
  else if constexpr (TB == 16) {  // 32 x 7 rows already cover what 16 x 13 do
    if (mb <= 10) EBSD_GRID(10);
    else if (mb <= 13) EBSD_GRID(13);
    else return hipErrorInvalidValue;
  } else {
    return hipErrorInvalidValue;
  }
#undef EBSD_GRID
  return hipGetLastError();
}

static hipError_t launch_grid(int n, const float2* spec_p, const float2* spec_l, const int32_t* pi,
                              const int32_t* li, int64_t k, const int32_t* centre, int kappa, int m, int int_keys,
                              const float2* tab, float* h, float* s, int32_t* si, hipStream_t stream) {
  if (k <= 0) return hipSuccess;
  const int bnd = band_of(n);
  if (bnd < 0 || grid_lds_bytes(n, m) > 160 * 1024) return hipErrorInvalidValue;
  const int64_t kmax = (int64_t(1) << 31) / 1024;  // blocks x threads of one dispatch below 2^31
  if (k > kmax) {
    const int64_t sc = (int64_t)(bnd + 1) * (2 * bnd + 1);
    for (int64_t s0 = 0; s0 < k; s0 += kmax) {
      const hipError_t e = launch_grid(n, pi ? spec_p : spec_p + s0 * sc, li ? spec_l : spec_l + s0 * sc,
                                       pi ? pi + s0 : nullptr, li ? li + s0 : nullptr, k - s0 < kmax ? k - s0 : kmax,
                                       centre ? centre + 2 * s0 : nullptr, kappa, m, int_keys, tab, h + s0,
                                       s ? s + 2 * s0 : nullptr, si ? si + 2 * s0 : nullptr, stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  // one block per CU by LDS: 32 x 32 threads, else 16 x 16
  const bool wide = grid_lds_bytes(n, m) > 80 * 1024;
  if (bnd + 1 <= 64)
    return wide ? grid_vj<2, 32>(n, bnd, spec_p, spec_l, pi, li, k, centre, kappa, m, int_keys, tab, h, s, si, stream)
                : grid_vj<4, 16>(n, bnd, spec_p, spec_l, pi, li, k, centre, kappa, m, int_keys, tab, h, s, si, stream);
  if (bnd + 1 <= 112)
    return wide ? grid_vj<4, 32>(n, bnd, spec_p, spec_l, pi, li, k, centre, kappa, m, int_keys, tab, h, s, si, stream)
                : grid_vj<7, 16>(n, bnd, spec_p, spec_l, pi, li, k, centre, kappa, m, int_keys, tab, h, s, si, stream);
  return hipErrorInvalidValue;
}

int subpixel_table_size(int n, int kappa) { return grid_table_size(n, kappa, (3 * kappa + 3) / 4); }
size_t subpixel_lds_bytes(int n, int kappa) { return grid_lds_bytes(n, (3 * kappa + 3) / 4); }
hipError_t launch_subpixel_tables(int n, int kappa, float2* tab, hipStream_t stream) {
  return launch_grid_tables(n, kappa, (3 * kappa + 3) / 4, tab, stream);
}

hipError_t launch_subpixel(int n, const float2* spec_p, const float2* spec_l, const int32_t* pi, const int32_t* li,
                           int64_t k, const int32_t* s_int, int kappa, const float2* tab, float* h_sub,
                           float* s_sub, hipStream_t stream) {
  return launch_grid(n, spec_p, spec_l, pi, li, k, s_int, kappa, (3 * kappa + 3) / 4, 0, tab, h_sub, s_sub,
                     nullptr, stream);
}

int window_table_size(int n, int max_shift) { return grid_table_size(n, 1, max_shift); }
hipError_t launch_window_tables(int n, int max_shift, float2* tab, hipStream_t stream) {
  return launch_grid_tables(n, 1, max_shift, tab, stream);
}
bool window_peak_supported(int n, int max_shift) {
  return band_of(n) > 0 && max_shift >= 0 && 2 * max_shift + 1 <= 13 * 16 && 2 * max_shift < n &&
         grid_lds_bytes(n, max_shift) <= 160 * 1024;
}
hipError_t launch_window_peak(int n, const float2* spec_p, const float2* spec_l, const int32_t* pi,
                              const int32_t* li, int64_t k, int max_shift, const float2* tab, float* h_int,
                              int32_t* s_int, hipStream_t stream) {
  return launch_grid(n, spec_p, spec_l, pi, li, k, nullptr, 1, max_shift, 1, tab, h_int, nullptr, s_int, stream);
}

hipError_t launch_window_scores(int n, const float2* spec_p, int64_t p, const float2* spec_l, int64_t l,
                                int max_shift, const float2* tab, float* scores, hipStream_t stream) {
  if (p <= 0 || l <= 0) return hipSuccess;
  const int bnd = band_of(n);
  if (bnd < 0 || !window_peak_supported(n, max_shift)) return hipErrorInvalidValue;
  if (bnd + 1 > 112) return hipErrorInvalidValue;
  const int64_t total = p * l;
  const int64_t kmax = (int64_t(1) << 31) / 1024;  // blocks x threads of one dispatch below 2^31
  const bool wide = grid_lds_bytes(n, max_shift) > 80 * 1024;
  for (int64_t k0 = 0; k0 < total; k0 += kmax) {
    const int64_t kc = total - k0 < kmax ? total - k0 : kmax;
    hipError_t e;
    if (bnd + 1 <= 64)
      e = wide ? grid_vj<2, 32>(n, bnd, spec_p, spec_l, nullptr, nullptr, kc, nullptr, 1, max_shift, 1, tab, scores,
                                nullptr, nullptr, stream, k0, l)
               : grid_vj<4, 16>(n, bnd, spec_p, spec_l, nullptr, nullptr, kc, nullptr, 1, max_shift, 1, tab, scores,
                                nullptr, nullptr, stream, k0, l);
    else
      e = wide ? grid_vj<4, 32>(n, bnd, spec_p, spec_l, nullptr, nullptr, kc, nullptr, 1, max_shift, 1, tab, scores,
                                nullptr, nullptr, stream, k0, l)
               : grid_vj<7, 16>(n, bnd, spec_p, spec_l, nullptr, nullptr, kc, nullptr, 1, max_shift, 1, tab, scores,
                                nullptr, nullptr, stream, k0, l);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ebsd

// Filtered spectra at 256 x 256 (same definition as k_spectra in
// k_spectra_xcf.hip: contrast normalisation, Hann window, forward 2-D DFT,
// band-pass cut at rho_max, FP64 energy, unit-energy band layout).  A 256^2
// transform does not fit one block's LDS, so it runs as three passes through
// a global intermediate:
//   rows     two real rows packed as one complex 256-point FFT (16 x 16,
//            one LDS exchange), separated into the Hermitian halves v <= B;
//   columns  256-point FFTs along y for 8 columns per block, band-pass,
//            band rows stored, FP64 energy partial per block;
//   scale    energy summed, band scaled to unit energy.
#include "ebsd_common.hpp"
#include "ebsd_internal.hpp"

#include <math.h>

namespace ebsd {

namespace {
constexpr int N = 256, R = 16, B = Plan<256>::B, NV = B + 1, NK = 2 * B + 1;
constexpr int COLS = 8;                        // columns per block in the column pass
constexpr int CGROUPS = (NV + COLS - 1) / COLS;

__device__ __forceinline__ cf root256(int k) {
  double s, c;
  sincospi(2.0 * (double)(k & (N - 1)) / (double)N, &s, &c);
  return cf{(float)c, (float)s};
}
}  // namespace

// mean and 1/std of each image (FP64 sums)
__global__ __launch_bounds__(256) void k_img_stats(const float* __restrict__ imgs, int npix, float2* __restrict__ st) {
  const int64_t k = blockIdx.x;
  const float* img = imgs + k * (int64_t)npix;
  double s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < npix; i += 256) {
    const double v = img[i];
    s1 += v;
    s2 += v * v;
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  __shared__ double red[8];
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = s1;
    red[4 + (threadIdx.x >> 6)] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double mean = (red[0] + red[1] + red[2] + red[3]) / npix;
    const double var = (red[4] + red[5] + red[6] + red[7]) / npix - mean * mean;
    st[k] = make_float2((float)mean, var > 0.0 ? (float)(1.0 / sqrt(var)) : 0.0f);
  }
}

// rows: block (image k, group g) handles row pairs (q, q + 128), q in [16 g, 16 g + 16)
__global__ __launch_bounds__(256) void k_rows256(const float* __restrict__ imgs, const float2* __restrict__ st,
                                                 int window, cf* __restrict__ vout) {
  __shared__ cf ys[16 * 16 * 17];  // [pair][c][b], b padded
  __shared__ cf tw[N];
  __shared__ float win[N];
  const int tid = threadIdx.x;
  const int64_t k = blockIdx.x >> 3;
  const int g = blockIdx.x & 7;
  const float* img = imgs + k * (int64_t)N * N;
  const float mean = st[k].x, istd = st[k].y;
  tw[tid] = root256(tid);
  {
    const float s = sinpif(((float)tid + 0.5f) / (float)N);
    win[tid] = window ? s * s : 1.0f;
  }
  __syncthreads();
  const int p = tid >> 4, b = tid & 15;
  const int q = 16 * g + p;
  {
    cf x[R];
    const float w0 = win[q] * istd, w1 = win[q + 128] * istd;
#pragma unroll
    for (int a = 0; a < R; ++a) {
      const int col = R * a + b;
      x[a] = cf{(img[q * N + col] - mean) * w0 * win[col], (img[(q + 128) * N + col] - mean) * w1 * win[col]};
    }
    DFT<R, -1>::run(x);
#pragma unroll
    for (int c = 1; c < R; ++c) x[c] = cmulc(x[c], tw[b * c]);
#pragma unroll
    for (int c = 0; c < R; ++c) ys[(p * 16 + c) * 17 + b] = x[c];
  }
  __syncthreads();
  const int c = tid & 15;
  cf z[R];
#pragma unroll
  for (int bb = 0; bb < R; ++bb) z[bb] = ys[(p * 16 + c) * 17 + bb];
  DFT<R, -1>::run(z);  // Z(v = c + 16 d)
  __syncthreads();
  cf* zs = ys;  // [pair][v], 16 x 256
#pragma unroll
  for (int d = 0; d < R; ++d) zs[p * N + c + R * d] = z[d];
  __syncthreads();
  // separate the packed rows: F_q(v) = (Z(v) + conj Z(-v)) / 2, F_{q+128}(v) = (Z(v) - conj Z(-v)) / 2i
  for (int t = tid; t < 16 * NV; t += 256) {
    const int pp = t / NV, v = t - pp * NV;
    const cf z1 = zs[pp * N + v], z2 = zs[pp * N + ((N - v) & (N - 1))];
    const int qq = 16 * g + pp;
    vout[(k * N + qq) * NV + v] = cf{0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y)};
    vout[(k * N + qq + 128) * NV + v] = cf{0.5f * (z1.y + z2.y), -0.5f * (z1.x - z2.x)};
  }
}

// columns: block (image k, group g) handles columns v in [8 g, 8 g + 8)
__global__ __launch_bounds__(256) void k_cols256(const cf* __restrict__ vin, FilterParams fp, cf* __restrict__ spec,
                                                 double* __restrict__ part) {
  __shared__ cf ys[COLS * 16 * 17];
  __shared__ cf tw[N];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int64_t k = blockIdx.x / CGROUPS;
  const int g = blockIdx.x - (int)(k * CGROUPS);
  tw[tid] = root256(tid);
  __syncthreads();
  const int col = tid >> 5, sub = tid & 31;  // 8 columns x 32 threads; 16 tasks per column per pass
  const int v = COLS * g + col;
  const bool vok = v < NV;
  if (sub < 16) {
    const int b = sub;
    cf x[R];
#pragma unroll
    for (int a = 0; a < R; ++a) x[a] = vok ? vin[(k * N + R * a + b) * NV + v] : cf{0.f, 0.f};
    DFT<R, -1>::run(x);
#pragma unroll
    for (int c = 1; c < R; ++c) x[c] = cmulc(x[c], tw[b * c]);
#pragma unroll
    for (int c = 0; c < R; ++c) ys[(col * 16 + c) * 17 + b] = x[c];
  }
  __syncthreads();
  double en = 0.0;
  if (sub < 16 && vok) {
    const int c = sub;
    cf z[R];
#pragma unroll
    for (int b = 0; b < R; ++b) z[b] = ys[(col * 16 + c) * 17 + b];
    DFT<R, -1>::run(z);  // X(u = c + 16 d, v)
    const float inv2hp = 1.0f / (2.0f * fp.sigma_hp * fp.sigma_hp);
    const float inv2lp = 1.0f / (2.0f * fp.sigma_lp * fp.sigma_lp);
    const float rmax2 = fp.rho_max * fp.rho_max;
    cf* out = spec + k * (int64_t)(NK * NV);
#pragma unroll
    for (int d = 0; d < R; ++d) {
      const int u = c + R * d;
      const int us = u >= N / 2 ? u - N : u;
      const int kk = u <= B ? u : (u >= N - B ? u - N + NK : -1);
      if (kk >= 0) {
        const float r2 = (float)(us * us + v * v);
        float h = 0.0f;
        if (r2 <= rmax2) h = (1.0f - expf(-r2 * inv2hp)) * expf(-r2 * inv2lp);
        const cf zz = cscale(z[d], h);
        out[kk * NV + v] = zz;
        en += (v == 0 ? 1.0 : 2.0) * ((double)zz.x * zz.x + (double)zz.y * zz.y);
      }
    }
  }
  en = wave_sum(en);
  if ((tid & 63) == 0) red[tid >> 6] = en;
  __syncthreads();
  if (tid == 0) part[k * CGROUPS + g] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_scale256(const double* __restrict__ part, cf* __restrict__ spec,
                                                  double* __restrict__ energy) {
  const int64_t k = blockIdx.x;
  __shared__ float sc;
  if (threadIdx.x == 0) {
    double e = 0.0;
    for (int g = 0; g < CGROUPS; ++g) e += part[k * CGROUPS + g];
    sc = e > 0.0 ? (float)(1.0 / sqrt(e)) : 0.0f;
    if (energy) energy[k] = e;
  }
  __syncthreads();
  cf* out = spec + k * (int64_t)(NK * NV);
  for (int i = threadIdx.x; i < NK * NV; i += 256) out[i] = cscale(out[i], sc);
}

size_t spectra256_scratch_bytes(int64_t k) {
  return (size_t)k * (sizeof(float2) + (size_t)N * NV * sizeof(cf) + CGROUPS * sizeof(double));
}

hipError_t launch_spectra256(const float* imgs, int64_t k, const FilterParams& fp, float2* spec, double* energy,
                             void* scratch, hipStream_t stream) {
  if (k <= 0) return hipSuccess;
  if (k * CGROUPS > (int64_t(1) << 31) / 256) return hipErrorInvalidValue;  // one dispatch below 2^31 items
  float2* st = (float2*)scratch;
  cf* v = (cf*)((char*)scratch + (size_t)k * sizeof(float2));
  double* part = (double*)((char*)v + (size_t)k * N * NV * sizeof(cf));
  hipLaunchKernelGGL(k_img_stats, dim3((unsigned)k), dim3(256), 0, stream, imgs, N * N, st);
  hipLaunchKernelGGL(k_rows256, dim3((unsigned)(k * 8)), dim3(256), 0, stream, imgs, st, fp.window, v);
  hipLaunchKernelGGL(k_cols256, dim3((unsigned)(k * CGROUPS)), dim3(256), 0, stream, v, fp, (cf*)spec, part);
  hipLaunchKernelGGL(k_scale256, dim3((unsigned)k), dim3(256), 0, stream, part, (cf*)spec, energy);
  return hipGetLastError();
}

}  // namespace ebsd

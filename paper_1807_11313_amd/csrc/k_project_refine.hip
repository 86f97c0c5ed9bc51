// Template projection, sub-pixel peak, library argmax and refinement kernels (gfx950).
#include "ebsd_common.hpp"
#include "ebsd_internal.hpp"

#include <math.h>

namespace ebsd {

// ---------------------------------------------------------------------------
// Gnomonic projection (section "SO(3) Library Generation"): pixel (i, j) of an
// n x n screen looks along d = normalise((i + 1/2)/n - PCx, (j + 1/2)/n - PCy, PCz)
// (detector frame x = +column, y = +row, z = source to screen; PC in screen
// widths); the crystal direction c = R d is looked up in the equirectangular
// master (row r at polar angle (r + 1/2) pi / H, column q at azimuth 2 pi q / W)
// with Keys cubic convolution (a = -0.5), periodic in azimuth, rows clamped.
__device__ __forceinline__ void keys4(float t, float* w) {
  // weights of taps at offsets -1, 0, 1, 2 for fractional position t in [0, 1)
  const float a = -0.5f;
  const float t2 = t * t, t3 = t2 * t;
  w[0] = a * (t3 - 2.0f * t2 + t);
  w[1] = (a + 2.0f) * t3 - (a + 3.0f) * t2 + 1.0f;
  const float s = 1.0f - t, s2 = s * s, s3 = s2 * s;
  w[2] = (a + 2.0f) * s3 - (a + 3.0f) * s2 + 1.0f;
  w[3] = a * (s3 - 2.0f * s2 + s);
}

__global__ __launch_bounds__(256) void k_project(const float* __restrict__ master, int mh, int mw,
                                                 const double* __restrict__ q,
                                                 const double* __restrict__ pc_per, double pcx,
                                                 double pcy, double pcz, int n,
                                                 float* __restrict__ out) {
  const int64_t k = blockIdx.y;
  const int pix = blockIdx.x * 256 + threadIdx.x;
  if (pix >= n * n) return;
  const double qw = q[4 * k], qx = q[4 * k + 1], qy = q[4 * k + 2], qz = q[4 * k + 3];
  const float r00 = (float)(1 - 2 * (qy * qy + qz * qz)), r01 = (float)(2 * (qx * qy - qw * qz)),
              r02 = (float)(2 * (qx * qz + qw * qy));
  const float r10 = (float)(2 * (qx * qy + qw * qz)), r11 = (float)(1 - 2 * (qx * qx + qz * qz)),
              r12 = (float)(2 * (qy * qz - qw * qx));
  const float r20 = (float)(2 * (qx * qz - qw * qy)), r21 = (float)(2 * (qy * qz + qw * qx)),
              r22 = (float)(1 - 2 * (qx * qx + qy * qy));
  if (pc_per) {
    pcx = pc_per[3 * k];
    pcy = pc_per[3 * k + 1];
    pcz = pc_per[3 * k + 2];
  }
  const int j = pix / n, i = pix - j * n;
  const float inv_n = 1.0f / (float)n;
  const float dx = ((float)i + 0.5f) * inv_n - (float)pcx;
  const float dy = ((float)j + 0.5f) * inv_n - (float)pcy;
  const float dz = (float)pcz;
  const float rn = rsqrtf(dx * dx + dy * dy + dz * dz);
  const float ux = dx * rn, uy = dy * rn, uz = dz * rn;
  const float cx = r00 * ux + r01 * uy + r02 * uz;
  const float cy = r10 * ux + r11 * uy + r12 * uz;
  const float cz = r20 * ux + r21 * uy + r22 * uz;
  const float theta = atan2f(sqrtf(cx * cx + cy * cy), cz);
  float phi = atan2f(cy, cx);
  if (phi < 0.0f) phi += 6.28318530717958647692f;
  float v = theta * ((float)mh * 0.318309886183790671538f) - 0.5f;
  const float u = phi * ((float)mw * 0.159154943091895335769f);
  v = fminf(fmaxf(v, 0.0f), (float)(mh - 1));
  const float v0f = floorf(v), u0f = floorf(u);
  float wv[4], wu[4];
  keys4(v - v0f, wv);
  keys4(u - u0f, wu);
  // phi is in [0, 2 pi] (rounding included), so u0 is in [0, mw]; the clamp
  // only guards the reads against a non-finite orientation.  Each periodic
  // azimuth tap index is then in [-1, mw + 2] and one conditional wrap each
  // way gives the same column as a modulo (mw >= 4)
  const int v0 = (int)v0f, u0 = min(max((int)u0f, 0), mw);
  int col[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    int c = u0 + b - 1;
    c += c < 0 ? mw : 0;
    c -= c >= mw ? mw : 0;
    col[b] = c;
  }
  float acc = 0.0f;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int row = min(max(v0 + a - 1, 0), mh - 1);
    const float* mrow = master + (int64_t)row * mw;
    float ra = 0.0f;
#pragma unroll
    for (int b = 0; b < 4; ++b) ra = __fmaf_rn(wu[b], mrow[col[b]], ra);
    acc = __fmaf_rn(wv[a], ra, acc);
  }
  out[k * (int64_t)n * n + pix] = acc;
}

// ---------------------------------------------------------------------------
// exp(2 pi i k / m), k in [0, m), FP64 evaluation.
__global__ void k_roots(int m, float2* out) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= m) return;
  double s, c;
  sincospi(2.0 * (double)k / (double)m, &s, &c);
  out[k] = make_float2((float)c, (float)s);
}

// ---------------------------------------------------------------------------
// Library argmax (section "Method Overview": best match = highest coefficient),
// ties to the smallest template index.
__global__ __launch_bounds__(256) void k_library_argmax(const float* __restrict__ scores, int64_t l,
                                                        int32_t* __restrict__ best,
                                                        float* __restrict__ best_h) {
  const int64_t p = blockIdx.x;
  const int tid = threadIdx.x;
  const float* s = scores + p * l;
  float bv = -INFINITY;
  int bi = 0x7fffffff;
  for (int64_t i = tid; i < l; i += 256) argmax_merge(bv, bi, s[i], (int)i);
  wave_argmax(bv, bi);
  __shared__ float rv[4];
  __shared__ int ri[4];
  if ((tid & 63) == 0) {
    rv[tid >> 6] = bv;
    ri[tid >> 6] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 4; ++w) argmax_merge(bv, bi, rv[w], ri[w]);
    if (bi < 0 || bi >= l) bi = 0;  // every score NaN: keep the index in range
    best[p] = bi;
    if (best_h) best_h[p] = bv;
  }
}

__global__ void k_gather_q(const double* __restrict__ lib_q, const int32_t* __restrict__ best,
                           int64_t p, double* __restrict__ best_q) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= p) return;
  const int64_t l = best[i];
#pragma unroll
  for (int c = 0; c < 4; ++c) best_q[4 * i + c] = lib_q[4 * l + c];
}

// ---------------------------------------------------------------------------
// Log-polar resampling (section "Orientation and Pattern Centre Refinement"):
// centre ((n-1)/2, (n-1)/2), n_rho radii log-spaced in [2, n/2 - 2] px, n_eta
// angles eta_m = 2 pi m / n_eta measured from +column toward +row, bilinear
// samples of the contrast-normalised image, each radius row mean-removed.
template <class T>
__global__ __launch_bounds__(256) void k_logpolar(const T* __restrict__ imgs, int n, int n_rho,
                                                  int n_eta, float* __restrict__ out) {
  const int64_t k = blockIdx.x;
  const int tid = threadIdx.x;
  const T* img = imgs + k * (int64_t)n * n;
  double s1 = 0.0, s2 = 0.0;
  for (int i = tid; i < n * n; i += 256) {
    const double v = ld_px(img[i]);
    s1 += v;
    s2 += v * v;
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  __shared__ double red[8];
  if ((tid & 63) == 0) {
    red[tid >> 6] = s1;
    red[4 + (tid >> 6)] = s2;
  }
  __syncthreads();
  const double mean = (red[0] + red[1] + red[2] + red[3]) / (double)(n * n);
  const double var = (red[4] + red[5] + red[6] + red[7]) / (double)(n * n) - mean * mean;
  const float fmean = (float)mean, inv_std = var > 0.0 ? (float)(1.0 / sqrt(var)) : 0.0f;
  const float c = 0.5f * (float)(n - 1);
  const double rmin = 2.0, rmax = 0.5 * n - 2.0;
  const int lane = tid & 63, wave = tid >> 6;
  float* o = out + k * (int64_t)n_rho * n_eta;
  // the angles' (cos, sin), the same for every radius; each lane keeps its
  // samples of a row in registers until the row mean is known, so every
  // output value is written once
  __shared__ float2 ang[1024];
  for (int m = tid; m < n_eta; m += 256) {
    float sn, cs;
    sincospif(2.0f * (float)m / (float)n_eta, &sn, &cs);
    ang[m] = make_float2(cs, sn);
  }
  __syncthreads();
  constexpr int MPL = 1024 / 64;  // samples per lane at the largest n_eta
  for (int row = wave; row < n_rho; row += 4) {
    const float r = (float)(rmin * pow(rmax / rmin, (double)row / (double)(n_rho - 1)));
    float sum = 0.0f;
    float xs[MPL];
#pragma unroll
    for (int i = 0; i < MPL; ++i) {
      const int m = lane + 64 * i;
      if (m < n_eta) {
        const float cs = ang[m].x, sn = ang[m].y;
        const float col = c + r * cs, rw = c + r * sn;
        const float r0f = floorf(rw), c0f = floorf(col);
        const float fr = rw - r0f, fc = col - c0f;
        const int r0 = (int)r0f, c0 = (int)c0f;
        const T* p = img + r0 * n + c0;
        const float val = (1.0f - fr) * ((1.0f - fc) * ld_px(p[0]) + fc * ld_px(p[1])) +
                          fr * ((1.0f - fc) * ld_px(p[n]) + fc * ld_px(p[n + 1]));
        const float x = (val - fmean) * inv_std;
        xs[i] = x;
        sum += x;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    const float mu = sum / (float)n_eta;
#pragma unroll
    for (int i = 0; i < MPL; ++i) {
      const int m = lane + 64 * i;
      if (m < n_eta) o[row * n_eta + m] = xs[i] - mu;
    }
  }
}

// Maximum of the trigonometric interpolant of the normalised eta
// correlation over D_int + a / kappa, |a| <= ceil(0.75 kappa), from its
// transform C(q), q in [0, n_eta / 2] (ties to the smallest a); thread 0
// writes gamma = 2 pi D / n_eta.  A block of 256 threads; rv / ri are
// 4-entry shared scratch.
__device__ __forceinline__ void eta_interpolate(const float* cqr, const float* cqi, int n_eta, int d_int,
                                                int kappa, float* rv, int* ri, double* gamma_out) {
  const int tid = threadIdx.x;
  const int m = (3 * kappa + 3) / 4;
  const int kn = kappa * n_eta;
  float best = -INFINITY;
  int besta = 0x7fffffff;
  for (int a = -m + tid; a <= m; a += 256) {
    const int ph = kappa * d_int + a;
    float v = cqr[0];
    for (int qq = 1; qq < n_eta / 2; ++qq) {
      int idx = (qq * ph) % kn;
      if (idx < 0) idx += kn;
      float sn, cs;
      sincospif(2.0f * (float)idx / (float)kn, &sn, &cs);
      v += 2.0f * (cqr[qq] * cs - cqi[qq] * sn);
    }
    // Nyquist term cos(pi t) = (-1)^d_int cos(pi a / kappa)
    const float ny = ((d_int & 1) ? -1.0f : 1.0f) * cospif((float)a / (float)kappa);
    v += cqr[n_eta / 2] * ny;
    v /= (float)n_eta;
    argmax_merge(best, besta, v, a + m);
  }
  wave_argmax(best, besta);
  __syncthreads();
  if ((tid & 63) == 0) {
    rv[tid >> 6] = best;
    ri[tid >> 6] = besta;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 4; ++w) argmax_merge(best, besta, rv[w], ri[w]);
    const double dsub = (double)d_int + (double)(besta - m) / (double)kappa;
    *gamma_out = 2.0 * 3.14159265358979323846 * dsub / (double)n_eta;
  }
}

// eta correlation c(D) = sum_k w_k sum_m Le[k][m] Lt[k][m - D] (Hann weights
// over radius), normalised; integer argmax (ties to the smallest D), then the
// maximum of its trigonometric interpolant over D_int + a / kappa,
// |a| <= ceil(0.75 kappa) (ties to the smallest a); gamma = 2 pi D / n_eta.
// Direct form, one lag per thread, every value read from LDS: any n_eta (the
// default grids take the transform form below).
__global__ __launch_bounds__(256) void k_eta_peak(const float* __restrict__ lp_e,
                                                  const float* __restrict__ lp_t, int n_rho,
                                                  int n_eta, int kappa, double* __restrict__ gamma) {
  extern __shared__ float fsm[];
  constexpr int RC = 8;  // radius rows staged per step
  float* le = fsm;                     // [RC][n_eta]
  float* lt = fsm + RC * n_eta;        // [RC][n_eta]
  float* cc = lt + RC * n_eta;         // [n_eta]
  float* cq = cc + n_eta;              // [2][n_eta / 2 + 1]
  const int64_t k = blockIdx.x;
  const int tid = threadIdx.x;
  const float* E = lp_e + k * (int64_t)n_rho * n_eta;
  const float* T = lp_t + k * (int64_t)n_rho * n_eta;
  constexpr int DMAX = 4;  // n_eta <= 1024
  float acc[DMAX];
#pragma unroll
  for (int j = 0; j < DMAX; ++j) acc[j] = 0.0f;
  float ee = 0.0f, tt = 0.0f;
  for (int r0 = 0; r0 < n_rho; r0 += RC) {
    const int rc = min(RC, n_rho - r0);
    __syncthreads();
    for (int t = tid; t < rc * n_eta; t += 256) {
      le[t] = E[r0 * n_eta + t];
      lt[t] = T[r0 * n_eta + t];
    }
    __syncthreads();
    for (int rr = 0; rr < rc; ++rr) {
      const float s = sinpif(((float)(r0 + rr) + 0.5f) / (float)n_rho);
      const float w = s * s;
      const float* er = le + rr * n_eta;
      const float* tr = lt + rr * n_eta;
#pragma unroll
      for (int j = 0; j < DMAX; ++j) {
        const int d = tid + 256 * j;
        if (d < n_eta) {
          float a = 0.0f;
          // m - d wraps at m = d
          for (int m = 0; m < d; ++m) a = __fmaf_rn(er[m], tr[m - d + n_eta], a);
          for (int m = d; m < n_eta; ++m) a = __fmaf_rn(er[m], tr[m - d], a);
          acc[j] = __fmaf_rn(w, a, acc[j]);
        }
      }
      if (tid < n_eta) {
        // per-thread partial energies over this row
        const float* trow = lt + rr * n_eta;
        float pe = 0.0f, pt = 0.0f;
        for (int m = tid; m < n_eta; m += 256) {
          pe = __fmaf_rn(er[m], er[m], pe);
          pt = __fmaf_rn(trow[m], trow[m], pt);
        }
        ee = __fmaf_rn(w, pe, ee);
        tt = __fmaf_rn(w, pt, tt);
      }
    }
  }
  // raw correlation into cc
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    const int d = tid + 256 * j;
    if (d < n_eta) cc[d] = acc[j];
  }
  // energies
  for (int off = 32; off > 0; off >>= 1) {
    ee += __shfl_xor(ee, off, 64);
    tt += __shfl_xor(tt, off, 64);
  }
  __shared__ float rsum[8];
  __shared__ float rv[4];
  __shared__ int ri[4];
  if ((tid & 63) == 0) {
    rsum[tid >> 6] = ee;
    rsum[4 + (tid >> 6)] = tt;
  }
  __syncthreads();
  const float norm = sqrtf((rsum[0] + rsum[1] + rsum[2] + rsum[3]) * (rsum[4] + rsum[5] + rsum[6] + rsum[7]));
  const float inv = norm > 0.0f ? 1.0f / norm : 0.0f;
  float bv = -INFINITY;
  int bi = 0x7fffffff;
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    const int d = tid + 256 * j;
    if (d < n_eta) {
      const float v = cc[d] * inv;
      cc[d] = v;
      argmax_merge(bv, bi, v, d);
    }
  }
  wave_argmax(bv, bi);
  if ((tid & 63) == 0) {
    rv[tid >> 6] = bv;
    ri[tid >> 6] = bi;
  }
  __syncthreads();
  for (int w = 0; w < 4; ++w) argmax_merge(bv, bi, rv[w], ri[w]);
  const int d_int = bi >= n_eta / 2 ? bi - n_eta : bi;
  // C(q) = sum_D c(D) exp(-2 pi i q D / n_eta), q in [0, n_eta / 2]
  const int nq = n_eta / 2 + 1;
  float* cqr = cq;
  float* cqi = cq + nq;
  for (int qq = tid; qq < nq; qq += 256) {
    float ar = 0.0f, ai = 0.0f;
    for (int d = 0; d < n_eta; ++d) {
      float sn, cs;
      sincospif(2.0f * (float)((qq * d) % n_eta) / (float)n_eta, &sn, &cs);
      ar = __fmaf_rn(cc[d], cs, ar);
      ai = __fmaf_rn(-cc[d], sn, ai);
    }
    cqr[qq] = ar;
    cqi[qq] = ai;
  }
  __syncthreads();
  eta_interpolate(cqr, cqi, n_eta, d_int, kappa, rv, ri, gamma + k);
}

// ---------------------------------------------------------------------------
// FP64 orientation updates (Equation 7 with the atan reading; log-polar z):
// with c = R d, a crystal rotated by Q in the detector frame has orientation
// R Q^T, i.e. quaternion q (x) conj(q_Q).
// With `beam` set, the shift was measured against a template projected at
// (pcx0, pcy0) and the pattern sits at pc_per[i]: the PC move translates the
// pattern by +n (dx, dy) px, which is taken off before the angles.
__global__ void k_update_xy(double* __restrict__ q, const float* __restrict__ s_sub, int64_t kk,
                            const double* __restrict__ pc_per, double pcz, int n, int beam, double pcx0,
                            double pcy0) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= kk) return;
  const double dd = (pc_per ? pc_per[3 * i + 2] : pcz) * (double)n;
  double sx = (double)s_sub[2 * i], sy = (double)s_sub[2 * i + 1];
  if (beam) {
    sx -= (double)n * (pc_per[3 * i] - pcx0);
    sy -= (double)n * (pc_per[3 * i + 1] - pcy0);
  }
  const double beta = atan(sx / dd);
  const double alpha = -atan(sy / dd);
  // conj(q_y(beta) q_x(alpha)) = conj(q_x(alpha)) conj(q_y(beta))
  const double cxi[4] = {cos(0.5 * alpha), -sin(0.5 * alpha), 0.0, 0.0};
  const double cyi[4] = {cos(0.5 * beta), 0.0, -sin(0.5 * beta), 0.0};
  double t[4], o[4];
  qmul(q + 4 * i, cxi, t);
  qmul(t, cyi, o);
  qstore(q + 4 * i, o);
}

__global__ void k_update_z(double* __restrict__ q, const double* __restrict__ gamma, int64_t kk) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= kk) return;
  const double g = gamma[i];
  const double czi[4] = {cos(0.5 * g), 0.0, 0.0, -sin(0.5 * g)};
  double o[4];
  qmul(q + 4 * i, czi, o);
  qstore(q + 4 * i, o);
}

// ---------------------------------------------------------------------------
hipError_t launch_project(int n, const float* master, int mh, int mw, const double* q, int64_t k,
                          const double* pc_per, double pcx, double pcy, double pcz, float* out,
                          hipStream_t stream) {
  if (k <= 0) return hipSuccess;
  if (k > 65535) {
    for (int64_t s = 0; s < k; s += 65535) {
      const int64_t c = k - s < 65535 ? k - s : 65535;
      hipError_t e = launch_project(n, master, mh, mw, q + 4 * s, c, pc_per ? pc_per + 3 * s : nullptr, pcx,
                                    pcy, pcz, out + s * (int64_t)n * n, stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  dim3 grid((unsigned)((n * n + 255) / 256), (unsigned)k);
  hipLaunchKernelGGL(k_project, grid, dim3(256), 0, stream, master, mh, mw, q, pc_per, pcx, pcy, pcz, n, out);
  return hipGetLastError();
}

hipError_t launch_roots(int m, float2* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_roots, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, m, out);
  return hipGetLastError();
}

hipError_t launch_library_argmax(const float* scores, int64_t p, int64_t l, int32_t* best,
                                 float* best_h, hipStream_t stream) {
  if (p <= 0) return hipSuccess;
  const int64_t pmax = (int64_t(1) << 31) / 256;  // blocks x threads of one dispatch below 2^31
  for (int64_t s = 0; s < p; s += pmax) {
    const int64_t pc = p - s < pmax ? p - s : pmax;
    hipLaunchKernelGGL(k_library_argmax, dim3((unsigned)pc), dim3(256), 0, stream, scores + s * l, l, best + s,
                       best_h + s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_gather_q(const double* lib_q, const int32_t* best, int64_t p, double* best_q,
                           hipStream_t stream) {
  if (p <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_q, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, stream, lib_q, best, p, best_q);
  return hipGetLastError();
}

hipError_t launch_logpolar(int n, const float* imgs, int64_t k, int n_rho, int n_eta, float* out,
                           hipStream_t stream) {
  if (k <= 0) return hipSuccess;
  if (k > (int64_t(1) << 31) / 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_logpolar<float>, dim3((unsigned)k), dim3(256), 0, stream, imgs, n, n_rho, n_eta, out);
  return hipGetLastError();
}

hipError_t launch_logpolar(int n, const __bf16* imgs, int64_t k, int n_rho, int n_eta, float* out,
                           hipStream_t stream) {
  if (k <= 0) return hipSuccess;
  if (k > (int64_t(1) << 31) / 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_logpolar<__bf16>, dim3((unsigned)k), dim3(256), 0, stream, imgs, n, n_rho, n_eta, out);
  return hipGetLastError();
}

// The same eta correlation through row transforms, for n_eta = NE = P1 x P2
// (P2 threads per radius row, RG rows at a time).  Row k is packed as
// z = Le[k] + i Lt[k] and transformed once (forward: radix P1 in registers
// over m = P2 a + j, twiddle, radix P2 over j); with S(q) = Z(q) + conj(Z(-q))
// and D(q) = Z(q) - conj(Z(-q)), Le's transform times the conjugate of Lt's
// is i S conj(D) / 4.  The weighted products are summed over rows in a
// fixed order into A(q), q in [0, NE / 2]; c(D) is the inverse transform of
// A, and the transform of the normalised c that the interpolation needs is
// A times the normalisation.  The energies are the direct weighted sums.
template <int NE>
__global__ __launch_bounds__(256) void k_eta_fft(const float* __restrict__ lp_e, const float* __restrict__ lp_t,
                                                 int n_rho, int kappa, double* __restrict__ gamma) {
  constexpr int P2 = NE >= 512 ? 32 : 16, P1 = NE / P2, RG = 256 / P2, NQ = NE / 2 + 1;
  constexpr int CPT = (P1 + P2 - 1) / P2, QPT = (NQ + 255) / 256;
  static_assert(P1 * P2 == NE && RG * P2 == 256, "row layout");
  extern __shared__ float fsm[];
  cf* yb = reinterpret_cast<cf*>(fsm);                // [RG][NE]
  cf* pr = yb + RG * NE;                              // [RG][NQ]
  cf* rt = pr + RG * NQ;                              // [NE] exp(+2 pi i t / NE)
  float* cc = reinterpret_cast<float*>(rt + NE);      // [NE]
  float* cqr = cc + NE;                               // [NQ]
  float* cqi = cqr + NQ;                              // [NQ]
  __shared__ float rsum[8];
  __shared__ float rv[4];
  __shared__ int ri[4];
  const int64_t k = blockIdx.x;
  const int tid = threadIdx.x, j = tid % P2, g = tid / P2;
  const float* E = lp_e + k * (int64_t)n_rho * NE;
  const float* T = lp_t + k * (int64_t)n_rho * NE;
  for (int t = tid; t < NE; t += 256) {
    float sn, cs;
    sincospif(2.0f * (float)t / (float)NE, &sn, &cs);
    rt[t] = cf{cs, sn};
  }
  cf acc[QPT];
#pragma unroll
  for (int i = 0; i < QPT; ++i) acc[i] = cf{0.f, 0.f};
  float ee = 0.0f, tt = 0.0f;
  cf* yg = yb + g * NE;
  cf* pg = pr + g * NQ;
  __syncthreads();
  for (int r0 = 0; r0 < n_rho; r0 += RG) {
    const int r = r0 + g;
    const bool rok = r < n_rho;
    const float sw = sinpif(((float)r + 0.5f) / (float)n_rho);
    const float w = rok ? sw * sw : 0.0f;
    cf x[P1];
    float pe = 0.0f, pt = 0.0f;
#pragma unroll
    for (int a = 0; a < P1; ++a) {
      const int m = P2 * a + j;
      const float ev = rok ? E[(int64_t)r * NE + m] : 0.0f;
      const float tv = rok ? T[(int64_t)r * NE + m] : 0.0f;
      x[a] = cf{ev, tv};
      pe = __fmaf_rn(ev, ev, pe);
      pt = __fmaf_rn(tv, tv, pt);
    }
    ee = __fmaf_rn(w, pe, ee);
    tt = __fmaf_rn(w, pt, tt);
    DFT<P1, -1>::run(x);
#pragma unroll
    for (int c = 1; c < P1; ++c) x[c] = cmulc(x[c], rt[(j * c) % NE]);
#pragma unroll
    for (int c = 0; c < P1; ++c) yg[c * P2 + j] = x[c];
    __syncthreads();
    cf h[CPT][P2];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int c = j + P2 * i;
      if (c < P1) {
#pragma unroll
        for (int b = 0; b < P2; ++b) h[i][b] = yg[c * P2 + b];
        DFT<P2, -1>::run(h[i]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int c = j + P2 * i;
      if (c < P1) {
#pragma unroll
        for (int d = 0; d < P2; ++d) yg[c + P1 * d] = h[i][d];  // Z(c + P1 d)
      }
    }
    __syncthreads();
    for (int q = j; q < NQ; q += P2) {
      const cf zq = yg[q], zm = yg[(NE - q) % NE];
      const cf sq = cf{zq.x + zm.x, zq.y - zm.y};
      const cf dq = cf{zq.x - zm.x, zq.y + zm.y};
      const cf p = cmulc(sq, dq);
      pg[q] = cf{-0.25f * w * p.y, 0.25f * w * p.x};
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
      const int q = tid + 256 * i;
      if (q < NQ) {
        cf sum = pr[q];
        for (int g2 = 1; g2 < RG; ++g2) sum = cadd(sum, pr[g2 * NQ + q]);
        acc[i] = cadd(acc[i], sum);
      }
    }
    __syncthreads();
  }
  // A(q) into pr[0 .. NQ), then c(D) = (1/NE) [A(0) + (-1)^D A(NE/2) + 2 sum_q Re(A(q) e^{2 pi i q D / NE})]
#pragma unroll
  for (int i = 0; i < QPT; ++i) {
    const int q = tid + 256 * i;
    if (q < NQ) pr[q] = acc[i];
  }
  for (int off = 32; off > 0; off >>= 1) {
    ee += __shfl_xor(ee, off, 64);
    tt += __shfl_xor(tt, off, 64);
  }
  if ((tid & 63) == 0) {
    rsum[tid >> 6] = ee;
    rsum[4 + (tid >> 6)] = tt;
  }
  __syncthreads();
  for (int d = tid; d < NE; d += 256) {
    float v = 0.0f;
    for (int q = 1; q < NE / 2; ++q) {
      const cf e = rt[(q * d) % NE];
      v = __fmaf_rn(pr[q].x, e.x, __fmaf_rn(-pr[q].y, e.y, v));
    }
    cc[d] = (pr[0].x + ((d & 1) ? -pr[NE / 2].x : pr[NE / 2].x) + 2.0f * v) / (float)NE;
  }
  __syncthreads();
  const float norm = sqrtf((rsum[0] + rsum[1] + rsum[2] + rsum[3]) * (rsum[4] + rsum[5] + rsum[6] + rsum[7]));
  const float inv = norm > 0.0f ? 1.0f / norm : 0.0f;
  float bv = -INFINITY;
  int bi = 0x7fffffff;
  for (int d = tid; d < NE; d += 256) argmax_merge(bv, bi, cc[d] * inv, d);
  wave_argmax(bv, bi);
  if ((tid & 63) == 0) {
    rv[tid >> 6] = bv;
    ri[tid >> 6] = bi;
  }
  __syncthreads();
  for (int w = 0; w < 4; ++w) argmax_merge(bv, bi, rv[w], ri[w]);
  const int d_int = bi >= NE / 2 ? bi - NE : bi;
  for (int q = tid; q < NQ; q += 256) {
    cqr[q] = pr[q].x * inv;
    cqi[q] = pr[q].y * inv;
  }
  __syncthreads();
  eta_interpolate(cqr, cqi, NE, d_int, kappa, rv, ri, gamma + k);
}

hipError_t launch_eta_peak(const float* lp_e, const float* lp_t, int64_t k, int n_rho, int n_eta,
                           int kappa, double* gamma, hipStream_t stream) {
  if (k <= 0) return hipSuccess;
  if (n_eta > 1024 || n_rho < 2 || k > (int64_t(1) << 31) / 256) return hipErrorInvalidValue;
  // the default grids (n_eta = 2 N) through row transforms
#define EBSD_ETAF(NE)                                                                                         \
  do {                                                                                                        \
    constexpr int P2 = NE >= 512 ? 32 : 16, NQ = NE / 2 + 1;                                                  \
    const size_t shf = sizeof(cf) * ((size_t)(256 / P2) * (NE + NQ) + NE) + sizeof(float) * (NE + 2 * NQ);    \
    (void)hipFuncSetAttribute((const void*)k_eta_fft<NE>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shf); \
    hipLaunchKernelGGL(k_eta_fft<NE>, dim3((unsigned)k), dim3(256), shf, stream, lp_e, lp_t, n_rho, kappa, gamma); \
    return hipGetLastError();                                                                                 \
  } while (0)
  switch (n_eta) {
    case 128: EBSD_ETAF(128);
    case 192: EBSD_ETAF(192);
    case 256: EBSD_ETAF(256);
    case 320: EBSD_ETAF(320);
    case 512: EBSD_ETAF(512);
    default: break;
  }
#undef EBSD_ETAF
  const size_t shm = sizeof(float) * ((size_t)2 * 8 * n_eta + n_eta + 2 * (n_eta / 2 + 1));
  (void)hipFuncSetAttribute((const void*)k_eta_peak, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL(k_eta_peak, dim3((unsigned)k), dim3(256), shm, stream, lp_e, lp_t, n_rho, n_eta, kappa, gamma);
  return hipGetLastError();
}

hipError_t launch_update_xy(double* q, const float* s_sub, int64_t k, const double* pc_per, double pcz,
                            int n, hipStream_t stream, const double* beam_pc0) {
  if (k <= 0) return hipSuccess;
  const int beam = beam_pc0 != nullptr && pc_per != nullptr;
  hipLaunchKernelGGL(k_update_xy, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, stream, q, s_sub, k, pc_per,
                     pcz, n, beam, beam ? beam_pc0[0] : 0.0, beam ? beam_pc0[1] : 0.0);
  return hipGetLastError();
}

// Affine map-wide PC model, one point per thread: separately rounded
// products and sums (no fused multiply-add), in the order
// (pc0 + (col - col0) d_col) + (row - row0) d_row.
__global__ void k_pc_map(PcModel m, int64_t kk, double* __restrict__ out) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= kk) return;
  const int64_t row = i / m.width;
  const double a = (double)(i - row * m.width) - m.col0;
  const double b = (double)row - m.row0;
#pragma unroll
  for (int c = 0; c < 3; ++c) out[3 * i + c] = (m.pc0[c] + a * m.d_col[c]) + b * m.d_row[c];
}

// Capture-range test orientations: entry (r, a, k) = q_ref[r] (x) conj(q_a(theta_k))
// (orientation R Q^T for a detector-frame rotation Q about axis a = x, y, z),
// stored at ((r * 3 + a) * nt + k); ref_of holds r (the reference's index).
__global__ void k_capture_orient(const double* __restrict__ q_ref, int64_t nr, const double* __restrict__ theta_deg,
                                 int nt, double* __restrict__ q, int32_t* __restrict__ ref_of) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nr * 3 * nt) return;
  const int k = (int)(i % nt);
  const int a = (int)((i / nt) % 3);
  const int64_t r = i / (3 * (int64_t)nt);
  const double h = 0.5 * theta_deg[k] * (3.14159265358979323846 / 180.0);
  const double sh = sin(h);
  const double cq[4] = {cos(h), a == 0 ? -sh : 0.0, a == 1 ? -sh : 0.0, a == 2 ? -sh : 0.0};
  double o[4];
  qmul(q_ref + 4 * r, cq, o);
  qstore(q + 4 * i, o);
  ref_of[i] = (int32_t)r;
}

// Full width at half maximum of each sampled curve above its floor, one
// thread per curve: level = (largest + smallest sample) / 2; from the first
// maximum, walk outwards to the first sample below the level on each side
// and interpolate linearly; a side that stays above reports the end of the
// sampled range.
__global__ void k_fwhm(const float* __restrict__ h, int64_t nc, const double* __restrict__ t, int nt,
                       double* __restrict__ width) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nc) return;
  const float* c = h + i * nt;
  int k0 = 0;
  float lo = c[0];
  for (int k = 1; k < nt; ++k) {
    if (c[k] > c[k0]) k0 = k;
    lo = fminf(lo, c[k]);
  }
  const double level = 0.5 * ((double)c[k0] + (double)lo);
  double e[2];
  for (int side = 0; side < 2; ++side) {
    const int step = side ? 1 : -1;
    int k = k0;
    e[side] = t[k0];
    while (k + step >= 0 && k + step < nt) {
      const double a = c[k], b = c[k + step];
      if (b < level) {
        e[side] = t[k] + (t[k + step] - t[k]) * (a - level) / (a - b);
        break;
      }
      k += step;
      e[side] = t[k];
    }
  }
  width[i] = e[1] - e[0];
}

hipError_t launch_capture_orient(const double* q_ref, int64_t nr, const double* theta_deg, int nt, double* q,
                                 int32_t* ref_of, hipStream_t stream) {
  const int64_t k = nr * 3 * nt;
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_capture_orient, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, stream, q_ref, nr, theta_deg,
                     nt, q, ref_of);
  return hipGetLastError();
}

hipError_t launch_fwhm(const float* h, int64_t nc, const double* t, int nt, double* width, hipStream_t stream) {
  if (nc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fwhm, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, stream, h, nc, t, nt, width);
  return hipGetLastError();
}

hipError_t launch_pc_map(const PcModel& m, int64_t k, double* out, hipStream_t stream) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pc_map, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, stream, m, k, out);
  return hipGetLastError();
}

hipError_t launch_update_z(double* q, const double* gamma, int64_t k, hipStream_t stream) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_update_z, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, stream, q, gamma, k);
  return hipGetLastError();
}

}  // namespace ebsd

// Equispaced orientation library and nearest-neighbour disorientations
// (section "SO(3) Spacing", Equation 6, Figure 2).
//
// Library: an S^2 x S^1 grid over SO(3) (equidistant polar rings on the
// sphere with azimuths in proportion to each ring's circumference, the circle
// split linearly), each point the rotation Rz(phi) Ry(theta) Rz(psi - phi),
// reduced to the cubic fundamental zone.  One thread per grid point; one
// block then compacts the kept points in grid order.
//
// Nearest neighbours: all pairs, one thread per orientation, candidate
// orientations staged through LDS.  The largest |w| over the 24 cubic
// equivalents of a misorientation m comes in closed form from the sorted
// magnitudes a1 >= a2 >= a3 >= a4 of its components: the identity and the
// three 180-degree turns about <100> give a1, the 90-degree turns about
// <100> and the 180-degree turns about <110> give (a1 + a2) / sqrt 2, the
// 120-degree turns about <111> give (a1 + a2 + a3 + a4) / 2.
#include "ebsd_internal.hpp"

#include <hip/hip_runtime.h>

namespace ebsd {

namespace {

constexpr double kTieEps = 1e-12;
constexpr double kPi = 3.14159265358979323846;

// The 24 proper cubic rotations as quaternions (w >= 0), identity first:
// 180 deg about <100>, +-90 deg about <100>, +-120 deg about <111>, 180 deg
// about <110>.
struct CubicOps {
  double q[24][4];
};

__device__ __forceinline__ CubicOps cubic_ops() {
  const double c = 0.70710678118654752440, h = 0.5;
  return CubicOps{{{1, 0, 0, 0},   {0, 1, 0, 0},   {0, 0, 1, 0},   {0, 0, 0, 1},   {c, c, 0, 0},
                   {c, -c, 0, 0},  {c, 0, c, 0},   {c, 0, -c, 0},  {c, 0, 0, c},   {c, 0, 0, -c},
                   {h, h, h, h},   {h, h, h, -h},  {h, h, -h, h},  {h, h, -h, -h}, {h, -h, h, h},
                   {h, -h, h, -h}, {h, -h, -h, h}, {h, -h, -h, -h}, {0, c, c, 0},  {0, c, -c, 0},
                   {0, c, 0, c},   {0, c, 0, -c},  {0, 0, c, c},   {0, 0, c, -c}}};
}

__device__ __forceinline__ void hamilton(const double* a, const double* b, double* o) {
  o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

// Sign so that w > 0, or, at |w| <= eps, the first component beyond eps is
// positive.
__device__ __forceinline__ void canonicalise(double* q) {
  bool flip;
  if (fabs(q[0]) > kTieEps) {
    flip = q[0] < 0.0;
  } else {
    flip = false;
    for (int c = 1; c < 4; ++c)
      if (fabs(q[c]) > kTieEps) {
        flip = q[c] < 0.0;
        break;
      }
  }
  if (flip)
    for (int c = 0; c < 4; ++c) q[c] = -q[c];
}

// a <= b lexicographically, components equal within eps.
__device__ __forceinline__ bool key_le(const double* a, const double* b) {
  for (int c = 0; c < 4; ++c)
    if (fabs(a[c] - b[c]) > kTieEps) return a[c] < b[c];
  return true;
}

__global__ void k_so3_grid(const int64_t* __restrict__ ring_off, int m, int n_psi, int64_t n_all,
                           double* __restrict__ q_all, unsigned char* __restrict__ keep) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= n_all) return;
  const int k = (int)(g % n_psi);
  const int64_t a = g / n_psi;
  // ring i holds azimuth indices [ring_off[i], ring_off[i + 1])
  int lo = 0, hi = m;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ring_off[mid] <= a) lo = mid;
    else hi = mid - 1;
  }
  const int i = lo;
  const int64_t n_i = ring_off[i + 1] - ring_off[i];
  const double theta = kPi * i / m;
  const double phi = 2.0 * kPi * (double)(a - ring_off[i]) / (double)n_i;
  const double psi = 2.0 * kPi * k / n_psi;
  const double ct = cos(0.5 * theta), st = sin(0.5 * theta);
  double q[4] = {ct * cos(0.5 * psi), -st * sin(phi - 0.5 * psi), st * cos(phi - 0.5 * psi), ct * sin(0.5 * psi)};
  canonicalise(q);
  const CubicOps ops = cubic_ops();
  double w[24], best = 0.0;
  for (int s = 0; s < 24; ++s) {
    const double* o = ops.q[s];
    w[s] = fabs(o[0] * q[0] - o[1] * q[1] - o[2] * q[2] - o[3] * q[3]);
    best = fmax(best, w[s]);
  }
  bool in = w[0] >= best - kTieEps;
  for (int s = 1; s < 24 && in; ++s) {
    if (w[s] < best - kTieEps) continue;
    double e[4];
    hamilton(ops.q[s], q, e);
    canonicalise(e);
    in = key_le(q, e);
  }
  for (int c = 0; c < 4; ++c) q_all[4 * g + c] = q[c];
  keep[g] = in ? 1 : 0;
}

// One block of 1024 threads walks the flags in order, 1024 at a time: a
// block-wide exclusive scan gives each kept point its output slot.  Points
// beyond cap are counted, not written.
__global__ __launch_bounds__(1024) void k_so3_compact(const double* __restrict__ q_all,
                                                      const unsigned char* __restrict__ keep, int64_t n_all,
                                                      double* __restrict__ q_out, int64_t cap,
                                                      int64_t* __restrict__ count) {
  __shared__ int wave_sum[16];
  __shared__ int64_t base;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) base = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < n_all; c0 += 1024) {
    const int64_t g = c0 + tid;
    const int f = g < n_all ? keep[g] : 0;
    const unsigned long long bal = __ballot(f);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wave_sum[wv] = __popcll(bal);
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      off += w < wv ? wave_sum[w] : 0;
      tot += wave_sum[w];
    }
    const int64_t slot = base + off + before;
    if (f && slot < cap)
      for (int c = 0; c < 4; ++c) q_out[4 * slot + c] = q_all[4 * g + c];
    __syncthreads();
    if (tid == 0) base += tot;
    __syncthreads();
  }
  if (tid == 0) *count = base;
}

// Largest |w| over the 24 cubic equivalents of the misorientation m.
__device__ __forceinline__ double cubic_max_w(const double* m) {
  double a1 = fabs(m[0]), a2 = fabs(m[1]), a3 = fabs(m[2]), a4 = fabs(m[3]);
  // sort descending (a 4-element network)
  double t;
#define EBSD_CSWAP(x, y) \
  if (x < y) {           \
    t = x;               \
    x = y;               \
    y = t;               \
  }
  EBSD_CSWAP(a1, a2) EBSD_CSWAP(a3, a4) EBSD_CSWAP(a1, a3) EBSD_CSWAP(a2, a4) EBSD_CSWAP(a2, a3)
#undef EBSD_CSWAP
  return fmax(a1, fmax((a1 + a2) * 0.70710678118654752440, 0.5 * (a1 + a2 + a3 + a4)));
}

// Each thread owns orientation a; disorientation to b is 2 acos(max |w| of
// the cubic equivalents of q_b (x) conj(q_a)); the largest max |w| wins,
// ties to the smaller index.
__global__ __launch_bounds__(256) void k_nn_disorientation(const double* __restrict__ q, int64_t n,
                                                           double* __restrict__ nn_deg,
                                                           int32_t* __restrict__ nn_idx) {
  __shared__ double tile[256][4];
  const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double qa[4] = {1, 0, 0, 0};
  if (a < n)
    for (int c = 0; c < 4; ++c) qa[c] = q[4 * a + c];
  const double ca[4] = {qa[0], -qa[1], -qa[2], -qa[3]};
  double best = -1.0;
  int64_t bi = -1;
  for (int64_t t0 = 0; t0 < n; t0 += 256) {
    const int64_t b = t0 + threadIdx.x;
    for (int c = 0; c < 4; ++c) tile[threadIdx.x][c] = b < n ? q[4 * b + c] : 0.0;
    __syncthreads();
    const int cnt = n - t0 < 256 ? (int)(n - t0) : 256;
    for (int j = 0; j < cnt; ++j) {
      double mq[4];
      hamilton(tile[j], ca, mq);
      const double f = cubic_max_w(mq);
      if (t0 + j != a && f > best) {
        best = f;
        bi = t0 + j;
      }
    }
    __syncthreads();
  }
  if (a < n) {
    nn_deg[a] = 2.0 * acos(fmin(1.0, best)) * (180.0 / kPi);
    nn_idx[a] = (int32_t)bi;
  }
}

}  // namespace

hipError_t launch_so3_library(const int64_t* ring_off, int m, int n_psi, int64_t n_all, double* q_all,
                              unsigned char* keep, double* q_out, int64_t cap, int64_t* count, hipStream_t stream) {
  if (n_all <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_so3_grid, dim3((unsigned)((n_all + 255) / 256)), dim3(256), 0, stream, ring_off, m, n_psi,
                     n_all, q_all, keep);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_so3_compact, dim3(1), dim3(1024), 0, stream, q_all, keep, n_all, q_out, cap, count);
  return hipGetLastError();
}

hipError_t launch_nn_disorientation(const double* q, int64_t n, double* nn_deg, int32_t* nn_idx,
                                    hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nn_disorientation, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, q, n, nn_deg,
                     nn_idx);
  return hipGetLastError();
}

}  // namespace ebsd

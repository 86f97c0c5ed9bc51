// Filtered spectra and cross-correlation kernels (gfx950).
//
// Spectra (sections "Fast Fourier Transform" and "SO(3) Sampling Frequency"):
// contrast normalisation, separable Hann window, forward 2-D DFT (Equation 4,
// unnormalised), band-pass H(rho) = (1 - exp(-rho^2 / 2 s_hp^2)) exp(-rho^2 / 2 s_lp^2)
// cut to zero beyond rho_max, FP64 energy, unit-energy scaling.
//
// Correlation (Equations 2, 3 and the spatial definition of r_fg, normalised
// by the autocorrelations): rho(s) = sum_u E(u) conj(T(u)) exp(+2 pi i u.s / N)
// for unit-energy spectra, evaluated on every cyclic shift by an inverse 2-D
// DFT that only touches the non-zero band, then reduced to its peak.
//
// Stored spectrum layout (band layout): complex64 S[kk][v], kk in [0, 2B + 1)
// with u = kk for kk <= B and u = kk - (2B + 1) otherwise (rows), v in [0, B]
// (the Hermitian half along columns, contiguous); B = 3N/8, outside of which
// the filter is zero.
//
// Every 1-D transform of length N = R1 * R2 is done in two in-register passes
// (radix R1, twiddle, radix R2) with one exchange through LDS in between;
// the 2-D inverse transform runs the column pass on the B + 1 non-zero
// columns only, and the row pass on pairs of rows packed as one complex
// transform (both rows' outputs are real).
#include "ebsd_common.hpp"
#include "ebsd_internal.hpp"

#include <math.h>

namespace ebsd {

template <int N>
struct Lay {
  static constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2, B = Plan<N>::B;
  static constexpr int NV = B + 1, NK = 2 * B + 1;
  static constexpr int SPEC = NV * NK;
  // padded strides (in complex elements) of the LDS exchange layouts
  static constexpr int XS = N + 4;   // [v][c][b]  column-pass exchange
  static constexpr int AS = NV + 1;  // [y][v]     column-pass output
  static constexpr int YS = N + 4;   // [q][c][b]  row-pass exchange
  static constexpr int ZS = N + 2;   // [q][v]     forward row-pass output
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  static constexpr int LDS = cmax(cmax(NV * XS, N * AS), cmax((N / 2) * YS, (N / 2) * ZS));
};

__device__ __forceinline__ int signed_shift(int k, int n) { return k >= n / 2 ? k - n : k; }

// exp(+2 pi i k / N), k in [0, N), into LDS (FP64 evaluation, rounded)
template <int N, int NT>
__device__ __forceinline__ void load_roots(cf* tw, int tid) {
  for (int k = tid; k < N; k += NT) {
    double s, c;
    sincospi(2.0 * (double)k / (double)N, &s, &c);
    tw[k] = cf{(float)c, (float)s};
  }
}

// ---------------------------------------------------------------------------
// Inverse 2-D transform of Z = E conj(T) over the band, calling epi(y, x, rho)
// for every shift (y = s_y mod N, x = s_x mod N).
template <int N, int NT, class Epi>
__device__ __forceinline__ void xcf_core(const cf* __restrict__ E, const cf* __restrict__ T,
                                         cf* lds, const cf* tw, int tid, Epi& epi) {
  using L = Lay<N>;
  constexpr int R1 = L::R1, R2 = L::R2, B = L::B, NV = L::NV, NK = L::NK;

  // column pass, radix R1 over u = R2 a + b, for every (v, b)
  constexpr int T1 = NV * R2;
  for (int t = tid; t < T1; t += NT) {
    const int v = t / R2, b = t - v * R2;
    cf x[R1];
#pragma unroll
    for (int a = 0; a < R1; ++a) {
      const int u = R2 * a + b;
      const int kk = u <= B ? u : (u >= N - B ? u - N + NK : -1);
      if (kk >= 0) {
        x[a] = cmulc(E[kk * NV + v], T[kk * NV + v]);
      } else {
        x[a] = cf{0.f, 0.f};
      }
    }
    DFT<R1, 1>::run(x);
#pragma unroll
    for (int c = 1; c < R1; ++c) x[c] = cmul(x[c], tw[b * c]);
#pragma unroll
    for (int c = 0; c < R1; ++c) lds[v * L::XS + c * R2 + b] = x[c];
  }
  __syncthreads();

  // column pass, radix R2 over b, for every (v, c): A(y = c + R1 d, v)
  constexpr int T2 = NV * R1, J2 = (T2 + NT - 1) / NT;
  cf h2[J2][R2];
#pragma unroll
  for (int j = 0; j < J2; ++j) {
    const int t = tid + j * NT;
    if (t < T2) {
      const int v = t / R1, c = t - v * R1;
#pragma unroll
      for (int b = 0; b < R2; ++b) h2[j][b] = lds[v * L::XS + c * R2 + b];
      DFT<R2, 1>::run(h2[j]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < J2; ++j) {
    const int t = tid + j * NT;
    if (t < T2) {
      const int v = t / R1, c = t - v * R1;
#pragma unroll
      for (int d = 0; d < R2; ++d) lds[(c + R1 * d) * L::AS + v] = h2[j][d];
    }
  }
  __syncthreads();

  // row pass on row pairs (q, q + N/2): S(v) = H_q(v) + i H_{q+N/2}(v) with the
  // Hermitian extension H_y(N - w) = conj(A(y, w)); radix R1 over v = R2 a + b
  constexpr int T3 = (N / 2) * R2, J3 = (T3 + NT - 1) / NT;
  cf h3[J3][R1];
#pragma unroll
  for (int j = 0; j < J3; ++j) {
    const int t = tid + j * NT;
    if (t < T3) {
      const int q = t / R2, b = t - q * R2;
#pragma unroll
      for (int a = 0; a < R1; ++a) {
        const int v = R2 * a + b;
        cf s = cf{0.f, 0.f};
        if (v == 0) {
          s = cf{lds[q * L::AS].x, lds[(q + N / 2) * L::AS].x};
        } else if (v <= B) {
          const cf p0 = lds[q * L::AS + v], p1 = lds[(q + N / 2) * L::AS + v];
          s = cf{p0.x - p1.y, p0.y + p1.x};
        } else if (v >= N - B) {
          const int w = N - v;
          const cf p0 = lds[q * L::AS + w], p1 = lds[(q + N / 2) * L::AS + w];
          s = cf{p0.x + p1.y, p1.x - p0.y};
        }
        h3[j][a] = s;
      }
      DFT<R1, 1>::run(h3[j]);
#pragma unroll
      for (int c = 1; c < R1; ++c) h3[j][c] = cmul(h3[j][c], tw[b * c]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < J3; ++j) {
    const int t = tid + j * NT;
    if (t < T3) {
      const int q = t / R2, b = t - q * R2;
#pragma unroll
      for (int c = 0; c < R1; ++c) lds[q * L::YS + c * R2 + b] = h3[j][c];
    }
  }
  __syncthreads();

  // row pass, radix R2: outputs x = c + R1 d; real part row q, imaginary part row q + N/2
  constexpr int T4 = (N / 2) * R1;
  for (int t = tid; t < T4; t += NT) {
    const int q = t / R1, c = t - q * R1;
    cf z[R2];
#pragma unroll
    for (int b = 0; b < R2; ++b) z[b] = lds[q * L::YS + c * R2 + b];
    DFT<R2, 1>::run(z);
#pragma unroll
    for (int d = 0; d < R2; ++d) {
      const int x = c + R1 * d;
      epi(q, x, z[d].x);
      epi(q + N / 2, x, z[d].y);
    }
  }
}

struct ArgmaxEpi {
  float m;
  int i, n, s;
  float* map;
  __device__ __forceinline__ void operator()(int y, int x, float v) {
    if (map) map[y * n + x] = v;
    if (s < 0 || (abs(signed_shift(y, n)) <= s && abs(signed_shift(x, n)) <= s))
      argmax_merge(m, i, v, y * n + x);
  }
};

template <int N, int NT>
__global__ __launch_bounds__(NT) void k_xcf_peak(const cf* __restrict__ spec_p, const cf* __restrict__ spec_l,
                                                 const int32_t* __restrict__ pi, const int32_t* __restrict__ li,
                                                 int max_shift, float* __restrict__ h_int,
                                                 int32_t* __restrict__ s_int, float* __restrict__ map) {
  using L = Lay<N>;
  __shared__ cf lds[L::LDS];
  __shared__ cf tw[N];
  __shared__ float redv[NT / 64];
  __shared__ int redi[NT / 64];
  const int tid = threadIdx.x;
  const int64_t k = blockIdx.x;
  load_roots<N, NT>(tw, tid);
  __syncthreads();
  ArgmaxEpi epi{-INFINITY, 0x7fffffff, N, max_shift, map ? map + k * N * N : nullptr};
  const int64_t ip = pi ? pi[k] : k, il = li ? li[k] : k;
  xcf_core<N, NT>(spec_p + ip * L::SPEC, spec_l + il * L::SPEC, lds, tw, tid, epi);
  float m = epi.m;
  int i = epi.i;
  wave_argmax(m, i);
  if ((tid & 63) == 0) {
    redv[tid >> 6] = m;
    redi[tid >> 6] = i;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < NT / 64; ++w) argmax_merge(m, i, redv[w], redi[w]);
    h_int[k] = m;
    if (i < 0 || i >= N * N) i = 0;  // every value NaN: report shift 0
    const int sy = i / N, sx = i - sy * N;
    s_int[2 * k] = signed_shift(sx, N);
    s_int[2 * k + 1] = signed_shift(sy, N);
  }
}

// ---------------------------------------------------------------------------
// Search kernel for N = 128 (R1 = 16, R2 = 8, B = 48), 8 waves per block.
// Every phase gives each wave one radix position, so the band tests, the
// spectrum row indices and the inter-pass twiddles are wave-uniform (scalar),
// and lanes run along the spectrum column v or the row pair q, so every LDS
// access is lane-contiguous.  The pattern's spectrum stays in registers
// while the block streams its chunk of templates.
//   phase 1  wave b, lane v:  radix 16 over u = 8a + b of E conj(T), twiddle
//   phase 2  wave c, lane v:  radix 8 over b -> A(y = c + 16 d, v)
//   phase 3  wave b, lane q:  radix 16 over v = 8a + b of the packed row pair
//                             (q, q + 64), twiddle
//   phase 4  wave c, lane q:  radix 8 over b -> rho(row q and q + 64, x = c + 16 d)
// Raw buffer view of one spectrum (gfx9 descriptor word 3: 32-bit data
// format, no stride; reads past the byte count return zero): a load then
// takes its lane offset in one VGPR and its uniform row offset in an SGPR,
// with no per-load address arithmetic.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t spectrum_rsrc(const cf* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<cf*>(p), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ cf buffer_cf(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
  return __builtin_bit_cast(cf, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <int N>
struct RootTable {
  cf w[N];
  constexpr RootTable() : w() {
    for (int k = 0; k < N; ++k) {
      w[k].x = (float)cx::cos2pi(k, N);
      w[k].y = (float)cx::sin2pi(k, N);
    }
  }
};
__constant__ RootTable<128> c_roots128 = RootTable<128>();

// CAND: template l of pattern p is spec_l[cand[p nl + l]] (a list of nl
// candidates per pattern, as the learned proposal makes; indices clamped to
// [0, lib_n)) instead of spec_l[l]
template <bool WINDOW, bool PERSIST, bool CAND = false>
__global__ __launch_bounds__(512, 4) void k_xcf_scores128(const cf* __restrict__ spec_p, int64_t np,
                                                          const cf* __restrict__ spec_l, int64_t nl,
                                                          int lchunk, int64_t nblk, int max_shift,
                                                          float* __restrict__ scores, int* __restrict__ queue,
                                                          const int32_t* __restrict__ cand = nullptr,
                                                          int64_t lib_n = 0) {
  constexpr int N = 128, R1 = 16, R2 = 8, B = 48, NV = 49;
  constexpr int SPEC = NV * (2 * B + 1);
  constexpr int GAP = band_gap_mask<N, R1, R2, B>();  // a = 7, 8, 9
  static_assert(GAP == 0x380, "band gap of the 128 plan");
  constexpr int AV = N + 1;  // A[v][y] row stride (odd: the phase-2 writes spread over banks)
  // X [c][b][v] (R1*R2*NV), A [v][y] (NV*AV), Y [c][b][q] (R1*R2*64) share one buffer
  constexpr int LDSN = (R1 * R2 * 64 > NV * AV) ? R1 * R2 * 64 : NV * AV;
  __shared__ cf lds[LDSN];
  static_assert((R1 * R2 - 1) * NV + 63 < LDSN, "phase-2 reads of lanes past the band stay in LDS");
  __shared__ float red[8];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  __shared__ int item;
  int64_t g;
  if constexpr (PERSIST) {
    if (tid == 0) item = atomicAdd(queue, 1);
    __syncthreads();
    g = item;
  } else {
    const int64_t per = (nblk + 7) / 8;
    g = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  }
  if (g >= nblk) return;
  const bool vlane = lane < NV;

  // inter-pass twiddles w^(wave c), c = 1..15: the same set in phases 1 and 3
  cf tw[R1];
#pragma unroll
  for (int c = 0; c < R1; ++c) tw[c] = c_roots128.w[(wave * c) & (N - 1)];

  while (g < nblk) {
  const int64_t chunk = g / np, p = g - chunk * np;
  // pattern spectrum values used by this lane in phase 1
  const cf* E = spec_p + p * SPEC;
  cf ev[R1];
#pragma unroll
  for (int a = 0; a < R1; ++a) {
    const int u = R2 * a + wave;
    const int kk = u <= B ? u : (u >= N - B ? u - N + 2 * B + 1 : -1);
    ev[a] = (kk >= 0 && vlane) ? E[kk * NV + lane] : cf{0.f, 0.f};
  }

  const int64_t l0 = chunk * lchunk;
  const int64_t l1 = l0 + lchunk < nl ? l0 + lchunk : nl;
  for (int64_t l = l0; l < l1; ++l) {
    int64_t tl = l;
    if constexpr (CAND) {
      tl = cand[p * nl + l];
      tl = tl < 0 ? 0 : (tl >= lib_n ? lib_n - 1 : tl);
    }
    const cf* T = spec_l + tl * SPEC;
    // phase 1 (ev is zero outside the band, so every lane loads from a
    // clamped in-band address without a branch and the product stays zero:
    // the loads are in flight together).  Wave 0 (b = 0) has unit twiddles
    // and compile-time rows; for the other waves input a = 6 (u = 48 + b) is
    // past the band edge too, so it is neither loaded nor added
    const auto phase1 = [&](auto w0c) {
      constexpr bool W0 = decltype(w0c)::value;
      constexpr int G1 = W0 ? GAP : (GAP | 0x40);
      const int b = W0 ? 0 : wave;
      cf x[R1];
      // buffer loads: one lane offset, uniform row offsets, no per-row VGPRs
      const unsigned voff = (unsigned)(vlane ? lane : NV - 1) * (unsigned)sizeof(cf);
      const __amdgpu_buffer_rsrc_t Tr = spectrum_rsrc(T, SPEC * (int)sizeof(cf));
#pragma unroll
      for (int a = 0; a < R1; ++a) {
        if ((G1 >> a) & 1) continue;
        const int u = R2 * a + b;
        const int kk = u <= B ? u : (u >= N - B ? u - N + 2 * B + 1 : 0);
        x[a] = buffer_cf(Tr, voff, kk * NV * (int)sizeof(cf));
      }
#pragma unroll
      for (int a = 0; a < R1; ++a)
        if (!((G1 >> a) & 1)) x[a] = cmulc(ev[a], x[a]);
      dft_zero<R1, 1, G1>(x);
      if constexpr (!W0) {
#pragma unroll
        for (int c = 1; c < R1; ++c) x[c] = cmul(x[c], tw[c]);
      }
      if (vlane) {
#pragma unroll
        for (int c = 0; c < R1; ++c) lds[(c * R2 + b) * NV + lane] = x[c];
      }
    };
    if (wave == 0) phase1(std::true_type{});
    else phase1(std::false_type{});
    __syncthreads();
    // phase 2: waves take c = wave and c = wave + 8
    cf h[2][R2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = wave + 8 * j;
#pragma unroll
      for (int b = 0; b < R2; ++b) h[j][b] = lds[(c * R2 + b) * NV + lane];  // lanes >= NV: in-bounds, never stored
      DFT<R2, 1>::run(h[j]);
    }
    __syncthreads();
    if (vlane) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int c = wave + 8 * j;
#pragma unroll
        for (int d = 0; d < R2; ++d) lds[lane * AV + c + R1 * d] = h[j][d];
      }
    }
    __syncthreads();
    // phase 3: wave b, lane q: packed rows q and q + 64
    // S(v) = A(q, v) + i A(q + 64, v) for 0 < v <= B, conj(A(q, N - v)) +
    // i conj(A(q + 64, N - v)) for v >= N - B, (A(q, 0).x, A(q + 64, 0).x)
    // at v = 0 and 0 in the gap: every row is read (clamped, no branch, so the
    // reads are in flight together) and the cases are uniform coefficients
    // c = +-1 or 0 (fma(c, y, x) = x + c y exactly)
    // (as in phase 1, wave 0 has unit twiddles and compile-time rows, and
    // for the other waves v = 48 + b is past the band edge)
    cf s[R1];
    const auto phase3 = [&](auto w0c) {
      constexpr bool W0 = decltype(w0c)::value;
      constexpr int G3 = W0 ? GAP : (GAP | 0x40);
      const int b = W0 ? 0 : wave;
      cf p0[R1], p1[R1];
      static_for<0, R1>([&](auto ai) {
        constexpr int a = decltype(ai)::value;
        if constexpr (!((G3 >> a) & 1)) {
          const int v = R2 * a + b;
          const int w = v <= B ? v : (v >= N - B ? N - v : 0);
          p0[a] = lds[w * AV + lane];
          p1[a] = lds[w * AV + lane + 64];
        }
      });
      static_for<0, R1>([&](auto ai) {
        constexpr int a = decltype(ai)::value;
        if constexpr (!((G3 >> a) & 1)) {
          const int v = R2 * a + b;
          const float c = v == 0 ? 0.f : (v >= N - B ? -1.f : 1.f);
          s[a] = cf{__fmaf_rn(-c, p1[a].y, p0[a].x), __fmaf_rn(c, p0[a].y, p1[a].x)};
        }
      });
      dft_zero<R1, 1, G3>(s);  // v = 8 a + b in the gap for a = 7, 8, 9 (and 6 for b > 0)
      if constexpr (!W0) {
#pragma unroll
        for (int c = 1; c < R1; ++c) s[c] = cmul(s[c], tw[c]);
      }
    };
    if (wave == 0) phase3(std::true_type{});
    else phase3(std::false_type{});
    __syncthreads();
#pragma unroll
    for (int c = 0; c < R1; ++c) lds[(c * R2 + wave) * 64 + lane] = s[c];
    __syncthreads();
    // phase 4: waves take c = wave and c = wave + 8; outputs x = c + 16 d
    float m = -INFINITY;
    const float mq0 = abs(signed_shift(lane, N)) <= max_shift ? 0.f : -INFINITY;
    const float mq1 = abs(signed_shift(lane + 64, N)) <= max_shift ? 0.f : -INFINITY;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = wave + 8 * j;
      cf z[R2];
#pragma unroll
      for (int b = 0; b < R2; ++b) z[b] = lds[(c * R2 + b) * 64 + lane];
      DFT<R2, 1>::run(z);
#pragma unroll
      for (int d = 0; d < R2; ++d) {
        if constexpr (WINDOW) {
          // the column test is uniform; the rows of this lane enter through
          // additive 0 / -inf masks (exact)
          const int x = c + R1 * d;
          if (abs(signed_shift(x, N)) <= max_shift) m = fmaxf(fmaxf(m, z[d].x + mq0), z[d].y + mq1);
        } else {
          m = fmaxf(fmaxf(m, z[d].x), z[d].y);  // one three-input maximum per output pair
        }
      }
    }
    m = wave_max(m);
    if (lane == 0) red[wave] = m;
    __syncthreads();
    if (tid == 0) {
      float r = red[0];
#pragma unroll
      for (int w = 1; w < 8; ++w) r = fmaxf(r, red[w]);
      scores[p * nl + l] = r;
    }
  }
  if constexpr (!PERSIST) break;
  __syncthreads();
  if (tid == 0) item = atomicAdd(queue, 1);
  __syncthreads();
  g = item;
  }
}

// ---------------------------------------------------------------------------
// The same wave-uniform search for N = R1 x R2 with R2 waves per block
// (64 = 8 x 8, 96 = 12 x 8, 160 = 10 x 16: sixteen small-radix waves beat
// ten radix-16 ones, whose registers allow only 2.5 waves per SIMD).  Phases 1-2 run the column
// transform with lanes along v (B + 1 <= 64 lanes); phases 3-4 run the row
// transform on row pairs (q, q + N/2) packed as one complex transform, with
// lanes along q in blocks of QB rows; where R1 is not a multiple of R2 the
// waves past R1 idle in the second radix pass.
__constant__ RootTable<64> c_roots64 = RootTable<64>();
__constant__ RootTable<96> c_roots96 = RootTable<96>();
__constant__ RootTable<160> c_roots160 = RootTable<160>();

template <int N>
__device__ __forceinline__ cf root_of(int k) {
  if constexpr (N == 64) return c_roots64.w[k];
  else if constexpr (N == 96) return c_roots96.w[k];
  else if constexpr (N == 128) return c_roots128.w[k];
  else return c_roots160.w[k];
}

#ifndef EBSD_SEARCHW_MINW64
#define EBSD_SEARCHW_MINW64 6
#endif
#ifndef EBSD_SEARCHW_T160
#define EBSD_SEARCHW_T160 1
#endif
template <int N>
struct WLay {
  static constexpr int R1 = N == 64 ? 8 : (N == 96 ? 12 : (N == 160 && EBSD_SEARCHW_T160 ? 10 : 16));
  static constexpr int R2 = N == 160 ? (EBSD_SEARCHW_T160 ? 16 : 10) : 8;
  static constexpr int B = Plan<N>::B, NV = B + 1, NK = 2 * B + 1, SPEC = NV * NK;
  static constexpr int NQ = N / 2;                      // packed row pairs
  static constexpr int QB = N == 160 ? 40 : NQ;         // rows per lane block
  static constexpr int NQB = (NQ + QB - 1) / QB;
  static constexpr int JC = (R1 + R2 - 1) / R2;         // second-pass radix positions per wave
  static constexpr int AV = N + 1;                      // A[v][y] row stride
  static constexpr int XN = R1 * R2 * NV, AN = NV * AV, YN = R1 * R2 * QB;
  // SEPA: A sits after X, so the second column pass writes each radix
  // position as soon as it is done and Y reuses X (used at 160, where X + A
  // fit in LDS and several row blocks read A again); otherwise A and Y
  // overwrite X and A in turn, after barriers
  static constexpr bool SEPA = N == 160;
  static constexpr int AOFF = SEPA ? XN : 0;
  static constexpr int YOFF = SEPA ? 0 : (NQB > 1 ? AN : 0);
  static constexpr int cmx(int a, int b) { return a > b ? a : b; }
  // templates per wave: at 64 the band columns (25) and packed row pairs
  // (32) of one template fill half a wave, so each 32-lane half takes its
  // own template, with its own LDS region
  static constexpr int TPW = N == 64 ? 2 : 1;
  static constexpr int SUB = 64 / TPW;                  // lanes per template
  static constexpr int LDSH = cmx(cmx(XN, AOFF + AN), YOFF + YN);
  static constexpr int LDSN = LDSH * TPW;
  static_assert(NV <= SUB && QB <= SUB, "a template's columns and row block fit its lanes");
  static constexpr int NT = R2 * 64;
  // waves per SIMD the register allocation must allow (occupancy beats the
  // few spills it costs): two 8-wave blocks per CU at 96 (128 VGPRs), at 64
  // as many as EBSD_SEARCHW_MINW64 asks; at 160 LDS allows one block
  static constexpr int MINW = N == 96 ? 4 : (N == 64 ? EBSD_SEARCHW_MINW64 : 1);
  // first-pass inputs a zero for every wave (u or v = R2 a + b between the
  // band edges): a = 4 at 64, 5 and 6 at 96, 7 to 9 at 128, 4 and 5 at 160;
  // skipped where the first radix splits as 4 x Q (not at 160, radix 10)
  static constexpr int GAP = band_gap_mask<N, R1, R2, B>();
  static constexpr bool ZGAP = R1 % 4 == 0 && R1 > 4;
  // template loads as raw buffer loads (measured: 1.03x at 64, neutral at
  // 160, 0.93x at 96, where the global-load form schedules better)
  static constexpr bool BUFLOAD = N != 96;
};

template <int N, bool WINDOW, bool PERSIST>
__global__ __launch_bounds__(WLay<N>::NT, WLay<N>::MINW) void k_xcf_scoresw(const cf* __restrict__ spec_p, int64_t np,
                                                             const cf* __restrict__ spec_l, int64_t nl, int lchunk,
                                                             int64_t nblk, int max_shift, float* __restrict__ scores,
                                                             int* __restrict__ queue) {
  using L = WLay<N>;
  constexpr int R1 = L::R1, R2 = L::R2, B = L::B, NV = L::NV, SPEC = L::SPEC, AV = L::AV;
  constexpr int NQ = L::NQ, QB = L::QB, NQB = L::NQB, JC = L::JC;
  constexpr int TPW = L::TPW, SUB = L::SUB;
  __shared__ cf lds[L::LDSN];
  static_assert((R1 * R2 - 1) * NV + SUB - 1 < L::LDSH, "phase-2 reads of lanes past the band stay in LDS");
  __shared__ float red[R2 * TPW];
  __shared__ int item;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // this lane's template (half of the wave at TPW = 2), lane within it, and
  // the template's LDS region
  const int half = TPW == 2 ? lane / SUB : 0;
  const int sl = TPW == 2 ? lane - half * SUB : lane;
  cf* const lt = lds + half * L::LDSH;
  int64_t g;
  if constexpr (PERSIST) {
    if (tid == 0) item = atomicAdd(queue, 1);
    __syncthreads();
    g = item;
  } else {
    const int64_t per = (nblk + 7) / 8;
    g = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  }
  if (g >= nblk) return;
  const bool vlane = sl < NV;

  while (g < nblk) {
    const int64_t chunk = g / np, p = g - chunk * np;
    const cf* E = spec_p + p * SPEC;
    // the pattern's phase-1 values, held in registers across the template loop
    cf ev[R1];
#pragma unroll
    for (int a = 0; a < R1; ++a) {
      const int u = R2 * a + wave;
      const int kk = u <= B ? u : (u >= N - B ? u - N + 2 * B + 1 : -1);
      ev[a] = (kk >= 0 && vlane) ? E[kk * NV + sl] : cf{0.f, 0.f};
    }
    const int64_t l0 = chunk * lchunk;
    const int64_t l1 = l0 + lchunk < nl ? l0 + lchunk : nl;
    for (int64_t l = l0; l < l1; l += TPW) {
      // at TPW = 2 the halves take templates l and l + 1; past the end of the
      // chunk both take l (the second result is not written)
      const bool two = TPW == 2 && l + 1 < l1;
      const int th = two ? half : 0;
      const cf* T = spec_l + l * SPEC;
      // phase 1: wave b, lane v: radix R1 over u = R2 a + b, twiddle.  The
      // cached pattern values are zero outside the band, so every lane loads
      // its template values from a clamped in-band address without a branch
      // (all R1 loads in flight together) and the products stay zero there
      {
        cf x[R1];
        const unsigned voff = (unsigned)(th * SPEC + (vlane ? sl : NV - 1)) * (unsigned)sizeof(cf);
        const __amdgpu_buffer_rsrc_t Tr = spectrum_rsrc(T, (two ? 2 : 1) * SPEC * (int)sizeof(cf));
#pragma unroll
        for (int a = 0; a < R1; ++a) {
          if (L::ZGAP && ((L::GAP >> a) & 1)) continue;  // neither loaded nor added
          const int u = R2 * a + wave;
          const int kk = u <= B ? u : (u >= N - B ? u - N + 2 * B + 1 : 0);
          if constexpr (L::BUFLOAD) x[a] = buffer_cf(Tr, voff, kk * NV * (int)sizeof(cf));
          else x[a] = *reinterpret_cast<const cf*>(reinterpret_cast<const char*>(T + kk * NV) + voff);
        }
#pragma unroll
        for (int a = 0; a < R1; ++a)
          if (!(L::ZGAP && ((L::GAP >> a) & 1))) x[a] = cmulc(ev[a], x[a]);
        if constexpr (L::ZGAP) dft_zero<R1, 1, L::GAP>(x);
        else DFT<R1, 1>::run(x);
#pragma unroll
        for (int c = 1; c < R1; ++c) x[c] = cmul(x[c], root_of<N>((wave * c) % N));
        if (vlane) {
#pragma unroll
          for (int c = 0; c < R1; ++c) lt[(c * R2 + wave) * NV + sl] = x[c];
        }
      }
      __syncthreads();
      // phase 2: wave takes c = wave + R2 j: radix R2 over b -> A(y = c + R1 d, v)
      if constexpr (L::SEPA) {
#pragma unroll
        for (int j = 0; j < JC; ++j) {
          const int c = wave + R2 * j;
          if (c < R1) {
            cf h[R2];
#pragma unroll
            for (int b = 0; b < R2; ++b) h[b] = lt[(c * R2 + b) * NV + sl];  // lanes >= NV: never stored
            DFT<R2, 1>::run(h);
            if (vlane) {
#pragma unroll
              for (int d = 0; d < R2; ++d) lt[L::AOFF + sl * AV + c + R1 * d] = h[d];
            }
          }
        }
      } else {
        cf h[JC][R2];
#pragma unroll
        for (int j = 0; j < JC; ++j) {
          const int c = wave + R2 * j;
          if (c < R1) {
#pragma unroll
            for (int b = 0; b < R2; ++b) h[j][b] = lt[(c * R2 + b) * NV + sl];  // lanes >= NV: in-bounds, never stored
            DFT<R2, 1>::run(h[j]);
          }
        }
        __syncthreads();
        if (vlane) {
#pragma unroll
          for (int j = 0; j < JC; ++j) {
            const int c = wave + R2 * j;
            if (c < R1) {
#pragma unroll
              for (int d = 0; d < R2; ++d) lt[sl * AV + c + R1 * d] = h[j][d];
            }
          }
        }
      }
      __syncthreads();
      const cf* A = lt + L::AOFF;
      float m = -INFINITY;
#pragma unroll
      for (int qb = 0; qb < NQB; ++qb) {
        const int q = qb * QB + sl;
        const bool qlane = sl < QB && q < NQ;
        const float mq0 = abs(signed_shift(q, N)) <= max_shift ? 0.f : -INFINITY;
        const float mq1 = abs(signed_shift(q + NQ, N)) <= max_shift ? 0.f : -INFINITY;
        // phase 3: wave b, lane q: radix R1 over v = R2 a + b of the packed rows (q, q + N/2)
        cf sv[R1];
#pragma unroll
        for (int a = 0; a < R1; ++a) {
          const int v = R2 * a + wave;
          if (!qlane) {
            sv[a] = cf{0.f, 0.f};
          } else if (v == 0) {
            sv[a] = cf{A[q].x, A[q + NQ].x};
          } else if (v <= B) {
            const cf p0 = A[v * AV + q], p1 = A[v * AV + q + NQ];
            sv[a] = cf{p0.x - p1.y, p0.y + p1.x};
          } else if (v >= N - B) {
            const int w = N - v;
            const cf p0 = A[w * AV + q], p1 = A[w * AV + q + NQ];
            sv[a] = cf{p0.x + p1.y, p1.x - p0.y};
          } else {
            sv[a] = cf{0.f, 0.f};
          }
        }
        if constexpr (L::ZGAP) dft_zero<R1, 1, L::GAP>(sv);  // the same band gap along v
        else DFT<R1, 1>::run(sv);
#pragma unroll
        for (int c = 1; c < R1; ++c) sv[c] = cmul(sv[c], root_of<N>((wave * c) % N));
        if constexpr (!L::SEPA && NQB == 1) __syncthreads();  // Y overwrites A, which other waves may still read
        if (sl < QB) {
#pragma unroll
          for (int c = 0; c < R1; ++c) lt[L::YOFF + (c * R2 + wave) * QB + sl] = sv[c];
        }
        __syncthreads();
        // phase 4: wave takes c = wave + R2 j: radix R2 over b -> x = c + R1 d
#pragma unroll
        for (int j = 0; j < JC; ++j) {
          const int c = wave + R2 * j;
          if (c < R1) {
            cf z[R2];
#pragma unroll
            for (int b = 0; b < R2; ++b) z[b] = lt[L::YOFF + (c * R2 + b) * QB + (sl < QB ? sl : 0)];
            DFT<R2, 1>::run(z);
            if (qlane) {
#pragma unroll
              for (int d = 0; d < R2; ++d) {
                if constexpr (WINDOW) {
                  // uniform column test; row masks additive 0 / -inf (exact)
                  const int x = c + R1 * d;
                  if (abs(signed_shift(x, N)) <= max_shift) m = fmaxf(m, fmaxf(z[d].x + mq0, z[d].y + mq1));
                } else {
                  m = fmaxf(m, fmaxf(z[d].x, z[d].y));
                }
              }
            }
          }
        }
        if (qb + 1 < NQB) __syncthreads();
      }
      if constexpr (TPW == 2) {
#pragma unroll
        for (int off = SUB / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));  // within the half
        if (sl == 0) red[wave * 2 + half] = m;
      } else {
        m = wave_max(m);
        if (lane == 0) red[wave] = m;
      }
      __syncthreads();
      if (tid == 0) {
        float r = red[0];
#pragma unroll
        for (int w = 1; w < R2; ++w) r = fmaxf(r, red[w * TPW]);
        scores[p * nl + l] = r;
        if (two) {
          float r1 = red[1];
#pragma unroll
          for (int w = 1; w < R2; ++w) r1 = fmaxf(r1, red[w * TPW + 1]);
          scores[p * nl + l + 1] = r1;
        }
      }
    }
    if constexpr (!PERSIST) break;
    __syncthreads();
    if (tid == 0) item = atomicAdd(queue, 1);
    __syncthreads();
    g = item;
  }
}

// ---------------------------------------------------------------------------
// The same search with every pass's work items spread over all threads of
// the block (96 and 160).  In the wave-uniform kernel above a wave owns one
// radix position and its lanes run along the band columns (37 at 96) or the
// packed row pairs (48 at 96, 40 per block at 160), and the second passes run
// R1 positions on R2 waves, so a third of the lanes and waves idle.  Here
// each pass is a list of (radix position, column or row) items, item t on
// thread t (a second round where there are more items than threads), so the
// same work takes fewer wave instructions.  A thread's items keep the same
// (position, column) for every template: its pattern values, template row
// offsets and row-pass input rows are set up once; twiddles come from a
// [b][c] table in LDS at a per-thread base.  The arithmetic on every value,
// including the exact zeros of the band gap, is that of the kernel above,
// so the scores are the same.
//
// A (the column-pass output) has a region of its own, apart from the one X
// and Y (the first and third passes' outputs) take in turn, so no pass waits
// for reads of the buffer it writes: 4 barriers per template where shared
// buffers need 6.  At 96 that is 65.6 KB, two 8-wave blocks per CU, whose
// barriers interleave (measured: two templates per 16-wave block, one block
// per CU, run 0.85x for the same work, though their items spread more evenly
// over the SIMDs); at 160 X and A already had separate regions.
template <int N>
struct FLay {
  using W = WLay<N>;
  static constexpr int NT = W::NT;
  static constexpr int cmx(int a, int b) { return a > b ? a : b; }
  static constexpr int XOFF = 0;                        // X, then Y (measured: 1.03x at 160 over A first)
  static constexpr int AOFF = cmx(W::XN, W::YN);
  static constexpr int LDSH = cmx(XOFF + cmx(W::XN, W::YN), AOFF + W::AN);
  static_assert(AOFF + W::AN <= XOFF || XOFF + cmx(W::XN, W::YN) <= AOFF, "A apart from X and Y");
};

// Where the band indices lo .. hi (one radix input over all its lanes) lie
// for a band of half-width B at size N.
constexpr int kPos = 0, kNeg = 1, kGap = 2, kStraddle = 3;
template <int N, int B>
constexpr int band_class_nb(int lo, int hi) {
  return hi <= B ? kPos : (lo >= N - B ? kNeg : ((lo > B && hi < N - B) ? kGap : kStraddle));
}

template <int N, bool WINDOW, bool PERSIST>
__global__ __launch_bounds__(FLay<N>::NT, WLay<N>::MINW) void k_xcf_scoresf(const cf* __restrict__ spec_p, int64_t np,
                                                             const cf* __restrict__ spec_l, int64_t nl,
                                                             int lchunk, int64_t nblk, int max_shift,
                                                             float* __restrict__ scores, int* __restrict__ queue) {
  using L = WLay<N>;
  using F = FLay<N>;
  constexpr int R1 = L::R1, R2 = L::R2, B = L::B, NV = L::NV, SPEC = L::SPEC, AV = L::AV;
  constexpr int NQ = L::NQ, QB = L::QB, NQB = L::NQB, NT = F::NT;
  constexpr int T1 = R2 * NV, T2 = R1 * NV, T3 = R2 * QB, T4 = R1 * QB;
  static_assert(T1 <= NT && T2 <= NT && T3 <= NT, "one round of items in passes 1-3");
  constexpr int R4 = (T4 + NT - 1) / NT;  // rounds of the last pass
  constexpr auto band_class = [](int lo, int hi) { return band_class_nb<N, WLay<N>::B>(lo, hi); };
  __shared__ cf lds[F::LDSH];
  __shared__ cf twt[R2 * R1];  // twt[b R1 + c] = w_N^(b c), b c < N
  __shared__ float red[NT / 64];
  __shared__ int item;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  for (int i = tid; i < R2 * R1; i += NT) twt[i] = root_of<N>((i / R1) * (i % R1));

  // pass-1 item: (b1, v1).  Input a (row u = R2 a + b1) lies for every b1
  // on the positive side of the band (row kk = u), on its negative side
  // (kk = u - N + 2B + 1), in its gap, or straddles an edge (per-lane row;
  // gap rows read row 0 and are multiplied by a cached zero)
  const bool act1 = tid < T1;
  const int b1 = act1 ? tid / NV : 0, v1 = act1 ? tid - b1 * NV : 0;
  const unsigned base1 = (unsigned)(b1 * NV + v1) * (unsigned)sizeof(cf), col1 = (unsigned)v1 * sizeof(cf);
  unsigned off1[R1];
#pragma unroll
  for (int a = 0; a < R1; ++a) {
    const int u = R2 * a + b1;
    const int kk = u <= B ? u : (u >= N - B ? u - N + 2 * B + 1 : 0);
    off1[a] = band_class(R2 * a, R2 * a + R2 - 1) == kStraddle ? (unsigned)(kk * NV + v1) * (unsigned)sizeof(cf) : 0u;
  }
  cf* const X = lds + F::XOFF;
  cf* const Y = lds + F::XOFF;
  cf* const A = lds + F::AOFF;
  // pass-2 item: (c2, v2)
  const bool act2 = tid < T2;
  const int c2 = act2 ? tid / NV : 0, v2 = act2 ? tid - c2 * NV : 0;
  // pass-3 item: (b3, q3 of the row block); for input a the band column
  // v = R2 a + b3 enters as A(v) (1 <= v <= B, k = +1), as the conjugate of
  // A(N - v) (v >= N - B, k = -1), through its real part only (v = 0, k = 0)
  // or not at all (the band gap, m = 0)
  const bool act3 = tid < T3;
  const int b3 = act3 ? tid / QB : 0, q3 = act3 ? tid - b3 * QB : 0;
  const int base3p = b3 * AV + q3, base3n = q3 - b3 * AV;  // A(R2 a + b3, q3) and A(N - R2 a - b3, q3) less the constant row
  int at3[R1];  // element index of A(row, q3) for the inputs that straddle a band edge
  float k3[R1], m3[R1];
#pragma unroll
  for (int a = 0; a < R1; ++a) {
    const int v = R2 * a + b3;
    const bool pos = v <= B, neg = v >= N - B;
    at3[a] = (pos ? v : (neg ? N - v : 0)) * AV + q3;
    k3[a] = (pos && v > 0) ? 1.0f : (neg ? -1.0f : 0.0f);
    m3[a] = (pos || neg) ? 1.0f : 0.0f;
  }

  int64_t g;
  if constexpr (PERSIST) {
    if (tid == 0) item = atomicAdd(queue, 1);
    __syncthreads();
    g = item;
  } else {
    const int64_t per = (nblk + 7) / 8;
    g = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    __syncthreads();  // the twiddle table
  }
  if (g >= nblk) return;

  while (g < nblk) {
    const int64_t chunk = g / np, p = g - chunk * np;
    const cf* E = spec_p + p * SPEC;
    cf ev[R1];
#pragma unroll
    for (int a = 0; a < R1; ++a) {
      const int u = R2 * a + b1;
      const int kk = u <= B ? u : (u >= N - B ? u - N + 2 * B + 1 : -1);
      ev[a] = (kk >= 0 && act1) ? E[kk * NV + v1] : cf{0.f, 0.f};
    }
    const int64_t l0 = chunk * lchunk;
    const int64_t l1 = l0 + lchunk < nl ? l0 + lchunk : nl;
    // pass-1 inputs of template T.  At 96 they are issued one template ahead
    // (before the last pass 4 of the template before), so that their latency
    // overlaps that pass and the barrier after it (measured 1.05x); at 160
    // the 20 registers they hold meanwhile make the kernel spill (0.93x)
    constexpr bool PREFETCH = N == 96;
    cf xn[R1];
    const auto load1 = [&](const cf* T) {
      const __amdgpu_buffer_rsrc_t Tr = spectrum_rsrc(T, SPEC * (int)sizeof(cf));
      static_for<0, R1>([&](auto ai) {
        constexpr int a = decltype(ai)::value;
        constexpr int cls = band_class(R2 * a, R2 * a + R2 - 1);
        if constexpr (L::ZGAP && ((L::GAP >> a) & 1)) return;  // neither loaded nor added
        unsigned vo;
        int so;
        if constexpr (cls == kPos) { vo = base1; so = R2 * a * NV * (int)sizeof(cf); }
        else if constexpr (cls == kNeg) { vo = base1; so = (R2 * a - N + 2 * B + 1) * NV * (int)sizeof(cf); }
        else if constexpr (cls == kGap) { vo = col1; so = 0; }
        else { vo = off1[a]; so = 0; }
        static_assert(cls != kNeg || R2 * a - N + 2 * B + 1 >= 0, "non-negative row offset");
        if constexpr (L::BUFLOAD) xn[a] = buffer_cf(Tr, vo, so);
        else xn[a] = *reinterpret_cast<const cf*>(reinterpret_cast<const char*>(T) + vo + so);
      });
    };
    if (PREFETCH && act1) load1(spec_l + l0 * SPEC);
    for (int64_t l = l0; l < l1; ++l) {
      // pass 1: item (b1, v1): radix R1 over u = R2 a + b1, twiddle
      if (act1) {
        if constexpr (!PREFETCH) load1(spec_l + l * SPEC);
        cf x[R1];
#pragma unroll
        for (int a = 0; a < R1; ++a)
          if (!(L::ZGAP && ((L::GAP >> a) & 1))) x[a] = cmulc(ev[a], xn[a]);
        if constexpr (L::ZGAP) dft_zero<R1, 1, L::GAP>(x);
        else DFT<R1, 1>::run(x);
        const cf* tw = twt + b1 * R1;
#pragma unroll
        for (int c = 1; c < R1; ++c) x[c] = cmul(x[c], tw[c]);
#pragma unroll
        for (int c = 0; c < R1; ++c) X[(c * R2 + b1) * NV + v1] = x[c];
      }
      __syncthreads();
      // pass 2: item (c2, v2): radix R2 over b -> A(y = c2 + R1 d, v2)
      if (act2) {
        cf h[R2];
#pragma unroll
        for (int b = 0; b < R2; ++b) h[b] = X[(c2 * R2 + b) * NV + v2];
        DFT<R2, 1>::run(h);
#pragma unroll
        for (int d = 0; d < R2; ++d) A[v2 * AV + c2 + R1 * d] = h[d];
      }
      __syncthreads();
      float m = -INFINITY;
#pragma unroll
      for (int qb = 0; qb < NQB; ++qb) {
        // pass 3: item (b3, q): radix R1 over v = R2 a + b3 of the packed rows (q, q + N/2)
        if (act3) {
          cf sv[R1];
          static_for<0, R1>([&](auto ai) {
            constexpr int a = decltype(ai)::value;
            // the columns v = R2 a + b3 of input a over all b3 (column 0, the
            // DC term, takes its real parts only: the coefficient form)
            constexpr int cls = a == 0 ? kStraddle : band_class(R2 * a, R2 * a + R2 - 1);
            if constexpr ((L::ZGAP && ((L::GAP >> a) & 1)) || cls == kGap) {
              sv[a] = cf{0.f, 0.f};
            } else if constexpr (cls == kPos) {
              const cf* pa = A + base3p + R2 * a * AV + qb * QB;
              const cf p0 = pa[0], p1 = pa[NQ];
              sv[a] = cf{p0.x - p1.y, p0.y + p1.x};
            } else if constexpr (cls == kNeg) {
              const cf* pa = A + base3n + (N - R2 * a) * AV + qb * QB;
              const cf p0 = pa[0], p1 = pa[NQ];
              sv[a] = cf{p0.x + p1.y, p1.x - p0.y};
            } else {
              const cf* pa = A + at3[a] + qb * QB;
              const cf p0 = pa[0], p1 = pa[NQ];
              sv[a] = cf{__fmaf_rn(-k3[a], p1.y, m3[a] * p0.x), __fmaf_rn(k3[a], p0.y, m3[a] * p1.x)};
            }
          });
          if constexpr (L::ZGAP) dft_zero<R1, 1, L::GAP>(sv);
          else DFT<R1, 1>::run(sv);
          const cf* tw = twt + b3 * R1;
#pragma unroll
          for (int c = 1; c < R1; ++c) sv[c] = cmul(sv[c], tw[c]);
#pragma unroll
          for (int c = 0; c < R1; ++c) Y[(c * R2 + b3) * QB + q3] = sv[c];
        }
        __syncthreads();
        if (PREFETCH && qb + 1 == NQB && act1 && l + 1 < l1) load1(spec_l + (l + 1) * SPEC);
        // pass 4: item (c4, q4): radix R2 over b -> x = c4 + R1 d
#pragma unroll
        for (int r = 0; r < R4; ++r) {
          const int t = tid + r * NT;
          if (t < T4) {
            const int c4 = t / QB, q4 = t - c4 * QB;
            const int qq = qb * QB + q4;
            cf z[R2];
#pragma unroll
            for (int b = 0; b < R2; ++b) z[b] = Y[(c4 * R2 + b) * QB + q4];
            DFT<R2, 1>::run(z);
            if (qq < NQ) {
              if constexpr (WINDOW) {
                const float mq0 = abs(signed_shift(qq, N)) <= max_shift ? 0.f : -INFINITY;
                const float mq1 = abs(signed_shift(qq + NQ, N)) <= max_shift ? 0.f : -INFINITY;
#pragma unroll
                for (int d = 0; d < R2; ++d) {
                  const int x = c4 + R1 * d;
                  const float mx = abs(signed_shift(x, N)) <= max_shift ? 0.f : -INFINITY;
                  m = fmaxf(m, fmaxf(z[d].x + mq0, z[d].y + mq1) + mx);
                }
              } else {
#pragma unroll
                for (int d = 0; d < R2; ++d) m = fmaxf(m, fmaxf(z[d].x, z[d].y));
              }
            }
          }
        }
        if (qb + 1 < NQB) __syncthreads();  // the next row block's pass 3 overwrites Y
      }
      m = wave_max(m);
      if (lane == 0) red[tid >> 6] = m;
      __syncthreads();
      if (tid == 0) {
        float r = red[0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) r = fmaxf(r, red[w]);
        scores[p * nl + l] = r;
      }
    }
    if constexpr (!PERSIST) break;
    __syncthreads();
    if (tid == 0) item = atomicAdd(queue, 1);
    __syncthreads();
    g = item;
  }
}

// ---------------------------------------------------------------------------
// Forward spectra of K images (pixels of type T: float or __bf16).
template <int N, int NT, class T>
__global__ __launch_bounds__(NT) void k_spectra(const T* __restrict__ imgs, int64_t img_stride,
                                                const int64_t* __restrict__ img_off, FilterParams fp,
                                                cf* __restrict__ spec, double* __restrict__ energy) {
  using L = Lay<N>;
  constexpr int R1 = L::R1, R2 = L::R2, B = L::B, NV = L::NV, NK = L::NK;
  __shared__ cf lds[L::LDS];
  __shared__ cf tw[N];
  __shared__ float win[N];
  __shared__ double red[2 * (NT / 64)];
  const int tid = threadIdx.x;
  const int64_t k = blockIdx.x;
  const T* img = imgs + (img_off ? img_off[k] : k * img_stride);
  load_roots<N, NT>(tw, tid);
  for (int i = tid; i < N; i += NT) {
    const float s = sinpif(((float)i + 0.5f) / (float)N);
    win[i] = fp.window ? s * s : 1.0f;
  }

  // mean and standard deviation in FP64
  double s1 = 0.0, s2 = 0.0;
  for (int i = tid; i < N * N; i += NT) {
    const double v = (double)ld_px(img[i]);
    s1 += v;
    s2 += v * v;
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if ((tid & 63) == 0) {
    red[tid >> 6] = s1;
    red[NT / 64 + (tid >> 6)] = s2;
  }
  __syncthreads();
  double t1 = 0.0, t2 = 0.0;
  for (int w = 0; w < NT / 64; ++w) {
    t1 += red[w];
    t2 += red[NT / 64 + w];
  }
  const double mean = t1 / (double)(N * N);
  const double var = t2 / (double)(N * N) - mean * mean;
  const float fmean = (float)mean;
  const float inv_std = var > 0.0 ? (float)(1.0 / sqrt(var)) : 0.0f;
  __syncthreads();

  // row pass, radix R1 on row pairs (q, q + N/2) packed as real + i imag
  constexpr int TF1 = (N / 2) * R2;
  for (int t = tid; t < TF1; t += NT) {
    const int q = t / R2, b = t - q * R2;
    cf x[R1];
    const float wq0 = win[q] * inv_std, wq1 = win[q + N / 2] * inv_std;
#pragma unroll
    for (int a = 0; a < R1; ++a) {
      const int col = R2 * a + b;
      const float v0 = (ld_px(img[q * N + col]) - fmean) * wq0 * win[col];
      const float v1 = (ld_px(img[(q + N / 2) * N + col]) - fmean) * wq1 * win[col];
      x[a] = cf{v0, v1};
    }
    DFT<R1, -1>::run(x);
#pragma unroll
    for (int c = 1; c < R1; ++c) x[c] = cmulc(x[c], tw[b * c]);
#pragma unroll
    for (int c = 0; c < R1; ++c) lds[q * L::YS + c * R2 + b] = x[c];
  }
  __syncthreads();

  // row pass, radix R2: Z_q(v = c + R1 d)
  constexpr int TF2 = (N / 2) * R1, JF2 = (TF2 + NT - 1) / NT;
  cf h2[JF2][R2];
#pragma unroll
  for (int j = 0; j < JF2; ++j) {
    const int t = tid + j * NT;
    if (t < TF2) {
      const int q = t / R1, c = t - q * R1;
#pragma unroll
      for (int b = 0; b < R2; ++b) h2[j][b] = lds[q * L::YS + c * R2 + b];
      DFT<R2, -1>::run(h2[j]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < JF2; ++j) {
    const int t = tid + j * NT;
    if (t < TF2) {
      const int q = t / R1, c = t - q * R1;
#pragma unroll
      for (int d = 0; d < R2; ++d) lds[q * L::ZS + c + R1 * d] = h2[j][d];
    }
  }
  __syncthreads();

  // separate the two packed rows: F_q(v) = (Z(v) + conj Z(-v)) / 2,
  // F_{q+N/2}(v) = (Z(v) - conj Z(-v)) / 2i, for v in [0, B]
  constexpr int TF3 = (N / 2) * NV, JF3 = (TF3 + NT - 1) / NT;
  cf h3[JF3][2];
#pragma unroll
  for (int j = 0; j < JF3; ++j) {
    const int t = tid + j * NT;
    if (t < TF3) {
      const int q = t / NV, v = t - q * NV;
      const cf z1 = lds[q * L::ZS + v];
      const cf zb = lds[q * L::ZS + (v == 0 ? 0 : N - v)];
      h3[j][0] = cf{0.5f * (z1.x + zb.x), 0.5f * (z1.y - zb.y)};
      h3[j][1] = cf{0.5f * (z1.y + zb.y), -0.5f * (z1.x - zb.x)};
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < JF3; ++j) {
    const int t = tid + j * NT;
    if (t < TF3) {
      const int q = t / NV, v = t - q * NV;
      lds[q * L::AS + v] = h3[j][0];
      lds[(q + N / 2) * L::AS + v] = h3[j][1];
    }
  }
  __syncthreads();

  // column pass, radix R1 over y = R2 a + b, for every (v, b)
  constexpr int TF4 = NV * R2, JF4 = (TF4 + NT - 1) / NT;
  cf h4[JF4][R1];
#pragma unroll
  for (int j = 0; j < JF4; ++j) {
    const int t = tid + j * NT;
    if (t < TF4) {
      const int v = t / R2, b = t - v * R2;
#pragma unroll
      for (int a = 0; a < R1; ++a) h4[j][a] = lds[(R2 * a + b) * L::AS + v];
      DFT<R1, -1>::run(h4[j]);
#pragma unroll
      for (int c = 1; c < R1; ++c) h4[j][c] = cmulc(h4[j][c], tw[b * c]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < JF4; ++j) {
    const int t = tid + j * NT;
    if (t < TF4) {
      const int v = t / R2, b = t - v * R2;
#pragma unroll
      for (int c = 0; c < R1; ++c) lds[v * L::XS + c * R2 + b] = h4[j][c];
    }
  }
  __syncthreads();

  // column pass, radix R2: X(u = c + R1 d, v); band-pass and energy
  constexpr int TF5 = NV * R1, JF5 = (TF5 + NT - 1) / NT;
  cf h5[JF5][R2];
  const float inv2hp = 1.0f / (2.0f * fp.sigma_hp * fp.sigma_hp);
  const float inv2lp = 1.0f / (2.0f * fp.sigma_lp * fp.sigma_lp);
  const float rmax2 = fp.rho_max * fp.rho_max;
  double en = 0.0;
#pragma unroll
  for (int j = 0; j < JF5; ++j) {
    const int t = tid + j * NT;
    if (t < TF5) {
      const int v = t / R1, c = t - v * R1;
#pragma unroll
      for (int b = 0; b < R2; ++b) h5[j][b] = lds[v * L::XS + c * R2 + b];
      DFT<R2, -1>::run(h5[j]);
#pragma unroll
      for (int d = 0; d < R2; ++d) {
        const int u = c + R1 * d;
        const int us = u >= N / 2 ? u - N : u;
        const float r2 = (float)(us * us + v * v);
        float h = 0.0f;
        if ((us >= -B && us <= B) && r2 <= rmax2 && us != -N / 2) {
          h = (1.0f - expf(-r2 * inv2hp)) * expf(-r2 * inv2lp);
        }
        const cf z = cscale(h5[j][d], h);
        h5[j][d] = z;
        en += (v == 0 ? 1.0 : 2.0) * ((double)z.x * (double)z.x + (double)z.y * (double)z.y);
      }
    }
  }
  en = wave_sum(en);
  if ((tid & 63) == 0) red[tid >> 6] = en;
  __syncthreads();
  double etot = 0.0;
  for (int w = 0; w < NT / 64; ++w) etot += red[w];
  const float scale = etot > 0.0 ? (float)(1.0 / sqrt(etot)) : 0.0f;
  cf* out = spec + k * L::SPEC;
#pragma unroll
  for (int j = 0; j < JF5; ++j) {
    const int t = tid + j * NT;
    if (t < TF5) {
      const int v = t / R1, c = t - v * R1;
#pragma unroll
      for (int d = 0; d < R2; ++d) {
        const int u = c + R1 * d;
        const int kk = u <= B ? u : (u >= N - B ? u - N + NK : -1);
        if (kk >= 0) out[kk * NV + v] = cscale(h5[j][d], scale);
      }
    }
  }
  if (tid == 0 && energy) energy[k] = etot;
}

// ---------------------------------------------------------------------------
int band_of(int n) {
  switch (n) {
    case 64: return Plan<64>::B;
    case 96: return Plan<96>::B;
    case 128: return Plan<128>::B;
    case 160: return Plan<160>::B;
    case 256: return Plan<256>::B;
    default: return -1;
  }
}
bool size_supported(int n) { return band_of(n) > 0; }
bool fft_supported(int n) { return n == 64 || n == 96 || n == 128 || n == 160; }

template <int N>
static constexpr int nt_xcf() { return N <= 96 ? 256 : 256; }
template <int N>
static constexpr int nt_spec() { return N <= 96 ? 256 : 512; }

#define EBSD_DISPATCH(n, CALL)        \
  switch (n) {                        \
    case 64: { constexpr int NN = 64; CALL; } break;   \
    case 96: { constexpr int NN = 96; CALL; } break;   \
    case 128: { constexpr int NN = 128; CALL; } break; \
    case 160: { constexpr int NN = 160; CALL; } break; \
    default: return hipErrorInvalidValue;              \
  }

// One dispatch holds fewer than 2^32 work-items per grid dimension; every
// launcher below keeps its 1-D grids under 2^31 by splitting the items.
constexpr int64_t kMaxItems = int64_t(1) << 31;

template <class T>
static hipError_t spectra_t(int n, const T* imgs, int64_t img_stride, int64_t k, const FilterParams& fp,
                            float2* spec, double* energy, hipStream_t stream) {
  if (k <= 0) return hipSuccess;
  const int64_t kmax = kMaxItems / 512;
  if (k > kmax) {
    const int64_t sc = (int64_t)(band_of(n) + 1) * (2 * band_of(n) + 1);
    for (int64_t s = 0; s < k; s += kmax) {
      const hipError_t e = spectra_t(n, imgs + s * img_stride, img_stride, k - s < kmax ? k - s : kmax, fp,
                                     spec + s * sc, energy ? energy + s : nullptr, stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  EBSD_DISPATCH(n, {
    constexpr int NT = nt_spec<NN>();
    hipLaunchKernelGGL((k_spectra<NN, NT, T>), dim3((unsigned)k), dim3(NT), 0, stream, imgs, img_stride,
                       (const int64_t*)nullptr, fp, (cf*)spec, energy);
  });
  return hipGetLastError();
}

hipError_t launch_spectra(int n, const float* imgs, int64_t img_stride, int64_t k,
                          const FilterParams& fp, float2* spec, double* energy,
                          hipStream_t stream) {
  return spectra_t(n, imgs, img_stride, k, fp, spec, energy, stream);
}

hipError_t launch_spectra(int n, const __bf16* imgs, int64_t img_stride, int64_t k,
                          const FilterParams& fp, float2* spec, double* energy,
                          hipStream_t stream) {
  return spectra_t(n, imgs, img_stride, k, fp, spec, energy, stream);
}

hipError_t launch_spectra_gather(int n, const float* imgs, const int64_t* img_off, int64_t k,
                                 const FilterParams& fp, float2* spec, double* energy, hipStream_t stream) {
  if (k <= 0) return hipSuccess;
  const int64_t kmax = kMaxItems / 512;
  if (k > kmax) {
    const int64_t sc = (int64_t)(band_of(n) + 1) * (2 * band_of(n) + 1);
    for (int64_t s = 0; s < k; s += kmax) {
      const hipError_t e = launch_spectra_gather(n, imgs, img_off + s, k - s < kmax ? k - s : kmax, fp,
                                                 spec + s * sc, energy ? energy + s : nullptr, stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  EBSD_DISPATCH(n, {
    constexpr int NT = nt_spec<NN>();
    hipLaunchKernelGGL((k_spectra<NN, NT, float>), dim3((unsigned)k), dim3(NT), 0, stream, imgs, (int64_t)0,
                       img_off, fp, (cf*)spec, energy);
  });
  return hipGetLastError();
}

// 96 and 160 run the search with its work items spread over the whole block
// (k_xcf_scoresf, scores bit-identical to the wave-uniform kernel's;
// measured 1.30x and 1.15x over every shift, 1.29x and 1.02x with a +-7
// window).  64 keeps two templates per wave, 128 its own kernel.
#ifndef EBSD_SEARCH_FLAT
#define EBSD_SEARCH_FLAT 1
#endif
template <int N, bool WINDOW>
constexpr bool search_flat() { return EBSD_SEARCH_FLAT && (N == 96 || N == 160); }

// Templates per block of the search.  At 128 a chunk of 64 (2.4 MB of band
// spectra) stays in one XCD's 4 MB L2 while the blocks running there stream
// their patterns, and halves the pattern re-reads of a 32-template chunk at
// the same time (measured); 128 or more templates no longer fit and raise
// the traffic again.  The other sizes keep 32.
static int search_lchunk(int n) { return n == 128 ? 64 : 32; }

hipError_t launch_xcf_scores(int n, const float2* spec_p, int64_t p, const float2* spec_l,
                             int64_t l, int max_shift, float* scores, hipStream_t stream) {
  if (p <= 0 || l <= 0) return hipSuccess;
  const int lchunk = search_lchunk(n);
  const int64_t nchunk = (l + lchunk - 1) / lchunk;
  // patterns per dispatch so that blocks x threads stays below 2^31
  const int64_t pmax = (kMaxItems / 1024 - 8) / nchunk;
  if (pmax < 1) return hipErrorInvalidValue;
  if (p > pmax) {
    const int64_t sc = (int64_t)(band_of(n) + 1) * (2 * band_of(n) + 1);
    for (int64_t s = 0; s < p; s += pmax) {
      const hipError_t e = launch_xcf_scores(n, spec_p + s * sc, p - s < pmax ? p - s : pmax, spec_l, l, max_shift,
                                             scores + s * l, stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int64_t nblk = p * nchunk;
  const int64_t grid = ((nblk + 7) / 8) * 8;
  if (n == 128) {
    if (max_shift < 0)
      hipLaunchKernelGGL((k_xcf_scores128<false, false>), dim3((unsigned)grid), dim3(512), 0, stream,
                         (const cf*)spec_p, p, (const cf*)spec_l, l, lchunk, nblk, max_shift, scores, nullptr);
    else
      hipLaunchKernelGGL((k_xcf_scores128<true, false>), dim3((unsigned)grid), dim3(512), 0, stream,
                         (const cf*)spec_p, p, (const cf*)spec_l, l, lchunk, nblk, max_shift, scores, nullptr);
    return hipGetLastError();
  }
  EBSD_DISPATCH(n, {
    constexpr int NT = WLay<NN>::NT;
    constexpr int NTF = FLay<NN>::NT;
    if (max_shift < 0) {
      if constexpr (search_flat<NN, false>())
        hipLaunchKernelGGL((k_xcf_scoresf<NN, false, false>), dim3((unsigned)grid), dim3(NTF), 0, stream,
                           (const cf*)spec_p, p, (const cf*)spec_l, l, lchunk, nblk, max_shift, scores, nullptr);
      else
        hipLaunchKernelGGL((k_xcf_scoresw<NN, false, false>), dim3((unsigned)grid), dim3(NT), 0, stream,
                           (const cf*)spec_p, p, (const cf*)spec_l, l, lchunk, nblk, max_shift, scores, nullptr);
    } else {
      if constexpr (search_flat<NN, true>())
        hipLaunchKernelGGL((k_xcf_scoresf<NN, true, false>), dim3((unsigned)grid), dim3(NTF), 0, stream,
                           (const cf*)spec_p, p, (const cf*)spec_l, l, lchunk, nblk, max_shift, scores, nullptr);
      else
        hipLaunchKernelGGL((k_xcf_scoresw<NN, true, false>), dim3((unsigned)grid), dim3(NT), 0, stream,
                           (const cf*)spec_p, p, (const cf*)spec_l, l, lchunk, nblk, max_shift, scores, nullptr);
    }
  });
  return hipGetLastError();
}

// Scores of each pattern against its own list of k candidate templates
// (scores[p k + j] for template cand[p k + j]), by the library search kernel
// (128 only; other sizes return hipErrorInvalidValue and the caller takes
// the single-pair kernel).
hipError_t launch_xcf_scores_cand(int n, const float2* spec_p, int64_t p, const float2* spec_l, int64_t l,
                                  const int32_t* cand, int k, int max_shift, float* scores, hipStream_t stream) {
  if (p <= 0 || k <= 0) return hipSuccess;
  if (l <= 0) return hipErrorInvalidValue;
  if (n != 128) return hipErrorInvalidValue;
  const int lchunk = search_lchunk(n);
  const int64_t nchunk = (k + lchunk - 1) / lchunk;
  const int64_t pmax = (kMaxItems / 1024 - 8) / nchunk;
  if (pmax < 1) return hipErrorInvalidValue;
  if (p > pmax) {
    const int64_t sc = (int64_t)(band_of(n) + 1) * (2 * band_of(n) + 1);
    for (int64_t s = 0; s < p; s += pmax) {
      const hipError_t e = launch_xcf_scores_cand(n, spec_p + s * sc, p - s < pmax ? p - s : pmax, spec_l, l,
                                                  cand + s * k, k, max_shift, scores + s * k, stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int64_t nblk = p * nchunk;
  const int64_t grid = ((nblk + 7) / 8) * 8;
  if (max_shift < 0)
    hipLaunchKernelGGL((k_xcf_scores128<false, false, true>), dim3((unsigned)grid), dim3(512), 0, stream,
                       (const cf*)spec_p, p, (const cf*)spec_l, (int64_t)k, lchunk, nblk, max_shift, scores, nullptr,
                       cand, l);
  else
    hipLaunchKernelGGL((k_xcf_scores128<true, false, true>), dim3((unsigned)grid), dim3(512), 0, stream,
                       (const cf*)spec_p, p, (const cf*)spec_l, (int64_t)k, lchunk, nblk, max_shift, scores, nullptr,
                       cand, l);
  return hipGetLastError();
}

hipError_t xcf_persistent_occupancy(int n, int max_shift, int* blocks_per_cu) {
  *blocks_per_cu = 0;
  if (n == 128) {
    return max_shift < 0
               ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_xcf_scores128<false, true>, 512, 0)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_xcf_scores128<true, true>, 512, 0);
  }
  EBSD_DISPATCH(n, {
    constexpr int NT = WLay<NN>::NT;
    if (max_shift < 0) {
      if constexpr (search_flat<NN, false>())
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_xcf_scoresf<NN, false, true>, FLay<NN>::NT, 0);
      else
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_xcf_scoresw<NN, false, true>, NT, 0);
    } else {
      if constexpr (search_flat<NN, true>())
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_xcf_scoresf<NN, true, true>, FLay<NN>::NT, 0);
      else
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_xcf_scoresw<NN, true, true>, NT, 0);
    }
  });
  return hipSuccess;
}

hipError_t launch_xcf_scores_persistent(int n, const float2* spec_p, int64_t p, const float2* spec_l, int64_t l,
                                        int max_shift, float* scores, int lchunk, int grid, int* queue,
                                        hipStream_t stream) {
  if (p <= 0 || l <= 0) return hipSuccess;
  if (lchunk < 1 || grid < 1) return hipErrorInvalidValue;
  const int64_t nchunk = (l + lchunk - 1) / lchunk;
  const int64_t nblk = p * nchunk;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  if (n == 128) {
    if (max_shift < 0)
      hipLaunchKernelGGL((k_xcf_scores128<false, true>), dim3((unsigned)grid), dim3(512), 0, stream,
                         (const cf*)spec_p, p, (const cf*)spec_l, l, lchunk, nblk, max_shift, scores, queue);
    else
      hipLaunchKernelGGL((k_xcf_scores128<true, true>), dim3((unsigned)grid), dim3(512), 0, stream,
                         (const cf*)spec_p, p, (const cf*)spec_l, l, lchunk, nblk, max_shift, scores, queue);
    return hipGetLastError();
  }
  EBSD_DISPATCH(n, {
    constexpr int NT = WLay<NN>::NT;
    constexpr int NTF = FLay<NN>::NT;
    if (max_shift < 0) {
      if constexpr (search_flat<NN, false>())
        hipLaunchKernelGGL((k_xcf_scoresf<NN, false, true>), dim3((unsigned)grid), dim3(NTF), 0, stream,
                           (const cf*)spec_p, p, (const cf*)spec_l, l, lchunk, nblk, max_shift, scores, queue);
      else
        hipLaunchKernelGGL((k_xcf_scoresw<NN, false, true>), dim3((unsigned)grid), dim3(NT), 0, stream,
                           (const cf*)spec_p, p, (const cf*)spec_l, l, lchunk, nblk, max_shift, scores, queue);
    } else {
      if constexpr (search_flat<NN, true>())
        hipLaunchKernelGGL((k_xcf_scoresf<NN, true, true>), dim3((unsigned)grid), dim3(NTF), 0, stream,
                           (const cf*)spec_p, p, (const cf*)spec_l, l, lchunk, nblk, max_shift, scores, queue);
      else
        hipLaunchKernelGGL((k_xcf_scoresw<NN, true, true>), dim3((unsigned)grid), dim3(NT), 0, stream,
                           (const cf*)spec_p, p, (const cf*)spec_l, l, lchunk, nblk, max_shift, scores, queue);
    }
  });
  return hipGetLastError();
}

hipError_t launch_xcf_peak(int n, const float2* spec_p, const float2* spec_l,
                           const int32_t* pi, const int32_t* li, int64_t k, int max_shift,
                           float* h_int, int32_t* s_int, float* map, hipStream_t stream) {
  if (k <= 0) return hipSuccess;
  const int64_t kmax = kMaxItems / 256;
  if (k > kmax) {
    const int64_t sc = (int64_t)(band_of(n) + 1) * (2 * band_of(n) + 1);
    for (int64_t s = 0; s < k; s += kmax) {
      // without index lists, pair k is (pattern k, template k)
      const hipError_t e = launch_xcf_peak(n, pi ? spec_p : spec_p + s * sc, li ? spec_l : spec_l + s * sc,
                                           pi ? pi + s : nullptr, li ? li + s : nullptr, k - s < kmax ? k - s : kmax,
                                           max_shift, h_int + s, s_int + 2 * s,
                                           map ? map + s * (int64_t)n * n : nullptr, stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  EBSD_DISPATCH(n, {
    constexpr int NT = nt_xcf<NN>();
    hipLaunchKernelGGL((k_xcf_peak<NN, NT>), dim3((unsigned)k), dim3(NT), 0, stream, (const cf*)spec_p,
                       (const cf*)spec_l, pi, li, max_shift, h_int, s_int, map);
  });
  return hipGetLastError();
}

}  // namespace ebsd

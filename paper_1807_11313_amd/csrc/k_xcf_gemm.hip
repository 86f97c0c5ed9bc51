// Windowed correlation search as split-precision DFT-GEMMs on MFMA (gfx950).
//
// For shifts restricted to |s_x|, |s_y| <= S, the band-limited correlation
// (Equations 2, 3 and the spatial definition of r_fg; see k_spectra_xcf.hip)
// is two dense products per pattern-template pair:
//   stage 1  A(s_y, v)     = sum_u  Z(u, v) W1(u, s_y),  W1 = exp(+2 pi i u s_y / N)
//   stage 2  rho(s_y, s_x) = Re sum_v A(s_y, v) C(v, s_x), C = w_v exp(+2 pi i v s_x / N)
// with Z = E conj(T) over the stored band (u in [-B, B], v in [0, B]) and
// w_0 = 1, w_v = 2 (Hermitian half).  Both run on MFMA with every operand
// split into two 16-bit halves, x = x_hi + x_lo (FP16 or BF16), products
// formed as hi*hi + hi*lo + lo*hi and accumulated in FP32; the BF16 form
// without the lo halves is the one-product variant.
//
// Stage 1 is computed transposed, A^T (v x s_y) = Z^T W1, with Z^T as the
// A operand of v_mfma_f32_16x16x32 (lane l: row v = l % 16, k = 8 (l / 16) + j)
// formed per pair on the VALU, and W1 as the B operand from LDS.  Its FP32
// accumulator tile (lane l: v = 4 (l / 16) + i, s_y = l % 16) is exactly the B
// operand layout of v_mfma_f32_16x16x16 (k = 4 (l / 16) + j, n = l % 16), so
// stage 2, rho^T (s_x x s_y) = C^T A^T, consumes it from registers after a
// split, with C^T as the constant A operand.  Each wave owns one pair at a
// time; the 8 waves of a block work through a chunk of templates against one
// pattern and share in LDS the constant fragments and, where it fits, the
// pattern's operand values in fragment order.  The next chunk's template
// values are loaded while the current chunk's products run, and consecutive
// MFMAs accumulate into different tiles.
#include "ebsd_common.hpp"
#include "ebsd_internal.hpp"

#include <math.h>

namespace ebsd {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Z (and the stage-1 output) is scaled by 2^12 before splitting so that the
// lo halves of typical band coefficients stay in the FP16 normal range, while
// |A| <= 2^12 sum_u |E||T| <= 2^11 stays far below the FP16 maximum.
constexpr float kZScale = 4096.0f;
constexpr float kZUnscale = 1.0f / 4096.0f;

#ifndef EBSD_GEMM_E_LIMIT
#define EBSD_GEMM_E_LIMIT (150 * 1024)
#endif
constexpr int kGemmELimit = EBSD_GEMM_E_LIMIT;

// patterns per block of the pattern-tiled search (0: one pattern per block)
#ifndef EBSD_GEMM_PATTERN_TILE
#define EBSD_GEMM_PATTERN_TILE 4
#endif
constexpr int kGemmPatternTile = EBSD_GEMM_PATTERN_TILE;
#ifndef EBSD_GEMM_INTERLEAVE
#define EBSD_GEMM_INTERLEAVE 1
#endif
#ifndef EBSD_GEMM_PAIRSYNC
#define EBSD_GEMM_PAIRSYNC 1
#endif
#ifndef EBSD_GEMM_SUPER
#define EBSD_GEMM_SUPER 0  // template blocks per super-tile; 0: 4, or 2 at 256 (L2 per XCD)
#endif

template <int N, int ST>
struct GemmLay {
  static constexpr int B = Plan<N>::B, NV = B + 1, NK = 2 * B + 1, SPEC = NV * NK;
  // With the filter cut at rho <= B, the rows u = +-B hold a non-zero value
  // only at v = 0 and the column v = B only at u = 0.  When B is a multiple of
  // 8 and 2B of 32 (N = 128, 256) those three entries are added exactly as
  // rank-one terms, and the products run on the 2B - 1 remaining rows (K
  // index k: band row k for k < B, row k + 2 for B <= k < 2B - 1, one zero
  // row) and B columns, with no padding.
  static constexpr bool FAST = (B % 8 == 0) && ((2 * B) % 32 == 0);
  static constexpr int KC = FAST ? (2 * B) / 32 : (NK + 31) / 32;  // 32-row chunks of K
  static constexpr int VT = FAST ? B / 16 : (NV + 15) / 16;        // 16-column tiles
  static constexpr int SLOTS = 16 * ST;         // shift slots s = slot - 8 ST
  // constant fragments: W1 [KC][ST][re, im(, -im)][hi, lo] x 64 lanes x 8 halves,
  //                     C  [VT][ST][re, -im][hi, lo] x 64 lanes x 4 halves;
  // the pre-negated -im part is kept when it fits, else Zi is negated per pair
  static constexpr int C_HALVES = VT * ST * 4 * 256;
  static constexpr bool NEGW = 2 * (KC * ST * 6 * 512 + C_HALVES) <= 150 * 1024;
  static constexpr int W1_PARTS = NEGW ? 3 : 2;
  static constexpr int W1_HALVES = KC * ST * 2 * W1_PARTS * 512;
  static constexpr int FRAG_BYTES = 2 * (W1_HALVES + C_HALVES);
  // pattern operand values in fragment order: [VT][KC] x 64 lanes x 8 complex,
  // kept in LDS when block-shared memory stays within kGemmELimit
  static constexpr int E_BYTES = VT * KC * 64 * 8 * 8;
  static constexpr bool ELDS = FRAG_BYTES + E_BYTES <= kGemmELimit;
  static constexpr int LDS_BYTES = FRAG_BYTES + (ELDS ? E_BYTES : 0);
};

// ---------------------------------------------------------------------------
// 16-bit halves: PREC 0 = FP16 hi + lo, 1 = BF16 hi + lo, 2 = BF16 hi only.
template <int PREC>
__device__ __forceinline__ void split2(float x, unsigned short& hi, unsigned short& lo) {
  if constexpr (PREC == 0) {
    const _Float16 h = (_Float16)x;
    const _Float16 l = (_Float16)(x - (float)h);
    hi = __builtin_bit_cast(unsigned short, h);
    lo = __builtin_bit_cast(unsigned short, l);
  } else {
    const __bf16 h = (__bf16)x;
    const __bf16 l = (__bf16)(x - (float)h);
    hi = __builtin_bit_cast(unsigned short, h);
    lo = __builtin_bit_cast(unsigned short, l);
  }
}

// x - hi for the FP16 half hi held in the low / high 16 bits of a packed
// dword: one mixed-precision FMA (-hi * 1 + x, exact in FP32) instead of a
// conversion and a subtraction.
__device__ __forceinline__ float sub_half_lo(unsigned packed, float x) {
  float r;
  asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(packed), "v"(x));
  return r;
}
__device__ __forceinline__ float sub_half_hi(unsigned packed, float x) {
  float r;
  asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(packed), "v"(x));
  return r;
}

// Splits two floats into packed (hi, hi) and (lo, lo) dwords.  FP16 uses the
// packed round-toward-zero conversion (the lo half carries the exact fp32
// remainder x - hi, so truncation costs at most one lo ulp).
template <int PREC>
__device__ __forceinline__ void split_pair(float a, float b, unsigned& hi, unsigned& lo) {
  if constexpr (PREC == 0) {
    hi = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(a, b));
    lo = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(sub_half_lo(hi, a), sub_half_hi(hi, b)));
  } else {
    // BF16, round to nearest even: both values by one packed conversion; the
    // hi halves back in FP32 are the top 16 bits, so x - hi is exact
    typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
    typedef float f2v __attribute__((ext_vector_type(2)));
    hi = __builtin_bit_cast(unsigned, __builtin_convertvector(f2v{a, b}, bf2));
    const float ha = __builtin_bit_cast(float, hi << 16), hb = __builtin_bit_cast(float, hi & 0xffff0000u);
    lo = __builtin_bit_cast(unsigned, __builtin_convertvector(f2v{a - ha, b - hb}, bf2));
  }
}

// Builds the constant fragments in FP64 and stores them split.
template <int N, int ST, int PREC>
__global__ void k_gemm_consts(unsigned short* __restrict__ frag) {
  using G = GemmLay<N, ST>;
  const int nw1 = G::W1_HALVES / 2;  // (hi, lo) pairs of W1
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nw1 + G::C_HALVES / 2) return;
  double val;
  int hi_at, lo_at;
  if (i < nw1) {
    // W1 element (kc, st, part, lane, j), part 0 re, 1 im, 2 -im
    constexpr int NP = G::W1_PARTS;
    const int j = i & 7, lane = (i >> 3) & 63, rest = i >> 9;
    const int part = rest % NP, st = (rest / NP) % ST, kc = (rest / NP) / ST;
    const int k = kc * 32 + 8 * (lane >> 4) + j;
    const int kk = G::FAST ? (k < G::B ? k : (k < 2 * G::B - 1 ? k + 2 : G::NK)) : k;
    const int slot = st * 16 + (lane & 15);
    const int s = slot - 8 * ST;
    if (kk < G::NK) {
      const int u = kk <= G::B ? kk : kk - G::NK;
      long ph = ((long)u * s) % N;
      if (ph < 0) ph += N;
      double sn, cs;
      sincospi(2.0 * (double)ph / (double)N, &sn, &cs);
      val = part == 0 ? cs : (part == 1 ? sn : -sn);
    } else {
      val = 0.0;
    }
    const int base = ((((kc * ST + st) * NP + part) * 2) * 64 + lane) * 8 + j;
    hi_at = base;
    lo_at = base + 512;
  } else {
    // C element (vt, sx, part, lane, j), part 0 re, 1 -im
    const int c = i - nw1;
    const int j = c & 3, lane = (c >> 2) & 63, rest = c >> 8;
    const int part = rest & 1, sx = (rest >> 1) % ST, vt = (rest >> 1) / ST;
    const int v = vt * 16 + 4 * (lane >> 4) + j;
    const int slot = sx * 16 + (lane & 15);
    const int s = slot - 8 * ST;
    if (v < (G::FAST ? G::B : G::NV)) {
      long ph = ((long)v * s) % N;
      if (ph < 0) ph += N;
      double sn, cs;
      sincospi(2.0 * (double)ph / (double)N, &sn, &cs);
      const double w = v == 0 ? 1.0 : 2.0;
      val = part == 0 ? w * cs : -w * sn;
    } else {
      val = 0.0;
    }
    const int base = G::W1_HALVES + ((((vt * ST + sx) * 2 + part) * 2) * 64 + lane) * 4 + j;
    hi_at = base;
    lo_at = base + 256;
  }
  unsigned short h, l;
  split2<PREC>((float)val, h, l);
  frag[hi_at] = h;
  frag[lo_at] = PREC == 2 ? (unsigned short)0 : l;
}

template <int PREC>
__device__ __forceinline__ f4 mfma32(const u4v& a, const u4v& b, const f4& c) {
  if constexpr (PREC == 0)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, a), __builtin_bit_cast(b8, b), c, 0, 0, 0);
}
template <int PREC>
__device__ __forceinline__ f4 mfma16(const u2v& a, const u2v& b, const f4& c) {
  if constexpr (PREC == 0)
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h4, a), __builtin_bit_cast(h4, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a), __builtin_bit_cast(s4, b), c, 0, 0, 0);
}

// Operand values of one (v tile, row chunk) for this lane: row v = vt 16 + lane % 16,
// band rows kk = kc 32 + 8 (lane / 16) + j.  Out-of-band rows and columns read a
// clamped address and are zeroed.
template <int N>
__device__ __forceinline__ void load_vals(const cf* __restrict__ S, int vt, int kc, int r16, int q4, cf* out) {
  constexpr int B = Plan<N>::B, NV = B + 1, NK = 2 * B + 1;
  if constexpr ((B % 8 == 0) && ((2 * B) % 32 == 0)) {
    // K rows of this lane group are contiguous band rows (k < B: row k,
    // else row k + 2); the one zero row at k = 2B - 1 reads a clamped row
    const int k0 = kc * 32 + 8 * q4;
    const int row0 = k0 < B ? k0 : k0 + 2;
    const cf* base = S + row0 * NV + vt * 16 + r16;
#pragma unroll
    for (int j = 0; j < 7; ++j) out[j] = base[j * NV];
    const bool pad = k0 + 7 == 2 * B - 1;
    const cf x = base[(pad ? 6 : 7) * NV];
    out[7] = pad ? cf{0.f, 0.f} : x;
    return;
  }
  const int v = vt * 16 + r16;
  const int vc = v < NV ? v : NV - 1;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int kk = kc * 32 + 8 * q4 + j;
    const int kc2 = kk < NK ? kk : NK - 1;
    const cf x = S[kc2 * NV + vc];
    out[j] = (v < NV && kk < NK) ? x : cf{0.f, 0.f};
  }
}

// exp(i pi k / 4), k in [0, 8)
__device__ __forceinline__ cf oct_root(int k) {
  constexpr float r = 0.70710678118654752440f;
  const float c[8] = {1.0f, r, 0.0f, -r, -1.0f, -r, 0.0f, r};
  return cf{c[k], c[(k + 6) & 7]};
}

// Staged fragments of 64 lanes x 8 complex values: value j of a lane sits at
// lane_base(frag, lane)[val_at(j)], with the 16-byte pairs (j / 2)
// lane-contiguous, so a 128-bit LDS read of one pair by 64 lanes touches
// consecutive addresses (lanes 64 bytes apart would put four of every eight
// lanes on the same banks).
template <class P>
__device__ __forceinline__ P* lane_base(P* frags, int frag, int lane) { return frags + frag * 512 + lane * 2; }
__device__ __forceinline__ constexpr int val_at(int j) { return (j >> 1) * 128 + (j & 1); }

template <int N, int ST, int PREC>
__global__ __launch_bounds__(512) void k_xcf_gemm(const cf* __restrict__ spec_p, int64_t np,
                                                  const cf* __restrict__ spec_l, int64_t nl, int lchunk,
                                                  int64_t nblk, int max_shift,
                                                  const unsigned short* __restrict__ frag_g,
                                                  float* __restrict__ scores) {
  using G = GemmLay<N, ST>;
  constexpr int VT = G::VT, KC = G::KC;
  constexpr bool TWO = PREC != 2;  // split products
  __shared__ __align__(16) unsigned char smem[G::LDS_BYTES];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t per = (nblk + 7) / 8;
  const int64_t g = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (g >= nblk) return;
  const int64_t chunk = g / np, p = g - chunk * np;
  const int r16 = lane & 15, q4 = lane >> 4;
  const cf* E = spec_p + p * G::SPEC;
  {
    const uint4* src = reinterpret_cast<const uint4*>(frag_g);
    uint4* dst = reinterpret_cast<uint4*>(smem);
    for (int i = tid; i < G::FRAG_BYTES / 16; i += 512) dst[i] = src[i];
    if constexpr (G::ELDS) {
      // pattern values in fragment order, pre-scaled: [vt][kc][lane][j]
      cf* es = reinterpret_cast<cf*>(smem + G::FRAG_BYTES);
      for (int f = wave; f < VT * KC; f += 8) {
        cf vals[8];
        load_vals<N>(E, f / KC, f % KC, r16, q4, vals);
#pragma unroll
        for (int j = 0; j < 8; ++j) lane_base(es, f, lane)[val_at(j)] = cscale(vals[j], kZScale);
      }
    }
  }
  __syncthreads();
  const u4v* w1f = reinterpret_cast<const u4v*>(smem);
  const u2v* cfr = reinterpret_cast<const u2v*>(smem + 2 * G::W1_HALVES);
  const cf* es = reinterpret_cast<const cf*>(smem + G::FRAG_BYTES);

  const int64_t l0 = chunk * lchunk;
  const int64_t l1 = l0 + lchunk < nl ? l0 + lchunk : nl;
  for (int64_t l = l0 + wave; l < l1; l += 8) {
    const cf* T = spec_l + l * G::SPEC;
    f4 rho[ST][ST];
#pragma unroll
    for (int a = 0; a < ST; ++a)
#pragma unroll
      for (int b = 0; b < ST; ++b) rho[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    cf tcur[8];
    load_vals<N>(T, 0, 0, r16, q4, tcur);
#pragma unroll 1
    for (int vt = 0; vt < VT; ++vt) {
      f4 ar[ST], ai[ST];
#pragma unroll
      for (int s = 0; s < ST; ++s) {
        ar[s] = f4{0.f, 0.f, 0.f, 0.f};
        ai[s] = f4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll 1
      for (int kc = 0; kc < KC; ++kc) {
        // prefetch the next chunk's template values
        int kn = kc + 1, vn = vt;
        if (kn == KC) {
          kn = 0;
          ++vn;
        }
        cf tnext[8];
        load_vals<N>(T, vn < VT ? vn : vt, kn, r16, q4, tnext);
        // Z = E conj(T), scaled, split into packed 16-bit halves
        cf ev[8];
        if constexpr (G::ELDS) {
#pragma unroll
          for (int j = 0; j < 8; ++j) ev[j] = lane_base(es, vt * KC + kc, lane)[val_at(j)];
        } else {
          load_vals<N>(E, vt, kc, r16, q4, ev);
#pragma unroll
          for (int j = 0; j < 8; ++j) ev[j] = cscale(ev[j], kZScale);
        }
        u4v zrh, zrl, zih, zil;
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
          const cf z0 = cmulc(ev[j], tcur[j]), z1 = cmulc(ev[j + 1], tcur[j + 1]);
          unsigned h, lo;
          split_pair<PREC>(z0.x, z1.x, h, lo);
          zrh[j / 2] = h;
          zrl[j / 2] = lo;
          split_pair<PREC>(z0.y, z1.y, h, lo);
          zih[j / 2] = h;
          zil[j / 2] = lo;
        }
        // Ar^T += Zr W1r + Zi (-W1i),  Ai^T += Zr W1i + Zi W1r; consecutive
        // MFMAs go to different accumulators
#pragma unroll
        for (int s = 0; s < ST; ++s) {
          const int fb = (kc * ST + s) * 2 * G::W1_PARTS * 64 + lane;  // [part][hi/lo][lane], u4v units
          const u4v wrh = w1f[fb], wrl = w1f[fb + 64];
          const u4v wih = w1f[fb + 128], wil = w1f[fb + 192];
          if constexpr (G::NEGW) {
            const u4v nwh = w1f[fb + 256], nwl = w1f[fb + 320];
            ar[s] = mfma32<PREC>(zrh, wrh, ar[s]);
            ai[s] = mfma32<PREC>(zrh, wih, ai[s]);
            ar[s] = mfma32<PREC>(zih, nwh, ar[s]);
            ai[s] = mfma32<PREC>(zih, wrh, ai[s]);
            if constexpr (TWO) {
              ar[s] = mfma32<PREC>(zrh, wrl, ar[s]);
              ai[s] = mfma32<PREC>(zrh, wil, ai[s]);
              ar[s] = mfma32<PREC>(zih, nwl, ar[s]);
              ai[s] = mfma32<PREC>(zih, wrl, ai[s]);
              ar[s] = mfma32<PREC>(zrl, wrh, ar[s]);
              ai[s] = mfma32<PREC>(zrl, wih, ai[s]);
              ar[s] = mfma32<PREC>(zil, nwh, ar[s]);
              ai[s] = mfma32<PREC>(zil, wrh, ai[s]);
            }
          } else {
            const u4v nzh = zih ^ 0x80008000u, nzl = zil ^ 0x80008000u;
            ar[s] = mfma32<PREC>(zrh, wrh, ar[s]);
            ai[s] = mfma32<PREC>(zrh, wih, ai[s]);
            ar[s] = mfma32<PREC>(nzh, wih, ar[s]);
            ai[s] = mfma32<PREC>(zih, wrh, ai[s]);
            if constexpr (TWO) {
              ar[s] = mfma32<PREC>(zrh, wrl, ar[s]);
              ai[s] = mfma32<PREC>(zrh, wil, ai[s]);
              ar[s] = mfma32<PREC>(nzh, wil, ar[s]);
              ai[s] = mfma32<PREC>(zih, wrl, ai[s]);
              ar[s] = mfma32<PREC>(zrl, wrh, ar[s]);
              ai[s] = mfma32<PREC>(zrl, wih, ai[s]);
              ar[s] = mfma32<PREC>(nzl, wih, ar[s]);
              ai[s] = mfma32<PREC>(zil, wrh, ai[s]);
            }
          }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) tcur[j] = tnext[j];
      }
      // stage 2: rho^T[s_x][s_y] += Cr^T Ar^T + (-Ci)^T Ai^T
      u2v brh[ST], brl[ST], bih[ST], bil[ST];
#pragma unroll
      for (int s = 0; s < ST; ++s) {
#pragma unroll
        for (int i = 0; i < 4; i += 2) {
          unsigned h, lo;
          split_pair<PREC>(ar[s][i], ar[s][i + 1], h, lo);
          brh[s][i / 2] = h;
          brl[s][i / 2] = lo;
          split_pair<PREC>(ai[s][i], ai[s][i + 1], h, lo);
          bih[s][i / 2] = h;
          bil[s][i / 2] = lo;
        }
      }
#pragma unroll
      for (int sx = 0; sx < ST; ++sx) {
        const int fb = (vt * ST + sx) * 4 * 64 + lane;  // [part][hi/lo][lane], u2v units
        const u2v crh = cfr[fb], crl = cfr[fb + 64];
        const u2v cih = cfr[fb + 128], cil = cfr[fb + 192];
#pragma unroll
        for (int sy = 0; sy < ST; ++sy) rho[sx][sy] = mfma16<PREC>(crh, brh[sy], rho[sx][sy]);
#pragma unroll
        for (int sy = 0; sy < ST; ++sy) rho[sx][sy] = mfma16<PREC>(cih, bih[sy], rho[sx][sy]);
        if constexpr (TWO) {
#pragma unroll
          for (int sy = 0; sy < ST; ++sy) {
            rho[sx][sy] = mfma16<PREC>(crh, brl[sy], rho[sx][sy]);
            rho[sx][sy] = mfma16<PREC>(cih, bil[sy], rho[sx][sy]);
          }
#pragma unroll
          for (int sy = 0; sy < ST; ++sy) {
            rho[sx][sy] = mfma16<PREC>(crl, brh[sy], rho[sx][sy]);
            rho[sx][sy] = mfma16<PREC>(cil, bih[sy], rho[sx][sy]);
          }
        }
      }
    }
    // rho^T tile [sx][sy]: lane holds s_x slot sx*16 + 4 q4 + i, s_y slot sy*16 + r16
    float cy[ST], cx4[ST][4];
#pragma unroll
    for (int a = 0; a < ST; ++a) {
      cy[a] = 0.0f;
#pragma unroll
      for (int i = 0; i < 4; ++i) cx4[a][i] = 0.0f;
    }
    if constexpr (G::FAST) {
      // the three band entries left out of the products (exp(2 pi i B s / N)
      // = exp(i pi (3 s mod 8) / 4) since B / N = 3/8)
      const cf za = cmulc(E[G::B * G::NV], T[G::B * G::NV]);              // u = +B, v = 0
      const cf zb = cmulc(E[(G::B + 1) * G::NV], T[(G::B + 1) * G::NV]);  // u = -B, v = 0
      const cf zc = cmulc(E[G::B], T[G::B]);                                // u = 0,  v = B
#pragma unroll
      for (int a = 0; a < ST; ++a) {
        const int syv = a * 16 + r16 - 8 * ST;
        const cf w = oct_root((3 * syv) & 7);
        cy[a] = (za.x * w.x - za.y * w.y) + (zb.x * w.x + zb.y * w.y);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int sxv = a * 16 + 4 * q4 + i - 8 * ST;
          const cf wx = oct_root((3 * sxv) & 7);
          cx4[a][i] = 2.0f * (zc.x * wx.x - zc.y * wx.y);
        }
      }
    }
    float m = -INFINITY;
#pragma unroll
    for (int sx = 0; sx < ST; ++sx)
#pragma unroll
      for (int sy = 0; sy < ST; ++sy)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int sxv = sx * 16 + 4 * q4 + i - 8 * ST, syv = sy * 16 + r16 - 8 * ST;
          const float val = __fmaf_rn(rho[sx][sy][i], kZUnscale, cy[sy] + cx4[sx][i]);
          if (abs(sxv) <= max_shift && abs(syv) <= max_shift) m = fmaxf(m, val);
        }
    m = wave_max(m);
    if (lane == 0) scores[p * nl + l] = m;
  }
}

// ---------------------------------------------------------------------------
int gemm_slot_tiles(int max_shift) { return (2 * max_shift + 1 + 15) / 16; }

#define EBSD_GEMM_SIZES(X) X(64) X(96) X(128) X(160) X(256)

// One row chunk of stage 1 for one 16-slot s_y tile: Ar^T += Zr W1r + Zi (-W1i),
// Ai^T += Zr W1i + Zi W1r, each product split into hi*hi + hi*lo + lo*hi
// (hi*hi only for plain BF16); consecutive MFMAs go to different accumulators.
template <int PREC, bool NEGW>
__device__ __forceinline__ void stage1_tile(const u4v& zrh, const u4v& zrl, const u4v& zih, const u4v& zil,
                                            const u4v* w1f, int fb, f4& ar, f4& ai) {
  constexpr bool TWO = PREC != 2;
  const u4v wrh = w1f[fb], wrl = w1f[fb + 64];
  const u4v wih = w1f[fb + 128], wil = w1f[fb + 192];
  if constexpr (NEGW) {
    const u4v nwh = w1f[fb + 256], nwl = w1f[fb + 320];
    ar = mfma32<PREC>(zrh, wrh, ar);
    ai = mfma32<PREC>(zrh, wih, ai);
    ar = mfma32<PREC>(zih, nwh, ar);
    ai = mfma32<PREC>(zih, wrh, ai);
    if constexpr (TWO) {
      ar = mfma32<PREC>(zrh, wrl, ar);
      ai = mfma32<PREC>(zrh, wil, ai);
      ar = mfma32<PREC>(zih, nwl, ar);
      ai = mfma32<PREC>(zih, wrl, ai);
      ar = mfma32<PREC>(zrl, wrh, ar);
      ai = mfma32<PREC>(zrl, wih, ai);
      ar = mfma32<PREC>(zil, nwh, ar);
      ai = mfma32<PREC>(zil, wrh, ai);
    }
  } else {
    const u4v nzh = zih ^ 0x80008000u, nzl = zil ^ 0x80008000u;
    ar = mfma32<PREC>(zrh, wrh, ar);
    ai = mfma32<PREC>(zrh, wih, ai);
    ar = mfma32<PREC>(nzh, wih, ar);
    ai = mfma32<PREC>(zih, wrh, ai);
    if constexpr (TWO) {
      ar = mfma32<PREC>(zrh, wrl, ar);
      ai = mfma32<PREC>(zrh, wil, ai);
      ar = mfma32<PREC>(nzh, wil, ar);
      ai = mfma32<PREC>(zih, wrl, ai);
      ar = mfma32<PREC>(zrl, wrh, ar);
      ai = mfma32<PREC>(zrl, wih, ai);
      ar = mfma32<PREC>(nzl, wih, ar);
      ai = mfma32<PREC>(zil, wrh, ai);
    }
  }
}

// Both 16-slot s_y tiles of one row chunk (ST = 2), with consecutive MFMAs
// cycling through the four accumulators so that no MFMA waits on the one
// just issued.
template <int PREC, bool NEGW>
__device__ __forceinline__ void stage1_tiles2(const u4v& zrh, const u4v& zrl, const u4v& zih, const u4v& zil,
                                              const u4v* w1f, int fb0, int fb1, f4* ar, f4* ai) {
  constexpr bool TWO = PREC != 2;
  const u4v wrh0 = w1f[fb0], wrl0 = w1f[fb0 + 64], wih0 = w1f[fb0 + 128], wil0 = w1f[fb0 + 192];
  const u4v wrh1 = w1f[fb1], wrl1 = w1f[fb1 + 64], wih1 = w1f[fb1 + 128], wil1 = w1f[fb1 + 192];
  u4v nwh0, nwl0, nwh1, nwl1, z2h, z2l;
  if constexpr (NEGW) {
    nwh0 = w1f[fb0 + 256];
    nwl0 = w1f[fb0 + 320];
    nwh1 = w1f[fb1 + 256];
    nwl1 = w1f[fb1 + 320];
    z2h = zih;
    z2l = zil;
  } else {
    nwh0 = wih0;
    nwl0 = wil0;
    nwh1 = wih1;
    nwl1 = wil1;
    z2h = zih ^ 0x80008000u;
    z2l = zil ^ 0x80008000u;
  }
  ar[0] = mfma32<PREC>(zrh, wrh0, ar[0]);
  ar[1] = mfma32<PREC>(zrh, wrh1, ar[1]);
  ai[0] = mfma32<PREC>(zrh, wih0, ai[0]);
  ai[1] = mfma32<PREC>(zrh, wih1, ai[1]);
  ar[0] = mfma32<PREC>(z2h, nwh0, ar[0]);
  ar[1] = mfma32<PREC>(z2h, nwh1, ar[1]);
  ai[0] = mfma32<PREC>(zih, wrh0, ai[0]);
  ai[1] = mfma32<PREC>(zih, wrh1, ai[1]);
  if constexpr (TWO) {
    ar[0] = mfma32<PREC>(zrh, wrl0, ar[0]);
    ar[1] = mfma32<PREC>(zrh, wrl1, ar[1]);
    ai[0] = mfma32<PREC>(zrh, wil0, ai[0]);
    ai[1] = mfma32<PREC>(zrh, wil1, ai[1]);
    ar[0] = mfma32<PREC>(z2h, nwl0, ar[0]);
    ar[1] = mfma32<PREC>(z2h, nwl1, ar[1]);
    ai[0] = mfma32<PREC>(zih, wrl0, ai[0]);
    ai[1] = mfma32<PREC>(zih, wrl1, ai[1]);
    ar[0] = mfma32<PREC>(zrl, wrh0, ar[0]);
    ar[1] = mfma32<PREC>(zrl, wrh1, ar[1]);
    ai[0] = mfma32<PREC>(zrl, wih0, ai[0]);
    ai[1] = mfma32<PREC>(zrl, wih1, ai[1]);
    ar[0] = mfma32<PREC>(z2l, nwh0, ar[0]);
    ar[1] = mfma32<PREC>(z2l, nwh1, ar[1]);
    ai[0] = mfma32<PREC>(zil, wrh0, ai[0]);
    ai[1] = mfma32<PREC>(zil, wrh1, ai[1]);
  }
}

// Pattern-tiled form: a block correlates PB patterns with 8 templates (one
// per wave).  The patterns' operand values of each (v tile, row chunk) step
// are staged once per block in LDS (a four-slot ring: during an even step
// waves w < PB stage step + 2 and the next PB waves step + 3, so one barrier
// closes each pair of steps; with EBSD_GEMM_PAIRSYNC=0 the two-slot form
// with a barrier per step) and every template value a wave loads serves PB patterns, so each pair
// costs SPEC / PB template bytes and SPEC / 8 pattern bytes of cache traffic
// instead of a full spectrum of each.  Blocks are numbered in super-tiles of
// a few template blocks, so the blocks running at one time on an XCD share
// their templates in its L2 and each streamed pattern block serves several.
template <int N, int ST, int PREC, int PB>
__global__ __launch_bounds__(512) void k_xcf_gemm_pt(const cf* __restrict__ spec_p, int64_t np,
                                                     const cf* __restrict__ spec_l, int64_t nl, int64_t npb,
                                                     int64_t nblk, int max_shift,
                                                     const unsigned short* __restrict__ frag_g,
                                                     float* __restrict__ scores) {
  using G = GemmLay<N, ST>;
  constexpr int VT = G::VT, KC = G::KC, NSTEP = VT * KC;
  constexpr bool TWO = PREC != 2;
  constexpr int EB = PB * 64 * 8;  // complex values per staging buffer
  constexpr int NSLOT = EBSD_GEMM_PAIRSYNC ? 4 : 2;
  __shared__ __align__(16) unsigned char smem[G::FRAG_BYTES + NSLOT * EB * sizeof(cf)];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t per = (nblk + 7) / 8;
  const int64_t g = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (g >= nblk) return;
  // super-tiles of TS template blocks: consecutive blocks (running at one time
  // on an XCD) cycle through the TS template blocks of one pattern block, so
  // each pattern block is read once per super-tile from HBM, not per
  // template block (the last super-tile may hold fewer template blocks).
  // TS x 8 template spectra stay in the XCD's L2: 4 x 8 x 38 KB at 128,
  // 2 x 8 x 150 KB at 256 (measured 1.05x at 128 and 256 over TS = 1)
  int64_t tb, pbk;
  {
    constexpr int TS = EBSD_GEMM_SUPER > 0 ? EBSD_GEMM_SUPER : (N >= 256 ? 2 : 4);
    const int64_t ntb = (nl + 7) / 8;
    const int64_t st = g / (TS * npb), tb0 = st * TS;
    const int64_t ts = ntb - tb0 < TS ? ntb - tb0 : TS;
    const int64_t r = g - tb0 * npb;
    pbk = r / ts;
    tb = tb0 + (r - pbk * ts);
  }
  const int64_t p0 = pbk * PB;
  const int64_t l = tb * 8 + wave;
  const bool lok = l < nl;
  const int r16 = lane & 15, q4 = lane >> 4;
  {
    const uint4* src = reinterpret_cast<const uint4*>(frag_g);
    uint4* dst = reinterpret_cast<uint4*>(smem);
    for (int i = tid; i < G::FRAG_BYTES / 16; i += 512) dst[i] = src[i];
  }
  const u4v* w1f = reinterpret_cast<const u4v*>(smem);
  const u2v* cfr = reinterpret_cast<const u2v*>(smem + 2 * G::W1_HALVES);
  cf* eb = reinterpret_cast<cf*>(smem + G::FRAG_BYTES);
  const cf* T = spec_l + (lok ? l : 0) * G::SPEC;
#if EBSD_GEMM_PAIRSYNC
  // waves w < 2 PB stage pattern p0 + w % PB of every other step (even
  // steps by w < PB, odd ones by the next PB waves), one barrier per pair
  const int sw = wave % PB;
  const bool stager = wave < 2 * PB;
  const int sodd = wave >= PB ? 1 : 0;
#else
  const int sw = wave;
  const bool stager = wave < PB;
  const int sodd = 0;
#endif
  const cf* Ew = spec_p + (p0 + sw < np ? p0 + sw : 0) * G::SPEC;
  const bool ewok = stager && p0 + sw < np;
  if (stager && sodd < NSTEP) {
    cf vals[8];
    load_vals<N>(Ew, sodd / KC, sodd % KC, r16, q4, vals);
#pragma unroll
    for (int j = 0; j < 8; ++j)
      lane_base(eb, sodd * PB + sw, lane)[val_at(j)] = ewok ? cscale(vals[j], kZScale) : cf{0.f, 0.f};
  }
  __syncthreads();

  f4 rho[PB][ST][ST];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int a = 0; a < ST; ++a)
#pragma unroll
      for (int b = 0; b < ST; ++b) rho[pb][a][b] = f4{0.f, 0.f, 0.f, 0.f};
  cf tcur[8];
  load_vals<N>(T, 0, 0, r16, q4, tcur);
#pragma unroll 1
  for (int vt = 0; vt < VT; ++vt) {
    f4 ar[PB][ST], ai[PB][ST];
#pragma unroll
    for (int pb = 0; pb < PB; ++pb)
#pragma unroll
      for (int s = 0; s < ST; ++s) {
        ar[pb][s] = f4{0.f, 0.f, 0.f, 0.f};
        ai[pb][s] = f4{0.f, 0.f, 0.f, 0.f};
      }
    // two steps per iteration for the split forms at 256 (the next step's
    // template values then need no register copies: 1.3-1.5 %); one for plain
    // BF16 and for four patterns per block, where two steps' registers spill
    constexpr int KU = TWO && PB <= 3 ? 2 : 1;
#pragma unroll KU
    for (int kc = 0; kc < KC; ++kc) {
      const int step = vt * KC + kc, buf = step & (NSLOT - 1);
      const bool more = step + 1 < NSTEP;
#if EBSD_GEMM_PAIRSYNC
      const int sstep = step + 2 + sodd;  // the step this wave stages now
      const bool stage_now = stager && (step & 1) == 0 && sstep < NSTEP;
#else
      const int sstep = step + 1;
      const bool stage_now = stager && more;
#endif
      const int kn = kc + 1 < KC ? kc + 1 : 0, vn = kc + 1 < KC ? vt : vt + 1;
      cf tnext[8], enext[8];
      load_vals<N>(T, more ? vn : vt, more ? kn : kc, r16, q4, tnext);
      if (stage_now) load_vals<N>(Ew, sstep / KC, sstep % KC, r16, q4, enext);
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) {
        const cf* ep = lane_base(static_cast<const cf*>(eb), buf * PB + pb, lane);
        u4v zrh, zrl, zih, zil;
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
          const cf z0 = cmulc(ep[val_at(j)], tcur[j]), z1 = cmulc(ep[val_at(j + 1)], tcur[j + 1]);
          unsigned h, lo;
          split_pair<PREC>(z0.x, z1.x, h, lo);
          zrh[j / 2] = h;
          zrl[j / 2] = lo;
          split_pair<PREC>(z0.y, z1.y, h, lo);
          zih[j / 2] = h;
          zil[j / 2] = lo;
        }
        if constexpr (ST == 2 && EBSD_GEMM_INTERLEAVE) {
          stage1_tiles2<PREC, G::NEGW>(zrh, zrl, zih, zil, w1f, (kc * ST) * 2 * G::W1_PARTS * 64 + lane,
                                       (kc * ST + 1) * 2 * G::W1_PARTS * 64 + lane, ar[pb], ai[pb]);
        } else {
#pragma unroll
          for (int s = 0; s < ST; ++s)
            stage1_tile<PREC, G::NEGW>(zrh, zrl, zih, zil, w1f, (kc * ST + s) * 2 * G::W1_PARTS * 64 + lane,
                                       ar[pb][s], ai[pb][s]);
        }
      }
      if (stage_now) {
#pragma unroll
        for (int j = 0; j < 8; ++j)
          lane_base(eb, (sstep & (NSLOT - 1)) * PB + sw, lane)[val_at(j)] =
              ewok ? cscale(enext[j], kZScale) : cf{0.f, 0.f};
      }
#if EBSD_GEMM_PAIRSYNC
      if ((step & 1) || step + 1 == NSTEP) __syncthreads();
#else
      __syncthreads();
#endif
#pragma unroll
      for (int j = 0; j < 8; ++j) tcur[j] = tnext[j];
    }
    // stage 2: rho^T[s_x][s_y] += Cr^T Ar^T + (-Ci)^T Ai^T
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      u2v brh[ST], brl[ST], bih[ST], bil[ST];
#pragma unroll
      for (int s = 0; s < ST; ++s) {
#pragma unroll
        for (int i = 0; i < 4; i += 2) {
          unsigned h, lo;
          split_pair<PREC>(ar[pb][s][i], ar[pb][s][i + 1], h, lo);
          brh[s][i / 2] = h;
          brl[s][i / 2] = lo;
          split_pair<PREC>(ai[pb][s][i], ai[pb][s][i + 1], h, lo);
          bih[s][i / 2] = h;
          bil[s][i / 2] = lo;
        }
      }
#pragma unroll
      for (int sx = 0; sx < ST; ++sx) {
        const int fb = (vt * ST + sx) * 4 * 64 + lane;
        const u2v crh = cfr[fb], crl = cfr[fb + 64];
        const u2v cih = cfr[fb + 128], cil = cfr[fb + 192];
#pragma unroll
        for (int sy = 0; sy < ST; ++sy) {
          rho[pb][sx][sy] = mfma16<PREC>(crh, brh[sy], rho[pb][sx][sy]);
          rho[pb][sx][sy] = mfma16<PREC>(cih, bih[sy], rho[pb][sx][sy]);
          if constexpr (TWO) {
            rho[pb][sx][sy] = mfma16<PREC>(crh, brl[sy], rho[pb][sx][sy]);
            rho[pb][sx][sy] = mfma16<PREC>(cih, bil[sy], rho[pb][sx][sy]);
            rho[pb][sx][sy] = mfma16<PREC>(crl, brh[sy], rho[pb][sx][sy]);
            rho[pb][sx][sy] = mfma16<PREC>(cil, bih[sy], rho[pb][sx][sy]);
          }
        }
      }
    }
  }
  if (!lok) return;
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const int64_t p = p0 + pb;
    if (p >= np) break;
    const cf* E = spec_p + p * G::SPEC;
    float cy[ST], cx4[ST][4];
#pragma unroll
    for (int a = 0; a < ST; ++a) {
      cy[a] = 0.0f;
#pragma unroll
      for (int i = 0; i < 4; ++i) cx4[a][i] = 0.0f;
    }
    if constexpr (G::FAST) {
      const cf za = cmulc(E[G::B * G::NV], T[G::B * G::NV]);              // u = +B, v = 0
      const cf zb = cmulc(E[(G::B + 1) * G::NV], T[(G::B + 1) * G::NV]);  // u = -B, v = 0
      const cf zc = cmulc(E[G::B], T[G::B]);                                // u = 0,  v = B
#pragma unroll
      for (int a = 0; a < ST; ++a) {
        const int syv = a * 16 + r16 - 8 * ST;
        const cf w = oct_root((3 * syv) & 7);
        cy[a] = (za.x * w.x - za.y * w.y) + (zb.x * w.x + zb.y * w.y);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int sxv = a * 16 + 4 * q4 + i - 8 * ST;
          const cf wx = oct_root((3 * sxv) & 7);
          cx4[a][i] = 2.0f * (zc.x * wx.x - zc.y * wx.y);
        }
      }
    }
    float m = -INFINITY;
#pragma unroll
    for (int sx = 0; sx < ST; ++sx)
#pragma unroll
      for (int sy = 0; sy < ST; ++sy)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int sxv = sx * 16 + 4 * q4 + i - 8 * ST, syv = sy * 16 + r16 - 8 * ST;
          const float val = __fmaf_rn(rho[pb][sx][sy][i], kZUnscale, cy[sy] + cx4[sx][i]);
          if (abs(sxv) <= max_shift && abs(syv) <= max_shift) m = fmaxf(m, val);
        }
    m = wave_max(m);
    if (lane == 0) scores[p * nl + l] = m;
  }
}

template <int N, int ST, int PREC>
static hipError_t run_gemm(const float2* spec_p, int64_t p, const float2* spec_l, int64_t l, int max_shift,
                           unsigned short* frag, float* scores, hipStream_t stream) {
  using G = GemmLay<N, ST>;
  if constexpr (G::FRAG_BYTES > 150 * 1024) {
    return hipErrorInvalidValue;  // constant fragments would not fit in LDS
  } else {
  const int nthr = G::W1_HALVES / 2 + G::C_HALVES / 2;
  hipLaunchKernelGGL((k_gemm_consts<N, ST, PREC>), dim3((nthr + 255) / 256), dim3(256), 0, stream, frag);
  // four patterns per block hold 32 accumulator tiles per wave at ST = 2
  // (at 256 the larger address arithmetic then spills, so three); wider
  // shift windows keep one pattern per block
  constexpr int PB = ST > 2 || kGemmPatternTile == 0 ? 0 : (N >= 256 && kGemmPatternTile > 3 ? 3 : kGemmPatternTile);
  if constexpr (PB > 0 && G::FRAG_BYTES + (EBSD_GEMM_PAIRSYNC ? 4 : 2) * PB * 64 * 8 * 8 <= 160 * 1024) {
    const int64_t ntb = (l + 7) / 8;
    // patterns per dispatch so that blocks x threads stays below 2^31
    const int64_t pmax = (((int64_t(1) << 31) / 512 - 8) / ntb) * PB;
    if (pmax < PB) return hipErrorInvalidValue;
    for (int64_t s = 0; s < p; s += pmax) {
      const int64_t pc = p - s < pmax ? p - s : pmax;
      const int64_t npb = (pc + PB - 1) / PB;
      const int64_t nblk = npb * ntb;
      const int64_t grid = ((nblk + 7) / 8) * 8;
      hipLaunchKernelGGL((k_xcf_gemm_pt<N, ST, PREC, PB>), dim3((unsigned)grid), dim3(512), 0, stream,
                         (const cf*)spec_p + s * G::SPEC, pc, (const cf*)spec_l, l, npb, nblk, max_shift, frag,
                         scores + s * l);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int lchunk = 32;
  const int64_t nchunk = (l + lchunk - 1) / lchunk;
  // patterns per dispatch so that blocks x threads stays below 2^31
  const int64_t pmax = ((int64_t(1) << 31) / 512 - 8) / nchunk;
  if (pmax < 1) return hipErrorInvalidValue;
  for (int64_t s = 0; s < p; s += pmax) {
    const int64_t pc = p - s < pmax ? p - s : pmax;
    const int64_t nblk = pc * nchunk;
    const int64_t grid = ((nblk + 7) / 8) * 8;
    hipLaunchKernelGGL((k_xcf_gemm<N, ST, PREC>), dim3((unsigned)grid), dim3(512), 0, stream,
                       (const cf*)spec_p + s * G::SPEC, pc, (const cf*)spec_l, l, lchunk, nblk, max_shift, frag,
                       scores + s * l);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
  }
}

size_t gemm_frag_bytes(int n, int max_shift) {
  const int st = gemm_slot_tiles(max_shift);
  if (st < 1 || st > 4) return 0;
  switch (n) {
#define EBSD_FB(NN)                                                        \
  case NN:                                                                 \
    switch (st) {                                                          \
      case 1: return GemmLay<NN, 1>::FRAG_BYTES;                          \
      case 2: return GemmLay<NN, 2>::FRAG_BYTES;                          \
      case 3: return GemmLay<NN, 3>::FRAG_BYTES;                          \
      default: return GemmLay<NN, 4>::FRAG_BYTES;                         \
    }
    EBSD_GEMM_SIZES(EBSD_FB)
#undef EBSD_FB
    default: return 0;
  }
}

bool gemm_supported(int n, int max_shift) {
  const size_t b = gemm_frag_bytes(n, max_shift);
  return max_shift >= 0 && b > 0 && b <= 150 * 1024;
}

hipError_t launch_xcf_gemm(int n, int precision, const float2* spec_p, int64_t p, const float2* spec_l, int64_t l,
                           int max_shift, unsigned short* frag, float* scores, hipStream_t stream) {
  if (p <= 0 || l <= 0) return hipSuccess;
  if (!gemm_supported(n, max_shift) || precision < 0 || precision > 2) return hipErrorInvalidValue;
  const int st = gemm_slot_tiles(max_shift);
#define EBSD_GP(NN, SS, PP) \
  if (n == NN && st == SS && precision == PP) return run_gemm<NN, SS, PP>(spec_p, p, spec_l, l, max_shift, frag, scores, stream);
#define EBSD_GS(NN) \
  EBSD_GP(NN, 1, 0) EBSD_GP(NN, 1, 1) EBSD_GP(NN, 1, 2) \
  EBSD_GP(NN, 2, 0) EBSD_GP(NN, 2, 1) EBSD_GP(NN, 2, 2) \
  EBSD_GP(NN, 3, 0) EBSD_GP(NN, 3, 1) EBSD_GP(NN, 3, 2) \
  EBSD_GP(NN, 4, 0) EBSD_GP(NN, 4, 1) EBSD_GP(NN, 4, 2)
  EBSD_GEMM_SIZES(EBSD_GS)
#undef EBSD_GS
#undef EBSD_GP
  return hipErrorInvalidValue;
}

}  // namespace ebsd

// Kernels of the proposal network (FP32): convolution and fully connected
// layers as tiled GEMMs on the FP32 matrix cores whose operands are read
// through index maps (the convolution's im2col never exists in memory),
// pooling, softmax cross-entropy, Adam, and the on-device training-data
// generator (random orientations, projection noise, binning,
// nearest-library labels).
#include "cnn_internal.hpp"
#include "ebsd_common.hpp"

#include <math.h>

namespace ebsd {
namespace cnn {

// ---------------------------------------------------------------------------
// Tiled FP32 GEMM on the matrix cores: C(m, n) = sum_k A(m, k) B(k, n) over k
// in the block's slice [z * kslice, (z + 1) * kslice) of [0, K).  TM x TN
// tiles (TM 64 or 128, TN 32, 64 or 128), KS-deep K steps through two LDS
// stages; wave w owns the (TM / 2) x (TN / 2) quarter (w & 1, w >> 1) as
// 16 x 16 tiles of v_mfma_f32_16x16x4f32 (A operand: lane l holds row l % 16,
// k = l / 16; B: k = l / 16, column l % 16; accumulator: rows 4 (l / 16) + r,
// column l % 16).  A::KFAST / B::KFAST choose which index runs along
// consecutive threads when the tile is loaded (the one that is contiguous in
// memory).  Larger tiles give each LDS operand read and each barrier more
// products: the launcher takes 128 rows and as many columns as N fills.
typedef float f4c __attribute__((ext_vector_type(4)));
#ifndef EBSD_TGEMM_KS
#define EBSD_TGEMM_KS 16
#endif
constexpr int KS = EBSD_TGEMM_KS;  // K depth of one step

// p[i] through a 32-bit byte offset from the (uniform) base, so that the
// load takes the base from scalar registers and one 32-bit offset per lane.
// Operands stay below 2^30 elements: batches of at most 4,096 patterns make
// the largest (the second layer's gradient map) 2^28.
__device__ __forceinline__ float ld32(const float* p, unsigned i) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(p) + (i << 2));
}
// p[i .. i + 3] in one 16-byte load (p 16-byte aligned, i a multiple of 4)
__device__ __forceinline__ f4c ld32x4(const float* p, unsigned i) {
  return *reinterpret_cast<const f4c*>(reinterpret_cast<const char*>(p) + (i << 2));
}
// p[(m + r ms) ld + k .. + 3] for r < CNT of a row-major matrix (k a
// multiple of 4): 16-byte loads when p is 16-byte aligned and ld a multiple
// of 4, else single ones
template <int CNT>
__device__ __forceinline__ void rows4(const float* p, int ld, int m, int k, int ms, f4c* v) {
  const unsigned o = (unsigned)m * (unsigned)ld + (unsigned)k, d = (unsigned)(ms * ld);
  if ((ld & 3) == 0 && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
#pragma unroll
    for (int r = 0; r < CNT; ++r) v[r] = ld32x4(p, o + r * d);
  } else {
#pragma unroll
    for (int r = 0; r < CNT; ++r)
#pragma unroll
      for (int j = 0; j < 4; ++j) v[r][j] = ld32(p, o + r * d + j);
  }
}

// The block's tile (x, y, z), numbered so that each XCD takes one run of
// consecutive tiles: the dispatcher hands block b to XCD b % 8, and tiles
// that share operand rows (the N tiles of one K slice) then meet in one L2.
__device__ __forceinline__ void xcd_tile(int& bx, int& by, int& bz) {
  const unsigned nx = gridDim.x, ny = gridDim.y, total = nx * ny * gridDim.z;
  const unsigned lin = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
  const unsigned xcd = lin & 7, q = lin >> 3, per = total >> 3, rem = total & 7;
  const unsigned item = xcd * per + min(xcd, rem) + q;
  bx = (int)(item % nx);
  by = (int)((item / nx) % ny);
  bz = (int)(item / (nx * ny));
}

// output maps that take a lane's four consecutive rows at once (QUAD)
template <class T, class = void>
struct OutQuad : std::false_type {};
template <class T>
struct OutQuad<T, std::void_t<decltype(T::QUAD)>> : std::bool_constant<T::QUAD> {};
template <class Out>
constexpr bool out_quad() { return OutQuad<Out>::value; }
// operand maps with a whole-step fetch (STEP), taken when stepwise(tile
// width) holds and the step and tile are whole.  KFAST false: a thread holds
// one row m (column n) of the tile and the values k0 + kw + ks r, ks = 256 /
// TM (TN), step().  KFAST true: the values of one k at rows (columns) m,
// m + 256 / KS, ..., stepk()
template <class T, class = void>
struct HasStep : std::false_type {};
template <class T>
struct HasStep<T, std::void_t<decltype(T::STEP)>> : std::bool_constant<T::STEP> {};

template <int TM, int TN, class A, class Bm, class Out>
__global__ __launch_bounds__(256) void k_tgemm(A a, Bm b, Out out, int M, int N, int K, int kslice) {
  static_assert((TM == 64 || TM == 128) && (TN == 32 || TN == 64 || TN == 128), "tile");
  constexpr int KRA = TM * KS / 256, KRB = TN * KS / 256;  // operand values per thread and step
  constexpr int TI = TM / 32, TJ = TN / 32;                 // 16 x 16 tiles per wave
  // two LDS stages: the operand values of the next K step are loaded into
  // registers while the matrix cores work on the current one, then stored
  // into the other stage (one barrier per step)
  __shared__ float as[2][KS][TM + 1];
  __shared__ float bs[2][KS][TN + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w & 1) * (TM / 2), wn = (w >> 1) * (TN / 2);
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int m0 = by * TM, n0 = bx * TN;
  const int kb = bz * kslice;
  const int ke = min(K, kb + kslice);
  f4c acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = f4c{0.f, 0.f, 0.f, 0.f};
  const int r16 = lane & 15, q4 = lane >> 4;
  // this thread's (m, k) and (k, n) positions in a KS-deep step
  int am[KRA], ak[KRA], bn[KRB], bk[KRB];
#pragma unroll
  for (int r = 0; r < KRA; ++r) {
    const int idx = tid + 256 * r;
    am[r] = A::KFAST ? idx / KS : idx % TM;
    ak[r] = A::KFAST ? idx % KS : idx / TM;
  }
#pragma unroll
  for (int r = 0; r < KRB; ++r) {
    const int idx = tid + 256 * r;
    bn[r] = Bm::KFAST ? idx / KS : idx % TN;
    bk[r] = Bm::KFAST ? idx % KS : idx / TN;
  }
  float ra[KRA], rb[KRB];
  // Whole-step fetches (see HasStep) for both operands, taken for every step
  // when the block's tile is whole and its K slice a whole number of steps;
  // otherwise every value goes through the bounds-tested maps.  The two loops
  // are compiled apart so that the bounds-tested path adds nothing (such as
  // its strength-reduced addresses) to the whole-step loop.
  auto fetch_steps = [&](int k0) {
    if (k0 >= ke) {
      // past the end: zeros for the stage nobody reads again
#pragma unroll
      for (int r = 0; r < KRA; ++r) ra[r] = 0.0f;
#pragma unroll
      for (int r = 0; r < KRB; ++r) rb[r] = 0.0f;
      return;
    }
    if constexpr (HasStep<A>::value && HasStep<Bm>::value) {
      if constexpr (A::KFAST) {
        // am[r] = tid / KS + (256 / KS) r and ak[r] = tid % KS for every r
        a.template stepk<KRA>(m0 + am[0], k0 + ak[0], 256 / KS, ra);
      } else {
        // am[r] = tid % TM and ak[r] = tid / TM + (256 / TM) r for every r
        a.template step<KRA>(m0 + am[0], k0, ak[0], 256 / TM, ra);
      }
      if constexpr (Bm::KFAST) {
        // bn[r] = tid / KS + (256 / KS) r and bk[r] = tid % KS for every r
        b.template stepk<KRB>(n0 + bn[0], k0 + bk[0], 256 / KS, rb);
      } else {
        // bn[r] = tid % TN and bk[r] = tid / TN + (256 / TN) r for every r
        b.template step<KRB>(n0 + bn[0], k0, bk[0], 256 / TN, rb);
      }
    }
  };
  auto fetch_tested = [&](int k0) {
#pragma unroll
    for (int r = 0; r < KRA; ++r) {
      const int m = m0 + am[r], k = k0 + ak[r];
      ra[r] = (m < M && k < ke) ? a(m, k) : 0.0f;
    }
#pragma unroll
    for (int r = 0; r < KRB; ++r) {
      const int n = n0 + bn[r], k2 = k0 + bk[r];
      rb[r] = (n < N && k2 < ke) ? b(k2, n) : 0.0f;
    }
  };
  auto stash = [&](int st) {
#pragma unroll
    for (int r = 0; r < KRA; ++r) as[st][ak[r]][am[r]] = ra[r];
#pragma unroll
    for (int r = 0; r < KRB; ++r) bs[st][bk[r]][bn[r]] = rb[r];
  };
  auto run = [&](auto whole) {
    constexpr bool W = decltype(whole)::value;
    auto fetch = [&](int k0) {
      if constexpr (W) fetch_steps(k0);
      else fetch_tested(k0);
    };
    fetch(kb);
    stash(0);
    __syncthreads();
    int st = 0;
    for (int k0 = kb; k0 < ke; k0 += KS) {
      // the next step's fetch and stash run unconditionally: past the end of
      // the slice zeros go to the stage nobody reads again.  With a
      // conditional stash the loads of one step could still count as
      // outstanding at the next step's zero-filled registers, and each step
      // would wait for its own A loads before it issued the B loads and its
      // products.
      fetch(k0 + KS);
#pragma unroll
      for (int k4 = 0; k4 < KS; k4 += 4) {
        float av[TI], bv[TJ];
#pragma unroll
        for (int i = 0; i < TI; ++i) av[i] = as[st][k4 + q4][wm + 16 * i + r16];
#pragma unroll
        for (int j = 0; j < TJ; ++j) bv[j] = bs[st][k4 + q4][wn + 16 * j + r16];
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
      }
      stash(st ^ 1);
      __syncthreads();
      st ^= 1;
    }
  };
  bool whole = false;
  if constexpr (HasStep<A>::value && HasStep<Bm>::value) {
    // a thread's A row (KFAST false) past M reads nothing: the whole tile is
    // required for both orders
    whole = (ke - kb) % KS == 0 && m0 + TM <= M && n0 + TN <= N && a.stepwise(TM) && b.stepwise(TN);
  }
  if (whole) run(std::true_type{});
  else run(std::false_type{});
  if constexpr (out_quad<Out>()) {
    // the four accumulator rows of a lane (m = 4 g .. 4 g + 3) go out together
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        const int m = m0 + wm + 16 * i + 4 * q4, n = n0 + wn + 16 * j + r16;
        if (m < M && n < N) out.quad(m, n, acc[i][j]);
      }
  } else {
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm + 16 * i + 4 * q4 + r, n = n0 + wn + 16 * j + r16;
          if (m < M && n < N) out(m, n, acc[i][j][r], bz);
        }
  }
}

// --- operand maps ---------------------------------------------------------
// Images are NCHW with H = W = 1 << lw.

// ---------------------------------------------------------------------------
// The same product with BF16 split operands on v_mfma_f32_16x16x32_bf16:
// every FP32 value x is split into x_hi = bf16(x) and x_lo = bf16(x - x_hi)
// (x - x_hi is exact), and a 16 x 16 x 32 tile takes the three products
// hi hi + hi lo + lo hi into an FP32 accumulator (the dropped lo lo term and
// the rounding of x_lo leave about 2^-16 of each product).  32-deep K steps
// through two LDS stages of hi / lo tiles stored [row][k] (80-byte rows, so
// the 16-byte fragment reads of 16 lanes meet 16 distinct bank quads);
// operand fragments: lane l holds row (column) l % 16, k = 8 (l / 16) + j.
// Operands split here: a thread of a KFAST-false one holds KR consecutive k
// of one row (one tap of a convolution: one bounds test) and stores its
// halves as 16-byte vectors; a thread of a KFAST one holds 4 consecutive k
// of each of its rows (16-byte loads where aligned) and stores 8-byte
// vectors.  Tiles may be 96 wide for a KFAST B.  Operands split
// ahead (PRESPLIT: the layer input ConvFwdSA, the weight rows SplitRows) are
// loaded and stored as halves, 16-byte vectors.  Used for the inference
// products, the training's fc and backward products (its convolutions stay
// FP32).
constexpr int KS2 = 32, LROW = 40;  // step depth; LDS row of 32 halves + 8 of padding
typedef __bf16 cnn_b8 __attribute__((ext_vector_type(8)));
typedef __bf16 cnn_bf2 __attribute__((ext_vector_type(2)));
typedef float cnn_f2 __attribute__((ext_vector_type(2)));
typedef unsigned cnn_u4 __attribute__((ext_vector_type(4)));
typedef unsigned cnn_u2 __attribute__((ext_vector_type(2)));
// two floats -> packed (hi, hi) and (lo, lo), round to nearest even
__device__ __forceinline__ void bf16_split2(float a, float b, unsigned& hi, unsigned& lo) {
  hi = __builtin_bit_cast(unsigned, __builtin_convertvector(cnn_f2{a, b}, cnn_bf2));
  const float ha = __builtin_bit_cast(float, hi << 16), hb = __builtin_bit_cast(float, hi & 0xffff0000u);
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector(cnn_f2{a - ha, b - hb}, cnn_bf2));
}

// operands whose BF16 halves were split ahead of the product (PRESPLIT),
// and among them the row-major ones (ROWS: SplitRows, used for B)
template <class T, class = void>
struct PreSplit : std::false_type {};
template <class T>
struct PreSplit<T, std::void_t<decltype(T::PRESPLIT)>> : std::bool_constant<T::PRESPLIT> {};
template <class T, class = void>
struct SplitRowsOp : std::false_type {};
template <class T>
struct SplitRowsOp<T, std::void_t<decltype(T::ROWS)>> : std::bool_constant<T::ROWS> {};
// B(k, n) = the BF16 halves of w[n][k], split ahead
// into rows of 2 k_len halves that interleave groups of 8: hi of k = 8 g ..
// 8 g + 7, then their lo (k_len a multiple of 32, rows 16-byte aligned), so
// a 32-deep step of one row is one 128-byte line of 8 16-byte chunks (chunk
// q: group q / 2, hi for even q, lo for odd).  k_tgemm_s gives each row 8
// lanes, lane q loading chunk q: a load instruction reads 8 whole lines.
struct SplitRows {
  static constexpr bool PRESPLIT = true;
  static constexpr bool ROWS = true;
  static constexpr bool KFAST = true;
  static constexpr bool STEP = true;
  const unsigned short* w;
  int k_len;
  __device__ bool stepwise(int) const { return true; }
  __device__ size_t hi_at(int n, int k) const { return (size_t)n * 2 * k_len + (k >> 3) * 16 + (k & 7); }
};

template <int TM, int TN, class A, class Bm, class Out>
__global__ __launch_bounds__(256) void k_tgemm_s(A a, Bm b, Out out, int M, int N, int K, int kslice) {
  static_assert((TM == 64 || TM == 128) && (TN == 32 || TN == 64 || TN == 128 || (TN == 96 && Bm::KFAST)),
                "tile (96 wide: K-fast B only)");
  constexpr int KRA = TM * KS2 / 256, KRB = TN * KS2 / 256;  // operand values per thread and step
  constexpr int TI = TM / 32, TJ = TN / 32;                   // 16 x 16 tiles per wave
  static_assert((A::KFAST || KRA % 8 == 0) && (Bm::KFAST || KRB % 8 == 0 || KRB == 4) && KRA % 2 == 0 &&
                    KRB % 2 == 0,
                "whole 16-byte vectors (or one 8-byte one) (KFAST false) or pairs (KFAST) per thread");
  __shared__ __attribute__((aligned(16))) unsigned short ah[2][TM][LROW], al[2][TM][LROW];
  __shared__ __attribute__((aligned(16))) unsigned short bh[2][TN][LROW], bl[2][TN][LROW];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w & 1) * (TM / 2), wn = (w >> 1) * (TN / 2);
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int m0 = by * TM, n0 = bx * TN;
  const int kb = bz * kslice;
  const int ke = min(K, kb + kslice);
  f4c acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = f4c{0.f, 0.f, 0.f, 0.f};
  const int r16 = lane & 15, g8 = (lane >> 4) * 8;
  // this thread's (m, k) and (k, n) positions in a step: KFAST false, KR
  // consecutive k of one row; KFAST true, one k of rows 256 / KS2 apart
  int am[KRA], ak[KRA], bn[KRB], bk[KRB];
#pragma unroll
  for (int r = 0; r < KRA; ++r) {
    am[r] = A::KFAST ? (tid + 256 * r) / KS2 : tid % TM;
    ak[r] = A::KFAST ? tid % KS2 : (tid / TM) * KRA + r;
  }
#pragma unroll
  for (int r = 0; r < KRB; ++r) {
    bn[r] = Bm::KFAST ? (tid + 256 * r) / KS2 : tid % TN;
    bk[r] = Bm::KFAST ? tid % KS2 : (tid / TN) * KRB + r;
  }
  float ra[KRA], rb[KRB];
  // a KFAST operand here: 4 consecutive k per thread (k0 + 4 (tid % 8)) of
  // rows tid / 8 + 32 r, fetched as 16-byte vectors where the operand allows
  // and stored as one 8-byte vector of hi and one of lo halves per row
  const int qk = 4 * (tid & 7), qr = tid >> 3;
  f4c va[A::KFAST ? TM / 32 : 1], vb[Bm::KFAST ? TN / 32 : 1];
  // a row-major pre-split B: 8 lanes per row, lane cq loading the row's
  // 16-byte chunk cq of the step, rows cr, cr + 32, ...
  const int cq = tid & 7, cr = tid >> 3;
  cnn_u4 bc[TN / 32];
  // a row's chunk cq of the step at k0 (bounds-tested: rows past R, k past ke
  // give zeros)
  auto chunk_at = [&](const SplitRows& w, int row, int R, int k0, cnn_u4& c) __attribute__((always_inline)) {
    const int kg = k0 + (cq >> 1) * 8;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k2 = kg + 2 * e;
      const bool ok0 = row < R && k2 < ke, ok1 = row < R && k2 + 1 < ke;
      const size_t o = ok0 ? w.hi_at(row, k2) + (cq & 1) * 8 : 0;
      c[e] = (ok0 ? (unsigned)w.w[o] : 0u) | (ok1 ? (unsigned)w.w[o + 1] << 16 : 0u);
    }
  };
  // pre-split A likewise: 256 / TM threads per row m, KPTA consecutive k each
  constexpr int TPM = 256 / TM, KPTA = KS2 / TPM;
  const int pm = tid / TPM, pka = (tid % TPM) * KPTA;
  unsigned ahv[KPTA / 2], alv[KPTA / 2];
  // the fetches return whether the A values are valid (a pre-split A's tap
  // outside the image: the stash stores zeros)
  auto fetch_steps = [&](int k0) __attribute__((always_inline)) -> int {
    int ok = 1;
    if constexpr (HasStep<A>::value && HasStep<Bm>::value) {
      if constexpr (PreSplit<A>::value) ok = a.template split_at<KPTA>(m0 + pm, k0 + pka, ahv, alv) ? 1 : 0;
      else if constexpr (A::KFAST) a.template stepk4<TM / 32>(m0 + qr, k0 + qk, 32, va);
      else a.template step<KRA>(m0 + am[0], k0, ak[0], 1, ra);
      if constexpr (SplitRowsOp<Bm>::value) {
#pragma unroll
        for (int j = 0; j < TN / 32; ++j)
          bc[j] = *reinterpret_cast<const cnn_u4*>(b.w + b.hi_at(n0 + cr + 32 * j, k0) + 8 * cq);
      } else if constexpr (Bm::KFAST) {
        b.template stepk4<TN / 32>(n0 + qr, k0 + qk, 32, vb);
      } else {
        b.template step<KRB>(n0 + bn[0], k0, bk[0], 1, rb);
      }
    }
    return ok;
  };
  auto fetch_tested = [&](int k0) __attribute__((always_inline)) -> int {
    if constexpr (PreSplit<A>::value) {
      const int m = m0 + pm;
#pragma unroll
      for (int e = 0; e < KPTA / 2; ++e) {
        const int k2 = k0 + pka + 2 * e;  // even: k2 and k2 + 1 share a group and a tap (ci even)
        a.pair_at(m, k2, m < M && k2 < ke, m < M && k2 + 1 < ke, ahv[e], alv[e]);
      }
    } else if constexpr (A::KFAST) {
#pragma unroll
      for (int r = 0; r < TM / 32; ++r)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int m = m0 + qr + 32 * r, k = k0 + qk + j;
          va[r][j] = (m < M && k < ke) ? a(m, k) : 0.0f;
        }
    } else {
#pragma unroll
      for (int r = 0; r < KRA; ++r) {
        const int m = m0 + am[r], k = k0 + ak[r];
        ra[r] = (m < M && k < ke) ? a(m, k) : 0.0f;
      }
    }
    if constexpr (SplitRowsOp<Bm>::value) {
#pragma unroll
      for (int j = 0; j < TN / 32; ++j) chunk_at(b, n0 + cr + 32 * j, N, k0, bc[j]);
    } else if constexpr (Bm::KFAST) {
#pragma unroll
      for (int r = 0; r < TN / 32; ++r)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n = n0 + qr + 32 * r, k2 = k0 + qk + j;
          vb[r][j] = (n < N && k2 < ke) ? b(k2, n) : 0.0f;
        }
    } else {
#pragma unroll
      for (int r = 0; r < KRB; ++r) {
        const int n = n0 + bn[r], k2 = k0 + bk[r];
        rb[r] = (n < N && k2 < ke) ? b(k2, n) : 0.0f;
      }
    }
    return 1;
  };
  // split and store one step's values into stage st
  auto stash = [&](int st, int ok) __attribute__((always_inline)) {
    if constexpr (PreSplit<A>::value) {
      if constexpr (KPTA >= 8) {
#pragma unroll
        for (int v = 0; v < KPTA / 8; ++v) {
          *reinterpret_cast<cnn_u4*>(&ah[st][pm][pka + 8 * v]) =
              ok ? cnn_u4{ahv[4 * v], ahv[4 * v + 1], ahv[4 * v + 2], ahv[4 * v + 3]} : cnn_u4{0u, 0u, 0u, 0u};
          *reinterpret_cast<cnn_u4*>(&al[st][pm][pka + 8 * v]) =
              ok ? cnn_u4{alv[4 * v], alv[4 * v + 1], alv[4 * v + 2], alv[4 * v + 3]} : cnn_u4{0u, 0u, 0u, 0u};
        }
      }
    } else if constexpr (A::KFAST) {
#pragma unroll
      for (int r = 0; r < TM / 32; ++r) {
        unsigned h0, l0, h1, l1;
        bf16_split2(va[r][0], va[r][1], h0, l0);
        bf16_split2(va[r][2], va[r][3], h1, l1);
        *reinterpret_cast<cnn_u2*>(&ah[st][qr + 32 * r][qk]) = cnn_u2{h0, h1};
        *reinterpret_cast<cnn_u2*>(&al[st][qr + 32 * r][qk]) = cnn_u2{l0, l1};
      }
    } else {
#pragma unroll
      for (int v = 0; v < KRA / 8; ++v) {
        cnn_u4 h, l;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          unsigned he, le;
          bf16_split2(ra[8 * v + 2 * e], ra[8 * v + 2 * e + 1], he, le);
          h[e] = he;
          l[e] = le;
        }
        *reinterpret_cast<cnn_u4*>(&ah[st][am[0]][ak[0] + 8 * v]) = h;
        *reinterpret_cast<cnn_u4*>(&al[st][am[0]][ak[0] + 8 * v]) = l;
      }
    }
    if constexpr (SplitRowsOp<Bm>::value) {
      unsigned short(*dst)[LROW] = (cq & 1) ? bl[st] : bh[st];
#pragma unroll
      for (int j = 0; j < TN / 32; ++j) *reinterpret_cast<cnn_u4*>(&dst[cr + 32 * j][(cq >> 1) * 8]) = bc[j];
    } else if constexpr (Bm::KFAST) {
#pragma unroll
      for (int r = 0; r < TN / 32; ++r) {
        unsigned h0, l0, h1, l1;
        bf16_split2(vb[r][0], vb[r][1], h0, l0);
        bf16_split2(vb[r][2], vb[r][3], h1, l1);
        *reinterpret_cast<cnn_u2*>(&bh[st][qr + 32 * r][qk]) = cnn_u2{h0, h1};
        *reinterpret_cast<cnn_u2*>(&bl[st][qr + 32 * r][qk]) = cnn_u2{l0, l1};
      }
    } else if constexpr (KRB == 4) {
      // 32-wide tiles: 4 consecutive k per thread, one 8-byte vector
      unsigned h0, l0, h1, l1;
      bf16_split2(rb[0], rb[1], h0, l0);
      bf16_split2(rb[2], rb[3], h1, l1);
      *reinterpret_cast<cnn_u2*>(&bh[st][bn[0]][bk[0]]) = cnn_u2{h0, h1};
      *reinterpret_cast<cnn_u2*>(&bl[st][bn[0]][bk[0]]) = cnn_u2{l0, l1};
    } else {
#pragma unroll
      for (int v = 0; v < KRB / 8; ++v) {
        cnn_u4 h, l;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          unsigned he, le;
          bf16_split2(rb[8 * v + 2 * e], rb[8 * v + 2 * e + 1], he, le);
          h[e] = he;
          l[e] = le;
        }
        *reinterpret_cast<cnn_u4*>(&bh[st][bn[0]][bk[0] + 8 * v]) = h;
        *reinterpret_cast<cnn_u4*>(&bl[st][bn[0]][bk[0] + 8 * v]) = l;
      }
    }
  };
  auto run = [&](auto whole) __attribute__((always_inline)) {
    constexpr bool W = decltype(whole)::value;
    auto fetch = [&](int k0) __attribute__((always_inline)) -> int {
      if constexpr (W) return fetch_steps(k0);
      else return fetch_tested(k0);
    };
    stash(0, fetch(kb));
    __syncthreads();
    int st = 0;
    for (int k0 = kb; k0 < ke; k0 += KS2) {
      // as in k_tgemm: the tested loop fetches and stashes unconditionally
      // (zeros past the end), the whole-step loop skips the step past the end
      const bool more = k0 + KS2 < ke;
      int ok = 1;
      if (!W || more) ok = fetch(k0 + KS2);
      cnn_u4 fa[TI][2], fb[TJ][2];
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        fa[i][0] = *reinterpret_cast<const cnn_u4*>(&ah[st][wm + 16 * i + r16][g8]);
        fa[i][1] = *reinterpret_cast<const cnn_u4*>(&al[st][wm + 16 * i + r16][g8]);
      }
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        fb[j][0] = *reinterpret_cast<const cnn_u4*>(&bh[st][wn + 16 * j + r16][g8]);
        fb[j][1] = *reinterpret_cast<const cnn_u4*>(&bl[st][wn + 16 * j + r16][g8]);
      }
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(cnn_b8, fa[i][0]),
                                                              __builtin_bit_cast(cnn_b8, fb[j][0]), acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(cnn_b8, fa[i][0]),
                                                              __builtin_bit_cast(cnn_b8, fb[j][1]), acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(cnn_b8, fa[i][1]),
                                                              __builtin_bit_cast(cnn_b8, fb[j][0]), acc[i][j], 0, 0, 0);
        }
      if (!W || more) stash(st ^ 1, ok);
      __syncthreads();
      st ^= 1;
    }
  };
  bool whole = false;
  if constexpr (HasStep<A>::value && HasStep<Bm>::value) {
    // K-fast operands are fetched in groups of 32 rows (stepk4)
    whole = (ke - kb) % KS2 == 0 && m0 + TM <= M && n0 + TN <= N && a.stepwise(A::KFAST ? 32 : TM) &&
            b.stepwise(Bm::KFAST ? 32 : TN);
  }
  if (whole) run(std::true_type{});
  else run(std::false_type{});
  if constexpr (out_quad<Out>()) {
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4), n = n0 + wn + 16 * j + r16;
        if (m < M && n < N) out.quad(m, n, acc[i][j]);
      }
  } else {
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r, n = n0 + wn + 16 * j + r16;
          if (m < M && n < N) out(m, n, acc[i][j][r], bz);
        }
  }
}

// Forward convolution, A(m, k) = the input pixel under tap t of channel c,
// with K ordered tap-major: k = t ci + c, t = 3 (dy + 1) + (dx + 1) (the
// weights are read from their tap-major copy, k_weights_tap, as WeightT).
// Output pixels are ordered by 2 x 2 pooling quad, m = ((b, Y, X), q), pixel
// (2 Y + q / 2, 2 X + q % 2), so that the four accumulator rows of a lane
// are one quad.  Offsets are 32-bit (inputs below 2^30 elements).  For
// ci >= 32 the values a thread loads in one 16- or 32-deep step (k = k0 +
// kw + ks r) share one tap: one bounds test, and the channels are ks planes
// apart.
struct ConvFwdA {
  static constexpr bool KFAST = false;
  static constexpr bool STEP = true;
  const float* in;
  int ci, lci, lw;  // lci = log2 ci
  __device__ void pix(int m, int& bb, int& y, int& x) const {
    const int lo = lw - 1, q = m & 3;
    x = 2 * ((m >> 2) & ((1 << lo) - 1)) + (q & 1);
    y = 2 * ((m >> (2 + lo)) & ((1 << lo) - 1)) + (q >> 1);
    bb = m >> (2 * lw);
  }
  __device__ float operator()(int m, int k) const {
    int bb, y, x;
    pix(m, bb, y, x);
    const int t = k >> lci, c = k & ((1 << lci) - 1);
    const int yy = y + t / 3 - 1, xx = x + t % 3 - 1, w = 1 << lw;
    if ((unsigned)yy >= (unsigned)w || (unsigned)xx >= (unsigned)w) return 0.0f;
    return in[(unsigned)(((((bb << lci) + c) << lw) + yy) << lw) + (unsigned)xx];
  }
  __device__ bool stepwise(int) const { return lci >= 5; }  // 32-deep steps share a tap too
  template <int CNT>
  __device__ void step(int m, int k0, int kw, int ks, float* v) const {
    int bb, y, x;
    pix(m, bb, y, x);
    const int t = k0 >> lci, c = (k0 & ((1 << lci) - 1)) + kw;
    const int yy = y + t / 3 - 1, xx = x + t % 3 - 1, w = 1 << lw;
    const bool inside = (unsigned)yy < (unsigned)w && (unsigned)xx < (unsigned)w;
    const unsigned base = (unsigned)(((((bb << lci) + c) << lw) + yy) << lw) + (unsigned)xx;
    const unsigned plane = (unsigned)ks << (2 * lw);
#pragma unroll
    for (int r = 0; r < CNT; ++r) v[r] = inside ? ld32(in, base + r * plane) : 0.0f;
  }
};
// Forward convolution reading an input already split for the BF16 products
// (k_tgemm_s): in[b][y][x] holds the ci channels' BF16 halves in groups of
// 8, hi of channels 8 g .. 8 g + 7 then their lo (2 ci halves per pixel,
// written by ConvReluPoolSplitOut).  K tap-major and output pixels
// quad-ordered as ConvFwdA.  split_at: a thread's KP consecutive k (one tap,
// channels c .. c + KP - 1, c a multiple of KP) as KP / 2 dwords of hi and
// of lo halves, loaded from the clamped pixel; false outside the image.
struct ConvFwdSA {
  static constexpr bool PRESPLIT = true;
  static constexpr bool KFAST = false;
  static constexpr bool STEP = true;
  const unsigned short* in;
  int ci, lci, lw;  // lci = log2 ci
  __device__ bool stepwise(int) const { return lci >= 5; }
  __device__ void pix(int m, int& bb, int& y, int& x) const {
    const int lo = lw - 1, q = m & 3;
    x = 2 * ((m >> 2) & ((1 << lo) - 1)) + (q & 1);
    y = 2 * ((m >> (2 + lo)) & ((1 << lo) - 1)) + (q >> 1);
    bb = m >> (2 * lw);
  }
  // hi half of channel c at pixel (bb, y, x); its lo is 8 halves on
  __device__ unsigned at(int bb, int y, int x, int c) const {
    return (((((unsigned)bb << lw) + (unsigned)y) << lw) + (unsigned)x) * (unsigned)(2 * ci) + (unsigned)((c >> 3) * 16 + (c & 7));
  }
  template <int KP>
  __device__ bool split_at(int m, int k, unsigned* h, unsigned* l) const {
    int bb, y, x;
    pix(m, bb, y, x);
    const int t = k >> lci, c = k & ((1 << lci) - 1);
    const int yy = y + t / 3 - 1, xx = x + t % 3 - 1, w = 1 << lw;
    const bool inside = (unsigned)yy < (unsigned)w && (unsigned)xx < (unsigned)w;
    const unsigned o = at(bb, min(max(yy, 0), w - 1), min(max(xx, 0), w - 1), c);
#pragma unroll
    for (int v = 0; v < KP / 8; ++v) {
      const cnn_u4 hv = *reinterpret_cast<const cnn_u4*>(in + o + 16 * v);
      const cnn_u4 lv = *reinterpret_cast<const cnn_u4*>(in + o + 16 * v + 8);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        h[4 * v + e] = hv[e];
        l[4 * v + e] = lv[e];
      }
    }
    return inside;
  }
  // channels c, c + 1 (c even) of tap k / ci at pixel m as (hi, lo) dwords;
  // ok0 / ok1: whether the two k are inside the product at all
  __device__ void pair_at(int m, int k, bool ok0, bool ok1, unsigned& h, unsigned& l) const {
    h = l = 0u;
    if (!ok0) return;
    int bb, y, x;
    pix(m, bb, y, x);
    const int t = k >> lci, c = k & ((1 << lci) - 1);
    const int yy = y + t / 3 - 1, xx = x + t % 3 - 1, w = 1 << lw;
    if ((unsigned)yy >= (unsigned)w || (unsigned)xx >= (unsigned)w) return;
    const unsigned o = at(bb, yy, xx, c);
    h = (unsigned)in[o] | (ok1 ? (unsigned)in[o + 1] << 16 : 0u);
    l = (unsigned)in[o + 8] | (ok1 ? (unsigned)in[o + 9] << 16 : 0u);
  }
};
// The pooled value of ConvReluPoolOut written split for the next layer's
// ConvFwdSA: out[b][Y][X] holds the co channels' halves in groups of 8
// (split inference only: no gradient positions)
struct ConvReluPoolSplitOut {
  static constexpr bool QUAD = true;
  unsigned short* out;
  const float* bias;
  int co, lw;  // lw: log2 of the pooled side
  __device__ void quad(int m, int n, const f4c& v) const {
    const int hw = 1 << (2 * lw);
    const int bb = (m >> 2) >> (2 * lw), p = (m >> 2) & (hw - 1);
    const float mx = fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3]));
    const float pv = fmaxf(mx + bias[n], 0.0f);
    unsigned h, l;
    bf16_split2(pv, 0.0f, h, l);
    const unsigned o = ((unsigned)bb * (unsigned)hw + (unsigned)p) * (unsigned)(2 * co) + (unsigned)((n >> 3) * 16 + (n & 7));
    out[o] = (unsigned short)h;
    out[o + 8] = (unsigned short)l;
  }
  __device__ void operator()(int, int, float, int) const {}
};
// pooled[b][n][Y][X] = max over the quad of max(acc + bias[n], 0), which is
// max(max over the quad of acc + bias[n], 0): adding the bias and clamping
// are monotone, so the value equals the unfused ReLU then max-pool exactly.
// With arg (training), arg[b][n][Y][X] = the quad position the pooled
// gradient flows back to: the first position q (order (0, 0), (0, 1),
// (1, 0), (1, 1)) whose ReLU output equals the pooled value, if that value is
// positive, else 4 (ReLU cut: no gradient).
struct ConvReluPoolOut {
  static constexpr bool QUAD = true;
  float* out;
  const float* bias;
  int co, lw;  // lw: log2 of the pooled side
  uint8_t* arg;
  __device__ void quad(int m, int n, const f4c& v) const {
    const int hw = 1 << (2 * lw);
    const int bb = (m >> 2) >> (2 * lw), p = (m >> 2) & (hw - 1);
    const float b = bias[n];
    const float mx = fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3]));
    const float pv = fmaxf(mx + b, 0.0f);
    const unsigned o = (unsigned)((bb * co + n) << (2 * lw)) + (unsigned)p;
    out[o] = pv;
    if (arg) {
      // v[q] + b == pv > 0 is max(v[q] + b, 0) == pv with a positive value
      const int q = !(pv > 0.0f) ? 4 : v[0] + b == pv ? 0 : v[1] + b == pv ? 1 : v[2] + b == pv ? 2 : 3;
      arg[o] = (uint8_t)q;
    }
  }
  __device__ void operator()(int, int, float, int) const {}
};
// B(k, n) = w[n][k]: the fc weights [classes][features], and the convolution
// weights in tap-major rows [co][9 ci] (k = t ci + c, see k_weights_tap)
struct WeightT {
  static constexpr bool KFAST = true;
  static constexpr bool STEP = true;
  const float* w;
  int k_len;
  __device__ float operator()(int k, int n) const { return w[(size_t)n * k_len + k]; }
  __device__ bool stepwise(int) const { return true; }
  template <int CNT>
  __device__ void stepk(int n, int k, int ns, float* v) const {
    const unsigned o = (unsigned)n * (unsigned)k_len + (unsigned)k, d = (unsigned)(ns * k_len);
#pragma unroll
    for (int r = 0; r < CNT; ++r) v[r] = ld32(w, o + r * d);
  }
  template <int CNT>
  __device__ void stepk4(int n, int k, int ns, f4c* v) const { rows4<CNT>(w, k_len, n, k, ns, v); }
};

// data gradient, A(m = (b, y, x), k) = g[b][o][y - dy + 1][x - dx + 1] with
// K tap-major as in the forward convolution: k = t co + o, t = 3 (dy + 1) +
// (dx + 1).  32-bit offsets (gradients below 2^30 elements); for co >= 32 a
// thread's values of one 16-deep step share one tap (one bounds test).
struct ConvBwdDataA {
  static constexpr bool KFAST = false;
  static constexpr bool STEP = true;
  const float* g;
  int lco, lw;  // lco = log2 co
  __device__ float operator()(int m, int k) const {
    const int w = 1 << lw;
    const int x = m & (w - 1), y = (m >> lw) & (w - 1), bb = m >> (2 * lw);
    const int t = k >> lco, o = k & ((1 << lco) - 1);
    const int yy = y - t / 3 + 1, xx = x - t % 3 + 1;
    if ((unsigned)yy >= (unsigned)w || (unsigned)xx >= (unsigned)w) return 0.0f;
    return g[(unsigned)(((((bb << lco) + o) << lw) + yy) << lw) + (unsigned)xx];
  }
  __device__ bool stepwise(int) const { return lco >= 5; }
  template <int CNT>
  __device__ void step(int m, int k0, int kw, int ks, float* v) const {
    const int w = 1 << lw;
    const int x = m & (w - 1), y = (m >> lw) & (w - 1), bb = m >> (2 * lw);
    const int t = k0 >> lco, o = (k0 & ((1 << lco) - 1)) + kw;
    const int yy = y - t / 3 + 1, xx = x - t % 3 + 1;
    const bool inside = (unsigned)yy < (unsigned)w && (unsigned)xx < (unsigned)w;
    const unsigned base = (unsigned)(((((bb << lco) + o) << lw) + yy) << lw) + (unsigned)xx;
    const unsigned plane = (unsigned)ks << (2 * lw);
#pragma unroll
    for (int r = 0; r < CNT; ++r) v[r] = inside ? ld32(g, base + r * plane) : 0.0f;
  }
};
// B(k = t co + o, n = c) = w[o][c][t], read from the tap-major rows wt[o][t ci
// + c] (contiguous in n).  For co >= 32 a thread's values of one step share
// the tap and lie ks rows apart.
struct WeightBwdData {
  static constexpr bool KFAST = false;
  static constexpr bool STEP = true;
  const float* wt;
  int ci, lco;
  __device__ float operator()(int k, int n) const {
    const int t = k >> lco, o = k & ((1 << lco) - 1);
    return wt[(unsigned)(o * 9 * ci + t * ci + n)];
  }
  __device__ bool stepwise(int) const { return lco >= 5; }
  template <int CNT>
  __device__ void step(int n, int k0, int kw, int ks, float* v) const {
    const int t = k0 >> lco, o = (k0 & ((1 << lco) - 1)) + kw;
    const unsigned base = (unsigned)(o * 9 * ci + t * ci + n), stride = (unsigned)(ks * 9 * ci);
#pragma unroll
    for (int r = 0; r < CNT; ++r) v[r] = ld32(wt, base + r * stride);
  }
};
// out[b][n][y][x] = acc
struct NchwOut {
  float* out;
  int c, lw;
  __device__ void operator()(int m, int n, float v, int) const {
    const int hw = 1 << (2 * lw);
    const int bb = m >> (2 * lw), p = m & (hw - 1);
    out[((size_t)bb * c + n) * hw + p] = v;
  }
};

// weight gradient, A(m = o, k = (b, y, x)) = g[b][o][y][x] (32-bit offsets:
// gradients below 2^30 elements).  Whole-step fetch: a thread's values of a
// step share k and lie ms rows apart.
struct ConvBwdWA {
  static constexpr bool KFAST = true;
  static constexpr bool STEP = true;
  const float* g;
  int co, lw;
  __device__ float operator()(int m, int k) const {
    const int hw = 1 << (2 * lw);
    return g[((unsigned)((k >> (2 * lw)) * co + m) << (2 * lw)) + (unsigned)(k & (hw - 1))];
  }
  __device__ bool stepwise(int) const { return true; }
  template <int CNT>
  __device__ void stepk(int m, int k, int ms, float* v) const {
    const int hw = 1 << (2 * lw);
    const unsigned base = ((unsigned)((k >> (2 * lw)) * co + m) << (2 * lw)) + (unsigned)(k & (hw - 1));
#pragma unroll
    for (int r = 0; r < CNT; ++r) v[r] = ld32(g, base + (unsigned)(r * ms) * (unsigned)hw);
  }
  // k_tgemm_s: k .. k + 3 (k a multiple of 4, one row of one plane) of rows
  // m + r ms, 16-byte loads
  template <int CNT>
  __device__ void stepk4(int m, int k, int ms, f4c* v) const {
    const int hw = 1 << (2 * lw);
    const unsigned base = ((unsigned)((k >> (2 * lw)) * co + m) << (2 * lw)) + (unsigned)(k & (hw - 1));
#pragma unroll
    for (int r = 0; r < CNT; ++r) v[r] = ld32x4(g, base + (unsigned)(r * ms) * (unsigned)hw);
  }
};
// B(k = (b, y, x), n) = in[b][c][y + dy - 1][x + dx - 1] with N tap-major,
// n = t ci + c, t = 3 dy + dx (the partial sums are put back into the stored
// [co][ci][3][3] order by the split sum).  When ci is a multiple of the tile
// width, a thread's values of a step (n, n + ns, ...) share one tap: one
// bounds test, channels ns planes apart.
struct ConvBwdWB {
  static constexpr bool KFAST = true;
  static constexpr bool STEP = true;
  const float* in;
  int lci, lw;  // lci = log2 ci
  __device__ float operator()(int k, int n) const {
    const int w = 1 << lw;
    const int x = k & (w - 1), y = (k >> lw) & (w - 1), bb = k >> (2 * lw);
    const int t = n >> lci, c = n & ((1 << lci) - 1);
    const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
    if ((unsigned)yy >= (unsigned)w || (unsigned)xx >= (unsigned)w) return 0.0f;
    return in[(unsigned)(((((bb << lci) + c) << lw) + yy) << lw) + (unsigned)xx];
  }
  __device__ bool stepwise(int tn) const { return (1 << lci) >= tn; }
  template <int CNT>
  __device__ void stepk(int n, int k, int ns, float* v) const {
    const int w = 1 << lw;
    const int x = k & (w - 1), y = (k >> lw) & (w - 1), bb = k >> (2 * lw);
    const int t = n >> lci, c = n & ((1 << lci) - 1);
    const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
    const bool inside = (unsigned)yy < (unsigned)w && (unsigned)xx < (unsigned)w;
    const unsigned base = (unsigned)(((((bb << lci) + c) << lw) + yy) << lw) + (unsigned)xx;
    const unsigned plane = (unsigned)ns << (2 * lw);
#pragma unroll
    for (int r = 0; r < CNT; ++r) v[r] = inside ? ld32(in, base + r * plane) : 0.0f;
  }
  // k_tgemm_s: k .. k + 3 (k a multiple of 4: pixels x .. x + 3 of one image
  // row) of columns n + r ns, each its own tap (ci >= 32: the 32 columns of a
  // group n0 + 32 r .. share one); a centre column of taps reads a 16-byte
  // vector, the side ones test their first or last pixel
  template <int CNT>
  __device__ void stepk4(int n, int k, int ns, f4c* v) const {
    const int w = 1 << lw;
    const int x = k & (w - 1), y = (k >> lw) & (w - 1), bb = k >> (2 * lw);
#pragma unroll
    for (int r = 0; r < CNT; ++r) {
      const int nr = n + r * ns, t = nr >> lci, c = nr & ((1 << lci) - 1);
      const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
      const bool iy = (unsigned)yy < (unsigned)w, i0 = iy && xx >= 0, i3 = iy && xx + 3 < w;
      const unsigned o = (unsigned)(((((bb << lci) + c) << lw) + yy) << lw) + (unsigned)xx;
      if (t % 3 == 1) {
        v[r] = iy ? ld32x4(in, o) : f4c{0.f, 0.f, 0.f, 0.f};
      } else {
        v[r][0] = i0 ? ld32(in, o) : 0.0f;
        v[r][1] = iy ? ld32(in, o + 1) : 0.0f;
        v[r][2] = iy ? ld32(in, o + 2) : 0.0f;
        v[r][3] = i3 ? ld32(in, o + 3) : 0.0f;
      }
    }
  }
};
// partial[z][m][n] = acc (split K, summed in a fixed order afterwards)
struct SplitOut {
  float* part;
  int M, N;
  __device__ void operator()(int m, int n, float v, int z) const { part[((size_t)z * M + m) * N + n] = v; }
};

// row-major matrices (the whole-step fetches use 32-bit offsets: operands
// below 2^30 elements)
struct RowK {  // A(m, k) = p[m * ld + k]
  static constexpr bool KFAST = true;
  static constexpr bool STEP = true;
  const float* p;
  int ld;
  __device__ float operator()(int m, int k) const { return p[(size_t)m * ld + k]; }
  __device__ bool stepwise(int) const { return true; }
  template <int CNT>
  __device__ void stepk(int m, int k, int ms, float* v) const {
    const unsigned o = (unsigned)m * (unsigned)ld + (unsigned)k, d = (unsigned)(ms * ld);
#pragma unroll
    for (int r = 0; r < CNT; ++r) v[r] = ld32(p, o + r * d);
  }
  // k_tgemm_s: k .. k + 3 of rows m + r ms (16-byte loads when ld is a
  // multiple of 4)
  template <int CNT>
  __device__ void stepk4(int m, int k, int ms, f4c* v) const { rows4<CNT>(p, ld, m, k, ms, v); }
};
struct ColK {  // A(m, k) = p[k * ld + m]
  static constexpr bool KFAST = false;
  static constexpr bool STEP = true;
  const float* p;
  int ld;
  __device__ float operator()(int m, int k) const { return p[(size_t)k * ld + m]; }
  __device__ bool stepwise(int) const { return true; }
  template <int CNT>
  __device__ void step(int m, int k0, int kw, int ks, float* v) const {
    const unsigned o = (unsigned)(k0 + kw) * (unsigned)ld + (unsigned)m, d = (unsigned)(ks * ld);
#pragma unroll
    for (int r = 0; r < CNT; ++r) v[r] = ld32(p, o + r * d);
  }
};
struct BRowN {  // B(k, n) = p[k * ld + n]
  static constexpr bool KFAST = false;
  static constexpr bool STEP = true;
  const float* p;
  int ld;
  __device__ float operator()(int k, int n) const { return p[(size_t)k * ld + n]; }
  __device__ bool stepwise(int) const { return true; }
  template <int CNT>
  __device__ void step(int n, int k0, int kw, int ks, float* v) const {
    const unsigned o = (unsigned)(k0 + kw) * (unsigned)ld + (unsigned)n, d = (unsigned)(ks * ld);
#pragma unroll
    for (int r = 0; r < CNT; ++r) v[r] = ld32(p, o + r * d);
  }
};
struct RowOut {  // C[m * ld + n] = acc (+ bias[n])
  float* out;
  const float* bias;
  int ld;
  __device__ void operator()(int m, int n, float v, int) const {
    out[(size_t)m * ld + n] = bias ? v + bias[n] : v;
  }
};

// K slice of a split into `splits` parts (a whole number of K steps) and the
// number of slices z that gemm launches: callers summing the partials use
// the same z
static int k_slice(int K, int splits) {
  splits = splits < 1 ? 1 : splits;
  const int kslice = (K + splits - 1) / splits;
  return (kslice + KS - 1) / KS * KS;
}
static int k_slices(int K, int splits) {
  const int kslice = k_slice(K, splits);
  return (K + kslice - 1) / kslice;
}

template <class A, class Bm, class Out>
static hipError_t gemm(A a, Bm b, Out out, int M, int N, int K, int splits, hipStream_t st, bool wide = false,
                       bool narrow = false) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int kslice = k_slice(K, splits);
  const int z = k_slices(K, splits) < 1 ? 1 : k_slices(K, splits);
  // wide: 128-row tiles and as many columns (up to 128) as N fills, taken
  // only while that grid still gives every compute unit two blocks (small
  // batches keep the 64 x 64 tiles, which make four times as many blocks)
  const int tn = N <= 32 ? 32 : N <= 64 ? 64 : 128;
  if (wide && (int64_t)((N + tn - 1) / tn) * ((M + 127) / 128) * z < 512) wide = false;
  if (wide && N <= 32) {
    hipLaunchKernelGGL((k_tgemm<128, 32, A, Bm, Out>), dim3((N + 31) / 32, (M + 127) / 128, z), dim3(256), 0, st,
                       a, b, out, M, N, K, kslice);
  } else if (wide && N <= 64) {
    hipLaunchKernelGGL((k_tgemm<128, 64, A, Bm, Out>), dim3((N + 63) / 64, (M + 127) / 128, z), dim3(256), 0, st,
                       a, b, out, M, N, K, kslice);
  } else if (wide) {
    hipLaunchKernelGGL((k_tgemm<128, 128, A, Bm, Out>), dim3((N + 127) / 128, (M + 127) / 128, z), dim3(256), 0,
                       st, a, b, out, M, N, K, kslice);
  } else if (narrow) {
    // narrow: 64 x 32 tiles (operands whose whole-step fetch needs tiles at
    // most 32 wide)
    hipLaunchKernelGGL((k_tgemm<64, 32, A, Bm, Out>), dim3((N + 31) / 32, (M + 63) / 64, z), dim3(256), 0, st, a, b,
                       out, M, N, K, kslice);
  } else {
    hipLaunchKernelGGL((k_tgemm<64, 64, A, Bm, Out>), dim3((N + 63) / 64, (M + 63) / 64, z), dim3(256), 0, st, a, b,
                       out, M, N, K, kslice);
  }
  return hipGetLastError();
}

// K slice of a split into `splits` parts for k_tgemm_s (a whole number of its
// 32-deep steps) and the number of slices z it launches
static int k_slice_s(int K, int splits) {
  splits = splits < 1 ? 1 : splits;
  const int kslice = (K + splits - 1) / splits;
  return (kslice + KS2 - 1) / KS2 * KS2;
}
static int k_slices_s(int K, int splits) {
  const int kslice = k_slice_s(K, splits);
  return (K + kslice - 1) / kslice;
}

// products with BF16 split operands (k_tgemm_s): 128-row tiles where allowed
// and the grid stays large, narrow 64 x 32 on request, else 64 x 64
template <class A, class Bm, class Out>
static hipError_t gemm_split(A a, Bm b, Out out, int M, int N, int K, hipStream_t st, int splits = 1,
                             bool wide_ok = true, bool narrow = false) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int kslice = k_slice_s(K, splits);
  const int z = k_slices_s(K, splits) < 1 ? 1 : k_slices_s(K, splits);
  const int tn = N <= 32 ? 32 : N <= 64 ? 64 : 128;
  // 128-row tiles once they still give 1,024 blocks (four per CU: timed
  // against 256, 512 and 2,048, the fc of a 2,048-pattern pass with its
  // 1,008 such blocks runs faster on 64 x 64 tiles)
  const bool wide = wide_ok && (int64_t)((N + tn - 1) / tn) * ((M + 127) / 128) * z >= 1024;
  if (wide && N <= 32) {
    hipLaunchKernelGGL((k_tgemm_s<128, 32, A, Bm, Out>), dim3((N + 31) / 32, (M + 127) / 128, z), dim3(256), 0, st,
                       a, b, out, M, N, K, kslice);
  } else if (wide && N <= 64) {
    hipLaunchKernelGGL((k_tgemm_s<128, 64, A, Bm, Out>), dim3((N + 63) / 64, (M + 127) / 128, z), dim3(256), 0, st,
                       a, b, out, M, N, K, kslice);
  } else if (wide) {
    hipLaunchKernelGGL((k_tgemm_s<128, 128, A, Bm, Out>), dim3((N + 127) / 128, (M + 127) / 128, z), dim3(256), 0,
                       st, a, b, out, M, N, K, kslice);
  } else if (narrow) {
    hipLaunchKernelGGL((k_tgemm_s<64, 32, A, Bm, Out>), dim3((N + 31) / 32, (M + 63) / 64, z), dim3(256), 0, st, a,
                       b, out, M, N, K, kslice);
  } else {
    hipLaunchKernelGGL((k_tgemm_s<64, 64, A, Bm, Out>), dim3((N + 63) / 64, (M + 63) / 64, z), dim3(256), 0, st, a,
                       b, out, M, N, K, kslice);
  }
  return hipGetLastError();
}

// part [z][M][N] -> out [M][N]: a block sums 64 consecutive outputs with G
// groups of 64 threads, group g taking the partials k = g, g + G, ...; the
// groups' sums are then added in group order (a fixed order, as the split
// itself is fixed).  G = 16 when the split is long (few outputs, many
// partials), else 1.  With nt > 0 the columns of part are tap-major, n =
// t ci + c (ci = 2^lci, nt = 9 ci), and go out in [c][t] order.
template <int G>
__global__ __launch_bounds__(64 * G) void k_split_sum(const float* __restrict__ part, int z, int64_t mn,
                                                      float* __restrict__ out, int nt, int lci) {
  __shared__ float acc[G][64];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  float s = 0.0f;
  if (i < mn)
    for (int k = g; k < z; k += G) s += part[(size_t)k * mn + i];
  int64_t o = i;
  if (nt > 0) {
    const int64_t m = i / nt;
    const int n = (int)(i - m * nt), t = n >> lci, c = n & ((1 << lci) - 1);
    o = m * nt + c * 9 + t;
  }
  if constexpr (G == 1) {
    if (i < mn) out[o] = s;
  } else {
    acc[g][lane] = s;
    __syncthreads();
    if (g == 0 && i < mn) {
      float t = acc[0][lane];
#pragma unroll
      for (int h = 1; h < G; ++h) t += acc[h][lane];
      out[o] = t;
    }
  }
}
static void split_sum(const float* part, int z, int64_t mn, float* out, hipStream_t st, int nt = 0, int lci = 0) {
  const unsigned blocks = (unsigned)((mn + 63) / 64);
  if (z >= 64) hipLaunchKernelGGL(k_split_sum<16>, dim3(blocks), dim3(1024), 0, st, part, z, mn, out, nt, lci);
  else hipLaunchKernelGGL(k_split_sum<1>, dim3(blocks), dim3(64), 0, st, part, z, mn, out, nt, lci);
}

// Bias gradient of a convolution, the sum over (b, pixel) of g[b][c][pixel].
// g is zero except at the recorded quad position of each pooled output,
// where it is the pooled gradient, so the sum runs over the pooled maps:
// block (c, z) sums images z, z + Z, ... of dpool where arg < 4 (first
// stage, in double)
__global__ __launch_bounds__(256) void k_channel_part(const uint8_t* __restrict__ arg, const float* __restrict__ dpool,
                                                      int bsz, int c, int lhw, int zs, double* __restrict__ part) {
  // the block's images bb = z, z + zs, ... and their hw = 2^lhw pixels as one
  // range, spread over all threads (the pooled maps of the last layers hold
  // 16 and 64 pixels)
  const int ch = blockIdx.x, z = blockIdx.y, hw = 1 << lhw;
  const int n = ((bsz - z + zs - 1) / zs) << lhw;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) {
    const size_t o = ((size_t)(z + zs * (j >> lhw)) * c + ch) * hw + (j & (hw - 1));
    s += arg[o] < 4 ? dpool[o] : 0.0f;
  }
  s = wave_sum(s);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)ch * zs + z] = red[0] + red[1] + red[2] + red[3];
}

// second stage, one wave per channel (zs <= 64): out[c] = sum_z part[c][z]
// by a fixed butterfly
__global__ __launch_bounds__(64) void k_channel_sum(const double* __restrict__ part, int zs,
                                                    float* __restrict__ out) {
  const int ch = blockIdx.x, z = threadIdx.x;
  const double s = wave_sum(z < zs ? part[(size_t)ch * zs + z] : 0.0);
  if (z == 0) out[ch] = (float)s;
}

// column sums of a [rows][cols] matrix: a block takes 64 columns, thread
// (x, y) of its 64 x 16 sums rows y, y + 16, ..., then the 16 partials are
// added in order
__global__ __launch_bounds__(1024) void k_col_sum(const float* __restrict__ a, int rows, int cols,
                                                  float* __restrict__ out) {
  __shared__ float red[16][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + tx;
  float s = 0.0f;
  if (j < cols)
    for (int r = ty; r < rows; r += 16) s += a[(size_t)r * cols + j];
  red[ty][tx] = s;
  __syncthreads();
  if (ty == 0 && j < cols) {
    float t = red[0][tx];
#pragma unroll
    for (int y = 1; y < 16; ++y) t += red[y][tx];
    out[j] = t;
  }
}

// Weight gradient of the first convolution (one input channel, 64 x 64):
// dW[o][t] = sum over (b, y, x) of g[b][o][y][x] in[b][y + dy - 1][x + dx - 1],
// t = 3 dy + dx.  g is the pooled gradient at each pooled output's recorded
// quad position and zero elsewhere, so the sum runs over the pooled maps.
// Block (b, group of OG channels) loads its pooled gradients and positions
// first, then stages image b with a zero border in LDS; a thread takes
// pooled positions i, i + 256, ... of each channel, and the block's nine sums
// per channel go to part[b][o][t] (fixed order: lanes, then waves), summed
// over b afterwards.
template <int OG>
__global__ __launch_bounds__(256) void k_wgrad_first(const float* __restrict__ x, const uint8_t* __restrict__ arg,
                                                     const float* __restrict__ dpool, int co,
                                                     float* __restrict__ part) {
  constexpr int W = kInSize, WP = W / 2, S = W + 2, PR = WP * WP / 256;
  __shared__ float xs[S * S];
  __shared__ float red[4][OG][9];
  const int bb = blockIdx.x, o0 = blockIdx.y * OG, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int q[OG][PR];
  float d[OG][PR];
#pragma unroll
  for (int oi = 0; oi < OG; ++oi)
#pragma unroll
    for (int r = 0; r < PR; ++r) {
      const size_t o = ((size_t)bb * co + o0 + oi) * (WP * WP) + tid + 256 * r;
      q[oi][r] = arg[o];
      d[oi][r] = dpool[o];
    }
  for (int i = tid; i < S * S; i += 256) {
    const int yy = i / S - 1, xx = i % S - 1;
    xs[i] = ((unsigned)yy < (unsigned)W && (unsigned)xx < (unsigned)W) ? x[((size_t)bb * W + yy) * W + xx] : 0.0f;
  }
  __syncthreads();
#pragma unroll
  for (int oi = 0; oi < OG; ++oi) {
    float acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = 0.0f;
#pragma unroll
    for (int r = 0; r < PR; ++r) {
      const int i = tid + 256 * r, qq = q[oi][r];
      const float dv = qq < 4 ? d[oi][r] : 0.0f;
      // full-resolution pixel of the quad position (any position when q = 4:
      // dv = 0 there), shifted by the border
      const int py = 2 * (i / WP) + ((qq >> 1) & 1), px = 2 * (i % WP) + (qq & 1);
      const float* xp = xs + py * S + px;
#pragma unroll
      for (int t = 0; t < 9; ++t) acc[t] = fmaf(dv, xp[(t / 3) * S + t % 3], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      float v = acc[t];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) red[w][oi][t] = v;
    }
  }
  __syncthreads();
  if (tid < OG * 9) {
    const int oi = tid / 9, t = tid % 9;
    part[((size_t)bb * co + o0 + oi) * 9 + t] = ((red[0][oi][t] + red[1][oi][t]) + red[2][oi][t]) + red[3][oi][t];
  }
}

// Convolution weights [co][ci][3][3] -> tap-major rows wt[o][t ci + c] =
// w[o][c][t], the four layers in one launch
__global__ void k_weights_tap(const float* __restrict__ params, Layout lay, float* __restrict__ wt) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= kTapWeights) return;
  int l = 0;
  while (l < 3 && j >= tap_weights_offset(l + 1)) ++l;
  const int ci = l ? kChannels[l - 1] : 1;
  const int64_t i = j - tap_weights_offset(l);
  const int64_t o = i / (9 * ci);
  const int rem = (int)(i - o * 9 * ci), t = rem / ci, c = rem - t * ci;
  wt[j] = params[lay.conv_w[l] + (o * ci + c) * 9 + t];
}

// BF16 halves (x_hi = bf16(x), x_lo = bf16(x - x_hi)) of rows floats rows of
// k_len (a multiple of 8) into the interleaved rows of SplitRows: a thread
// takes one group of 8
__global__ void k_split_rows(const float* __restrict__ x, int64_t rows, int k_len, unsigned short* __restrict__ w) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;  // group index
  const int gpr = k_len >> 3;
  if (g >= rows * gpr) return;
  const int64_t n = g / gpr;
  const int kg = (int)(g - n * gpr);
  const float* src = x + n * k_len + 8 * kg;
  unsigned short* dst = w + n * 2 * k_len + 16 * kg;
  cnn_u4 h, l;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    unsigned he, le;
    bf16_split2(src[2 * e], src[2 * e + 1], he, le);
    h[e] = he;
    l[e] = le;
  }
  *reinterpret_cast<cnn_u4*>(dst) = h;
  *reinterpret_cast<cnn_u4*>(dst + 8) = l;
}

// The first convolution (one input channel: K = 9) with its bias, ReLU and
// 2 x 2 max pool on the vector ALUs, which suit a 9-deep product better
// than 16- or 32-deep matrix steps: a thread takes one pooled pixel, its
// 4 x 4 input patch in registers and every channel (the weights, the same
// for every lane, come through the scalar cache).  Pooled value and
// gradient position as ConvReluPoolOut; SPLIT: the pooled map written in
// ConvReluPoolSplitOut's split layout instead.  w: [32][9], x: [bsz][64][64].
template <bool SPLIT>
__global__ __launch_bounds__(256) void k_conv1_pool(const float* __restrict__ x, const float* __restrict__ w,
                                                    const float* __restrict__ bias, int64_t bsz,
                                                    float* __restrict__ out, uint8_t* __restrict__ arg,
                                                    unsigned short* __restrict__ sout) {
  constexpr int S = kInSize, PS = S / 2, C = kChannels[0];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= bsz * PS * PS) return;
  const int X = (int)(i & (PS - 1)), Y = (int)((i / PS) & (PS - 1));
  const int64_t bb = i / (PS * PS);
  const float* img = x + bb * S * S;
  float pt[4][4];  // input rows 2 Y - 1 .. 2 Y + 2, columns 2 X - 1 .. 2 X + 2 (zero padding)
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int yy = 2 * Y - 1 + r, xx = 2 * X - 1 + s;
      pt[r][s] = ((unsigned)yy < (unsigned)S && (unsigned)xx < (unsigned)S) ? img[yy * S + xx] : 0.0f;
    }
  for (int c0 = 0; c0 < C; c0 += 8) {
    float pv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = c0 + e;
      float wt[9];
#pragma unroll
      for (int t = 0; t < 9; ++t) wt[t] = w[c * 9 + t];
      float v[4];  // quad positions (0, 0), (0, 1), (1, 0), (1, 1)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float a = 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) a = __builtin_fmaf(pt[(q >> 1) + t / 3][(q & 1) + t % 3], wt[t], a);
        v[q] = a;
      }
      const float b = bias[c];
      const float mx = fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3]));
      const float pool = fmaxf(mx + b, 0.0f);
      pv[e] = pool;
      if constexpr (!SPLIT) {
        const int64_t o = ((bb * C + c) * PS + Y) * PS + X;
        out[o] = pool;
        if (arg) {
          const int q = !(pool > 0.0f) ? 4 : v[0] + b == pool ? 0 : v[1] + b == pool ? 1 : v[2] + b == pool ? 2 : 3;
          arg[o] = (uint8_t)q;
        }
      }
    }
    if constexpr (SPLIT) {
      cnn_u4 h, l;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        unsigned he, le;
        bf16_split2(pv[2 * e], pv[2 * e + 1], he, le);
        h[e] = he;
        l[e] = le;
      }
      unsigned short* dst = sout + ((bb * PS + Y) * PS + X) * (2 * C) + 2 * c0;
      *reinterpret_cast<cnn_u4*>(dst) = h;
      *reinterpret_cast<cnn_u4*>(dst + 8) = l;
    }
  }
}

// gradient through the ReLU and the 2 x 2 max pool: the pooled gradient goes to the
// quad position arg recorded by the forward pass (4: to none of them)
__global__ void k_unpool_bwd(const uint8_t* __restrict__ arg, const float* __restrict__ dpool, int64_t planes,
                             int lw_out, float* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int wo = 1 << lw_out;
  if (i >= planes * wo * wo) return;
  const int64_t pl = i >> (2 * lw_out);
  const int y = (int)((i >> lw_out) & (wo - 1)), x = (int)(i & (wo - 1));
  const size_t base = (pl << (2 * lw_out + 2)) + (size_t)(2 * y) * (2 * wo) + 2 * x;
  const int q = arg[i];
  const float d = dpool[i];
  *reinterpret_cast<float2*>(g + base) = float2{q == 0 ? d : 0.0f, q == 1 ? d : 0.0f};
  *reinterpret_cast<float2*>(g + base + 2 * wo) = float2{q == 2 ? d : 0.0f, q == 3 ? d : 0.0f};
}

// softmax cross-entropy per row: loss_row[b], dz = (softmax - onehot) / B
__global__ __launch_bounds__(1024) void k_softmax_xent(const float* __restrict__ z, const int32_t* __restrict__ y,
                                                       int l, int bsz, float* __restrict__ dz,
                                                       double* __restrict__ loss_row) {
  const int bb = blockIdx.x;
  const float* zr = z + (size_t)bb * l;
  __shared__ float redf[16];
  __shared__ double redd[16];
  float mx = -INFINITY;
  for (int i = threadIdx.x; i < l; i += 1024) mx = fmaxf(mx, zr[i]);
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0) redf[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = redf[0];
#pragma unroll
  for (int k = 1; k < 16; ++k) mx = fmaxf(mx, redf[k]);
  double s = 0.0;
  for (int i = threadIdx.x; i < l; i += 1024) s += exp((double)(zr[i] - mx));
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) redd[threadIdx.x >> 6] = s;
  __syncthreads();
  s = redd[0];
#pragma unroll
  for (int k = 1; k < 16; ++k) s += redd[k];
  const int lab = y[bb];
  const float inv = 1.0f / (float)bsz;
  for (int i = threadIdx.x; i < l; i += 1024) {
    const float p = (float)(exp((double)(zr[i] - mx)) / s);
    dz[(size_t)bb * l + i] = (p - (i == lab ? 1.0f : 0.0f)) * inv;
  }
  if (threadIdx.x == 0) loss_row[bb] = log(s) - (double)(zr[lab] - mx);
}

// mean of the per-row losses (lane sums, then a fixed butterfly)
__global__ __launch_bounds__(64) void k_mean_loss(const double* __restrict__ loss_row, int bsz,
                                                  float* __restrict__ loss) {
  double s = 0.0;
  for (int i = threadIdx.x; i < bsz; i += 64) s += loss_row[i];
  s = wave_sum(s);
  if (threadIdx.x == 0) *loss = (float)(s / bsz);
}

// Adam (Kingma and Ba), bias-corrected step sizes precomputed on the host;
// the weights 1 - b1 and 1 - b2 come rounded from double (1.0f - 0.999f
// would be 1.3e-5 off 0.001)
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr_t, float b1, float b2, float omb1, float omb2,
                       float eps_t) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float vi = b2 * v[i] + omb2 * (gi * gi);
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr_t * mi / (sqrtf(vi) + eps_t);
}

// ---------------------------------------------------------------------------
// Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror and
// Shaw, SC 2011), counter (i_lo, i_hi, stream, 0), key (seed_lo, seed_hi).
__device__ __forceinline__ uint4 philox(uint64_t i, uint32_t stream, uint64_t seed) {
  uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32), c2 = stream, c3 = 0u;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}
// uniform in (0, 1]: (53 bits + 1/2) / 2^53 (the top value rounds to 1)
__device__ __forceinline__ double unit(uint32_t a, uint32_t b) {
  const uint64_t x = ((uint64_t)a << 21) ^ (uint64_t)(b >> 11);  // 53 bits
  return ((double)(x & ((1ull << 53) - 1)) + 0.5) * (1.0 / 9007199254740992.0);
}
__device__ __forceinline__ float2 normal2(uint4 r) {
  const double u1 = unit(r.x, r.y), u2 = unit(r.z, r.w);
  const double rad = sqrt(-2.0 * log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  return make_float2((float)(rad * c), (float)(rad * s));
}

// He-normal initial weights (biases zero): std sqrt(2 / fan_in)
__global__ void k_init_params(float* __restrict__ w, int64_t begin, int64_t count, float stdv, uint64_t seed,
                              uint32_t stream) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const float2 z = normal2(philox((uint64_t)i, stream, seed));
  w[begin + i] = stdv * z.x;
}

// random orientation (Shoemake's uniform quaternion) and in-plane pattern
// centre offset for sample index s
__global__ void k_sample_setup(int64_t first, int64_t bsz, uint64_t seed, double pcx, double pcy, double pcz,
                               double max_off_frac, double* __restrict__ q, double* __restrict__ pc) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= bsz) return;
  const uint64_t s = (uint64_t)(first + j);
  const uint4 r0 = philox(s, 1u, seed), r1 = philox(s, 2u, seed);
  const double u1 = unit(r0.x, r0.y), u2 = unit(r0.z, r0.w), u3 = unit(r1.x, r1.y);
  double s2, c2, s3, c3;
  sincospi(2.0 * u2, &s2, &c2);
  sincospi(2.0 * u3, &s3, &c3);
  const double a = sqrt(1.0 - u1), b = sqrt(u1);
  double v[4] = {b * c3, a * s2, a * c2, b * s3};
  qstore(q + 4 * j, v);
  const double ox = (2.0 * unit(r1.z, r1.w) - 1.0) * max_off_frac;
  const uint4 r2 = philox(s, 3u, seed);
  const double oy = (2.0 * unit(r2.x, r2.y) - 1.0) * max_off_frac;
  pc[3 * j] = pcx + ox;
  pc[3 * j + 1] = pcy + oy;
  pc[3 * j + 2] = pcz;
}

// Noise (when `noisy`: the pattern scaled to a mean count level, Poisson by
// its normal approximation, plus Gaussian read noise fixing the pattern's
// SNR), f x f block-mean binning to 64 x 64 (f = n / 64) and
// (x - mean) / std.  One block per pattern.
template <class T>
__global__ __launch_bounds__(256) void k_noise_bin(const T* __restrict__ clean, int n, int64_t first,
                                                   uint64_t seed, float counts, float snr, int noisy,
                                                   float* __restrict__ x) {
  __shared__ float bin[64 * 64];
  __shared__ double red[8];
  const int64_t j = blockIdx.x;
  const int tid = threadIdx.x;
  const T* img = clean + (size_t)j * n * n;
  double s1 = 0.0, s2 = 0.0;
  for (int i = tid; i < n * n; i += 256) {
    const double v = ld_px(img[i]);
    s1 += v;
    s2 += v * v;
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if ((tid & 63) == 0) {
    red[tid >> 6] = s1;
    red[4 + (tid >> 6)] = s2;
  }
  __syncthreads();
  const double mean = (red[0] + red[1] + red[2] + red[3]) / ((double)n * n);
  const double var = (red[4] + red[5] + red[6] + red[7]) / ((double)n * n) - mean * mean;
  const double ct = var > 0.0 && mean > 0.0 ? sqrt(var) / mean : 0.0;
  double var_g = ct > 0.0 ? (counts * ct / snr) * (counts * ct / snr) - counts : 0.0;
  double c_eff = counts;
  if (var_g < 0.0) {
    c_eff = ct > 0.0 ? (snr / ct) * (snr / ct) : counts;
    var_g = 0.0;
  }
  const float scale = !noisy ? 1.0f : (mean > 0.0 ? (float)(c_eff / mean) : 0.0f);
  const float sg = (float)sqrt(var_g);
  const int f = n / 64;
  const uint64_t s = (uint64_t)(first + j);
  __syncthreads();
  for (int o = tid; o < 64 * 64; o += 256) {
    const int by = o >> 6, bx = o & 63;
    float acc = 0.0f;
    for (int dy = 0; dy < f; ++dy)
      for (int dx = 0; dx < f; ++dx) {
        const int pix = (by * f + dy) * n + bx * f + dx;
        float v = ld_px(img[pix]) * scale;
        if (noisy) {
          const float2 z = normal2(philox((s << 20) ^ (uint64_t)pix, 4u, seed));
          v += sqrtf(fmaxf(v, 0.0f)) * z.x + sg * z.y;
        }
        acc += v;
      }
    bin[o] = acc / (float)(f * f);
  }
  __syncthreads();
  s1 = 0.0;
  s2 = 0.0;
  for (int o = tid; o < 64 * 64; o += 256) {
    const double v = bin[o];
    s1 += v;
    s2 += v * v;
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  __syncthreads();
  if ((tid & 63) == 0) {
    red[tid >> 6] = s1;
    red[4 + (tid >> 6)] = s2;
  }
  __syncthreads();
  const double m2 = (red[0] + red[1] + red[2] + red[3]) / 4096.0;
  const double v2 = (red[4] + red[5] + red[6] + red[7]) / 4096.0 - m2 * m2;
  const float fm = (float)m2, is = v2 > 0.0 ? (float)(1.0 / sqrt(v2)) : 0.0f;
  for (int o = tid; o < 64 * 64; o += 256) x[(size_t)j * 4096 + o] = (bin[o] - fm) * is;
}

// The 24 proper rotations of the cubic point group as quaternions.
__constant__ double c_cubic_q[24][4] = {
    {1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1},
    {0.70710678118654752, 0.70710678118654752, 0, 0}, {0.70710678118654752, -0.70710678118654752, 0, 0},
    {0.70710678118654752, 0, 0.70710678118654752, 0}, {0.70710678118654752, 0, -0.70710678118654752, 0},
    {0.70710678118654752, 0, 0, 0.70710678118654752}, {0.70710678118654752, 0, 0, -0.70710678118654752},
    {0.5, 0.5, 0.5, 0.5}, {0.5, 0.5, 0.5, -0.5}, {0.5, 0.5, -0.5, 0.5}, {0.5, 0.5, -0.5, -0.5},
    {0.5, -0.5, 0.5, 0.5}, {0.5, -0.5, 0.5, -0.5}, {0.5, -0.5, -0.5, 0.5}, {0.5, -0.5, -0.5, -0.5},
    {0, 0.70710678118654752, 0.70710678118654752, 0}, {0, 0.70710678118654752, -0.70710678118654752, 0},
    {0, 0.70710678118654752, 0, 0.70710678118654752}, {0, 0.70710678118654752, 0, -0.70710678118654752},
    {0, 0, 0.70710678118654752, 0.70710678118654752}, {0, 0, 0.70710678118654752, -0.70710678118654752}};

// label[j] = library orientation of smallest cubic disorientation from q[j]
// (largest |<q, s (x) q_l>|; ties: smallest index).  One block per sample.
__global__ __launch_bounds__(256) void k_nearest_library(const double* __restrict__ q, const double* __restrict__ lib,
                                                         int l, int32_t* __restrict__ label) {
  const int64_t j = blockIdx.x;
  const double a[4] = {q[4 * j], q[4 * j + 1], q[4 * j + 2], q[4 * j + 3]};
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int i = threadIdx.x; i < l; i += 256) {
    const double* b = lib + 4 * (size_t)i;
    double m = 0.0;
    for (int s = 0; s < 24; ++s) {
      double sb[4];
      qmul(c_cubic_q[s], b, sb);
      m = fmax(m, fabs(a[0] * sb[0] + a[1] * sb[1] + a[2] * sb[2] + a[3] * sb[3]));
    }
    if (m > best) {  // i increases: ties keep the smaller index
      best = m;
      bi = i;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double b2 = __shfl_xor(best, off, 64);
    const int i2 = __shfl_xor(bi, off, 64);
    if (b2 > best || (b2 == best && i2 < bi)) {
      best = b2;
      bi = i2;
    }
  }
  __shared__ double rv[4];
  __shared__ int ri[4];
  if ((threadIdx.x & 63) == 0) {
    rv[threadIdx.x >> 6] = best;
    ri[threadIdx.x >> 6] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w)
      if (rv[w] > best || (rv[w] == best && ri[w] < bi)) {
        best = rv[w];
        bi = ri[w];
      }
    label[j] = bi;
  }
}

// The k largest scores of each row, in decreasing order (ties: smaller
// index first; NaN scores count as -inf).  One block per row; the row is
// staged in LDS.
__global__ __launch_bounds__(256) void k_topk(const float* __restrict__ z, int l, int k, int32_t* __restrict__ idx) {
  extern __shared__ float row[];
  const int64_t b = blockIdx.x;
  for (int i = threadIdx.x; i < l; i += 256) {
    const float v = z[(size_t)b * l + i];
    row[i] = v != v ? -INFINITY : v;
  }
  __shared__ float rv[4];
  __shared__ int ri[4];
  __shared__ int pick;
  __syncthreads();
  for (int t = 0; t < k; ++t) {
    float best = -INFINITY;
    int bi = 0x7fffffff;
    for (int i = threadIdx.x; i < l; i += 256) argmax_merge(best, bi, row[i], i);
    wave_argmax(best, bi);
    if ((threadIdx.x & 63) == 0) {
      rv[threadIdx.x >> 6] = best;
      ri[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < 4; ++w) argmax_merge(best, bi, rv[w], ri[w]);
      pick = bi;
      idx[b * k + t] = bi;
    }
    __syncthreads();
    // a taken entry becomes NaN, which never wins a comparison (k <= l)
    if (threadIdx.x == 0) row[pick] = __int_as_float(0x7fc00000);
    __syncthreads();
  }
}

// The same selection for k <= kTopKWave by a threshold.  Lane j of wave 0
// takes the largest of threads 4j .. 4j + 3's entries (i = t + 256 r); T =
// the k-th largest of these 64 group maxima (ranked by value, then lane), so
// at least k entries are >= T and the k best are among them.  The entries
// >= T (typically a few dozen of thousands) are collected and wave 0 orders
// them by (score, then index), the total order of k_topk: a bitonic sort in
// registers for at most 64 of them, else k rounds of a wave argmax; more
// than kTopKCand (heavy ties at T) falls back to k_topk's block argmax.
constexpr int kTopKWave = 64, kTopKCand = 1024;
__device__ __forceinline__ bool topk_before(float va, int ia, float vb, int ib) {
  return va > vb || (va == vb && ia < ib);
}
__global__ __launch_bounds__(256) void k_topk_wave(const float* __restrict__ z, int l, int k,
                                                   int32_t* __restrict__ idx) {
  extern __shared__ float row[];
  __shared__ float tmax[256];
  __shared__ float cv[kTopKCand];
  __shared__ int ci[kTopKCand];
  __shared__ int ncand;
  __shared__ float thr;
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  float mt = -INFINITY;
  for (int i = tid; i < l; i += 256) {
    const float v = z[(size_t)b * l + i];
    const float vv = v != v ? -INFINITY : v;
    row[i] = vv;
    mt = fmaxf(mt, vv);
  }
  tmax[tid] = mt;
  if (tid == 0) ncand = 0;
  __syncthreads();
  if (w == 0) {
    const float g = fmaxf(fmaxf(tmax[4 * lane], tmax[4 * lane + 1]), fmaxf(tmax[4 * lane + 2], tmax[4 * lane + 3]));
    int rank = 0;
    for (int u = 0; u < 64; ++u) {
      const float o = __shfl(g, u, 64);
      rank += (o > g || (o == g && u < lane)) ? 1 : 0;
    }
    if (rank == k - 1) thr = g;  // ranks are a permutation of 0 .. 63
  }
  __syncthreads();
  const float t = thr;
  for (int i = tid; i < l; i += 256) {
    const float v = row[i];
    if (v >= t) {
      const int p = atomicAdd(&ncand, 1);
      if (p < kTopKCand) {
        cv[p] = v;
        ci[p] = i;
      }
    }
  }
  __syncthreads();
  const int m = ncand;
  if (m <= 64) {
    if (w == 0) {
      float v = lane < m ? cv[lane] : -INFINITY;
      int i = lane < m ? ci[lane] : 0x7fffffff;
      for (int size = 2; size <= 64; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
          const float ov = __shfl_xor(v, stride, 64);
          const int oi = __shfl_xor(i, stride, 64);
          // runs of `size` lanes alternate direction until the last pass;
          // the lower lane of a pair keeps the earlier entry of its run
          const bool fwd = (lane & size) == 0 || size == 64;
          const bool lower = (lane & stride) == 0;
          const bool other_first = topk_before(ov, oi, v, i);
          if (lower == fwd ? other_first : topk_before(v, i, ov, oi)) {
            v = ov;
            i = oi;
          }
        }
      if (lane < k) idx[b * k + lane] = i;
    }
  } else if (m <= kTopKCand) {
    if (w == 0) {
      // a lane caches its best candidate; only the owner of a pick rescans
      auto best = [&](float& bv, int& bi, int& slot) {
        bv = -INFINITY;
        bi = 0x7fffffff;
        slot = -1;
        for (int e = lane; e < m; e += 64)
          if (topk_before(cv[e], ci[e], bv, bi)) {
            bv = cv[e];
            bi = ci[e];
            slot = e;
          }
      };
      float mv;
      int mi, ms;
      best(mv, mi, ms);
      for (int r = 0; r < k; ++r) {
        float bv = mv;
        int bi = mi;
        wave_argmax(bv, bi);
        if (lane == 0) idx[b * k + r] = bi;
        if (bi == mi && ms >= 0) {
          cv[ms] = __int_as_float(0x7fc00000);  // NaN never wins a comparison
          best(mv, mi, ms);
        }
      }
    }
  } else {
    __shared__ float rv[4];
    __shared__ int ri[4];
    __shared__ int pick;
    for (int r = 0; r < k; ++r) {
      float bv = -INFINITY;
      int bi = 0x7fffffff;
      for (int i = tid; i < l; i += 256) argmax_merge(bv, bi, row[i], i);
      wave_argmax(bv, bi);
      if (lane == 0) {
        rv[w] = bv;
        ri[w] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        for (int u = 1; u < 4; ++u) argmax_merge(bv, bi, rv[u], ri[u]);
        pick = bi;
        idx[b * k + r] = bi;
      }
      __syncthreads();
      if (tid == 0) row[pick] = __int_as_float(0x7fc00000);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// host side

namespace {
inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }
inline int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}
}  // namespace

Layout layout_of(int n_classes) {
  Layout lay;
  int64_t off = 0;
  int ci = 1;
  for (int i = 0; i < 4; ++i) {
    lay.conv_w[i] = off;
    off += (int64_t)kChannels[i] * ci * 9;
    lay.conv_b[i] = off;
    off += kChannels[i];
    ci = kChannels[i];
  }
  lay.fc_w = off;
  off += (int64_t)n_classes * kFeatures;
  lay.fc_b = off;
  off += n_classes;
  lay.total = off;
  lay.classes = n_classes;
  return lay;
}

hipError_t init_params(float* params, const Layout& lay, uint64_t seed, hipStream_t st) {
  hipError_t e = hipMemsetAsync(params, 0, sizeof(float) * lay.total, st);
  if (e != hipSuccess) return e;
  int ci = 1;
  for (int i = 0; i < 4; ++i) {
    const int64_t cnt = (int64_t)kChannels[i] * ci * 9;
    hipLaunchKernelGGL(k_init_params, dim3(nb(cnt)), dim3(256), 0, st, params, lay.conv_w[i], cnt,
                       (float)sqrt(2.0 / (ci * 9)), seed, (uint32_t)(10 + i));
    ci = kChannels[i];
  }
  const int64_t cnt = (int64_t)lay.classes * kFeatures;
  hipLaunchKernelGGL(k_init_params, dim3(nb(cnt)), dim3(256), 0, st, params, lay.fc_w, cnt,
                     (float)sqrt(1.0 / kFeatures), seed, 20u);
  return hipGetLastError();
}

// forward (after prepare on the same parameters); act holds p_i (i = 0..3),
// in training arg_i, and the logits; split: inference products with BF16
// split operands (k_tgemm_s), the weights' halves made by prepare
hipError_t prepare(const float* params, const Layout& lay, const Acts& act, bool split, hipStream_t st) {
  hipLaunchKernelGGL(k_weights_tap, dim3(nb(kTapWeights)), dim3(256), 0, st, params, lay, act.wt);
  if (split) {
    // layers 2-4 (the first stays FP32); layer i's rows start at twice its
    // tap-major offset
    for (int i = 1, ci = kChannels[0]; i < 4; ci = kChannels[i], ++i) {
      const int k_len = 9 * ci;
      hipLaunchKernelGGL(k_split_rows, dim3(nb((int64_t)kChannels[i] * k_len / 8)), dim3(256), 0, st,
                         act.wt + tap_weights_offset(i), (int64_t)kChannels[i], k_len,
                         act.wts + 2 * tap_weights_offset(i));
    }
    hipLaunchKernelGGL(k_split_rows, dim3(nb((int64_t)lay.classes * kFeatures / 8)), dim3(256), 0, st,
                       params + lay.fc_w, (int64_t)lay.classes, kFeatures, act.fcs);
  }
  return hipGetLastError();
}

hipError_t forward(const float* params, const Layout& lay, const float* x, int64_t bsz, const Acts& act,
                   hipStream_t st, bool train, bool split) {
  // training: only the fc takes split operands (its output feeds the smooth
  // softmax, while a convolution's output decides the ReLU and pool choices)
  const bool fc_split = split;
  split = split && !train;
  const float* a = x;
  int ci = 1, w = kInSize;
  hipError_t e;
  for (int i = 0; i < 4; ++i) {
    const int co = kChannels[i], lw = ilog2(w);
    const int M = (int)(bsz * w * w), K = ci * 9;
    const int lci = ilog2(ci);
    // each convolution pools in its epilogue: only the pooled maps (and, in
    // training, the gradient positions) are written
    const float* bias = params + lay.conv_b[i];
    if (i == 0) {
      static_assert(kChannels[0] % 8 == 0, "first layer: channel groups of 8");
      const unsigned blocks = nb(bsz * (kInSize / 2) * (kInSize / 2));
      if (split)
        hipLaunchKernelGGL(k_conv1_pool<true>, dim3(blocks), dim3(256), 0, st, x, params + lay.conv_w[0], bias, bsz,
                           nullptr, nullptr, reinterpret_cast<unsigned short*>(act.p[0]));
      else
        hipLaunchKernelGGL(k_conv1_pool<false>, dim3(blocks), dim3(256), 0, st, x, params + lay.conv_w[0], bias,
                           bsz, act.p[0], train ? act.arg[0] : nullptr, nullptr);
      e = hipGetLastError();
    } else if (!split) {
      const ConvReluPoolOut o{act.p[i], bias, co, lw - 1, train ? act.arg[i] : nullptr};
      e = gemm(ConvFwdA{a, ci, lci, lw}, WeightT{act.wt + tap_weights_offset(i), K}, o, M, co, K, 1, st, true);
    } else {
      // split inference: the pooled maps are written split for the next
      // layer's BF16 products (in the FP32 maps' buffers, the same bytes; the
      // first layer's by k_conv1_pool), the last one as FP32 features for the fc
      const unsigned short* sa = reinterpret_cast<const unsigned short*>(a);
      const ConvReluPoolSplitOut so{reinterpret_cast<unsigned short*>(act.p[i]), bias, co, lw - 1};
      const SplitRows wb{act.wts + 2 * tap_weights_offset(i), K};
      if (i < 3)
        e = gemm_split(ConvFwdSA{sa, ci, lci, lw}, wb, so, M, co, K, st);
      else
        e = gemm_split(ConvFwdSA{sa, ci, lci, lw}, wb, ConvReluPoolOut{act.p[3], bias, co, lw - 1, nullptr}, M, co,
                       K, st);
    }
    if (e != hipSuccess) return e;
    a = act.p[i];
    ci = co;
    w /= 2;
  }
  const RowOut o{act.logits, params + lay.fc_b, lay.classes};
  if (fc_split && train)
    return gemm_split(RowK{a, kFeatures}, WeightT{params + lay.fc_w, kFeatures}, o, (int)bsz, lay.classes, kFeatures,
                      st);
  return split ? gemm_split(RowK{a, kFeatures}, SplitRows{act.fcs, kFeatures}, o, (int)bsz, lay.classes,
                            kFeatures, st)
               : gemm(RowK{a, kFeatures}, WeightT{params + lay.fc_w, kFeatures}, o, (int)bsz, lay.classes, kFeatures, 1,
                      st, true);
}

static int splits_for(int64_t k_len, int64_t tiles) {
  // enough blocks to fill the chip, slices of at least 1024
  int64_t s = (1024 + tiles - 1) / tiles;
  const int64_t maxs = (k_len + 1023) / 1024;
  if (s > maxs) s = maxs;
  if (s < 1) s = 1;
  return (int)s;
}

hipError_t backward(const float* params, const Layout& lay, const float* x, const int32_t* labels, int64_t bsz,
                    const Acts& act, float* grad, float* part, size_t part_floats, double* loss_row, float* loss,
                    hipStream_t st, bool split) {
  hipError_t e;
  const int L = lay.classes;
  hipLaunchKernelGGL(k_softmax_xent, dim3((unsigned)bsz), dim3(1024), 0, st, act.logits, labels, L, (int)bsz,
                     act.dz, loss_row);
  hipLaunchKernelGGL(k_mean_loss, dim3(1), dim3(64), 0, st, loss_row, (int)bsz, loss);
  // fc: dW = dz^T f, db = column sums of dz, df = dz W
  {
    const ColK fa{act.dz, L};
    const BRowN fb{act.p[3], kFeatures};
    const RowOut fo{grad + lay.fc_w, nullptr, kFeatures};
    e = split ? gemm_split(fa, fb, fo, L, kFeatures, (int)bsz, st) : gemm(fa, fb, fo, L, kFeatures, (int)bsz, 1, st, true);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_col_sum, dim3((L + 63) / 64), dim3(1024), 0, st, act.dz, (int)bsz, L, grad + lay.fc_b);
  {
    // df = dz W: few output tiles and a long K (= L), so K is split and the
    // partials are summed in a fixed order
    const int tiles = (int)(((bsz + 63) / 64) * ((kFeatures + 63) / 64));
    int s = (512 + tiles - 1) / tiles;
    const int smax = (L + 255) / 256;
    s = s > smax ? smax : (s < 1 ? 1 : s);
    while ((size_t)s * bsz * kFeatures > part_floats && s > 1) s = (s + 1) / 2;
    const int z = split ? k_slices_s(L, s) : k_slices(L, s);
    const RowK da{act.dz, L};
    const BRowN db{params + lay.fc_w, kFeatures};
    const SplitOut dout{part, (int)bsz, kFeatures};
    e = split ? gemm_split(da, db, dout, (int)bsz, kFeatures, L, st, s)
              : gemm(da, db, dout, (int)bsz, kFeatures, L, s, st);
    if (e != hipSuccess) return e;
    split_sum(part, z, (int64_t)bsz * kFeatures, act.dp[3], st);
  }
  int w = kInSize >> 3;  // conv4 input side (8)
  for (int i = 3; i >= 0; --i) {
    const int co = kChannels[i], ci = i ? kChannels[i - 1] : 1, lw = ilog2(w);
    const float* in = i ? act.p[i - 1] : x;
    if (i == 0) {
      // the first layer needs no input gradient: its weight gradient reads
      // the pooled gradient directly, and g_0 is never formed
      static_assert(kChannels[0] % 8 == 0 && (kInSize / 2) * (kInSize / 2) % 256 == 0, "first-layer shape");
      if ((size_t)bsz * co * 9 > part_floats) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_wgrad_first<8>, dim3((unsigned)bsz, co / 8), dim3(256), 0, st, x, act.arg[0], act.dp[0],
                         co, part);
      split_sum(part, (int)bsz, (int64_t)co * 9, grad + lay.conv_w[0], st);
    } else {
      hipLaunchKernelGGL(k_unpool_bwd, dim3(nb(bsz * co * (w / 2) * (w / 2))), dim3(256), 0, st, act.arg[i],
                         act.dp[i], (int64_t)(bsz * co), lw - 1, act.g[i]);
      // weight gradient, split over (b, y, x); 32-wide tiles when ci < 64
      // (the tap-major columns of a tile then share a tap)
      const int K = (int)(bsz * w * w), N = ci * 9;
      if (split && ci % 32 == 0) {
        // 96-wide tiles (three taps of 32 channels; N = 9 ci divides into
        // them): each K slice of the gradient is read N / 96 times
#ifdef EBSD_WG_TM64
        const int tm = 64;
#else
        const int tm = co >= 128 ? 128 : 64;
#endif
        const int64_t tiles = (int64_t)((co + tm - 1) / tm) * (N / 96);
        int s = splits_for(K, tiles);
        while ((size_t)s * co * N > part_floats && s > 1) s = (s + 1) / 2;
        const int z = k_slices_s(K, s), kslice = k_slice_s(K, s);
        const ConvBwdWA wa{act.g[i], co, lw};
        const ConvBwdWB wb{in, ilog2(ci), lw};
        const SplitOut wo{part, co, N};
        const dim3 grid(N / 96, (co + tm - 1) / tm, z);
        if (tm == 64)
          hipLaunchKernelGGL((k_tgemm_s<64, 96, ConvBwdWA, ConvBwdWB, SplitOut>), grid, dim3(256), 0, st, wa, wb, wo,
                             co, N, K, kslice);
        else
          hipLaunchKernelGGL((k_tgemm_s<128, 96, ConvBwdWA, ConvBwdWB, SplitOut>), grid, dim3(256), 0, st, wa, wb,
                             wo, co, N, K, kslice);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        split_sum(part, z, (int64_t)co * N, grad + lay.conv_w[i], st, N, ilog2(ci));
      } else {
      const bool narrow = ci < 64;
      const int tn = narrow ? 32 : 64;
      const int64_t tiles = (int64_t)((co + 63) / 64) * ((N + tn - 1) / tn);
      int s = splits_for(K, tiles);
      while ((size_t)s * co * N > part_floats && s > 1) s = (s + 1) / 2;
      const int z = split ? k_slices_s(K, s) : k_slices(K, s);
      const ConvBwdWA wa{act.g[i], co, lw};
      const ConvBwdWB wb{in, ilog2(ci), lw};
      const SplitOut wo{part, co, N};
      e = split ? gemm_split(wa, wb, wo, co, N, K, st, s, false, narrow) : gemm(wa, wb, wo, co, N, K, s, st, false, narrow);
      if (e != hipSuccess) return e;
      split_sum(part, z, (int64_t)co * N, grad + lay.conv_w[i], st, N, ilog2(ci));
      }
    }
    {
      const int zs = (int)(bsz < 64 ? bsz : 64);
      double* cpart = reinterpret_cast<double*>(part);  // the weight-gradient partials are summed already
      hipLaunchKernelGGL(k_channel_part, dim3(co, zs), dim3(256), 0, st, act.arg[i], act.dp[i], (int)bsz, co,
                         2 * (lw - 1), zs, cpart);
      hipLaunchKernelGGL(k_channel_sum, dim3(co), dim3(64), 0, st, cpart, zs, grad + lay.conv_b[i]);
    }
    if (i > 0) {
      const ConvBwdDataA ga{act.g[i], ilog2(co), lw};
      const WeightBwdData gb{act.wt + tap_weights_offset(i), ci, ilog2(co)};
      const NchwOut go{act.dp[i - 1], ci, lw};
      e = split ? gemm_split(ga, gb, go, (int)(bsz * w * w), ci, co * 9, st)
                : gemm(ga, gb, go, (int)(bsz * w * w), ci, co * 9, 1, st, true);
      if (e != hipSuccess) return e;
    }
    w *= 2;
  }
  return hipGetLastError();
}

hipError_t adam(float* params, const float* grad, float* m, float* v, int64_t n, int64_t step, float lr,
                hipStream_t st) {
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
  const float lr_t = (float)(lr * sqrt(c2) / c1);
  const float eps_t = (float)(eps * sqrt(c2));
  hipLaunchKernelGGL(k_adam, dim3(nb(n)), dim3(256), 0, st, params, grad, m, v, n, lr_t, (float)b1, (float)b2,
                     (float)(1.0 - b1), (float)(1.0 - b2), eps_t);
  return hipGetLastError();
}

hipError_t sample_setup(int64_t first, int64_t bsz, uint64_t seed, double pcx, double pcy, double pcz,
                        double max_off_frac, double* q, double* pc, hipStream_t st) {
  hipLaunchKernelGGL(k_sample_setup, dim3(nb(bsz)), dim3(256), 0, st, first, bsz, seed, pcx, pcy, pcz,
                     max_off_frac, q, pc);
  return hipGetLastError();
}

template <class T>
static hipError_t noise_bin_t(const T* clean, int n, int64_t bsz, int64_t first, uint64_t seed, float counts,
                              float snr, int noisy, float* x, hipStream_t st) {
  if (bsz > (int64_t(1) << 31) / 256) return hipErrorInvalidValue;  // one dispatch below 2^31 items
  if (n % kInSize != 0 || n < kInSize) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_noise_bin<T>, dim3((unsigned)bsz), dim3(256), 0, st, clean, n, first, seed, counts, snr,
                     noisy, x);
  return hipGetLastError();
}

hipError_t noise_bin(const float* clean, int n, int64_t bsz, int64_t first, uint64_t seed, float counts, float snr,
                     int noisy, float* x, hipStream_t st) {
  return noise_bin_t(clean, n, bsz, first, seed, counts, snr, noisy, x, st);
}

hipError_t noise_bin(const __bf16* clean, int n, int64_t bsz, int64_t first, uint64_t seed, float counts,
                     float snr, int noisy, float* x, hipStream_t st) {
  return noise_bin_t(clean, n, bsz, first, seed, counts, snr, noisy, x, st);
}

hipError_t nearest_library(const double* q, int64_t bsz, const double* lib, int l, int32_t* label,
                           hipStream_t st) {
  if (bsz > (int64_t(1) << 31) / 256) return hipErrorInvalidValue;  // one dispatch below 2^31 items
  hipLaunchKernelGGL(k_nearest_library, dim3((unsigned)bsz), dim3(256), 0, st, q, lib, l, label);
  return hipGetLastError();
}

hipError_t topk(const float* z, int64_t rows, int l, int k, int32_t* idx, hipStream_t st) {
  if (rows > (int64_t(1) << 31) / 256) return hipErrorInvalidValue;  // one dispatch below 2^31 items
  const size_t shm = sizeof(float) * (size_t)l;
  if (shm > 160 * 1024) return hipErrorInvalidValue;
  // (the threshold form adds 9 KB of its own to the row in LDS)
  if (k <= kTopKWave && shm + 1024 * (size_t)(1 + 2 * kTopKCand / 256) + 64 <= 160 * 1024) {
    const hipError_t e =
        hipFuncSetAttribute((const void*)k_topk_wave, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_topk_wave, dim3((unsigned)rows), dim3(256), shm, st, z, l, k, idx);
    return hipGetLastError();
  }
  const hipError_t e = hipFuncSetAttribute((const void*)k_topk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_topk, dim3((unsigned)rows), dim3(256), shm, st, z, l, k, idx);
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace ebsd

// Shared device-side building blocks for the gfx950 template-matching path:
// a plain complex type, compile-time roots of unity, small in-register DFTs
// (radix 2, 3, 4, 5 and their products), and wavefront reductions.
//
// Transform convention (Equation 4 without its unitary factor, which cancels
// in the normalised correlation): forward X(u) = sum_x x(x) exp(-2 pi i u x / N),
// inverse x(s) = sum_u X(u) exp(+2 pi i u s / N).  DIR = -1 is forward,
// DIR = +1 is inverse.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>
#include <utility>

namespace ebsd {

struct cf {
  float x, y;
};

// A pattern pixel widened to FP32 (patterns may be stored as FP32 or BF16).
__device__ __forceinline__ float ld_px(float v) { return v; }
__device__ __forceinline__ float ld_px(__bf16 v) { return (float)v; }

__device__ __forceinline__ cf cmake(float a, float b) { return cf{a, b}; }
__device__ __forceinline__ cf cadd(cf a, cf b) { return cf{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cf csub(cf a, cf b) { return cf{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cf cmul(cf a, cf b) {
  return cf{__fmaf_rn(a.x, b.x, -a.y * b.y), __fmaf_rn(a.x, b.y, a.y * b.x)};
}
// a * conj(b)
__device__ __forceinline__ cf cmulc(cf a, cf b) {
  return cf{__fmaf_rn(a.x, b.x, a.y * b.y), __fmaf_rn(a.y, b.x, -a.x * b.y)};
}
__device__ __forceinline__ cf cconj(cf a) { return cf{a.x, -a.y}; }
__device__ __forceinline__ cf cscale(cf a, float s) { return cf{a.x * s, a.y * s}; }
// multiply by s*i, s = +-1
template <int S>
__device__ __forceinline__ cf cmuli(cf a) {
  return S > 0 ? cf{-a.y, a.x} : cf{a.y, -a.x};
}

// ---------------------------------------------------------------------------
// Compile-time trigonometry (Taylor series after reduction to [-pi/4, pi/4]),
// used only to form constant twiddles of the small DFTs.
namespace cx {
constexpr double PI = 3.14159265358979323846264338327950288;
constexpr double sin_t(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cos_t(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi k / n for integers (exact octant reduction)
constexpr double cos2pi(long k, long n) {
  k %= n;
  if (k < 0) k += n;
  // angle = 2 pi k / n in [0, 2 pi); reduce with exact rational arithmetic
  long k8 = 8 * k;  // angle in units of pi/4: k8 / n
  long oct = k8 / n;
  double r = (double)(k8 - oct * n) / (double)n * (PI / 4.0);  // remainder in [0, pi/4)
  switch (oct) {
    case 0: return cos_t(r);
    case 1: return sin_t(PI / 4.0 - r);
    case 2: return -sin_t(r);
    case 3: return -cos_t(PI / 4.0 - r);
    case 4: return -cos_t(r);
    case 5: return -sin_t(PI / 4.0 - r);
    case 6: return sin_t(r);
    default: return cos_t(PI / 4.0 - r);
  }
}
constexpr double sin2pi(long k, long n) { return cos2pi(k * 4 - n, 4 * n); }
}  // namespace cx

// w = exp(DIR * 2 pi i K / R) as compile-time constants
template <long K, long R, int DIR>
struct Tw {
  static constexpr float re = (float)cx::cos2pi(K, R);
  static constexpr float im = (float)(DIR * cx::sin2pi(K, R));
};

// multiply by exp(DIR * 2 pi i K / R); trivial angles become swaps / negations
template <long K, long R, int DIR>
__device__ __forceinline__ cf twiddle(cf a) {
  constexpr long k = ((K % R) + R) % R;
  if constexpr (k == 0) {
    return a;
  } else if constexpr (4 * k == R) {
    return cmuli<DIR>(a);
  } else if constexpr (2 * k == R) {
    return cf{-a.x, -a.y};
  } else if constexpr (4 * k == 3 * R) {
    return cmuli<-DIR>(a);
  } else {
    constexpr float c = Tw<k, R, DIR>::re, s = Tw<k, R, DIR>::im;
    return cf{__fmaf_rn(a.x, c, -a.y * s), __fmaf_rn(a.x, s, a.y * c)};
  }
}

// static for-loop over [B, E) with an integral_constant index
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// ---------------------------------------------------------------------------
// In-register DFT of length R on x[0..R) (natural order in and out).
template <int R, int DIR>
struct DFT;

template <int DIR>
struct DFT<1, DIR> {
  __device__ __forceinline__ static void run(cf*) {}
};

template <int DIR>
struct DFT<2, DIR> {
  __device__ __forceinline__ static void run(cf* x) {
    cf a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <int DIR>
struct DFT<3, DIR> {
  __device__ __forceinline__ static void run(cf* x) {
    constexpr float c = -0.5f;
    constexpr float s = (float)(DIR * 0.86602540378443864676372317075294);
    cf a = x[0], b = x[1], d = x[2];
    cf t = cadd(b, d);
    cf u = csub(b, d);
    x[0] = cadd(a, t);
    cf m = cf{__fmaf_rn(t.x, c, a.x), __fmaf_rn(t.y, c, a.y)};
    // +- i s u
    cf r = cf{-u.y * s, u.x * s};
    x[1] = cadd(m, r);
    x[2] = csub(m, r);
  }
};

template <int DIR>
struct DFT<4, DIR> {
  __device__ __forceinline__ static void run(cf* x) {
    cf a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]);
    cf b0 = cadd(x[1], x[3]), b1 = cmuli<DIR>(csub(x[1], x[3]));
    x[0] = cadd(a0, b0);
    x[2] = csub(a0, b0);
    x[1] = cadd(a1, b1);
    x[3] = csub(a1, b1);
  }
};

template <int DIR>
struct DFT<5, DIR> {
  __device__ __forceinline__ static void run(cf* x) {
    constexpr float c1 = (float)cx::cos2pi(1, 5), c2 = (float)cx::cos2pi(2, 5);
    constexpr float s1 = (float)(DIR * cx::sin2pi(1, 5)), s2 = (float)(DIR * cx::sin2pi(2, 5));
    cf a = x[0];
    cf t1 = cadd(x[1], x[4]), t2 = cadd(x[2], x[3]);
    cf u1 = csub(x[1], x[4]), u2 = csub(x[2], x[3]);
    x[0] = cadd(a, cadd(t1, t2));
    cf m1 = cf{a.x + c1 * t1.x + c2 * t2.x, a.y + c1 * t1.y + c2 * t2.y};
    cf m2 = cf{a.x + c2 * t1.x + c1 * t2.x, a.y + c2 * t1.y + c1 * t2.y};
    // i (s1 u1 + s2 u2) and i (s2 u1 - s1 u2)
    float p1 = s1 * u1.x + s2 * u2.x, q1 = s1 * u1.y + s2 * u2.y;
    float p2 = s2 * u1.x - s1 * u2.x, q2 = s2 * u1.y - s1 * u2.y;
    x[1] = cf{m1.x - q1, m1.y + p1};
    x[4] = cf{m1.x + q1, m1.y - p1};
    x[2] = cf{m2.x - q2, m2.y + p2};
    x[3] = cf{m2.x + q2, m2.y - p2};
  }
};

// smallest factor used to split a composite radix
template <int R>
constexpr int split_factor() {
  return (R % 4 == 0 && R != 4) ? 4 : (R % 2 == 0 && R != 2) ? 2 : (R % 3 == 0 && R != 3) ? 3 : 5;
}

// Composite R = P * Q: input u = Q a + b, output y = c + P d.
//   t_b(c) = sum_a x(Q a + b) w_P^{a c};  t_b(c) *= w_R^{b c};
//   X(c + P d) = sum_b t_b(c) w_Q^{b d}.
template <int R, int DIR>
struct DFT {
  static constexpr int P = split_factor<R>();
  static constexpr int Q = R / P;
  __device__ __forceinline__ static void run(cf* x) {
    cf t[R];
    static_for<0, Q>([&](auto bi) {
      constexpr int b = decltype(bi)::value;
      cf v[P];
      static_for<0, P>([&](auto ai) { v[decltype(ai)::value] = x[Q * decltype(ai)::value + b]; });
      DFT<P, DIR>::run(v);
      static_for<0, P>([&](auto ci) {
        constexpr int c = decltype(ci)::value;
        t[c * Q + b] = twiddle<(long)b * c, R, DIR>(v[c]);
      });
    });
    static_for<0, P>([&](auto ci) {
      constexpr int c = decltype(ci)::value;
      DFT<Q, DIR>::run(&t[c * Q]);
      static_for<0, Q>([&](auto di) {
        constexpr int d = decltype(di)::value;
        x[c + P * d] = t[c * Q + d];
      });
    });
  }
};

// Length-R DFT for R = 4 Q with Q > 1 (the split of DFT<R>: same twiddles and
// output order) of inputs some of which are known to be zero: bit j of ZM
// marks x[j] == 0, x[j] is then not read.  Dropping the additions of exact
// zeros leaves every output equal to that of DFT<R, DIR> up to the sign of
// zero results.  At most one input of each first-stage butterfly pair
// (j, j + 2Q) may be zero.
template <int R, int DIR, int ZM>
__device__ __forceinline__ void dft_zero(cf* x) {
  constexpr int Q = R / 4;
  static_assert(R % 4 == 0 && Q > 1 && split_factor<R>() == 4, "radix 4 x Q");
  cf t[R];
  static_for<0, Q>([&](auto bi) {
    constexpr int b = decltype(bi)::value;
    constexpr bool z0 = (ZM >> b) & 1, z1 = (ZM >> (Q + b)) & 1, z2 = (ZM >> (2 * Q + b)) & 1,
                   z3 = (ZM >> (3 * Q + b)) & 1;
    static_assert(!(z0 && z2) && !(z1 && z3), "a butterfly pair with two zero inputs");
    cf a0, a1, b0, d1;
    if constexpr (z0) {
      a0 = x[2 * Q + b];
      a1 = cf{-x[2 * Q + b].x, -x[2 * Q + b].y};
    } else if constexpr (z2) {
      a0 = a1 = x[b];
    } else {
      a0 = cadd(x[b], x[2 * Q + b]);
      a1 = csub(x[b], x[2 * Q + b]);
    }
    if constexpr (z1) {
      b0 = x[3 * Q + b];
      d1 = cf{-x[3 * Q + b].x, -x[3 * Q + b].y};
    } else if constexpr (z3) {
      b0 = d1 = x[Q + b];
    } else {
      b0 = cadd(x[Q + b], x[3 * Q + b]);
      d1 = csub(x[Q + b], x[3 * Q + b]);
    }
    const cf b1 = cmuli<DIR>(d1);
    const cf v[4] = {cadd(a0, b0), cadd(a1, b1), csub(a0, b0), csub(a1, b1)};
    static_for<0, 4>([&](auto ci) {
      constexpr int c = decltype(ci)::value;
      t[c * Q + b] = twiddle<(long)b * c, R, DIR>(v[c]);
    });
  });
  static_for<0, 4>([&](auto ci) {
    constexpr int c = decltype(ci)::value;
    DFT<Q, DIR>::run(&t[c * Q]);
    static_for<0, Q>([&](auto di) {
      constexpr int d = decltype(di)::value;
      x[c + 4 * d] = t[c * Q + d];
    });
  });
}

// Inputs a of a first radix-R1 pass over u = R2 a + b (any b in [0, R2)) that
// fall between the band edges B and N - B, i.e. are zero for every b.
template <int N, int R1, int R2, int B>
constexpr int band_gap_mask() {
  int m = 0;
  for (int a = 0; a < R1; ++a)
    if (R2 * a > B && R2 * a + R2 - 1 < N - B) m |= 1 << a;
  return m;
}

// ---------------------------------------------------------------------------
// Per-size plan of the two-pass decomposition N = R1 * R2 used for every
// 2-D transform, and the band half-width B of the filtered spectra (the
// band-pass filter is exactly zero for rho > 3N/8).
template <int N>
struct Plan;
template <>
struct Plan<64> {
  static constexpr int R1 = 8, R2 = 8, B = 24;
};
template <>
struct Plan<96> {
  static constexpr int R1 = 12, R2 = 8, B = 36;
};
template <>
struct Plan<128> {
  static constexpr int R1 = 16, R2 = 8, B = 48;
};
template <>
struct Plan<160> {
  static constexpr int R1 = 16, R2 = 10, B = 60;
};
template <>
struct Plan<256> {
  static constexpr int R1 = 16, R2 = 16, B = 96;
};

// ---------------------------------------------------------------------------
// Wavefront (64 lanes) and block reductions.
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
// (value, index) lexicographic maximum: larger value, then smaller index
__device__ __forceinline__ void argmax_merge(float& v, int& i, float v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}
__device__ __forceinline__ void wave_argmax(float& v, int& i) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    float v2 = __shfl_xor(v, off, 64);
    int i2 = __shfl_xor(i, off, 64);
    argmax_merge(v, i, v2, i2);
  }
}

// ---------------------------------------------------------------------------
// FP64 quaternions (w, x, y, z): Hamilton product and storage normalised
// with w >= 0.
__device__ __forceinline__ void qmul(const double* a, const double* b, double* o) {
  o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}
__device__ __forceinline__ void qstore(double* q, const double* v) {
  const double s = 1.0 / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3]);
  const double sg = v[0] < 0.0 ? -s : s;
#pragma unroll
  for (int c = 0; c < 4; ++c) q[c] = v[c] * sg;
}

}  // namespace ebsd

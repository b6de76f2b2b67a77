// Fixed-size DFTs held in registers, for the batched 1D transforms of the Fourier-domain grid
// certificate (the paper evaluates its convolutions in the Fourier domain, section 2).
//
// dft<N>(v) replaces v[0..N) by its forward DFT, V_k = sum_n v_n exp(-2 pi i n k / N), for
// N in {2, 3, 4, 5} directly and for composite N = A * B (A, B in that set or composite
// themselves) by one Cooley-Tukey split: B-point transforms of the A decimated subsequences,
// the twiddles exp(-2 pi i a kb / N), then A-point transforms across them. Twiddles are
// compile-time constants (trigonometry evaluated by constexpr series), and the trivial ones
// (1, -1, +-i) cost no multiplication.
#pragma once

#include <hip/hip_runtime.h>

namespace sfw {
namespace fftr {

// ---------------------------------------------------------------- compile-time trigonometry

constexpr double kPi = 3.14159265358979323846264338327950288;

// Taylor series on |x| <= pi / 4 (13 terms: error far below double rounding there).
__host__ __device__ constexpr double sin_small(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int n = 1; n < 13; ++n) {
    term *= -x2 / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
__host__ __device__ constexpr double cos_small(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int n = 1; n < 13; ++n) {
    term *= -x2 / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}

// cos and sin of 2 pi m / n for integers, by exact octant reduction of the fraction m / n.
__host__ __device__ constexpr double cos2pi(long m, long n) {
  m %= n;
  if (m < 0) m += n;
  // angle = 2 pi m / n in [0, 2 pi): fold with cos(2pi - a) = cos a, cos(pi - a) = -cos a
  if (2 * m > n) m = n - m;                  // [0, pi]
  double sign = 1.0;
  if (4 * m > n) {                           // (pi/2, pi]
    m = n - 2 * m;                           // angle' = pi - angle = 2 pi (n/2 - m)/n
    // represent pi - angle as 2 pi m' / (2n) with m' = n - 2m
    n = 2 * n;
    sign = -1.0;
  }
  const double a = 2.0 * kPi * (double)m / (double)n;  // [0, pi/2]
  return sign * (8 * m > n ? sin_small(kPi / 2 - a) : cos_small(a));
}
__host__ __device__ constexpr double sin2pi(long m, long n) {
  // sin(2 pi m / n) = cos(2 pi (m - n/4) / n) = cos(2 pi (4m - n) / (4n))
  return cos2pi(4 * m - n, 4 * n);
}

template <int N>
struct Twiddles {
  float re[N], im[N];  // exp(-2 pi i m / N)
  __host__ __device__ constexpr Twiddles() : re(), im() {
    for (int m = 0; m < N; ++m) {
      re[m] = (float)cos2pi(m, N);
      im[m] = (float)-sin2pi(m, N);
    }
  }
};

// ---------------------------------------------------------------- complex helpers

__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) {
  return make_float2(a.x - b.x, a.y - b.y);
}
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }
__host__ __device__ __forceinline__ float2 mul_pi(float2 a) { return make_float2(-a.y, a.x); }

// v * exp(-2 pi i m / N); m is a compile-time constant after unrolling, so the branches fold.
template <int N>
__host__ __device__ __forceinline__ float2 twiddle(float2 v, int m) {
  constexpr Twiddles<N> T{};
  m %= N;
  if (m == 0) return v;
  if (2 * m == N) return make_float2(-v.x, -v.y);
  if (4 * m == N) return mul_mi(v);
  if (4 * m == 3 * N) return mul_pi(v);
  return cmul(v, make_float2(T.re[m], T.im[m]));
}

// ---------------------------------------------------------------- DFTs

// Split of composite sizes N = A * B (0 for the direct sizes).
template <int N>
struct Split;
template <> struct Split<6> { static constexpr int A = 2, B = 3; };
template <> struct Split<8> { static constexpr int A = 2, B = 4; };
template <> struct Split<9> { static constexpr int A = 3, B = 3; };
template <> struct Split<10> { static constexpr int A = 2, B = 5; };
template <> struct Split<12> { static constexpr int A = 4, B = 3; };
template <> struct Split<15> { static constexpr int A = 3, B = 5; };
template <> struct Split<16> { static constexpr int A = 4, B = 4; };

template <int N>
struct Dft {
  // n = a + A b, k = kb + B ka:
  // V[kb + B ka] = sum_a W_A^{a ka} W_N^{a kb} sum_b v[a + A b] W_B^{b kb}
  __host__ __device__ __forceinline__ static void run(float2* v) {
    constexpr int A = Split<N>::A, B = Split<N>::B;
    float2 y[N];
#pragma unroll
    for (int a = 0; a < A; ++a) {
      float2 t[B];
#pragma unroll
      for (int b = 0; b < B; ++b) t[b] = v[a + A * b];
      Dft<B>::run(t);
#pragma unroll
      for (int kb = 0; kb < B; ++kb) y[a * B + kb] = twiddle<N>(t[kb], a * kb);
    }
#pragma unroll
    for (int kb = 0; kb < B; ++kb) {
      float2 t[A];
#pragma unroll
      for (int a = 0; a < A; ++a) t[a] = y[a * B + kb];
      Dft<A>::run(t);
#pragma unroll
      for (int ka = 0; ka < A; ++ka) v[kb + B * ka] = t[ka];
    }
  }
};

template <>
struct Dft<2> {
  __host__ __device__ __forceinline__ static void run(float2* v) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <>
struct Dft<3> {
  __host__ __device__ __forceinline__ static void run(float2* v) {
    const float s = 0.86602540378443865f;  // sin(2 pi / 3)
    const float2 t1 = cadd(v[1], v[2]);
    const float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
    const float2 d = csub(v[1], v[2]);
    const float2 t3 = make_float2(s * d.y, -s * d.x);  // -i s (v1 - v2)
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
  }
};

template <>
struct Dft<4> {
  __host__ __device__ __forceinline__ static void run(float2* v) {
    const float2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    const float2 c = cadd(v[1], v[3]), d = mul_mi(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
  }
};

template <>
struct Dft<5> {
  __host__ __device__ __forceinline__ static void run(float2* v) {
    const float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;  // cos(2pi/5), cos(4pi/5)
    const float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;   // sin(2pi/5), sin(4pi/5)
    const float2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const float2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const float2 x0 = v[0];
    const float2 p1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
    const float2 p2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
    // q1 = -i (s1 b1 + s2 b2), q2 = -i (s2 b1 - s1 b2)
    const float2 q1 = mul_mi(make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
    const float2 q2 = mul_mi(make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
    v[0] = make_float2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
    v[1] = cadd(p1, q1);
    v[4] = csub(p1, q1);
    v[2] = cadd(p2, q2);
    v[3] = csub(p2, q2);
  }
};

}  // namespace fftr
}  // namespace sfw

// Lengths with a two-stage plan, listed as X(L, R1, R2) with L = R1 * R2: the lengths from 16
// to 256 that split into two factors with a register DFT above (most balanced split, powers
// of two first).
#define SFW_FX_LENGTHS(X) \
  X(16, 4, 4)             \
  X(18, 6, 3)             \
  X(20, 5, 4)             \
  X(24, 6, 4)             \
  X(25, 5, 5)             \
  X(27, 9, 3)             \
  X(30, 6, 5)             \
  X(32, 8, 4)             \
  X(36, 6, 6)             \
  X(40, 8, 5)             \
  X(45, 9, 5)             \
  X(48, 8, 6)             \
  X(50, 10, 5)            \
  X(54, 9, 6)             \
  X(60, 10, 6)            \
  X(64, 8, 8)             \
  X(72, 9, 8)             \
  X(75, 15, 5)            \
  X(80, 10, 8)            \
  X(81, 9, 9)             \
  X(90, 10, 9)            \
  X(96, 12, 8)            \
  X(100, 10, 10)          \
  X(108, 12, 9)           \
  X(120, 12, 10)          \
  X(128, 16, 8)           \
  X(135, 15, 9)           \
  X(144, 12, 12)          \
  X(150, 15, 10)          \
  X(160, 16, 10)          \
  X(180, 15, 12)          \
  X(192, 16, 12)          \
  X(225, 15, 15)          \
  X(240, 16, 15)          \
  X(256, 16, 16)


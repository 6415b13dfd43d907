// Device-side helpers shared by the image-formation kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace sar {

// ---------------------------------------------------------------------------
// complex arithmetic on float2 (x = real, y = imaginary)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a += b * s (s real)
// a += b * c (complex)
__device__ __forceinline__ void cfma_c(float2& a, float2 b, float2 c) {
  a.x = fmaf(b.x, c.x, fmaf(-b.y, c.y, a.x));
  a.y = fmaf(b.x, c.y, fmaf(b.y, c.x, a.y));
}

__device__ __forceinline__ void cfma(float2& a, float2 b, float s) {
  a.x = fmaf(b.x, s, a.x);
  a.y = fmaf(b.y, s, a.y);
}

// exp(j 2 pi t) for t given in cycles (float64); the fractional part is taken
// in float64, then the hardware sine/cosine (which take revolutions) run on it.
__device__ __forceinline__ float2 cis_cycles(double t) {
  const double fr = __builtin_amdgcn_fract(t);  // t - floor(t) in one instruction
  const float r = (float)fr;
  return make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
}
// streaming (non-temporal) loads and stores of one complex value: lines read or
// written once are marked for early eviction instead of displacing reused ones
typedef float f2_vec __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 load_stream(const float2* p) {
  const f2_vec v = __builtin_nontemporal_load((const f2_vec*)p);
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void store_stream(float2* p, float2 v) {
  const f2_vec w = {v.x, v.y};
  __builtin_nontemporal_store(w, (f2_vec*)p);
}
// two adjacent complex values in one 16-byte streaming store (p 16-byte aligned)
typedef float f4_vec __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void store_stream2(float2* p, float2 v0, float2 v1) {
  const f4_vec w = {v0.x, v0.y, v1.x, v1.y};
  __builtin_nontemporal_store(w, (f4_vec*)p);
}

// the same with the argument formed and reduced in float32 (precision diagnostic)
__device__ __forceinline__ float2 cis_cycles_f32(float t) {
  const float r = __builtin_amdgcn_fractf(t);
  return make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
}

// ---------------------------------------------------------------------------
// compile-time loops and twiddles
// ---------------------------------------------------------------------------
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

constexpr double ct_sin_taylor(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int i = 1; i < 16; ++i) {
    term *= -x2 / ((2.0 * i) * (2.0 * i + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ct_cos_taylor(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int i = 1; i < 16; ++i) {
    term *= -x2 / ((2.0 * i - 1.0) * (2.0 * i));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi k / n, exact at multiples of a quarter turn
constexpr double ct_cos2pi(long k, long n) {
  k = ((k % n) + n) % n;
  const long q = (4 * k) / n;
  const long r = 4 * k - q * n;
  const double t = 1.5707963267948966 * (double)r / (double)n;
  const double c = r == 0 ? 1.0 : ct_cos_taylor(t);
  const double s = r == 0 ? 0.0 : ct_sin_taylor(t);
  switch (q & 3) {
    case 0: return c;
    case 1: return -s;
    case 2: return -c;
    default: return s;
  }
}
constexpr double ct_sin2pi(long k, long n) {
  k = ((k % n) + n) % n;
  const long q = (4 * k) / n;
  const long r = 4 * k - q * n;
  const double t = 1.5707963267948966 * (double)r / (double)n;
  const double c = r == 0 ? 1.0 : ct_cos_taylor(t);
  const double s = r == 0 ? 0.0 : ct_sin_taylor(t);
  switch (q & 3) {
    case 0: return s;
    case 1: return c;
    case 2: return -s;
    default: return -c;
  }
}

constexpr int ct_log2(int n) { return n <= 1 ? 0 : 1 + ct_log2(n / 2); }
constexpr int ct_bitrev(int v, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1) << (bits - 1 - i);
  return r;
}

// x * exp(SIGN j 2 pi J / LEN) with J, LEN compile-time
template <int J, int LEN, int SIGN>
__device__ __forceinline__ float2 twiddle_mul(float2 x) {
  constexpr int jm = ((J % LEN) + LEN) % LEN;
  if constexpr (jm == 0) {
    return x;
  } else if constexpr (4 * jm == LEN) {           // exp(SIGN j pi/2) = SIGN j
    return SIGN > 0 ? make_float2(-x.y, x.x) : make_float2(x.y, -x.x);
  } else if constexpr (2 * jm == LEN) {
    return make_float2(-x.x, -x.y);
  } else if constexpr (4 * jm == 3 * LEN) {
    return SIGN > 0 ? make_float2(x.y, -x.x) : make_float2(-x.y, x.x);
  } else {
    constexpr float c = (float)ct_cos2pi(jm, LEN);
    constexpr float s = (float)(SIGN * ct_sin2pi(jm, LEN));
    return make_float2(x.x * c - x.y * s, x.x * s + x.y * c);
  }
}

// In-register radix-2 decimation-in-frequency DFT of size N (power of two):
// X[k] = sum_n x[n] exp(SIGN j 2 pi n k / N).  Input in natural order, output
// X[k] left in x[bitrev(k)].
template <int N, int SIGN>
__device__ __forceinline__ void reg_dft_dif(float2 (&x)[N]) {
  static_assert((N & (N - 1)) == 0, "power of two");
  if constexpr (N >= 2) {
    static_for<0, ct_log2(N)>([&](auto sc) __attribute__((always_inline)) {
      constexpr int stage = decltype(sc)::value;
      constexpr int len = N >> stage;
      constexpr int half = len / 2;
      static_for<0, N / len>([&](auto gc) __attribute__((always_inline)) {
        constexpr int start = decltype(gc)::value * len;
        static_for<0, half>([&](auto jc) __attribute__((always_inline)) {
          constexpr int j = decltype(jc)::value;
          const float2 a = x[start + j];
          const float2 b = x[start + j + half];
          x[start + j] = cadd(a, b);
          x[start + j + half] = twiddle_mul<j, len, SIGN>(csub(a, b));
        });
      });
    });
  }
}

// XCD-aware remap of a linear block id: the hardware deals consecutive block
// ids round-robin over the 8 XCDs; remap so that each XCD receives one
// contiguous range of work ids (neighbouring tiles share that XCD's L2).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nblocks) {
  constexpr uint32_t kXcd = 8;
  if (nblocks % kXcd != 0) return bid;
  const uint32_t per = nblocks / kXcd;
  return (bid % kXcd) * per + bid / kXcd;
}

}  // namespace sar

// Steps a3 and a6: batched 1-D FFTs along a strided axis whose batch
// dimension is contiguous in memory (frequency, or the transverse mode index
// times z, is always the fastest index in this library's layouts).
//
// Four-step decomposition L = L1 * L2 of
//   X[k2 + L2 k1] = sum_{l1} w_L1^{l1 k1} w_L^{l1 k2} sum_{l2} x[l1 + L1 l2] w_L2^{l2 k2}:
// each thread loads one stride-L1 subsequence of one batch column straight
// from HBM into registers, runs an unrolled L2-point DFT with compile-time
// twiddles, applies the inter-step twiddle (built from two entries of a
// float64-generated table),
// exchanges through LDS once, and finishes with an L1-point register DFT.
// A block handles BC adjacent batch columns so loads and stores move BC*8
// contiguous bytes per row.  The epilogue fuses the crop to the image's
// centred modes and a per-output scale (deapodisation or +-1 signs).  Inputs
// are read once, with streaming loads; outputs use streaming stores only where
// no later kernel reads them soon (the image), since the next pass reads the
// others straight back.

#include "device_common.hpp"
#include "launch.hpp"
#include "sar_internal.hpp"

namespace sar {
namespace {

template <int L1, int L2, int BC, int SIGN>
struct FftBody {
  using Args = FftLines;
  static constexpr int kThreads = (L1 > L2 ? L1 : L2) * BC;
  static __device__ __forceinline__ void run(const FftLines& a, uint32_t blk, uint32_t nblk);
};

template <int L1, int L2, int BC, int SIGN>
__device__ __forceinline__ void FftBody<L1, L2, BC, SIGN>::run(const FftLines& a, uint32_t blk, uint32_t nblk) {
  constexpr int L = L1 * L2;
  constexpr int RS = (L2 + 1) * BC;  // padded LDS row (one l1) to spread banks
  extern __shared__ float2 lds[];     // [L1][L2 + 1][BC]
  const int64_t nbc = (a.B + BC - 1) / BC;
  // consecutive column groups share cache lines when BC * 8 < 128 bytes: the
  // remap runs them back to back on one XCD so the second finds them in L2
  const int64_t bid = xcd_remap(blk, nblk);
  const int64_t o = bid / nbc;
  const int64_t bc = bid - o * nbc;
  const int b = threadIdx.x % BC;
  const int t = threadIdx.x / BC;
  const int64_t bg = bc * BC + b;
  const bool bv = bg < a.B;
  const float2* __restrict__ in = a.in + o * a.s_in_o + (bv ? bg : 0);

  if (t < L1) {
    float2 v[L2];
#pragma unroll
    for (int l2 = 0; l2 < L2; ++l2)
      v[l2] = bv ? load_stream(&in[(int64_t)(t + L1 * l2) * a.s_in_l]) : make_float2(0.f, 0.f);
    reg_dft_dif<L2, SIGN>(v);
    // inter-step twiddles w_L^(t k2) from two table reads, w^t and w^(TB t):
    // w^(t k2) = (w^(TB t))^(k2 / TB) (w^t)^(k2 % TB), at most about nine
    // roundings each (the table reads they replace were a third of the
    // pass's memory instructions)
    constexpr int TB = L2 < 8 ? L2 : 8;
    float2 p1[TB], pB[(L2 + TB - 1) / TB];
    p1[0] = make_float2(1.f, 0.f);
    pB[0] = make_float2(1.f, 0.f);
    {
      const float2 w1 = a.tw[t];
#pragma unroll
      for (int j = 1; j < TB; ++j) p1[j] = cmul(p1[j - 1], w1);
      const float2 wB = a.tw[(TB * t) % L];
#pragma unroll
      for (int j = 1; j < (L2 + TB - 1) / TB; ++j) pB[j] = cmul(pB[j - 1], wB);
    }
    static_for<0, L2>([&](auto kc) __attribute__((always_inline)) {
      constexpr int k2 = decltype(kc)::value;
      float2 y = v[ct_bitrev(k2, ct_log2(L2))];
      if constexpr (k2 != 0) y = cmul(y, cmul(pB[k2 / TB], p1[k2 % TB]));
      lds[t * RS + k2 * BC + b] = y;
    });
  }
  __syncthreads();
  if (t < L2) {
    float2 v[L1];
#pragma unroll
    for (int l1 = 0; l1 < L1; ++l1) v[l1] = lds[l1 * RS + t * BC + b];
    reg_dft_dif<L1, SIGN>(v);
    if (bv) {
      float2* __restrict__ out = a.out + o * a.s_out_o + bg;
      static_for<0, L1>([&](auto kc) __attribute__((always_inline)) {
        constexpr int k1 = decltype(kc)::value;
        const int k = t + L2 * k1;
        int P;
        if (a.centred) {
          const int h = a.n_out / 2;
          P = k < a.n_out - h ? k + h : (k >= L - h ? k - L + h : -1);
        } else {
          P = k;
        }
        if (P >= 0) {
          float2 y = v[ct_bitrev(k1, ct_log2(L1))];
          if (a.scale) y = cscale(y, a.scale[P]);
          if (a.nt_out)
            store_stream(&out[(int64_t)P * a.s_out_k], y);
          else
            out[(int64_t)P * a.s_out_k] = y;
        }
      });
    }
  }
}

// ---------------------------------------------------------------------------
// Any length 2^a 3^b 5^c (the non-power-of-two image sides and oversampled
// grids): a block holds BC batch columns of the whole line in LDS and runs
// self-sorting (Stockham) radix-8/4/2/3/5 passes on it.  Pass p with radix R,
// after passes whose radices multiply to Ns, maps butterfly j (k = j mod Ns)
// from x[j + q L/R] to x'[(j / Ns) Ns R + k + q Ns] after the twiddles
// w_{Ns R}^(q k) and an R-point DFT; the last pass leaves X in natural order.
// Each pass reads all its butterflies into registers, waits for the block, and
// writes them back, so one LDS buffer serves in place; every thread issues all
// its global loads (at most 32) before using any.  The epilogue is that of the
// power-of-two kernel plus the shifted, complex-scaled placement of odd
// inverse lengths.
constexpr int kMixMaxPasses = 16;
constexpr int kMixThreads = 512;
constexpr int kMixMaxElems = 4096;                        // L x BC complex values in LDS
constexpr int kMixPerThread = kMixMaxElems / kMixThreads;  // 8

struct FftMixedArgs {
  FftLines f;
  int lbc;    // log2 of the batch columns per block
  int npass;
  uint64_t radices;  // radix of pass p in bits [4p, 4p + 4) (no per-pass array:
                     // a fused batch copies its arguments to registers)
  // n / d as umulhi(n, ceil(2^32 / d)), exact for n < 2^16, d <= 4096 (checked
  // exhaustively); this one for the length, the passes' Ns computed in the kernel
  uint32_t mag_l;
};

// ceil(2^32 / d) for 2 <= d <= 4096 (0 for d = 1): in float64 the quotient is
// exact when d is a power of two and otherwise at least 1/d from an integer,
// far more than its rounding, so the ceiling is exact
__device__ __forceinline__ uint32_t magic_div(int d) {
  return d <= 1 ? 0u : (uint32_t)ceil(4294967296.0 / (double)d);
}

// R-point DFT in natural order, X[m] = sum_n a[n] exp(SIGN j 2 pi n m / R)
template <int R, int SIGN>
__device__ __forceinline__ void small_dft(float2 (&a)[R]) {
  if constexpr ((R & (R - 1)) == 0) {
    reg_dft_dif<R, SIGN>(a);   // output in bit-reversed order
    float2 t[R];
#pragma unroll
    for (int m = 0; m < R; ++m) t[m] = a[ct_bitrev(m, ct_log2(R))];
#pragma unroll
    for (int m = 0; m < R; ++m) a[m] = t[m];
  } else {
    float2 t[R];
    static_for<0, R>([&](auto mc) __attribute__((always_inline)) {
      constexpr int m = decltype(mc)::value;
      float2 acc = a[0];
      static_for<1, R>([&](auto nc) __attribute__((always_inline)) {
        constexpr int n = decltype(nc)::value;
        acc = cadd(acc, twiddle_mul<(m * n) % R, R, SIGN>(a[n]));
      });
      t[m] = acc;
    });
#pragma unroll
    for (int m = 0; m < R; ++m) a[m] = t[m];
  }
}

template <int R, int SIGN>
__device__ __forceinline__ void stockham_pass(float2* __restrict__ x, int L, int lbc, int Ns, uint32_t mag_ns,
                                              uint32_t mag_l, const float2* __restrict__ tw) {
  constexpr int U = (kMixPerThread + R - 1) / R;  // butterflies per thread at most
  const int BC = 1 << lbc;
  const int m = L / R;
  const int nb = m << lbc;            // butterflies of the block
  const int tstep = L / (Ns * R);     // w_{Ns R} = tw[tstep]
  float2 v[U][R];
  int dst[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int i = threadIdx.x + u * kMixThreads;
    dst[u] = -1;
    if (i < nb) {
      const int b = i & (BC - 1);
      const int j = i >> lbc;
      const int g = mag_ns ? (int)__umulhi((uint32_t)j, mag_ns) : j;  // j / Ns
      const int k = j - g * Ns;
#pragma unroll
      for (int q = 0; q < R; ++q) v[u][q] = x[((j + q * m) << lbc) + b];
      if (k != 0) {
        const int e = tstep * k;
#pragma unroll
        for (int q = 1; q < R; ++q) {
          const int t = q * e;
          v[u][q] = cmul(v[u][q], tw[t - L * (int)__umulhi((uint32_t)t, mag_l)]);  // (q e) mod L
        }
      }
      small_dft<R, SIGN>(v[u]);
      dst[u] = ((g * Ns * R + k) << lbc) + b;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (dst[u] >= 0) {
#pragma unroll
      for (int q = 0; q < R; ++q) x[dst[u] + ((q * Ns) << lbc)] = v[u][q];
    }
  __syncthreads();
}

template <int SIGN>
struct FftMixedBody {
  using Args = FftMixedArgs;
  static constexpr int kThreads = kMixThreads;
  static constexpr int kMinWavesPerEU = 4;  // up to four blocks per CU (32 KiB of LDS each)
  static __device__ __forceinline__ void run(const FftMixedArgs& m, uint32_t blk, uint32_t) {
    extern __shared__ float2 lds[];
    const FftLines& a = m.f;
    const int L = a.L;
    const int lbc = m.lbc;
    const int BC = 1 << lbc;
    const int ne = L << lbc;
    const int64_t nbc = (a.B + BC - 1) / BC;
    const int64_t o = blk / nbc;
    const int64_t bc = blk - o * nbc;
    float2* x = lds;
    {
      const float2* __restrict__ in = a.in + o * a.s_in_o + bc * BC;
      float2 t[kMixPerThread];
#pragma unroll
      for (int u = 0; u < kMixPerThread; ++u) {
        const int i = threadIdx.x + u * kMixThreads;
        const int b = i & (BC - 1);
        t[u] = (i < ne && bc * BC + b < a.B) ? load_stream(&in[(int64_t)(i >> lbc) * a.s_in_l + b])
                                             : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < kMixPerThread; ++u) {
        const int i = threadIdx.x + u * kMixThreads;
        if (i < ne) x[i] = t[u];
      }
    }
    __syncthreads();
    int Ns = 1;
    for (int p = 0; p < m.npass; ++p) {
      const int R = (int)((m.radices >> (4 * p)) & 15u);
      const uint32_t mg = magic_div(Ns);
      if (R == 8)
        stockham_pass<8, SIGN>(x, L, lbc, Ns, mg, m.mag_l, a.tw);
      else if (R == 4)
        stockham_pass<4, SIGN>(x, L, lbc, Ns, mg, m.mag_l, a.tw);
      else if (R == 2)
        stockham_pass<2, SIGN>(x, L, lbc, Ns, mg, m.mag_l, a.tw);
      else if (R == 3)
        stockham_pass<3, SIGN>(x, L, lbc, Ns, mg, m.mag_l, a.tw);
      else
        stockham_pass<5, SIGN>(x, L, lbc, Ns, mg, m.mag_l, a.tw);
      Ns *= R;
    }
    float2* __restrict__ out = a.out + o * a.s_out_o + bc * BC;
    const int h = a.n_out / 2;
    for (int i = threadIdx.x; i < ne; i += kMixThreads) {
      const int b = i & (BC - 1);
      const int k = i >> lbc;
      if (bc * BC + b >= a.B) continue;
      int P;
      if (a.centred == 1)
        P = k < a.n_out - h ? k + h : (k >= L - h ? k - L + h : -1);
      else if (a.centred == 2)
        P = k + h < L ? k + h : k + h - L;
      else
        P = k;
      if (P < 0) continue;
      float2 v = x[i];
      if (a.centred == 2)
        v = cmul(v, a.cscale[P]);
      else if (a.scale)
        v = cscale(v, a.scale[P]);
      float2* dst = &out[(int64_t)P * a.s_out_k + b];
      if (a.nt_out)
        store_stream(dst, v);
      else
        *dst = v;
    }
  }
};

sar_status launch_mixed(const FftLines& a, LaunchSink& sink) {
  FftMixedArgs m{};
  m.f = a;
  int n = a.L;
  for (int r : {8, 4, 2, 3, 5})
    while (n % r == 0) {
      if (m.npass == kMixMaxPasses) return fail(SAR_ERR_UNSUPPORTED, "FFT length has too many factors");
      m.radices |= (uint64_t)r << (4 * m.npass++);
      n /= r;
    }
  if (n != 1) return fail(SAR_ERR_UNSUPPORTED, "FFT length not a product of 2, 3 and 5: " + std::to_string(a.L));
  if (a.L > kMixMaxElems) return fail(SAR_ERR_UNSUPPORTED, "FFT length too long: " + std::to_string(a.L));
  // batch columns per block: up to 16 (128-byte row segments) while the
  // block's lines fit its 32 KiB of LDS
  int bc = 1;
  while (bc < 16 && 2 * bc * a.L <= kMixMaxElems && bc < a.B) bc *= 2;
  while ((1 << m.lbc) < bc) ++m.lbc;
  m.mag_l = (uint32_t)(((1ull << 32) + (uint64_t)a.L - 1) / (uint64_t)a.L);
  const int64_t nblk = (a.B + bc - 1) / bc * a.n_outer;
  if (nblk <= 0) return SAR_OK;
  if (nblk > 0x7fffffffLL) return fail(SAR_ERR_UNSUPPORTED, "FFT batch too large");
  const size_t lds = (size_t)a.L * bc * sizeof(float2);
  if (a.sign < 0) return launch_body<FftMixedBody<-1>>(sink, (uint32_t)nblk, lds, m, "fft launch");
  return launch_body<FftMixedBody<+1>>(sink, (uint32_t)nblk, lds, m, "fft launch");
}

template <int L1, int L2, int BC>
sar_status launch_lb(const FftLines& a, LaunchSink& sink) {
  const size_t lds = (size_t)L1 * (L2 + 1) * BC * sizeof(float2);
  const int64_t nbc = (a.B + BC - 1) / BC;
  const int64_t nblk = nbc * a.n_outer;
  if (nblk <= 0) return SAR_OK;
  if (nblk > 0x7fffffffLL) return fail(SAR_ERR_UNSUPPORTED, "FFT batch too large");
  if (a.sign < 0) return launch_body<FftBody<L1, L2, BC, -1>>(sink, (uint32_t)nblk, lds, a, "fft launch");
  return launch_body<FftBody<L1, L2, BC, +1>>(sink, (uint32_t)nblk, lds, a, "fft launch");
}

}  // namespace

bool is_5smooth(int64_t v) {
  if (v < 1) return false;
  for (int r : {2, 3, 5})
    while (v % r == 0) v /= r;
  return v == 1;
}

sar_status launch_fft_lines(const FftLines& a, LaunchSink& sink) {
  // shifted placement (odd lengths) only in the mixed-radix kernel
  if (a.centred == 2 || (a.L & (a.L - 1)) != 0) return launch_mixed(a, sink);
  // batch columns per block chosen so one block's LDS stays near 64 KiB; where
  // L is not a square, L1 > L2 so that every thread of the block loads and
  // transforms in the first pass (the load-bound one)
  switch (a.L) {
    case 8: return launch_lb<4, 2, 16>(a, sink);
    case 16: return launch_lb<4, 4, 16>(a, sink);
    case 32: return launch_lb<8, 4, 16>(a, sink);
    case 64: return launch_lb<8, 8, 16>(a, sink);
    case 128: return launch_lb<16, 8, 16>(a, sink);
    case 256: return launch_lb<16, 16, 16>(a, sink);
    case 512: return launch_lb<32, 16, 16>(a, sink);
    case 1024: return launch_lb<32, 32, 8>(a, sink);
    case 2048: return launch_lb<64, 32, 4>(a, sink);
    case 4096: return launch_lb<64, 64, 2>(a, sink);
    default: return launch_mixed(a, sink);
  }
}

}  // namespace sar

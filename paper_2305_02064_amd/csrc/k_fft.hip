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
          P = k < h ? k + h : (k >= L - h ? k - L + h : -1);
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

sar_status launch_fft_lines(const FftLines& a, LaunchSink& sink) {
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
    default: return fail(SAR_ERR_UNSUPPORTED, "FFT length not supported: " + std::to_string(a.L));
  }
}

}  // namespace sar

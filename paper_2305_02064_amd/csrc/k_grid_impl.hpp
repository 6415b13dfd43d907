#pragma once
// Steps a1 + a2 (kernel template; one translation unit per kernel width): multi-planar multistatic compensation (Eq. (11)) fused into
// Kaiser-Bessel gridding of the irregular virtual samples onto the oversampled
// uniform (x', y') grid (the spreading half of the type-1 NUFFT that stands in
// for FT_2D of Eq. (16), Sec. III).
//
// Output-stationary design: one wavefront owns an 8 x 8 tile of grid cells for
// 64 consecutive frequencies (lane = frequency) and keeps the 64 complex
// accumulators in registers.  It walks the sorted records of every sample
// whose W x W support touches the tile (rows of base cells, each a contiguous
// run in the cell-sorted list), compensates the sample's echo once per
// frequency with the float64 phase argument k * beta reduced modulo one cycle,
// and adds the clipped separable taps.  Sample records are staged in LDS 64 at
// a time (one lane per record) and read back as broadcasts; echo rows are
// prefetched eight samples ahead into a ring of registers.  Which taps of a sample land inside the
// tile depends on its base-cell offset (A, B) relative to the tile; a uniform
// binary dispatch selects a fully unrolled body for that offset so every
// accumulator index is static.  Tiles partition the grid, so each cell is
// written exactly once with plain coalesced stores: no atomics, no zeroing
// pass, and a fixed summation order.

#include <hip/hip_fp16.h>

#include "device_common.hpp"
#include "sar_internal.hpp"

namespace sar {
namespace grid_impl {

constexpr int T = kTile;

struct GridArgs {
  const void* rec;
  const int32_t* cell_start;
  const void* echo;
  float echo_scale;
  const double* fcc;  // f / c per frequency
  float2* grid;       // [my][mx][nf]
  int mx, my, nf;
  int ntx, nty;
};

template <int LO, int HI, typename F>
__device__ __forceinline__ void dispatch_range(int idx, F&& f) {
  if constexpr (HI - LO == 1) {
    f(std::integral_constant<int, LO>{});
  } else {
    constexpr int MID = (LO + HI) / 2;
    if (idx < MID)
      dispatch_range<LO, MID>(idx, f);
    else
      dispatch_range<MID, HI>(idx, f);
  }
}

template <int ET>
__device__ __forceinline__ float2 load_echo(const void* echo, int64_t idx, float scale) {
  if constexpr (ET == SAR_ECHO_C64) {
    return ((const float2*)echo)[idx];
  } else {
    const __half2 h = ((const __half2*)echo)[idx];
    const float2 v = __half22float2(h);
    return make_float2(v.x * scale, v.y * scale);
  }
}

template <int W, int ET>
__global__ __launch_bounds__(64) void k_grid(GridArgs a) {
  constexpr int NB = T + W - 1;       // base-cell offsets per axis touching a tile
  constexpr int NSEG = 2 * NB;        // each row may split in two at the x wrap
  constexpr int D = 8;                // echo prefetch depth (samples)
  constexpr int RW = (int)(sizeof(SampleRec<W>) / sizeof(uint4));
  static_assert(sizeof(SampleRec<W>) % sizeof(uint4) == 0, "record is a whole number of 16-byte words");
  __shared__ int seg_s[NSEG];
  __shared__ int seg_off[NSEG + 1];
  __shared__ uint4 recs[64 * RW];     // records of the current chunk of 64 samples

  const uint32_t work = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = (int)(work % (uint32_t)a.ntx);
  const uint32_t rest = work / (uint32_t)a.ntx;
  const int ty = (int)(rest % (uint32_t)a.nty);
  const int fchunk = (int)(rest / (uint32_t)a.nty);
  const int tx0 = tx * T, ty0 = ty * T;
  const int lane = threadIdx.x;
  const int f = fchunk * 64 + lane;
  const bool active = f < a.nf;
  const int fl = active ? f : a.nf - 1;
  const double fcc = a.fcc[fl];
  const SampleRec<W>* __restrict__ rec = (const SampleRec<W>*)a.rec;

  // runs of base cells: row j (A = j - (W-1)), x in [tx0 - (W-1), tx0 + T)
  if (lane < NB) {
    int cy = ty0 + lane - (W - 1);
    cy = cy < 0 ? cy + a.my : cy;
    const int64_t row = (int64_t)cy * a.mx;
    const int xlo = tx0 - (W - 1);
    const int xhi = tx0 + T;
    int s0, e0, s1 = 0, e1 = 0;
    if (xlo >= 0) {
      s0 = a.cell_start[row + xlo];
      e0 = a.cell_start[row + xhi];
    } else {
      s0 = a.cell_start[row + a.mx + xlo];
      e0 = a.cell_start[row + a.mx];
      s1 = a.cell_start[row];
      e1 = a.cell_start[row + xhi];
    }
    seg_s[2 * lane] = s0;
    seg_s[2 * lane + 1] = s1;
    seg_off[2 * lane] = e0 - s0;
    seg_off[2 * lane + 1] = e1 - s1;
  }
  __syncthreads();
  if (lane == 0) {
    int run = 0;
    for (int k = 0; k < NSEG; ++k) {
      const int l = seg_off[k];
      seg_off[k] = run;
      run += l;
    }
    seg_off[NSEG] = run;
  }
  __syncthreads();
  const int total = __builtin_amdgcn_readfirstlane(seg_off[NSEG]);

  float2 acc[T][T];
#pragma unroll
  for (int r = 0; r < T; ++r)
#pragma unroll
    for (int c = 0; c < T; ++c) acc[r][c] = make_float2(0.f, 0.f);

  for (int c0 = 0; c0 < total; c0 += 64) {
    const int n_c = __builtin_amdgcn_readfirstlane(min(64, total - c0));
    // lane j stages the record of the chunk's j-th sample in LDS
    int srcv = 0, av = 0;
    if (lane < n_c) {
      const int t = c0 + lane;
      int k = 0;
      while (seg_off[k + 1] <= t) ++k;
      const int s = seg_s[k] + (t - seg_off[k]);
      const uint4* rp = (const uint4*)(rec + s);
#pragma unroll
      for (int q = 0; q < RW; ++q) recs[lane * RW + q] = rp[q];
      srcv = rec[s].src;
      av = k / 2 - (W - 1);
    }
    __syncthreads();

    // echo prefetch ring (D samples ahead); slots are selected by a uniform
    // switch so every ring register keeps a static index
    float2 ring[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      ring[d] = make_float2(0.f, 0.f);
      if (d < n_c) {
        const int sd = __builtin_amdgcn_readlane(srcv, d);
        ring[d] = load_echo<ET>(a.echo, (int64_t)sd * a.nf + fl, a.echo_scale);
      }
    }
    for (int j = 0; j < n_c; ++j) {
      const int jn = j + D;
      const bool pre = jn < n_c;
      const int sn = __builtin_amdgcn_readlane(srcv, pre ? jn : 0);
      const int64_t en = (int64_t)sn * a.nf + fl;
      float2 ev = make_float2(0.f, 0.f);
      dispatch_range<0, D>(j & (D - 1), [&](auto dc) __attribute__((always_inline)) {
        constexpr int d = decltype(dc)::value;
        ev = ring[d];
        if (pre) ring[d] = load_echo<ET>(a.echo, en, a.echo_scale);
      });
      SampleRec<W> r;
      {
        uint4 w4[RW];
#pragma unroll
        for (int q = 0; q < RW; ++q) w4[q] = recs[j * RW + q];
        __builtin_memcpy(&r, w4, sizeof(r));
      }
      const int A = __builtin_amdgcn_readlane(av, j);
      // compensation: s_hat = s exp(+j 2 pi f beta / c)
      const float2 v = cmul(ev, cis_cycles(r.beta * fcc));
      int b = __builtin_amdgcn_readfirstlane((int)r.cx) - tx0;
      if (b < -(W - 1)) b += a.mx;
      if (b >= T) b -= a.mx;
      const int idx = (A + (W - 1)) * NB + (b + (W - 1));
      dispatch_range<0, NB * NB>(idx, [&](auto ic) __attribute__((always_inline)) {
        constexpr int I = decltype(ic)::value;
        constexpr int AA = I / NB - (W - 1);
        constexpr int BB = I % NB - (W - 1);
        static_for<0, W>([&](auto jc) __attribute__((always_inline)) {
          constexpr int jj = decltype(jc)::value;
          constexpr int rr = AA + jj;
          if constexpr (rr >= 0 && rr < T) {
            const float2 vy = cscale(v, r.wy[jj]);
            static_for<0, W>([&](auto kc) __attribute__((always_inline)) {
              constexpr int kk = decltype(kc)::value;
              constexpr int cc = BB + kk;
              if constexpr (cc >= 0 && cc < T) cfma(acc[rr][cc], vy, r.wx[kk]);
            });
          }
        });
      });
    }
    __syncthreads();
  }

  if (active) {
#pragma unroll
    for (int r = 0; r < T; ++r)
#pragma unroll
      for (int c = 0; c < T; ++c)
        a.grid[((int64_t)(ty0 + r) * a.mx + (tx0 + c)) * a.nf + f] = acc[r][c];
  }
}

template <int W>
sar_status grid_w(const Plan& p, const void* d_echo, float echo_scale, const Workspace& ws, float2* grid,
                  hipStream_t stream) {
  GridArgs a;
  a.rec = ws.rec;
  a.cell_start = ws.cell_start;
  a.echo = d_echo;
  a.echo_scale = echo_scale;
  a.fcc = p.d_fcc;
  a.grid = grid;
  a.mx = p.mx;
  a.my = p.my;
  a.nf = p.nf;
  a.ntx = p.mx / T;
  a.nty = p.my / T;
  const int nfc = (p.nf + 63) / 64;
  const int64_t nblk = (int64_t)a.ntx * a.nty * nfc;
  if (p.echo_type == SAR_ECHO_C64)
    k_grid<W, SAR_ECHO_C64><<<(unsigned)nblk, 64, 0, stream>>>(a);
  else
    k_grid<W, SAR_ECHO_F16X2><<<(unsigned)nblk, 64, 0, stream>>>(a);
  return check_hip(hipGetLastError(), "gridding launch");
}

}  // namespace grid_impl

#define SAR_INSTANTIATE_GRID(W)                                                                    \
  sar_status launch_gridding_w##W(const Plan& p, const void* d_echo, float echo_scale,              \
                                  const Workspace& ws, float2* grid, hipStream_t stream) {          \
    return grid_impl::grid_w<W>(p, d_echo, echo_scale, ws, grid, stream);                          \
  }

}  // namespace sar

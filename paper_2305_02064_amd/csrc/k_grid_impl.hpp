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
// and adds the clipped separable taps.  Echo rows are streamed through LDS in
// chunks of 8 samples with the direct global-to-LDS loads of gfx950: at the
// start of chunk c the wave waits once, moves the chunk's echo values into
// registers, and issues the loads of chunk c+1 (whose source rows were fetched
// a chunk earlier), so memory latency overlaps the arithmetic of a whole
// chunk.  Sample records arrive through scalar loads.  Which taps of a sample land inside the
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
  const int32_t* order;  // source row of each sorted sample
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

// asynchronous copy of one dword per lane from global memory into LDS at
// lds_base + 4 * lane (the direct global-to-LDS load of gfx950)
__device__ __forceinline__ void dma_dword(const void* src, void* lds_base) {
  __builtin_amdgcn_global_load_lds(src, (void __attribute__((address_space(3)))*)lds_base, 4, 0, 0);
}

template <int W, int ET>
__global__ __launch_bounds__(64) void k_grid(GridArgs a) {
  constexpr int NB = T + W - 1;       // base-cell offsets per axis touching a tile
  constexpr int NSEG = 2 * NB;        // each row may split in two at the x wrap
  constexpr int CH = 8;               // samples per pipeline chunk
  constexpr int EB = ET == SAR_ECHO_C64 ? 512 : 256;  // echo bytes per sample and wave
  __shared__ int seg_s[NSEG];
  __shared__ int seg_off[NSEG + 1];
  __shared__ __attribute__((aligned(16))) char echobuf[CH * EB];

  const uint32_t work = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = (int)(work % (uint32_t)a.ntx);
  const uint32_t rest = work / (uint32_t)a.ntx;
  const int ty = (int)(rest % (uint32_t)a.nty);
  const int fchunk = (int)(rest / (uint32_t)a.nty);
  const int tx0 = tx * T, ty0 = ty * T;
  const int lane = threadIdx.x;
  const int fbase = fchunk * 64;
  const int f = fbase + lane;
  const bool active = f < a.nf;
  const int fl = active ? f : a.nf - 1;
  const double fcc = a.fcc[fl];
  // records are read-only here: read through the constant address space they
  // are fetched with scalar loads
  typedef const __attribute__((address_space(4))) uint32_t* cword_ptr;
  const cword_ptr crec = (cword_ptr)a.rec;
  auto load_rec = [&](int sidx) __attribute__((always_inline)) {
    constexpr int RD = (int)(sizeof(SampleRec<W>) / 4);
    uint32_t w[RD];
    const cword_ptr p = crec + (int64_t)sidx * RD;
#pragma unroll
    for (int q = 0; q < RD; ++q) w[q] = p[q];
    SampleRec<W> out;
    __builtin_memcpy(&out, w, sizeof(out));
    return out;
  };

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
  const int nchunk = (total + CH - 1) / CH;

  // sorted-list index of the chunk's lane-th sample (lanes >= chunk size: -1)
  auto chunk_index = [&](int c) __attribute__((always_inline)) -> int {
    const int t = c * CH + lane;
    if (lane >= CH || t >= total) return -1;
    int k = 0;
    while (seg_off[k + 1] <= t) ++k;
    return seg_s[k] + (t - seg_off[k]);
  };
  // echo rows of a chunk into LDS with direct global-to-LDS loads
  auto stage_echo = [&](int c, int srcv) __attribute__((always_inline)) {
    const int n = min(CH, total - c * CH);
    for (int k = 0; k < n; ++k) {
      const int src = __builtin_amdgcn_readlane(srcv, k);
      if constexpr (ET == SAR_ECHO_C64) {
        const float* row = (const float*)a.echo + (int64_t)src * a.nf * 2;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int fi = fbase * 2 + h * 64 + lane;   // float index within the row
          dma_dword(row + (fi < 2 * a.nf ? fi : 0), echobuf + k * EB + h * 256);
        }
      } else {
        const uint32_t* row = (const uint32_t*)a.echo + (int64_t)src * a.nf;
        const int fi = fbase + lane;
        dma_dword(row + (fi < a.nf ? fi : 0), echobuf + k * EB);
      }
    }
  };

  float2 acc[T][T];
#pragma unroll
  for (int r = 0; r < T; ++r)
#pragma unroll
    for (int c = 0; c < T; ++c) acc[r][c] = make_float2(0.f, 0.f);

  // pipeline: echo of chunk c+1 and source rows of chunk c+2 are in flight
  // while chunk c is processed from registers
  int sidx0 = chunk_index(0);
  int sidx1 = chunk_index(1);
  int src0 = sidx0 >= 0 ? a.order[sidx0] : 0;
  int src1 = sidx1 >= 0 ? a.order[sidx1] : 0;
  if (nchunk > 0) stage_echo(0, src0);
  for (int c = 0; c < nchunk; ++c) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int n = __builtin_amdgcn_readfirstlane(min(CH, total - c * CH));
    // the chunk's echo values (re, im interleaved) in one register vector,
    // indexed below with a uniform sample index
    typedef float evec __attribute__((ext_vector_type(2 * CH)));
    evec ev;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      float2 t2;
      if constexpr (ET == SAR_ECHO_C64) {
        t2 = *(const float2*)(echobuf + k * EB + lane * 8);
      } else {
        t2 = __half22float2(*(const __half2*)(echobuf + k * EB + lane * 4));
        t2 = make_float2(t2.x * a.echo_scale, t2.y * a.echo_scale);
      }
      ev[2 * k] = t2.x;
      ev[2 * k + 1] = t2.y;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (c + 1 < nchunk) stage_echo(c + 1, src1);
    const int sidx2 = chunk_index(c + 2);
    const int src2 = sidx2 >= 0 ? a.order[sidx2] : 0;
    SampleRec<W> r = load_rec(__builtin_amdgcn_readlane(sidx0, 0));
    for (int k = 0; k < n; ++k) {
      // consume the current record (its scalar load was issued one sample ago)
      int A = (int)r.cy - ty0;
      if (A < -(W - 1)) A += a.my;
      if (A >= T) A -= a.my;
      int b = (int)r.cx - tx0;
      if (b < -(W - 1)) b += a.mx;
      if (b >= T) b -= a.mx;
      const int idx = __builtin_amdgcn_readfirstlane((A + (W - 1)) * NB + (b + (W - 1)));
      const double arg = r.beta * fcc;
      const SampleRec<W> rc = r;
      // scalar loads return out of order and can only be waited for all
      // together: issue the next record's load only after the current one
      // has been consumed
      asm volatile("" ::: "memory");
      if (k + 1 < n) r = load_rec(__builtin_amdgcn_readlane(sidx0, k + 1));
      const float2 e = make_float2(ev[2 * k], ev[2 * k + 1]);
      // compensation: s_hat = s exp(+j 2 pi f beta / c)
      const float2 v = cmul(e, cis_cycles(arg));
      dispatch_range<0, NB * NB>(idx, [&](auto ic) __attribute__((always_inline)) {
        constexpr int I = decltype(ic)::value;
        constexpr int AA = I / NB - (W - 1);
        constexpr int BB = I % NB - (W - 1);
        static_for<0, W>([&](auto jc) __attribute__((always_inline)) {
          constexpr int jj = decltype(jc)::value;
          constexpr int rr = AA + jj;
          if constexpr (rr >= 0 && rr < T) {
            const float2 vy = cscale(v, rc.wy[jj]);
            static_for<0, W>([&](auto kc) __attribute__((always_inline)) {
              constexpr int kk = decltype(kc)::value;
              constexpr int cc = BB + kk;
              if constexpr (cc >= 0 && cc < T) cfma(acc[rr][cc], vy, rc.wx[kk]);
            });
          }
        });
      });
    }
    sidx0 = sidx1;
    sidx1 = sidx2;
    src1 = src2;
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
  a.order = ws.order;
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

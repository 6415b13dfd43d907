// Steps a1 + a2 (kernel template; one translation unit per kernel width):
// multi-planar multistatic compensation (Eq. (11)) fused into Kaiser-Bessel
// gridding of the irregular virtual samples onto the oversampled uniform
// (x', y') grid (the spreading half of the type-1 NUFFT that stands in for
// FT_2D of Eq. (16), Sec. III).
//
// Output-stationary design: one wavefront owns a tile of 4 x 8 grid cells for
// 128 frequencies; lane l carries frequencies fbase + l and fbase + 64 + l and
// keeps 2 x 32 complex accumulators in registers.  It walks every sample
// whose W x W support touches the tile (rows of first-tap cells, each a
// contiguous run in the cell-sorted list), compensates the sample's echo with
// the float64 phase argument k * beta reduced modulo one cycle, and adds the
// clipped separable taps.  Which taps land inside the tile depends on the
// sample's cell offset (A, B) relative to the tile; a uniform binary dispatch
// selects a fully unrolled body for that offset, so every accumulator index is
// static.  Tiles partition the grid, so each cell is written exactly once with
// coalesced streaming stores (marked for early eviction, so they do not push
// echo rows out of L2): no atomics, no zeroing pass, a fixed summation order.
//
// Echo rows are streamed through LDS in chunks of 8 samples with the direct
// global-to-LDS loads of gfx950: at the start of chunk c the wave waits once,
// moves the chunk's echo values into a register vector (indexed with the
// uniform sample index), and issues the loads of chunk c+1, whose source rows
// were fetched a chunk earlier.  Residual paths and cell offsets of a chunk
// are gathered lane-parallel a chunk ahead, so all of its compensation phases
// are computed together at the chunk start; kernel weights arrive through
// scalar loads one sample ahead.  Carrying two
// frequencies per lane spreads each sample visit's scalar work (dispatch,
// weights) over twice the arithmetic.
#pragma once

#include <hip/hip_fp16.h>

#include <cstddef>

#include "device_common.hpp"
#include "launch.hpp"
#include "sar_internal.hpp"

// Repeats M(I) for I = 0 .. 255 (covers NBY * NBX up to (4 + 7) * (8 + 7) = 165
// for 8 x 4 tiles and (8 + 5) * (8 + 5) = 169 for 8 x 8 tiles up to 6 taps).
#define SAR_GRID_R4(M, B) M((B)) M((B) + 1) M((B) + 2) M((B) + 3)
#define SAR_GRID_R16(M, B) SAR_GRID_R4(M, B) SAR_GRID_R4(M, (B) + 4) SAR_GRID_R4(M, (B) + 8) SAR_GRID_R4(M, (B) + 12)
#define SAR_GRID_R64(M, B) \
  SAR_GRID_R16(M, B) SAR_GRID_R16(M, (B) + 16) SAR_GRID_R16(M, (B) + 32) SAR_GRID_R16(M, (B) + 48)
#define SAR_GRID_CASES(M) SAR_GRID_R64(M, 0) SAR_GRID_R64(M, 64) SAR_GRID_R64(M, 128) SAR_GRID_R64(M, 192)

namespace sar {
namespace grid_impl {

// Tile configurations: TX x TY cells per wave, FPL frequencies per lane (64 *
// FPL per wave), CH samples per pipeline chunk (two chunk buffers per wave),
// and the waves per SIMD the register allocator is asked for:
//   0: 4 x 4 cells, 2 frequencies: 64 accumulator registers, chunks of 4, four
//      waves per SIMD up to 4 taps (the occupancy outweighs the extra halo);
//   1: 8 x 8 cells, 1 frequency: less halo, no idle lanes for sweeps of at most
//      64 frequencies (128 accumulators, three waves);
//   2: 8 x 4 cells, 2 frequencies: less halo than tile 0 for 5- and 6-tap kernels.
// Widths beyond those of kGridTileWidths would spill registers and are not
// compiled for tiles 1 and 2.
template <int TC>
struct TileCfg;
template <>
struct TileCfg<0> {
  static constexpr int TX = 4, TY = 4, FPL = 2, CH = 4;
  static constexpr int waves(int W) { return W <= 4 ? 4 : (W <= 6 ? 3 : 2); }
};
template <>
struct TileCfg<1> {
  static constexpr int TX = 8, TY = 8, FPL = 1, CH = 6;
  static constexpr int waves(int W) { return W <= 4 ? 3 : 2; }
};
template <>
struct TileCfg<2> {
  static constexpr int TX = 8, TY = 4, FPL = 2, CH = 6;
  static constexpr int waves(int W) { return W <= 4 ? 3 : 2; }
};
template <int TC>
constexpr bool tile_matches_host() {
  return TileCfg<TC>::TX == kGridTiles[TC][0] && TileCfg<TC>::TY == kGridTiles[TC][1] &&
         TileCfg<TC>::FPL == kGridTiles[TC][2];
}
static_assert(tile_matches_host<0>() && tile_matches_host<1>() && tile_matches_host<2>(),
              "host table of tile configurations");

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
  // over-full unions (four-wave kernel only): per union the first overflow
  // slot (-1: not split), the slot list (union, part), partial grids per slot
  const int32_t* uofs;
  const int2* slots;
  float2* partial;    // [slot][64 cells][nf]
  const int32_t* nslots_used;
  int max_slots;
  int part_len;       // samples of a union's stream per part
  int nmain;          // blocks of the union grid (the rest take overflow slots)
};

// value of lane k of a float64 register pair
__device__ __forceinline__ double readlane_f64(double v, int k) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffLL), k);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), k);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// asynchronous copies from global memory into LDS (the direct global-to-LDS
// loads of gfx950): one dword, or 16 bytes, per lane to lds_base + size * lane
__device__ __forceinline__ void dma_dword(const void* src, void* lds_base) {
  __builtin_amdgcn_global_load_lds(src, (void __attribute__((address_space(3)))*)lds_base, 4, 0, 0);
}
__device__ __forceinline__ void dma_quad(const void* src, void* lds_base) {
  __builtin_amdgcn_global_load_lds(src, (void __attribute__((address_space(3)))*)lds_base, 16, 0, 0);
}

// echo-type template value of the precision diagnostic: complex64 echo with the
// compensation argument k * beta formed and reduced in float32
constexpr int kEchoC64Fp32Args = 2;

template <int W, int ET, int TC>
struct GridBody {
  using Args = GridArgs;
  static constexpr int kThreads = 64;
  // waves per SIMD asked of the register allocator (see TileCfg)
  static constexpr int kMinWavesPerEU = TileCfg<TC>::waves(W);
  static __device__ __forceinline__ void run(const GridArgs& a, uint32_t blk, uint32_t nblk);
};

template <int W, int ET, int TC>
__device__ __forceinline__ void GridBody<W, ET, TC>::run(const GridArgs& a, uint32_t blk, uint32_t nblk) {
  constexpr int TX = TileCfg<TC>::TX;
  constexpr int TY = TileCfg<TC>::TY;
  constexpr int FPL = TileCfg<TC>::FPL;
  constexpr int NBX = TX + W - 1;     // last-tap column offsets touching a tile
  constexpr int NBY = TY + W - 1;     // last-tap row offsets touching a tile
  constexpr int NSEG = 2 * NBY;       // each row of cells may split at the x wrap
  constexpr int CH = TileCfg<TC>::CH;  // samples per pipeline chunk
  constexpr int EBH = 512;            // bytes per sample and 64 frequencies of compensated values
  constexpr int EB = FPL * EBH;       // bytes per sample of one chunk buffer
  constexpr int NW = 2 * W;           // weight words per sample (wx then wy)
  constexpr int WS = (NW + 3) / 4 * 4;      // padded to 16-byte blocks for 128-bit reads
  constexpr int NWQ = (CH * WS + 63) / 64;  // weight loads per chunk (64 words each)
  constexpr int BUF = CH * EB + NWQ * 256;  // one chunk buffer: values, then weights
  static_assert(NBY * NBX <= 256, "pattern chain covers 256 patterns");
  __shared__ int seg_s[NSEG];
  __shared__ int seg_off[NSEG + 1];
  __shared__ __attribute__((aligned(16))) char cbuf[2][BUF];

  // row-major tile order (x fastest, frequency chunk slowest); measured
  // faster than narrower strip orders for the serpentine scans
  const uint32_t work = xcd_remap(blk, nblk);
  const int tx = (int)(work % (uint32_t)a.ntx);
  const uint32_t rest = work / (uint32_t)a.ntx;
  const int ty = (int)(rest % (uint32_t)a.nty);
  const int fchunk = (int)(rest / (uint32_t)a.nty);
  const int tx0 = tx * TX, ty0 = ty * TY;
  const int lane = threadIdx.x;
  const int fbase = fchunk * 64 * FPL;
  int fq[FPL];
  double fcc[FPL];
#pragma unroll
  for (int h = 0; h < FPL; ++h) {
    fq[h] = fbase + 64 * h + lane;
    fcc[h] = a.fcc[fq[h] < a.nf ? fq[h] : a.nf - 1];
  }
  // runs of first-tap cells: row j (y offset j - (W-1)), x in [tx0 - (W-1), tx0 + TX)
  if (lane < NBY) {
    int cy = ty0 + lane - (W - 1);
    cy = cy < 0 ? cy + a.my : cy;
    const int64_t row = (int64_t)cy * a.mx;
    const int xlo = tx0 - (W - 1);
    const int xhi = tx0 + TX;
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

  // sorted-list index of the chunk's lane-th sample (lanes >= chunk size: -1);
  // chunks are asked for in increasing order, so each lane keeps the segment
  // it reached last time and only moves forward
  int kseg = 0;
  auto chunk_index = [&](int c) __attribute__((always_inline)) -> int {
    const int t = c * CH + lane;
    if (lane >= CH || t >= total) return -1;
    while (seg_off[kseg + 1] <= t) ++kseg;
    return seg_s[kseg] + (t - seg_off[kseg]);
  };
  // per-sample fields gathered lane-parallel (lane k: the chunk's k-th sample)
  const SampleRec<W>* __restrict__ grec = (const SampleRec<W>*)a.rec;
  auto gather_beta = [&](int sidx) __attribute__((always_inline)) -> double {
    return sidx >= 0 ? grec[sidx].beta : 0.0;
  };
  // the last-tap cell (cx low half, cy high half) is gathered a chunk ahead
  // and turned into the tap pattern only when the chunk is processed: using
  // the loaded value at once would wait for every earlier vector load,
  // including the direct loads of the next chunk, and serialise the pipeline
  auto gather_cxy = [&](int sidx) __attribute__((always_inline)) -> uint32_t {
    return sidx >= 0 ? *(const uint32_t*)&grec[sidx].cx : 0u;
  };
  auto pattern_of = [&](uint32_t cxy) __attribute__((always_inline)) -> int {
    int aa = (int)(cxy >> 16) - ty0;       // last-tap row offset in [0, NBY) after the wrap
    int bb = (int)(cxy & 0xffffu) - tx0;   // last-tap column offset in [0, NBX)
    aa += aa < 0 ? a.my : 0;
    bb += bb < 0 ? a.mx : 0;
    return aa * NBX + bb;
  };
  // Chunk c into buffer b with direct global-to-LDS loads: the echo rows of
  // its samples (frequency-major, compensated in place later) and their
  // kernel weights (lane L loads word L % WS of the chunk's sample L / WS;
  // words NW..WS-1 are padding).
  // 16-byte echo loads need every complex pair (2 frequencies) inside the row.
  constexpr int RF = (int)(sizeof(SampleRec<W>) / 4);           // record size in words
  constexpr int WOFF = (int)(offsetof(SampleRec<W>, wx) / 4);   // first weight word
  const bool quad_ok = (a.nf & 1) == 0;
  auto stage = [&](int c, int b, int srcv, int sidxv) __attribute__((always_inline)) {
    const int n = min(CH, total - c * CH);
    char* buf = cbuf[b];
    for (int k = 0; k < n; ++k) {
      const int src = __builtin_amdgcn_readlane(srcv, k);
      if constexpr (ET != SAR_ECHO_F16X2) {
        const float* row = (const float*)a.echo + (int64_t)src * a.nf * 2;
        if (FPL == 2 && quad_ok) {
          // one 16-byte load per lane covers the 128 frequencies (2 per lane)
          const int fi = fbase * 2 + 4 * lane;
          dma_quad(row + (fi < 2 * a.nf ? fi : 0), buf + k * EB);
        } else {
#pragma unroll
          for (int q = 0; q < 2 * FPL; ++q) {
            const int fi = fbase * 2 + q * 64 + lane;   // float index within the row
            dma_dword(row + (fi < 2 * a.nf ? fi : 0), buf + k * EB + q * 256);
          }
        }
      } else {
        // half pairs land in the first half of the sample's slot
        const uint32_t* row = (const uint32_t*)a.echo + (int64_t)src * a.nf;
#pragma unroll
        for (int q = 0; q < FPL; ++q) {
          const int fi = fbase + q * 64 + lane;
          dma_dword(row + (fi < a.nf ? fi : 0), buf + k * EB + q * 256);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NWQ; ++q) {
      const int L = q * 64 + lane;
      const int k = L / WS;
      const int wd = L - k * WS;
      const int si = __shfl(sidxv, k < n ? k : 0);   // a sample of this chunk
      const float* src = (const float*)a.rec + (int64_t)si * RF + WOFF + (wd < NW ? wd : 0);
      dma_dword(src, buf + CH * EB + q * 256);
    }
  };

  float2 acc[TY][TX][FPL];
#pragma unroll
  for (int r = 0; r < TY; ++r)
#pragma unroll
    for (int c = 0; c < TX; ++c)
#pragma unroll
      for (int h = 0; h < FPL; ++h) acc[r][c][h] = make_float2(0.f, 0.f);

  // pipeline: while chunk c is processed from buffer c & 1, the echo rows and
  // weights of chunk c+1 fill the other buffer, and the residual paths,
  // patterns and source rows of the chunks after are gathered
  int sidx0 = chunk_index(0);
  int sidx1 = chunk_index(1);
  double beta0 = gather_beta(sidx0);
  uint32_t cxy0 = gather_cxy(sidx0);
  int src1 = sidx1 >= 0 ? a.order[sidx1] : 0;
  if (nchunk > 0) stage(0, 0, sidx0 >= 0 ? a.order[sidx0] : 0, sidx0);
  for (int c = 0; c < nchunk; ++c) {
    char* buf = cbuf[c & 1];
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int n = __builtin_amdgcn_readfirstlane(min(CH, total - c * CH));
    const int idx0 = pattern_of(cxy0);
    // compensation in place, two samples at a time (chunks hold an even
    // number of slots; a spare slot is processed but never read):
    // s_hat = s exp(+j 2 pi f beta / c), k * beta in float64 reduced modulo a
    // cycle, then hardware sine and cosine (which overlap the other vector
    // work, so every frequency takes its own phase)
    static_assert(CH % 2 == 0, "compensation pairs");
    for (int k = 0; k < n; k += 2) {
      float2 t2[2][FPL];
      double bk[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        bk[u] = readlane_f64(beta0, k + u);
#pragma unroll
        for (int h = 0; h < FPL; ++h) {
          if constexpr (ET != SAR_ECHO_F16X2) {
            t2[u][h] = *(const float2*)(buf + (k + u) * EB + h * EBH + lane * 8);
          } else {
            const float2 w2 = __half22float2(*(const __half2*)(buf + (k + u) * EB + h * 256 + lane * 4));
            t2[u][h] = make_float2(w2.x * a.echo_scale, w2.y * a.echo_scale);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int h = 0; h < FPL; ++h)
          if constexpr (ET == kEchoC64Fp32Args)
            *(float2*)(buf + (k + u) * EB + h * EBH + lane * 8) =
                cmul(t2[u][h], cis_cycles_f32((float)bk[u] * (float)fcc[h]));
          else
            *(float2*)(buf + (k + u) * EB + h * EBH + lane * 8) = cmul(t2[u][h], cis_cycles(bk[u] * fcc[h]));
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (c + 1 < nchunk) stage(c + 1, (c + 1) & 1, src1, sidx1);
    const int sidx2 = chunk_index(c + 2);
    const int src2 = sidx2 >= 0 ? a.order[sidx2] : 0;
    const double beta1 = gather_beta(sidx1);
    const uint32_t cxy1 = gather_cxy(sidx1);
    // one sample with its tap pattern fixed at compile time: I = row offset *
    // NBX + column offset of its last tap relative to the tile
    int k = 0;
    // LDS addresses (32-bit) of this lane's values and of the weights
    typedef __attribute__((address_space(3))) char lds_char;
    const uint32_t vbase = (uint32_t)(uintptr_t)(lds_char*)buf + 8u * (uint32_t)lane;
    const uint32_t wbase = (uint32_t)(uintptr_t)(lds_char*)(buf + CH * EB);
    auto visit = [&](auto ic) __attribute__((always_inline)) {
      constexpr int I = decltype(ic)::value;
      constexpr int AA = I / NBX - (W - 1);   // first-tap row offset
      constexpr int BB = I % NBX - (W - 1);   // first-tap column offset
      // The sample's two compensated values and its weights, read and
      // waited for in one block: the next chunk's direct loads into the other
      // buffer stay in flight (a compiler-visible LDS read would wait for them).
      typedef float f2v __attribute__((ext_vector_type(2)));
      typedef float f4v __attribute__((ext_vector_type(4)));
      f2v r0, r1 = {0.f, 0.f};
      f4v q0, q1, q2 = {0.f, 0.f, 0.f, 0.f}, q3 = {0.f, 0.f, 0.f, 0.f};
      const uint32_t va = vbase + (uint32_t)(k * EB);
      const uint32_t wa = wbase + (uint32_t)(k * WS * 4);
      static_assert(EBH == 512, "value offsets in the read block");
      if constexpr (FPL == 2 && WS == 8) {
        asm volatile(
            "ds_read_b64 %0, %4\n\tds_read_b64 %1, %4 offset:512\n\t"
            "ds_read_b128 %2, %5\n\tds_read_b128 %3, %5 offset:16\n\ts_waitcnt lgkmcnt(0)"
            : "=&v"(r0), "=&v"(r1), "=&v"(q0), "=&v"(q1)
            : "v"(va), "v"(wa)
            : "memory");
      } else if constexpr (FPL == 2 && WS == 12) {
        asm volatile(
            "ds_read_b64 %0, %5\n\tds_read_b64 %1, %5 offset:512\n\t"
            "ds_read_b128 %2, %6\n\tds_read_b128 %3, %6 offset:16\n\tds_read_b128 %4, %6 offset:32\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(r0), "=&v"(r1), "=&v"(q0), "=&v"(q1), "=&v"(q2)
            : "v"(va), "v"(wa)
            : "memory");
      } else if constexpr (FPL == 2) {
        static_assert(WS == 16, "weight block of 8, 12 or 16 words");
        asm volatile(
            "ds_read_b64 %0, %6\n\tds_read_b64 %1, %6 offset:512\n\t"
            "ds_read_b128 %2, %7\n\tds_read_b128 %3, %7 offset:16\n\t"
            "ds_read_b128 %4, %7 offset:32\n\tds_read_b128 %5, %7 offset:48\n\ts_waitcnt lgkmcnt(0)"
            : "=&v"(r0), "=&v"(r1), "=&v"(q0), "=&v"(q1), "=&v"(q2), "=&v"(q3)
            : "v"(va), "v"(wa)
            : "memory");
      } else if constexpr (WS == 8) {
        static_assert(FPL == 1, "one or two frequencies per lane");
        asm volatile(
            "ds_read_b64 %0, %3\n\tds_read_b128 %1, %4\n\tds_read_b128 %2, %4 offset:16\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(r0), "=&v"(q0), "=&v"(q1)
            : "v"(va), "v"(wa)
            : "memory");
      } else {
        static_assert(FPL == 1 && WS == 12, "one-frequency tiles are built for kernels of 3 to 6 taps");
        asm volatile(
            "ds_read_b64 %0, %4\n\tds_read_b128 %1, %5\n\tds_read_b128 %2, %5 offset:16\n\t"
            "ds_read_b128 %3, %5 offset:32\n\ts_waitcnt lgkmcnt(0)"
            : "=&v"(r0), "=&v"(q0), "=&v"(q1), "=&v"(q2)
            : "v"(va), "v"(wa)
            : "memory");
      }
      float wv[16] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w,
                      q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w};
      float wx[W], wy[W];
#pragma unroll
      for (int q = 0; q < W; ++q) {
        wx[q] = wv[q];
        wy[q] = wv[W + q];
      }
      float2 v[FPL];
      v[0] = make_float2(r0.x, r0.y);
      if constexpr (FPL == 2) v[1] = make_float2(r1.x, r1.y);
      static_for<0, W>([&](auto jc) __attribute__((always_inline)) {
        constexpr int jj = decltype(jc)::value;
        constexpr int rr = AA + jj;
        if constexpr (rr >= 0 && rr < TY) {
          float2 vy[FPL];
#pragma unroll
          for (int h = 0; h < FPL; ++h) vy[h] = cscale(v[h], wy[jj]);
          static_for<0, W>([&](auto kc) __attribute__((always_inline)) {
            constexpr int kk = decltype(kc)::value;
            constexpr int cc = BB + kk;
            if constexpr (cc >= 0 && cc < TX) {
#pragma unroll
              for (int h = 0; h < FPL; ++h) cfma(acc[rr][cc][h], vy[h], wx[kk]);
            }
          });
        }
      });
    };
    // The sorted list walks the tile's cells in increasing pattern index, so
    // the chunk enters the chain of patterns once, at its first sample's
    // pattern, and falls through the later ones in order: per sample only one
    // compare and the loop branch remain.  A sample whose pattern lies behind
    // the chain's position re-enters it, and an index outside the chain (not
    // produced by the record kernel) is skipped, so every sample is visited
    // at most once and the loop always ends.
    int cur = __builtin_amdgcn_readlane(idx0, 0);
    for (;;) {
      switch (cur) {
#define SAR_GRID_CASE(I)                                                   \
  case (I):                                                                \
    if constexpr ((I) < NBY * NBX) {                                       \
      while (cur == (I)) {                                                 \
        visit(std::integral_constant<int, (I)>{});                         \
        if (++k >= n) goto chunk_done;                                     \
        cur = __builtin_amdgcn_readlane(idx0, k);                          \
      }                                                                    \
    }                                                                      \
    [[fallthrough]];
        SAR_GRID_CASES(SAR_GRID_CASE)
#undef SAR_GRID_CASE
        default:
          break;
      }
      if (cur < 0 || cur >= NBY * NBX) {
        if (++k >= n) break;
        cur = __builtin_amdgcn_readlane(idx0, k);
      }
    }
  chunk_done:
    sidx0 = sidx1;
    sidx1 = sidx2;
    src1 = src2;
    beta0 = beta1;
    cxy0 = cxy1;
  }

#pragma unroll
  for (int h = 0; h < FPL; ++h) {
    if (fq[h] < a.nf) {
#pragma unroll
      for (int r = 0; r < TY; ++r)
#pragma unroll
        for (int c = 0; c < TX; ++c)
          store_stream(&a.grid[((int64_t)(ty0 + r) * a.mx + (tx0 + c)) * a.nf + fq[h]], acc[r][c][h]);
    }
  }
}

template <int W, int TC>
sar_status grid_w(const Plan& p, const void* d_echo, float echo_scale, const Workspace& ws, float2* grid,
                  LaunchSink& sink) {
  constexpr int TX = TileCfg<TC>::TX;
  constexpr int TY = TileCfg<TC>::TY;
  constexpr int FPL = TileCfg<TC>::FPL;
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
  a.ntx = p.mx / TX;
  a.nty = p.my / TY;
  const int nfc = (p.nf + 64 * FPL - 1) / (64 * FPL);
  const int64_t nblk = (int64_t)a.ntx * a.nty * nfc;
  if (p.flags & SAR_FP32_ARGS) {  // precision diagnostic, compiled for W = 4 only
    if constexpr (W == 4)
      return launch_body<GridBody<W, kEchoC64Fp32Args, TC>>(sink, (uint32_t)nblk, 0, a, "gridding launch");
    return fail(SAR_ERR_UNSUPPORTED, "SAR_FP32_ARGS is compiled for a 4-tap lateral kernel");
  }
  if (p.echo_type == SAR_ECHO_C64)
    return launch_body<GridBody<W, SAR_ECHO_C64, TC>>(sink, (uint32_t)nblk, 0, a, "gridding launch");
  return launch_body<GridBody<W, SAR_ECHO_F16X2, TC>>(sink, (uint32_t)nblk, 0, a, "gridding launch");
}

}  // namespace grid_impl
}  // namespace sar

#include "k_grid_union.hpp"

namespace sar {
// Each tile configuration is compiled for the kernel widths of
// kGridTileWidths; the plan only selects a compiled one.
#define SAR_INSTANTIATE_GRID(W)                                                                    \
  sar_status launch_gridding_w##W(const Plan& p, const void* d_echo, float echo_scale,              \
                                  const Workspace& ws, float2* grid, LaunchSink& sink) {            \
    if constexpr ((W) >= kGridTileWidths[1][0] && (W) <= kGridTileWidths[1][1]) {                  \
      if (p.grid_tile == 1) return grid_impl::grid_w<W, 1>(p, d_echo, echo_scale, ws, grid, sink);  \
    }                                                                                              \
    if constexpr ((W) >= kGridTileWidths[2][0] && (W) <= kGridTileWidths[2][1]) {                  \
      if (p.grid_tile == 2) return grid_impl::grid_w<W, 2>(p, d_echo, echo_scale, ws, grid, sink);  \
    }                                                                                              \
    if constexpr ((W) >= kGridTileWidths[3][0] && (W) <= kGridTileWidths[3][1]) {                  \
      if (p.grid_tile == 3) return grid_impl::grid_union_w<W>(p, d_echo, echo_scale, ws, grid, sink); \
    }                                                                                              \
    return grid_impl::grid_w<W, 0>(p, d_echo, echo_scale, ws, grid, sink);                        \
  }

}  // namespace sar

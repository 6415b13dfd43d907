// Steps a1 + a2, multi-wave form (included by k_grid_impl.hpp): compensation
// (Eq. (11)) and Kaiser-Bessel gridding with each compensated echo value
// shared by the four waves of a workgroup.
//
// A workgroup owns a union of 8 x 8 grid cells for 128 frequencies (two
// adjacent ones per lane, so a lane reads a sample's values with one 16-byte
// LDS load and writes each cell with one 16-byte store).  Wave w owns the union's rows w and w + 4, all 8 columns: 2 x 8 x 2
// complex accumulators per lane.  Every sample whose W x W support touches
// the union covers W consecutive rows, so for W <= 4 it lands in at most one
// row of each wave (for W = 5 in both rows of a wave when its first tap row is
// the wave's first row) and every wave visits nearly every sample once: the
// waves stay in step.  The union's samples (rows of first-tap cells, contiguous runs of
// the cell-sorted list) stream through LDS in chunks of 16: the four waves
// stage a chunk's echo rows and kernel weights with gfx950's direct
// global-to-LDS loads, then each compensates a quarter of the chunk in place
// (float64 argument k * beta reduced modulo one cycle, hardware sine and
// cosine) and the workgroup forms each sample's W x W weight products once;
// after a barrier every wave walks the chunk, adding one product row times
// the values into its accumulators through a fully unrolled body per tap
// pattern.  Compared with one wave per 4 x 4 tile, a sample is compensated
// 1.9 instead of 3.1 times on average, and a visit does no per-row scaling.
// Rows of cells partition the grid: each value is written once with streaming
// stores, no atomics, a fixed summation order.
//
// Irregular density: a union whose sample stream is longer than a part
// (a dwelling hand piles thousands of samples into a few cells) is split.  A
// planning kernel takes ceil(length / part) - 1 overflow slots for it; the
// union's own workgroup walks the first part and writes the grid, extra
// workgroups (one per slot and frequency chunk) walk the later parts into
// partial grids, and a combining kernel adds the partials in part order.  The
// sum is therefore the same on every run, whichever slots a union gets.
#pragma once

namespace sar {
namespace grid_impl {

constexpr int kUnionWaves = 4;
constexpr int kUnionX = 8;     // cells along x per union
constexpr int kUnionY = 8;     // rows per union (two per wave, four apart)
constexpr int kUnionCh = 16;   // samples per chunk

// whether pattern I (see pattern_of) puts a tap row on one of the wave's rows
template <int W, int NBX, int NWV, int RPW>
constexpr bool union_has_tap(int I) {
  const int fr = I / NBX - (NWV - 1) - (W - 1);
  const int r0 = fr <= 0 ? 0 : (fr + NWV - 1) / NWV;
  return r0 < RPW && NWV * r0 - fr < W;
}

template <int W, int ET>
struct GridUnionBody {
  using Args = GridArgs;
  static constexpr int kThreads = 64 * kUnionWaves;
  static constexpr int kMinWavesPerEU = 4;
  static __device__ __forceinline__ void run(const GridArgs& a, uint32_t blk, uint32_t nblk);
};

template <int W, int ET>
__device__ __forceinline__ void GridUnionBody<W, ET>::run(const GridArgs& a, uint32_t blk, uint32_t nblk) {
  static_assert(W >= 2 && W <= 5, "tap rows of a sample meet at most two rows of a wave");
  constexpr int NWV = kUnionWaves;
  constexpr int UX = kUnionX;
  constexpr int UY = kUnionY;
  constexpr int RPW = UY / NWV;       // rows per wave
  constexpr int FPL = 2;              // frequencies per lane
  constexpr int CH = kUnionCh;
  constexpr int NBX = UX + W - 1;     // last-tap column offsets touching the union
  constexpr int NBY = UY + W - 1;     // last-tap row offsets touching the union
  constexpr int NA = NBY + NWV - 1;   // row offsets relative to a wave's first row
  constexpr int NSEG = 2 * NBY;       // each row of cells may split at the x wrap
  constexpr int EB = FPL * 512;       // bytes of one sample's compensated values
  constexpr int NW = 2 * W;           // weight words per sample (wx then wy)
  constexpr int WS = (NW + 3) / 4 * 4;
  constexpr int PR = W <= 4 ? 4 : 8;            // floats per product row (16 or 32 bytes)
  constexpr int PSZ = W <= 4 ? 16 : W * PR;     // floats of products per sample
  constexpr int VOFF = 0;
  constexpr int WOFF = CH * EB;                 // raw weights (direct loads)
  constexpr int POFF = WOFF + CH * WS * 4;      // products [CH][rows][PR]
  constexpr int BUF = POFF + CH * PSZ * 4;
  static_assert(NA * NBX <= 256, "pattern chain covers 256 patterns");
  static_assert(CH * WS <= 64 * NWV, "weights of a chunk in one direct load per wave");
  static_assert(CH * 16 == 64 * NWV, "one product row entry per thread and chunk (4-tap layout)");
  __shared__ int seg_s[NSEG];
  __shared__ int seg_off[NSEG + 1];
  __shared__ __attribute__((aligned(16))) char cbuf[2][BUF];

  const int nux = a.ntx;  // unions along x (mx / 8)
  const int nuy = a.nty;
  int ux, uy, fchunk, slot = -1, part = 0;
  if ((int)blk < a.nmain) {
    const uint32_t work = xcd_remap(blk, (uint32_t)a.nmain);
    ux = (int)(work % (uint32_t)nux);
    const uint32_t rest = work / (uint32_t)nux;
    uy = (int)(rest % (uint32_t)nuy);
    fchunk = (int)(rest / (uint32_t)nuy);
  } else {
    // an overflow slot: a later part of a split union
    const int nfc = a.nmain / (nux * nuy);
    const int o = (int)blk - a.nmain;
    slot = o / nfc;
    fchunk = o - slot * nfc;
    const int used = min(*a.nslots_used, a.max_slots);
    if (slot >= used) return;
    const int2 e = a.slots[slot];
    if (e.x < 0) return;
    ux = e.x % nux;
    uy = e.x / nux;
    part = e.y & 0xffff;
  }
  const int ux0 = ux * UX, uy0 = uy * UY;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int fbase = fchunk * 64 * FPL;
  int fq[FPL];
  double fcc[FPL];
#pragma unroll
  for (int h = 0; h < FPL; ++h) {
    fq[h] = fbase + FPL * lane + h;
    fcc[h] = a.fcc[fq[h] < a.nf ? fq[h] : a.nf - 1];
  }
  // runs of first-tap cells: row j (y offset j - (W-1)), x in [ux0 - (W-1), ux0 + UX)
  if (threadIdx.x < NBY) {
    const int j = threadIdx.x;
    int cy = uy0 + j - (W - 1);
    cy = cy < 0 ? cy + a.my : cy;
    const int64_t row = (int64_t)cy * a.mx;
    const int xlo = ux0 - (W - 1);
    const int xhi = ux0 + UX;
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
    seg_s[2 * j] = s0;
    seg_s[2 * j + 1] = s1;
    seg_off[2 * j] = e0 - s0;
    seg_off[2 * j + 1] = e1 - s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int k = 0; k < NSEG; ++k) {
      const int l = seg_off[k];
      seg_off[k] = run;
      run += l;
    }
    seg_off[NSEG] = run;
  }
  __syncthreads();
  const int total_all = __builtin_amdgcn_readfirstlane(seg_off[NSEG]);
  // stream positions [t0, t1) of this block: the whole union, its first part
  // (split union), or a later part (overflow slot)
  int t0 = 0, t1 = total_all;
  if (slot >= 0) {
    t0 = part * a.part_len;
    t1 = min(total_all, t0 + a.part_len);
  } else if (a.max_slots > 0 && a.uofs[uy * nux + ux] >= 0) {
    t1 = min(total_all, a.part_len);
  }
  const int total = t1 - t0;
  const int nchunk = (total + CH - 1) / CH;

  // sorted-list index of the chunk's lane-th sample (lanes >= CH or past the
  // end: -1); chunks are asked for in increasing order, so each lane keeps
  // the segment it reached last time
  int kseg = 0;
  auto chunk_index = [&](int c) __attribute__((always_inline)) -> int {
    const int t = t0 + c * CH + lane;
    if (lane >= CH || t >= t1) return -1;
    while (seg_off[kseg + 1] <= t) ++kseg;
    return seg_s[kseg] + (t - seg_off[kseg]);
  };
  const SampleRec<W>* __restrict__ grec = (const SampleRec<W>*)a.rec;
  auto gather_beta = [&](int sidx) __attribute__((always_inline)) -> double {
    return sidx >= 0 ? grec[sidx].beta : 0.0;
  };
  // last-tap cell gathered a chunk ahead, turned into the pattern only when
  // the chunk is processed (a use at once would wait for all earlier loads)
  auto gather_cxy = [&](int sidx) __attribute__((always_inline)) -> uint32_t {
    return sidx >= 0 ? *(const uint32_t*)&grec[sidx].cx : 0u;
  };
  // pattern of a sample for this wave: (last-tap row relative to the wave's
  // first row, shifted to >= 0) x NBX + last-tap column relative to the
  // union, or -1 when none of the wave's rows is among the sample's tap rows
  // (such samples are skipped, not walked through empty bodies)
  auto pattern_of = [&](uint32_t cxy) __attribute__((always_inline)) -> int {
    int aa = (int)(cxy >> 16) - uy0;
    int bb = (int)(cxy & 0xffffu) - ux0;
    aa += aa < 0 ? a.my : 0;
    bb += bb < 0 ? a.mx : 0;
    const int fr = aa - wv - (W - 1);                        // first tap row from the wave's first row
    const int r0 = fr <= 0 ? 0 : (fr + NWV - 1) / NWV;       // the wave's first row at or after it
    const bool tap = r0 < RPW && NWV * r0 - fr < W;
    return tap ? (aa - wv + NWV - 1) * NBX + bb : -1;
  };
  constexpr int RF = (int)(sizeof(SampleRec<W>) / 4);
  constexpr int WREC = (int)(offsetof(SampleRec<W>, wx) / 4);
  const bool quad_ok = (a.nf & 1) == 0;
  // chunk c into buffer b: wave wv stages the echo rows of samples
  // k = wv, wv + 4, ... and waves 0 and 1 the kernel weights
  auto stage = [&](int c, int b, int srcv, int sidxv) __attribute__((always_inline)) {
    const int n = min(CH, total - c * CH);
    char* buf = cbuf[b];
    for (int k = wv; k < n; k += NWV) {
      const int src = __builtin_amdgcn_readlane(srcv, k);
      if constexpr (ET != SAR_ECHO_F16X2) {
        const float* row = (const float*)a.echo + (int64_t)src * a.nf * 2;
        if (quad_ok) {
          const int fi = fbase * 2 + 4 * lane;
          dma_quad(row + (fi < 2 * a.nf ? fi : 0), buf + VOFF + k * EB);
        } else {
#pragma unroll
          for (int q = 0; q < 2 * FPL; ++q) {
            const int fi = fbase * 2 + q * 64 + lane;
            dma_dword(row + (fi < 2 * a.nf ? fi : 0), buf + VOFF + k * EB + q * 256);
          }
        }
      } else {
        const uint32_t* row = (const uint32_t*)a.echo + (int64_t)src * a.nf;
#pragma unroll
        for (int q = 0; q < FPL; ++q) {
          const int fi = fbase + q * 64 + lane;
          dma_dword(row + (fi < a.nf ? fi : 0), buf + VOFF + k * EB + q * 256);
        }
      }
    }
    if (wv < (CH * WS + 63) / 64) {
      const int L = wv * 64 + lane;
      const int k = L / WS;
      const int wd = L - k * WS;
      const int si = __shfl(sidxv, k < n ? k : 0);
      const float* src = (const float*)a.rec + (int64_t)si * RF + WREC + (wd < NW ? wd : 0);
      dma_dword(src, buf + WOFF + wv * 256);
    }
  };

  float2 acc[RPW][UX][FPL];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int c = 0; c < UX; ++c)
#pragma unroll
      for (int h = 0; h < FPL; ++h) acc[r][c][h] = make_float2(0.f, 0.f);

  int sidx0 = chunk_index(0);
  int sidx1 = chunk_index(1);
  double beta0 = gather_beta(sidx0);
  uint32_t cxy0 = gather_cxy(sidx0);
  int src1 = sidx1 >= 0 ? a.order[sidx1] : 0;
  if (nchunk > 0) stage(0, 0, sidx0 >= 0 ? a.order[sidx0] : 0, sidx0);
  for (int c = 0; c < nchunk; ++c) {
    char* buf = cbuf[c & 1];
    // the chunk's direct loads (every wave's) have landed, and every wave is
    // done with the buffer the next stage overwrites
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int n = __builtin_amdgcn_readfirstlane(min(CH, total - c * CH));
    const int idx0 = pattern_of(cxy0);
    // compensation of this wave's quarter of the chunk, in place:
    // s_hat = s exp(+j 2 pi f beta / c), float64 argument reduced mod a cycle
    for (int k = wv; k < n; k += NWV) {
      const double bk = readlane_f64(beta0, k);
      // the row sits in LDS in frequency order (complex64, or half pairs in
      // the first half of the slot); the lane's two values are adjacent
      float2 t2[FPL];
      if constexpr (ET != SAR_ECHO_F16X2) {
        const float4 t4 = *(const float4*)(buf + VOFF + k * EB + lane * 16);
        t2[0] = make_float2(t4.x, t4.y);
        t2[1] = make_float2(t4.z, t4.w);
      } else {
        const __half2* hp = (const __half2*)(buf + VOFF + k * EB + lane * 8);
#pragma unroll
        for (int h = 0; h < FPL; ++h) {
          const float2 w2 = __half22float2(hp[h]);
          t2[h] = make_float2(w2.x * a.echo_scale, w2.y * a.echo_scale);
        }
      }
      float2 u2[FPL];
#pragma unroll
      for (int h = 0; h < FPL; ++h) {
        if constexpr (ET == kEchoC64Fp32Args)
          u2[h] = cmul(t2[h], cis_cycles_f32((float)bk * (float)fcc[h]));
        else
          u2[h] = cmul(t2[h], cis_cycles(bk * fcc[h]));
      }
      *(float4*)(buf + VOFF + k * EB + lane * 16) = make_float4(u2[0].x, u2[0].y, u2[1].x, u2[1].y);
    }
    // weight products: entry e = (sample, tap row jj, tap column kk) holds
    // wx[kk] wy[jj] (one entry per thread for up to 4 taps)
#pragma unroll
    for (int e = threadIdx.x; e < CH * PSZ; e += 64 * NWV) {
      const int k = e / PSZ;
      const int r = e - k * PSZ;
      const int jj = r / PR;
      const int kk = r - jj * PR;
      float pr = 0.f;
      if (k < n && jj < W && kk < W) {
        const float* wk = (const float*)(buf + WOFF) + k * WS;
        pr = wk[kk] * wk[W + jj];
      }
      ((float*)(buf + POFF))[e] = pr;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (c + 1 < nchunk) stage(c + 1, (c + 1) & 1, src1, sidx1);
    const int sidx2 = chunk_index(c + 2);
    const int src2 = sidx2 >= 0 ? a.order[sidx2] : 0;
    const double beta1 = gather_beta(sidx1);
    const uint32_t cxy1 = gather_cxy(sidx1);
    int k = 0;
    typedef __attribute__((address_space(3))) char lds_char;
    const uint32_t vbase = (uint32_t)(uintptr_t)(lds_char*)buf + (uint32_t)(VOFF + 16 * lane);
    const uint32_t pbase = (uint32_t)(uintptr_t)(lds_char*)(buf + POFF);
    // one sample with its tap pattern fixed at compile time: I = (row offset
    // of its last tap from this wave's first row + NWV - 1) * NBX + column
    // offset of its last tap from the union
    auto visit = [&](auto ic) __attribute__((always_inline)) {
      constexpr int I = decltype(ic)::value;
      constexpr int AP = I / NBX - (NWV - 1);   // last-tap row offset from the wave's first row
      constexpr int BB = I % NBX;               // last-tap column offset
      constexpr int FR = AP - (W - 1);          // first-tap row offset
      // the wave's row r (offset 4 r) takes tap row 4 r - FR if that is in [0, W);
      // a 5-tap sample whose first tap row is the wave's first row also meets
      // the wave's second row (tap row 4)
      constexpr int R0 = (FR <= 0) ? 0 : (FR + NWV - 1) / NWV;
      constexpr int JJ = NWV * R0 - FR;
      constexpr bool TWO = R0 + 1 < RPW && JJ + NWV < W;
      if constexpr (R0 < RPW && JJ >= 0 && JJ < W) {
        typedef float f4v __attribute__((ext_vector_type(4)));
        f4v r;
        float wp[W], wq[W];
        const uint32_t va = vbase + (uint32_t)(k * EB);
        const uint32_t pa = pbase + (uint32_t)(k * PSZ * 4);
        if constexpr (W <= 4) {
          f4v q;
          asm volatile(
              "ds_read_b128 %0, %2\n\t"
              "ds_read_b128 %1, %3 offset:%4\n\ts_waitcnt lgkmcnt(0)"
              : "=&v"(r), "=&v"(q)
              : "v"(va), "v"(pa), "i"(JJ * 16)
              : "memory");
          const float q4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
          for (int i = 0; i < W; ++i) wp[i] = q4[i];
        } else if constexpr (!TWO) {
          f4v q;
          float q5;
          asm volatile(
              "ds_read_b128 %0, %3\n\t"
              "ds_read_b128 %1, %4 offset:%5\n\t"
              "ds_read_b32 %2, %4 offset:%6\n\ts_waitcnt lgkmcnt(0)"
              : "=&v"(r), "=&v"(q), "=&v"(q5)
              : "v"(va), "v"(pa), "i"(JJ * PR * 4), "i"(JJ * PR * 4 + 16)
              : "memory");
          wp[0] = q.x; wp[1] = q.y; wp[2] = q.z; wp[3] = q.w; wp[4] = q5;
        } else {
          f4v q, s4;
          float q5, s5;
          asm volatile(
              "ds_read_b128 %0, %5\n\t"
              "ds_read_b128 %1, %6 offset:%7\n\t"
              "ds_read_b32 %2, %6 offset:%8\n\t"
              "ds_read_b128 %3, %6 offset:%9\n\t"
              "ds_read_b32 %4, %6 offset:%10\n\ts_waitcnt lgkmcnt(0)"
              : "=&v"(r), "=&v"(q), "=&v"(q5), "=&v"(s4), "=&v"(s5)
              : "v"(va), "v"(pa), "i"(JJ * PR * 4), "i"(JJ * PR * 4 + 16), "i"((JJ + NWV) * PR * 4),
                "i"((JJ + NWV) * PR * 4 + 16)
              : "memory");
          wp[0] = q.x; wp[1] = q.y; wp[2] = q.z; wp[3] = q.w; wp[4] = q5;
          wq[0] = s4.x; wq[1] = s4.y; wq[2] = s4.z; wq[3] = s4.w; wq[4] = s5;
        }
        const float2 v[FPL] = {make_float2(r.x, r.y), make_float2(r.z, r.w)};
        static_for<0, W>([&](auto kc) __attribute__((always_inline)) {
          constexpr int kk = decltype(kc)::value;
          constexpr int cc = BB - (W - 1) + kk;
          if constexpr (cc >= 0 && cc < UX) {
#pragma unroll
            for (int h = 0; h < FPL; ++h) {
              cfma(acc[R0][cc][h], v[h], wp[kk]);
              if constexpr (TWO) cfma(acc[R0 + 1][cc][h], v[h], wq[kk]);
            }
          }
        });
      }
    };
    int cur = __builtin_amdgcn_readlane(idx0, 0);
    for (;;) {
      switch (cur) {
#define SAR_UNION_CASE(I)                                                  \
  case (I):                                                                \
    if constexpr ((I) < NA * NBX && union_has_tap<W, NBX, NWV, RPW>(I)) {  \
      while (cur == (I)) {                                                 \
        visit(std::integral_constant<int, (I)>{});                         \
        if (++k >= n) goto chunk_done;                                     \
        cur = __builtin_amdgcn_readlane(idx0, k);                          \
      }                                                                    \
    }                                                                      \
    [[fallthrough]];
        SAR_GRID_CASES(SAR_UNION_CASE)
#undef SAR_UNION_CASE
        default:
          break;
      }
      if (cur < 0 || cur >= NA * NBX) {
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

  // the store addresses are formed only here: an opaque lane offset keeps the
  // compiler from hoisting 32 of them, live across the whole chunk loop
  int off = lane;
  asm volatile("" : "+v"(off));
  // the grid (cell rows mx apart) or the slot's partial grid (rows UX apart)
  float2* gbase;
  int64_t rstride;
  if (slot < 0) {
    gbase = a.grid + ((int64_t)(uy0 + wv) * a.mx + ux0) * a.nf;
    rstride = (int64_t)a.mx * a.nf;
  } else {
    gbase = a.partial + ((int64_t)slot * UX * UY + wv * UX) * a.nf;
    rstride = (int64_t)UX * a.nf;
  }
  // the lane's two adjacent frequencies: one 16-byte store per cell when both
  // exist and the cells start on 16 bytes (even nf)
  const int f0 = fbase + FPL * off;
  if (f0 < a.nf) {
    float2* g = gbase + f0;
    if (quad_ok) {
#pragma unroll
      for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int c = 0; c < UX; ++c)
          store_stream2(g + NWV * r * rstride + (int64_t)c * a.nf, acc[r][c][0], acc[r][c][1]);
    } else {
      const bool second = f0 + 1 < a.nf;
#pragma unroll
      for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int c = 0; c < UX; ++c) {
          float2* q = g + NWV * r * rstride + (int64_t)c * a.nf;
          store_stream(q, acc[r][c][0]);
          if (second) store_stream(q + 1, acc[r][c][1]);
        }
    }
  }
}

// Split planning: one thread per union counts its stream (the samples whose
// first-tap cell lies in [x0 - (W-1), x0 + 8) x [y0 - (W-1), y0 + 8)) and takes
// ceil(count / part) - 1 consecutive overflow slots; a union whose slots would
// pass the end of the slot table runs unsplit (its slots are marked unused).
// A slot holds (union, part | parts << 16).
template <int W>
struct UnionPlanBody {
  struct Args {
    const int32_t* cell_start;
    int mx, my, nux, nuy;
    int part_len, max_slots;
    int32_t* counter;
    int32_t* uofs;
    int2* slots;
  };
  static constexpr int kThreads = 256;
  static __device__ __forceinline__ void run(const Args& a, uint32_t b, uint32_t) {
    const int u = (int)b * kThreads + threadIdx.x;
    if (u >= a.nux * a.nuy) return;
    const int x0 = (u % a.nux) * kUnionX, y0 = (u / a.nux) * kUnionY;
    int n = 0;
    for (int j = 0; j < kUnionY + W - 1; ++j) {
      int cy = y0 + j - (W - 1);
      cy = cy < 0 ? cy + a.my : cy;
      const int64_t row = (int64_t)cy * a.mx;
      const int xlo = x0 - (W - 1), xhi = x0 + kUnionX;
      if (xlo >= 0)
        n += a.cell_start[row + xhi] - a.cell_start[row + xlo];
      else
        n += a.cell_start[row + a.mx] - a.cell_start[row + a.mx + xlo] + a.cell_start[row + xhi] -
             a.cell_start[row];
    }
    const int extra = (n + a.part_len - 1) / a.part_len - 1;
    if (extra <= 0) {
      a.uofs[u] = -1;
      return;
    }
    const int ofs = atomicAdd(a.counter, extra);
    const bool fits = ofs + extra <= a.max_slots;
    a.uofs[u] = fits ? ofs : -1;
    for (int q = 0; q < extra && ofs + q < a.max_slots; ++q)
      a.slots[ofs + q] = fits ? make_int2(u, (q + 1) | (extra << 16)) : make_int2(-1, 0);
  }
};

// Adds the partial grids of a split union to the grid, in part order.  The
// union's 64 cells x nf values are shared out over the blocks of its overflow
// slots (one value range per slot), so the combine runs with as many blocks
// as slots; each value still sums its parts 1, 2, ... in order.
struct UnionCombineBody {
  struct Args {
    const int2* slots;
    const int32_t* counter;
    const float2* partial;
    float2* grid;
    int mx, nf, nux, max_slots;
  };
  static constexpr int kThreads = 256;
  static __device__ __forceinline__ void run(const Args& a, uint32_t b, uint32_t) {
    const int s = (int)b;
    if (s >= min(*a.counter, a.max_slots)) return;
    const int2 e = a.slots[s];
    if (e.x < 0) return;
    const int part = e.y & 0xffff;     // 1 .. parts
    const int parts = e.y >> 16;
    const int s0 = s - (part - 1);     // the union's first slot
    const int x0 = (e.x % a.nux) * kUnionX, y0 = (e.x / a.nux) * kUnionY;
    const int per = kUnionX * kUnionY * a.nf;
    const int lo = (int)((int64_t)per * (part - 1) / parts);
    const int hi = (int)((int64_t)per * part / parts);
    for (int i = lo + threadIdx.x; i < hi; i += kThreads) {
      const int cell = i / a.nf;
      const int f = i - cell * a.nf;
      float2* g = a.grid + ((int64_t)(y0 + cell / kUnionX) * a.mx + x0 + cell % kUnionX) * a.nf + f;
      float2 v = *g;
      const float2* pp = a.partial + (int64_t)s0 * per + i;
      int q = 0;
      for (; q + 4 <= parts; q += 4) {   // four loads in flight, added in order
        const float2 p0 = pp[(int64_t)q * per], p1 = pp[(int64_t)(q + 1) * per];
        const float2 p2 = pp[(int64_t)(q + 2) * per], p3 = pp[(int64_t)(q + 3) * per];
        v = cadd(cadd(cadd(cadd(v, p0), p1), p2), p3);
      }
      for (; q < parts; ++q) v = cadd(v, pp[(int64_t)q * per]);
      *g = v;
    }
  }
};

template <int W>
sar_status grid_union_launch(const Plan& p, const GridArgs& a, int64_t nblk, LaunchSink& sink) {
  if (p.flags & SAR_FP32_ARGS) {
    if constexpr (W == 4)
      return launch_body<GridUnionBody<W, kEchoC64Fp32Args>>(sink, (uint32_t)nblk, 0, a, "gridding launch");
    return fail(SAR_ERR_UNSUPPORTED, "SAR_FP32_ARGS is compiled for a 4-tap lateral kernel");
  }
  if (p.echo_type == SAR_ECHO_C64)
    return launch_body<GridUnionBody<W, SAR_ECHO_C64>>(sink, (uint32_t)nblk, 0, a, "gridding launch");
  return launch_body<GridUnionBody<W, SAR_ECHO_F16X2>>(sink, (uint32_t)nblk, 0, a, "gridding launch");
}

template <int W>
sar_status grid_union_w(const Plan& p, const void* d_echo, float echo_scale, const Workspace& ws, float2* grid,
                        LaunchSink& sink) {
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
  a.ntx = p.mx / kUnionX;
  a.nty = p.my / kUnionY;
  const int nfc = (p.nf + 127) / 128;
  const int nunion = a.ntx * a.nty;
  a.uofs = ws.uofs;
  a.slots = (const int2*)ws.slots;
  a.partial = ws.partial;
  a.nslots_used = ws.split_count;
  a.max_slots = ws.max_slots;
  a.part_len = kUnionPartLen;
  a.nmain = nunion * nfc;
  const int64_t nblk = (int64_t)a.nmain + (int64_t)a.max_slots * nfc;
  if (a.max_slots > 0) {
    typename UnionPlanBody<W>::Args pa{ws.cell_start, p.mx, p.my, a.ntx, a.nty, kUnionPartLen, a.max_slots,
                                       ws.split_count, ws.uofs, (int2*)ws.slots};
    sar_status st = launch_body<UnionPlanBody<W>>(sink, (uint32_t)((nunion + 255) / 256), 0, pa, "gridding launch");
    if (st != SAR_OK) return st;
  }
  sar_status st = grid_union_launch<W>(p, a, nblk, sink);
  if (st != SAR_OK || a.max_slots == 0) return st;
  UnionCombineBody::Args ca{(const int2*)ws.slots, ws.split_count, ws.partial, grid, p.mx, p.nf, a.ntx, a.max_slots};
  return launch_body<UnionCombineBody>(sink, (uint32_t)a.max_slots, 0, ca, "gridding launch");
}

}  // namespace grid_impl
}  // namespace sar

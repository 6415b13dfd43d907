// Step a0: virtual elements, residual path and sorted gridding records.
//
// Every Tx/Rx pair of every shot becomes a virtual element at the pair's
// midpoint projected onto the plane Z_0 (Eqs. (3)-(4)); its residual path
// beta (Eqs. (7), (12)) is kept for the phase compensation applied in the
// gridding kernel.  The elements are then sorted by the oversampled grid cell
// of their first kernel tap (per-cell counts and their scan give each cell's
// start; a stable radix sort gives the order) so that the gridding kernel can
// walk every sample whose support touches a tile as a handful of contiguous
// runs.  Within a cell the order is by source index, so results are
// reproducible.

#include "device_common.hpp"
#include "launch.hpp"
#include "sar_internal.hpp"

namespace sar {
namespace {

struct GeoArgs {
  const double* pos;     // [n_pos][3]
  const double* pair;    // [n_pair][4]: midpoint offset x, y; multistatic beta term; |d|^2 / 4
  int64_t n_v;
  int n_pair;
  double xc, yc;         // lateral centre of the image grid
  double gsx, gsy;       // metres -> oversampled cells
  int mx, my;
  double z_ref;
  double beta_sign;      // 2 sign(Z_0 - z_c), or 0 without compensation
  double kb_beta, inv_i0_beta;
  double z_c, amp_inv_r2;  // amplitude half: reference depth and 1 / (z_c - Z_0)^2 (0: off)
  int fp32;              // precision diagnostic: offsets and beta in float32
};

// Modified Bessel function of the first kind, order 0, by its power series
// I0(x) = sum_k (x^2/4)^k / (k!)^2 in nested form with a fixed number of
// terms: for the arguments of a width-W kernel (x <= beta < 2.9 W at
// oversampling up to 4) the first 4W + 4 terms leave a relative truncation
// below 3e-12 (below 1e-14 for W >= 5), far under the float32 rounding of the
// stored weights, and the unrolled, branch-free recurrence keeps the
// per-weight cost flat.
template <int K>
__device__ __forceinline__ double bessel_i0_series(double x) {
  const double q = 0.25 * x * x;
  double acc = 1.0;
  static_for<0, K>([&](auto ic) __attribute__((always_inline)) {
    constexpr int k = K - decltype(ic)::value;
    constexpr double inv_k2 = 1.0 / ((double)k * (double)k);
    acc = fma(acc, q * inv_k2, 1.0);
  });
  return acc;
}

// Kaiser-Bessel kernel of width W (cells), normalised to 1 at the centre.
template <int W>
__device__ __forceinline__ float kb_weight(double d, double beta, double inv_i0_beta) {
  const double z = d * (2.0 / (double)W);
  const double r = 1.0 - z * z;
  if (r <= 0.0) return 0.f;
  return (float)(bessel_i0_series<4 * W + 4>(beta * sqrt(r)) * inv_i0_beta);
}

// grid coordinate in [0, m) and first-tap cell for a kernel of width W
__device__ __forceinline__ void grid_coord(double rel, double scale, int m, int W, double& g, int& c0) {
  double t = rel * scale;
  t -= floor(t / (double)m) * (double)m;
  if (t >= (double)m) t -= (double)m;
  g = t;
  c0 = (int)floor(t - 0.5 * W) + 1;
}

// the same in float32 (precision diagnostic)
__device__ __forceinline__ void grid_coord_f32(float rel, float scale, int m, int W, double& g, int& c0) {
  float t = rel * scale;
  t -= floorf(t / (float)m) * (float)m;
  if (t >= (float)m) t -= (float)m;
  g = t;
  c0 = (int)floorf(t - 0.5f * (float)W) + 1;
}

// grid coordinates of virtual sample (shot m, pair l); keys and records call
// this one function, so both place a sample in the same cell
__device__ __forceinline__ void sample_cells(const GeoArgs& g, int64_t m, int l, int W, double& gx, int& cx,
                                             double& gy, int& cy) {
  if (g.fp32) {
    const float xv = (float)g.pos[3 * m + 0] + (float)g.pair[4 * l + 0];
    const float yv = (float)g.pos[3 * m + 1] + (float)g.pair[4 * l + 1];
    grid_coord_f32(xv - (float)g.xc, (float)g.gsx, g.mx, W, gx, cx);
    grid_coord_f32(yv - (float)g.yc, (float)g.gsy, g.my, W, gy, cy);
  } else {
    const double xv = g.pos[3 * m + 0] + g.pair[4 * l + 0];
    const double yv = g.pos[3 * m + 1] + g.pair[4 * l + 1];
    grid_coord(xv - g.xc, g.gsx, g.mx, W, gx, cx);
    grid_coord(yv - g.yc, g.gsy, g.my, W, gy, cy);
  }
}

__device__ __forceinline__ int wrap(int c, int m) { return c < 0 ? c + m : (c >= m ? c - m : c); }

struct ZeroBody {
  struct Args {
    int32_t* p;
    int64_t n;
    int32_t* one;  // one more word to clear (may be null)
  };
  static constexpr int kThreads = 256;
  static __device__ __forceinline__ void run(const Args& a, uint32_t b, uint32_t) {
    const int64_t i = (int64_t)b * kThreads + threadIdx.x;
    if (i < a.n) a.p[i] = 0;
    if (i == 0 && a.one) *a.one = 0;
  }
};

// per virtual sample: first-tap cell (the sort key), counted per cell
template <int W>
struct KeysBody {
  struct Args {
    GeoArgs g;
    int32_t* key;
    int32_t* count;
  };
  static constexpr int kThreads = 256;
  static __device__ __forceinline__ void run(const Args& a, uint32_t b, uint32_t) {
    const int64_t n = (int64_t)b * kThreads + threadIdx.x;
    if (n >= a.g.n_v) return;
    const int64_t m = n / a.g.n_pair;
    const int l = (int)(n - m * a.g.n_pair);
    double gx, gy;
    int cx, cy;
    sample_cells(a.g, m, l, W, gx, cx, gy, cy);
    const int k = wrap(cy, a.g.my) * a.g.mx + wrap(cx, a.g.mx);
    a.key[n] = k;
    atomicAdd(&a.count[k], 1);
  }
};

// ---- exclusive scans of counts (two passes, three beyond 1024 chunks) -----
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanChunk = kScanThreads * kScanItems;

__device__ __forceinline__ int block_exclusive_scan(int v, int* smem_waves, int& total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  if (lane == 63) smem_waves[wave] = incl;
  __syncthreads();
  if (wave == 0) {
    const int nw = blockDim.x >> 6;
    int w = lane < nw ? smem_waves[lane] : 0;
    int wi = w;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int t = __shfl_up(wi, off, 64);
      if (lane >= off) wi += t;
    }
    if (lane < nw) smem_waves[lane] = wi - w;  // exclusive wave offsets
    if (lane == nw - 1) smem_waves[64] = wi;   // block total
  }
  __syncthreads();
  total = smem_waves[64];
  return incl - v + smem_waves[wave];
}

// pass 1: scan within chunks of kScanChunk counts, chunk totals to bsum
struct ScanLocalBody {
  struct Args {
    int32_t* data;
    int64_t n;
    int32_t* bsum;
  };
  static constexpr int kThreads = kScanThreads;
  static __device__ __forceinline__ void run(const Args& a, uint32_t b, uint32_t) {
    __shared__ int smem[65];
    const int64_t base = (int64_t)b * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      v[i] = (base + i < a.n) ? a.data[base + i] : 0;
      s += v[i];
    }
    int total;
    int run_ = block_exclusive_scan(s, smem, total);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (base + i < a.n) a.data[base + i] = run_;
      run_ += v[i];
    }
    if (threadIdx.x == 0) a.bsum[b] = total;
  }
};

// pass 2 (one block): exclusive scan of the chunk totals; grand total out
struct ScanSumsBody {
  struct Args {
    int32_t* bsum;
    int nb;
    int32_t* total_out;
  };
  static constexpr int kThreads = kScanThreads;
  static __device__ __forceinline__ void run(const Args& a, uint32_t, uint32_t) {
    __shared__ int smem[65];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < a.nb; c0 += kScanChunk) {
      const int base = c0 + threadIdx.x * kScanItems;
      int v[kScanItems];
      int s = 0;
#pragma unroll
      for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < a.nb) ? a.bsum[base + i] : 0;
        s += v[i];
      }
      int total;
      int run_ = block_exclusive_scan(s, smem, total) + carry;
#pragma unroll
      for (int i = 0; i < kScanItems; ++i) {
        if (base + i < a.nb) a.bsum[base + i] = run_;
        run_ += v[i];
      }
      __syncthreads();
      if (threadIdx.x == 0) carry += total;
      __syncthreads();
    }
    if (threadIdx.x == 0) *a.total_out = carry;
  }
};

// pass 3: add each chunk's offset
struct ScanAddBody {
  struct Args {
    int32_t* data;
    int64_t n;
    const int32_t* bsum;
  };
  static constexpr int kThreads = kScanThreads;
  static __device__ __forceinline__ void run(const Args& a, uint32_t b, uint32_t) {
    const int64_t base = (int64_t)b * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    const int off = a.bsum[b];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
      if (base + i < a.n) a.data[base + i] += off;
  }
};

// passes 2 + 3 in one for up to kScanFuseChunks chunks: each block sums the
// raw totals of the chunks before its own (integer sums, so the offsets equal
// those of the separate pass) and block 0 also writes the grand total
constexpr int kScanFuseChunks = 1024;
struct ScanAddSumsBody {
  struct Args {
    int32_t* data;
    int64_t n;
    const int32_t* bsum;   // raw chunk totals
    int nb;
    int32_t* total_out;
  };
  static constexpr int kThreads = kScanThreads;
  static __device__ __forceinline__ void run(const Args& a, uint32_t b, uint32_t) {
    __shared__ int smem[65];
    const int upto = b == 0 ? a.nb : (int)b;   // block 0: every chunk, for the total
    int v = threadIdx.x < upto ? a.bsum[threadIdx.x] : 0;
    int total;
    const int excl = block_exclusive_scan(v, smem, total);
    // the sum of the chunks before b is the exclusive prefix at thread b
    // (block 0: all of them, its own offset is 0)
    __shared__ int off_s;
    if (b != 0 && threadIdx.x == (int)b - 1) off_s = excl + v;
    if (b == 0 && threadIdx.x == 0) {
      off_s = 0;
      *a.total_out = total;
    }
    __syncthreads();
    const int off = off_s;
    const int64_t base = (int64_t)b * kScanChunk + (int64_t)threadIdx.x * kScanItems;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
      if (base + i < a.n) a.data[base + i] += off;
  }
};

// ---- stable least-significant-digit radix sort of the samples by cell -----
// Each pass orders (key, index) pairs by one DB-bit digit of the key and keeps
// the order of equal digits, so after the last pass the samples are sorted by
// cell and, within a cell, by source index: the same order on every run,
// whatever the cell counts (a dwelling hand can put thousands of samples in
// one cell).  A pass is a per-tile digit histogram, an exclusive scan of the
// histograms in digit-major order (the scan kernels above) and a scatter that
// ranks equal digits within its tile in index order.  Every thread loads its
// 16 elements of the tile at once, so a tile's loads are all in flight together.
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;                          // elements per thread per tile
constexpr int kSortTile = kSortThreads * kSortRounds;    // 4096 elements

template <int DB>
struct RadixHistBody {
  static constexpr int NB = 1 << DB;
  struct Args {
    const int32_t* key;
    int64_t n;
    int shift;
    int ntiles;     // histogram stride: hist[digit * ntiles + tile]
    int32_t* hist;
  };
  static constexpr int kThreads = kSortThreads;
  static __device__ __forceinline__ void run(const Args& a, uint32_t b, uint32_t) {
    __shared__ int cnt[NB];
    int k[kSortRounds];
    const int64_t base = (int64_t)b * kSortTile + threadIdx.x;
#pragma unroll
    for (int j = 0; j < kSortRounds; ++j) {
      const int64_t i = base + (int64_t)j * kSortThreads;
      k[j] = i < a.n ? a.key[i] : -1;
    }
    for (int d = threadIdx.x; d < NB; d += kSortThreads) cnt[d] = 0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortRounds; ++j)
      if (k[j] >= 0) atomicAdd(&cnt[(k[j] >> a.shift) & (NB - 1)], 1);
    __syncthreads();
    for (int d = threadIdx.x; d < NB; d += kSortThreads) a.hist[(int64_t)d * a.ntiles + b] = cnt[d];
  }
};

template <int DB>
struct RadixScatterBody {
  static constexpr int NB = 1 << DB;
  struct Args {
    const int32_t* key_in;
    const int32_t* val_in;  // null: the element's own index (first pass)
    int32_t* key_out;       // null: keys not needed after this pass
    int32_t* val_out;
    int64_t n;
    int shift;
    int ntiles;
    const int32_t* offs;    // exclusive scan of the histograms, digit-major
  };
  static constexpr int kThreads = kSortThreads;
  static __device__ __forceinline__ void run(const Args& a, uint32_t b, uint32_t) {
    constexpr int kWaves = kSortThreads / 64;
    __shared__ int base_d[NB];             // next output slot per digit
    __shared__ int wcnt[kWaves][NB];       // per-wave digit counts of a round
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    int kk[kSortRounds], vv[kSortRounds];
    const int64_t base = (int64_t)b * kSortTile + tid;
#pragma unroll
    for (int j = 0; j < kSortRounds; ++j) {
      const int64_t i = base + (int64_t)j * kSortThreads;
      const bool valid = i < a.n;
      kk[j] = valid ? a.key_in[i] : -1;
      vv[j] = valid ? (a.val_in ? a.val_in[i] : (int)i) : 0;
    }
    for (int d = tid; d < NB; d += kSortThreads) {
      base_d[d] = a.offs[(int64_t)d * a.ntiles + b];
#pragma unroll
      for (int w = 0; w < kWaves; ++w) wcnt[w][d] = 0;
    }
    __syncthreads();
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;   // lanes below this one
    // per round, only the digits present are touched: the first lane of each
    // digit group in a wave posts the group's count, and after the round adds
    // it to the digit's next slot and clears its post (integer additions, so
    // the slots do not depend on their order)
#pragma unroll
    for (int j = 0; j < kSortRounds; ++j) {
      const bool valid = kk[j] >= 0;
      const int d = (kk[j] >> a.shift) & (NB - 1);
      // lanes of this wave holding the same digit: they agree on every digit bit
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < DB; ++bit) {
        const bool set = (d >> bit) & 1;
        const uint64_t m = __ballot(set);
        peers &= set ? m : ~m;
      }
      const int rank_w = __popcll(peers & lt);
      const bool lead = valid && rank_w == 0;
      const int group = __popcll(peers);
      if (lead) wcnt[wave][d] = group;
      __syncthreads();
      if (valid) {
        int pos = base_d[d] + rank_w;
        for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
        if (a.key_out) a.key_out[pos] = kk[j];
        a.val_out[pos] = vv[j];
      }
      __syncthreads();
      if (lead) {
        atomicAdd(&base_d[d], group);
        wcnt[wave][d] = 0;
      }
    }
  }
};

// One thread per sorted slot: the record of the slot's sample, its geometry
// recomputed in float64 (float32 for the precision diagnostic) from the shot
// position.
template <int W>
struct RecordsBody {
  struct Args {
    GeoArgs g;
    const int32_t* order;
    SampleRec<W>* rec;
  };
  static constexpr int kThreads = 256;
  static __device__ __forceinline__ void run(const Args& a, uint32_t b, uint32_t) {
    const int64_t s = (int64_t)b * kThreads + threadIdx.x;
    if (s >= a.g.n_v) return;
    const int64_t n = a.order[s];
    const int64_t m = n / a.g.n_pair;
    const int l = (int)(n - m * a.g.n_pair);
    double gx, gy;
    int cx, cy;
    sample_cells(a.g, m, l, W, gx, cx, gy, cy);
    SampleRec<W> r;
    r.src = (int32_t)n;
    r.cx = (int16_t)wrap(wrap(cx, a.g.mx) + W - 1, a.g.mx);
    r.cy = (int16_t)wrap(wrap(cy, a.g.my) + W - 1, a.g.my);
    if (a.g.fp32)
      r.beta = (float)a.g.beta_sign * ((float)a.g.pos[3 * m + 2] - (float)a.g.z_ref) + (float)a.g.pair[4 * l + 2];
    else
      r.beta = a.g.beta_sign * (a.g.pos[3 * m + 2] - a.g.z_ref) + a.g.pair[4 * l + 2];
    const double fx = (double)cx - gx;
    const double fy = (double)cy - gy;
    // amplitude half of the compensation (ratio of the amplitudes of Eqs. (9)
    // and (10) for a scatterer at the reference depth straight ahead of the
    // virtual element), folded into the x weights
    float amp = 1.0f;
    if (a.g.amp_inv_r2 != 0.0) {
      const double h = a.g.z_c - a.g.pos[3 * m + 2];
      amp = (float)((a.g.pair[4 * l + 3] + h * h) * a.g.amp_inv_r2);
    }
#pragma unroll
    for (int j = 0; j < W; ++j) {
      r.wx[j] = amp * kb_weight<W>(fx + j, a.g.kb_beta, a.g.inv_i0_beta);
      r.wy[j] = kb_weight<W>(fy + j, a.g.kb_beta, a.g.inv_i0_beta);
    }
    a.rec[s] = r;
  }
};

uint32_t blocks_for(int64_t n, int threads) { return (uint32_t)((n + threads - 1) / threads); }

// one radix pass: digit histograms per tile, their scan, the stable scatter
template <int DB, typename Scan>
sar_status radix_pass(LaunchSink& sink, const int32_t* kin, const int32_t* vin, int32_t* kout, int32_t* vout,
                      int64_t n_v, int shift, int ntiles, int32_t* hist, Scan& scan) {
  const char* what = "geometry/sort launch";
  const int64_t nhist = (int64_t)(1 << DB) * ntiles;
  sar_status st;
  if ((st = launch_body<RadixHistBody<DB>>(sink, ntiles, 0, {kin, n_v, shift, ntiles, hist}, what)) != SAR_OK)
    return st;
  if ((st = scan(hist, nhist, hist + nhist + 1)) != SAR_OK) return st;
  return launch_body<RadixScatterBody<DB>>(sink, ntiles, 0, {kin, vin, kout, vout, n_v, shift, ntiles, hist}, what);
}

template <int W>
sar_status geometry_sort_w(const Plan& p, const double* d_pos, int64_t n_pos, int64_t n_pos_grid,
                           const Workspace& ws, LaunchSink& sink) {
  const int64_t n_v = n_pos * p.n_pair;
  const int64_t n_v_grid = n_pos_grid * p.n_pair;
  const int64_t ncell = (int64_t)p.mx * p.my;
  GeoArgs g;
  g.pos = d_pos;
  g.pair = p.d_pair;
  g.n_v = n_v;
  g.n_pair = p.n_pair;
  g.xc = p.xc;
  g.yc = p.yc;
  g.gsx = (double)p.mx / ((double)p.nx * p.dx);
  g.gsy = (double)p.my / ((double)p.ny * p.dy);
  g.mx = p.mx;
  g.my = p.my;
  g.z_ref = p.z_ref;
  g.beta_sign = p.beta_sign;
  g.kb_beta = p.kb_beta;
  g.z_c = p.z_focus;
  g.amp_inv_r2 = p.amp_inv_r2;
  g.fp32 = (p.flags & SAR_FP32_ARGS) ? 1 : 0;
  // 1 / I0(beta) evaluated with the same series on the host
  {
    const double q = 0.25 * p.kb_beta * p.kb_beta;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 80; ++k) {
      term *= q / ((double)k * (double)k);
      sum += term;
      if (term < 1e-17 * sum) break;
    }
    g.inv_i0_beta = 1.0 / sum;
  }
  sar_status st;
  const char* what = "geometry/sort launch";
  if ((st = launch_body<ZeroBody>(sink, blocks_for(ncell + 1, 256), 0, {ws.cell_start, ncell + 1, ws.split_count},
                                  what)) != SAR_OK)
    return st;
  if ((st = launch_body<KeysBody<W>>(sink, blocks_for(n_v_grid, 256), 0, {g, ws.key, ws.cell_start}, what)) !=
      SAR_OK)
    return st;
  // cell starts: exclusive scan of the per-cell counts
  auto scan = [&](int32_t* data, int64_t n, int32_t* bsum) -> sar_status {
    const int nb = (int)((n + kScanChunk - 1) / kScanChunk);
    sar_status s2;
    if ((s2 = launch_body<ScanLocalBody>(sink, nb, 0, {data, n, bsum}, what)) != SAR_OK) return s2;
    if (nb <= kScanFuseChunks) return launch_body<ScanAddSumsBody>(sink, nb, 0, {data, n, bsum, nb, data + n}, what);
    if ((s2 = launch_body<ScanSumsBody>(sink, 1, 0, {bsum, nb, data + n}, what)) != SAR_OK) return s2;
    return launch_body<ScanAddBody>(sink, nb, 0, {data, n, bsum}, what);
  };
  if ((st = scan(ws.cell_start, ncell, ws.cell_start + ncell + 1)) != SAR_OK) return st;
  // sorted order: LSD radix passes over the key bits of the largest cell index,
  // as few as digits of up to 11 bits allow (the histogram stride and the
  // grids follow n_pos_grid, so a fused batch's launch sequence does not
  // depend on the call's n_pos)
  const int ntiles = (int)((n_v_grid + kSortTile - 1) / kSortTile);
  int bits = 1;
  while ((int64_t)1 << bits < ncell) ++bits;
  const int npass = (bits + 10) / 11;
  const int db = std::max(8, (bits + npass - 1) / npass);
  for (int q = 0; q < npass && ntiles > 0; ++q) {
    const int32_t* kin = (q & 1) ? ws.key_alt : ws.key;
    int32_t* kout = q + 1 == npass ? nullptr : ((q & 1) ? ws.key : ws.key_alt);
    int32_t* vout = ((npass - 1 - q) & 1) ? ws.order_alt : ws.order;
    const int32_t* vin = q == 0 ? nullptr : (((npass - q) & 1) ? ws.order_alt : ws.order);
    switch (db) {
      case 8: st = radix_pass<8>(sink, kin, vin, kout, vout, n_v, db * q, ntiles, ws.hist, scan); break;
      case 9: st = radix_pass<9>(sink, kin, vin, kout, vout, n_v, db * q, ntiles, ws.hist, scan); break;
      case 10: st = radix_pass<10>(sink, kin, vin, kout, vout, n_v, db * q, ntiles, ws.hist, scan); break;
      default: st = radix_pass<11>(sink, kin, vin, kout, vout, n_v, db * q, ntiles, ws.hist, scan); break;
    }
    if (st != SAR_OK) return st;
  }
  return launch_body<RecordsBody<W>>(sink, blocks_for(n_v_grid, 256), 0,
                                     {g, ws.order, (SampleRec<W>*)ws.rec}, what);
}

}  // namespace

sar_status launch_geometry_sort(const Plan& p, const double* d_pos, int64_t n_pos, int64_t n_pos_grid,
                                const Workspace& ws, LaunchSink& sink) {
  switch (p.w) {
    case 3: return geometry_sort_w<3>(p, d_pos, n_pos, n_pos_grid, ws, sink);
    case 4: return geometry_sort_w<4>(p, d_pos, n_pos, n_pos_grid, ws, sink);
    case 5: return geometry_sort_w<5>(p, d_pos, n_pos, n_pos_grid, ws, sink);
    case 6: return geometry_sort_w<6>(p, d_pos, n_pos, n_pos_grid, ws, sink);
    case 7: return geometry_sort_w<7>(p, d_pos, n_pos, n_pos_grid, ws, sink);
    case 8: return geometry_sort_w<8>(p, d_pos, n_pos, n_pos_grid, ws, sink);
    default: return fail(SAR_ERR_UNSUPPORTED, "kernel width not compiled");
  }
}

}  // namespace sar

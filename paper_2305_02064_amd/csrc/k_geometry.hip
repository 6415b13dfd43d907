// Step a0: virtual elements, residual path and sorted gridding records.
//
// Every Tx/Rx pair of every shot becomes a virtual element at the pair's
// midpoint projected onto the plane Z_0 (Eqs. (3)-(4)); its residual path
// beta (Eqs. (7), (12)) is kept for the phase compensation applied in the
// gridding kernel.  The elements are then counting-sorted by the oversampled
// grid cell of their first kernel tap so that the gridding kernel can walk
// every sample whose support touches a tile as a handful of contiguous runs.
// Within a cell the order is by source index, so results are reproducible.

#include "device_common.hpp"
#include "launch.hpp"
#include "sar_internal.hpp"

namespace sar {
namespace {

struct GeoArgs {
  const double* pos;     // [n_pos][3]
  const double* pair;    // [n_pair][4]: midpoint offset x, y; multistatic beta term; unused
  int64_t n_v;
  int n_pair;
  double xc, yc;         // lateral centre of the image grid
  double gsx, gsy;       // metres -> oversampled cells
  int mx, my;
  double z_ref;
  double beta_sign;      // 2 sign(Z_0 - z_c), or 0 without compensation
  double kb_beta, inv_i0_beta;
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
  };
  static constexpr int kThreads = 256;
  static __device__ __forceinline__ void run(const Args& a, uint32_t b, uint32_t) {
    const int64_t i = (int64_t)b * kThreads + threadIdx.x;
    if (i < a.n) a.p[i] = 0;
  }
};

// per virtual sample: first-tap cell (the sort key) and its rank in the cell
template <int W>
struct KeysBody {
  struct Args {
    GeoArgs g;
    int32_t* key;
    int32_t* rank;
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
    a.rank[n] = atomicAdd(&a.count[k], 1);
  }
};

// ---- exclusive scan of the per-cell counts (three passes) -----------------
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

struct ScatterBody {
  struct Args {
    int64_t n_v;
    const int32_t* key;
    const int32_t* rank;
    const int32_t* start;
    int32_t* order;
  };
  static constexpr int kThreads = 256;
  static __device__ __forceinline__ void run(const Args& a, uint32_t b, uint32_t) {
    const int64_t n = (int64_t)b * kThreads + threadIdx.x;
    if (n >= a.n_v) return;
    a.order[a.start[a.key[n]] + a.rank[n]] = (int32_t)n;
  }
};

// One thread per cell: order the cell's samples by source index.
struct SortCellsBody {
  struct Args {
    int64_t ncell;
    const int32_t* start;
    int32_t* order;
  };
  static constexpr int kThreads = 256;
  static __device__ __forceinline__ void run(const Args& a, uint32_t b, uint32_t) {
    const int64_t c = (int64_t)b * kThreads + threadIdx.x;
    if (c >= a.ncell) return;
    const int s0 = a.start[c], s1 = a.start[c + 1];
    for (int i = s0 + 1; i < s1; ++i) {
      const int v = a.order[i];
      int j = i - 1;
      while (j >= s0 && a.order[j] > v) {
        a.order[j + 1] = a.order[j];
        --j;
      }
      a.order[j + 1] = v;
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
#pragma unroll
    for (int j = 0; j < W; ++j) {
      r.wx[j] = kb_weight<W>(fx + j, a.g.kb_beta, a.g.inv_i0_beta);
      r.wy[j] = kb_weight<W>(fy + j, a.g.kb_beta, a.g.inv_i0_beta);
    }
    a.rec[s] = r;
  }
};

uint32_t blocks_for(int64_t n, int threads) { return (uint32_t)((n + threads - 1) / threads); }

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
  if ((st = launch_body<ZeroBody>(sink, blocks_for(ncell + 1, 256), 0, {ws.cell_start, ncell + 1}, what)) != SAR_OK)
    return st;
  if ((st = launch_body<KeysBody<W>>(sink, blocks_for(n_v_grid, 256), 0, {g, ws.key, ws.rank, ws.cell_start},
                                     what)) != SAR_OK)
    return st;
  const int nb = (int)((ncell + kScanChunk - 1) / kScanChunk);
  int32_t* bsum = ws.cell_start + ncell + 1;
  if ((st = launch_body<ScanLocalBody>(sink, nb, 0, {ws.cell_start, ncell, bsum}, what)) != SAR_OK) return st;
  if ((st = launch_body<ScanSumsBody>(sink, 1, 0, {bsum, nb, ws.cell_start + ncell}, what)) != SAR_OK) return st;
  if ((st = launch_body<ScanAddBody>(sink, nb, 0, {ws.cell_start, ncell, bsum}, what)) != SAR_OK) return st;
  if ((st = launch_body<ScatterBody>(sink, blocks_for(n_v_grid, 256), 0,
                                     {n_v, ws.key, ws.rank, ws.cell_start, ws.order}, what)) != SAR_OK)
    return st;
  if ((st = launch_body<SortCellsBody>(sink, blocks_for(ncell, 256), 0, {ncell, ws.cell_start, ws.order}, what)) !=
      SAR_OK)
    return st;
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

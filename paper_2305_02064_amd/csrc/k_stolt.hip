// Steps a4 + a5: range-migration filter and Stolt map with the z transform
// (and its single-plane form for 2-D images).
//
// For every (k_x, k_y) column of the spectrum, each frequency sample f_i
// becomes a non-uniform sample at k_z = sqrt(4 k_i^2 - k_x^2 - k_y^2)
// (Eq. (14); evanescent samples are dropped) with value
// S k_z exp(-j k_z Z_0) (Eq. (15), P = 1), or S 4k exp(-j k_z Z_0) with the
// optional Jacobian dk_z/dk = 4k/k_z of the change of variables.  The Stolt map plus the inverse
// transform along z is the non-uniform sum
//   Z(z_w) = sum_i F_i exp(+j k_z,i z_w),  z_w = z0 + w dz,
// a 1-D type-1 NUFFT at the positions theta_i = k_z,i dz: float64 pre-phase
// exp(j k_z (z_mid - Z_0)) and grid position, exponential-of-semicircle
// spreading into an oversampled LDS grid of MZ cells, an inverse four-step
// FFT in registers with one LDS exchange, and deapodisation of the nz centred
// outputs.
//
// A column is handled by a group of 16 lanes (4 columns per wavefront).  Each
// lane takes a contiguous run of frequencies, whose k_z positions are
// monotone and close together, accumulates them in a small register window of
// cells and flushes it to the shared grid with LDS atomics, so few lanes hit
// the same cell at once.  The +-1 factor (-1)^P (and (-1)^Q) that lets the
// next step use plain inverse DFTs on centred mode indices of an even axis is
// folded in here (an odd axis is shifted and phase-corrected by its inverse
// transform instead).

#include "device_common.hpp"
#include "es_poly.hpp"
#include "launch.hpp"
#include "sar_internal.hpp"

namespace sar {
namespace {

constexpr int kWaves = 1;   // wavefronts per block
constexpr int kG = 16;      // lanes per column
constexpr int kCols = kWaves * 64 / kG;  // columns per block

struct StoltArgs {
  const float2* spec;  // [ny][nx][nf]
  float2* zc;          // [ny][nx][nz]
  const double* k;     // [nf]
  const float* deapz;  // [nz]
  const float2* tw;    // exp(+j 2 pi i / MZ), i < MZ
  int nx, ny, nf, nz;
  double dkx, dky;
  double zmid_minus_zref_cyc;  // (z_mid - Z_0) / (2 pi)
  double dz_cells;             // dz * MZ / (2 pi)
  int dcf;             // 1: filter factor 4k (k_z times the Jacobian dk_z/dk = 4k/k_z)
  int sgx, sgy;        // 1: fold (-1)^P (resp. (-1)^Q) in (even nx, ny)
  int64_t ncol;
};

// The WZ weights of the exponential-of-semicircle kernel
// exp(beta (sqrt(1 - z^2) - 1)) at z = 2 d_s / WZ, d_s = tau + s - WZ/2 the
// distance of tap s from the sample, as polynomials in t = 2 tau - 1 (fitted
// per tap, es_poly.hpp; error about exp(-beta), the kernel's own value at the
// edge of its support): WZ x degree FMAs per sample instead of a square root
// and an exponential per tap
template <int WZ>
__device__ __forceinline__ void es_taps(float t, float (&w)[WZ]) {
  using P = EsPoly<WZ>;
#pragma unroll
  for (int s = 0; s < WZ; ++s) {
    float v = P::c[s][0];
#pragma unroll
    for (int j = 1; j <= P::kDeg; ++j) v = fmaf(v, t, P::c[s][j]);
    w[s] = v;
  }
}

// square root of a positive, normal float64: hardware reciprocal square root
// refined by two Newton steps (relative error far below 1e-12, ample for the
// k_z of a phase argument)
__device__ __forceinline__ double sqrt_pos(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * r;
  double s = x * r;
  s = fma(h, fma(-s, s, x), s);
  s = fma(h, fma(-s, s, x), s);
  return s;
}

// F32: the precision diagnostic (k_z, its pre-phase and grid position in
// float32 instead of float64)
template <int MZ, int WZ, bool F32>
struct StoltBody {
  using Args = StoltArgs;
  static constexpr int kThreads = 64 * kWaves;
  static __device__ __forceinline__ void run(const StoltArgs& a, uint32_t blk, uint32_t nblk);
};

template <int MZ, int WZ, bool F32>
__device__ __forceinline__ void StoltBody<MZ, WZ, F32>::run(const StoltArgs& a, uint32_t blk, uint32_t nblk) {
  constexpr int L2 = MZ / kG;       // points per lane in the first FFT pass
  constexpr int WWIN = WZ + 2;      // register window of cells per lane
  constexpr int RB = 8;             // samples per lane whose loads are in flight together
  constexpr int SB = 4;             // samples whose arithmetic is interleaved
  static_assert(MZ % kG == 0 && MZ <= 1024, "Stolt grid of 64..1024 cells");
  // LDS row of one column: MZ cells, then read back as the [16][L2 + 1]
  // padded transposition of the four-step FFT (one pad entry per row, so the
  // 16 lanes of a column write to distinct banks); 4 more entries shift the
  // rows of a wave's 4 columns onto different banks
  constexpr int RS = kG * (L2 + 1) + 4;
  __shared__ float2 grid[kCols][RS];
  const float2* __restrict__ tw = a.tw;       // twiddles and deapodisation:
  const float* __restrict__ deap = a.deapz;   // small tables, cached reads
  const int cl = threadIdx.x / kG;   // column slot in the block
  const int gl = threadIdx.x % kG;   // lane within the column's group
  float2* g = grid[cl];
  const int per = (a.nf + kG - 1) / kG;  // contiguous frequencies per lane
  const int64_t ngroups = (a.ncol + kCols - 1) / kCols;

  // one batch of the lane's run: wavenumbers and spectrum values, all loads
  // issued before any is used (a bit of `valid` per sample marks the ones
  // inside the run, so no loaded value is touched before its use)
  double kb[RB];
  float2 sb[RB];
  uint32_t valid = 0;
  auto load_batch = [&](int64_t colc, int r0) __attribute__((always_inline)) {
    const float2* __restrict__ sp = a.spec + colc * a.nf;
    valid = 0;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int i = gl * per + r0 + r;
      const bool ok = r0 + r < per && i < a.nf;
      const int ic = ok ? i : 0;
      kb[r] = a.k[ic];
      sb[r] = sp[ic];
      valid |= (uint32_t)ok << r;
    }
  };
  auto column_of = [&](int64_t grp) __attribute__((always_inline)) {
    const int64_t col = grp * kCols + cl;
    return col < a.ncol ? col : (int64_t)0;
  };
  if ((int64_t)blk < ngroups) load_batch(column_of(blk), 0);

  for (int64_t grp = blk; grp < ngroups; grp += nblk) {
    const int64_t col = grp * kCols + cl;
    const bool live = col < a.ncol;
    const int64_t colc = live ? col : 0;
    const int Q = (int)(colc / a.nx);
    const int P = (int)(colc - (int64_t)Q * a.nx);
    for (int c = gl; c < MZ; c += kG) g[c] = make_float2(0.f, 0.f);
    __syncthreads();

    // spreading: each lane accumulates its run of samples in a register window
    // of WWIN cells starting at cell wb and flushes it with LDS atomics when a
    // sample's support leaves the window
    if (live) {
      const double kx = (double)(P - a.nx / 2) * a.dkx;
      const double ky = (double)(Q - a.ny / 2) * a.dky;
      const double kp2 = kx * kx + ky * ky;
      const float kxf = (float)(P - a.nx / 2) * (float)a.dkx;
      const float kyf = (float)(Q - a.ny / 2) * (float)a.dky;
      const float kp2f = kxf * kxf + kyf * kyf;
      const float sgn = (((P & a.sgx) ^ (Q & a.sgy)) & 1) ? -1.f : 1.f;
      float2 win[WWIN];
#pragma unroll
      for (int s2 = 0; s2 < WWIN; ++s2) win[s2] = make_float2(0.f, 0.f);
      int wb = 0;
      bool open = false;
      auto flush = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int s2 = 0; s2 < WWIN; ++s2) {
          if (win[s2].x != 0.f || win[s2].y != 0.f) {
            const int c = (wb + s2) & (MZ - 1);
            atomicAdd(&g[c].x, win[s2].x);
            atomicAdd(&g[c].y, win[s2].y);
          }
          win[s2] = make_float2(0.f, 0.f);
        }
      };
      for (int r0 = 0; r0 < per; r0 += RB) {
        if (r0 > 0) load_batch(colc, r0);
        // SB samples at a time: first their k_z, pre-phase, value, first
        // cell and tap weights, with no branch, so the compiler interleaves
        // the samples' long dependency chains; then their window updates
#pragma unroll
        for (int r1 = 0; r1 < RB; r1 += SB) {
          float2 vv[SB];
          float ww[SB][WZ];
          int cc[SB];
          bool okk[SB];
#pragma unroll
          for (int q = 0; q < SB; ++q) {
            const int r = r1 + q;
            bool ok = (valid >> r) & 1u;
            float kzs;   // filter factor: k_z, or 4k with the Jacobian
            float2 ph;   // pre-phase exp(j k_z (z_mid - Z_0))
            double gc;   // grid position (cells), not wrapped
            if constexpr (F32) {
              const float k = (float)kb[r];
              const float kz2 = 4.f * k * k - kp2f;
              ok = ok && kz2 > 0.f;
              const float kzf = __builtin_sqrtf(ok ? kz2 : 1.f);   // evanescent: dropped below
              ph = cis_cycles_f32(kzf * (float)a.zmid_minus_zref_cyc);
              gc = (double)(kzf * (float)a.dz_cells);
              kzs = a.dcf ? 4.f * k : kzf;
            } else {
              const double k = kb[r];
              const double kz2 = 4.0 * k * k - kp2;
              ok = ok && kz2 > 0.0;
              const double kz = sqrt_pos(ok ? kz2 : 1.0);            // evanescent: dropped below
              kzs = a.dcf ? (float)(4.0 * k) : (float)kz;
              ph = cis_cycles(kz * a.zmid_minus_zref_cyc);
              gc = kz * a.dz_cells;
            }
            vv[q] = cscale(cmul(sb[r], ph), kzs * sgn);
            const double a0 = gc - 0.5 * WZ;
            const double c0d = floor(a0) + 1.0;
            cc[q] = (int)c0d;
            es_taps<WZ>((float)(2.0 * (c0d - a0) - 1.0), ww[q]);
            okk[q] = ok;
          }
#pragma unroll
          for (int q = 0; q < SB; ++q) {
            if (!okk[q]) continue;
            const int c0 = cc[q];
            if (!open || c0 < wb || c0 + WZ > wb + WWIN) {
              if (open) flush();
              wb = c0;
              open = true;
            }
            // tap s lands in window cell o + s, o = c0 - wb in 0 .. WWIN - WZ
            const int o = c0 - wb;
#pragma unroll
            for (int s2 = 0; s2 < WWIN; ++s2) {
              const float w0 = s2 < WZ ? ww[q][s2] : 0.f;
              const float w1 = s2 >= 1 && s2 - 1 < WZ ? ww[q][s2 - 1] : 0.f;
              const float w2 = s2 >= 2 && s2 - 2 < WZ ? ww[q][s2 - 2] : 0.f;
              cfma(win[s2], vv[q], o == 0 ? w0 : (o == 1 ? w1 : w2));
            }
          }
        }
      }
      if (open) flush();
    }
    // the next group's first batch loads while this group's transform runs
    if (grp + nblk < ngroups) load_batch(column_of(grp + nblk), 0);
    __syncthreads();

    // inverse DFT of the MZ cells: four-step with L1 = 16 lanes x L2 points
    // X[k2 + L2 k1] = sum_l1 w_16^(l1 k1) w_MZ^(l1 k2) sum_l2 x[l1 + 16 l2] w_L2^(l2 k2)
    float2 v1[L2];
#pragma unroll
    for (int l2 = 0; l2 < L2; ++l2) v1[l2] = g[gl + kG * l2];
    reg_dft_dif<L2, +1>(v1);
    __syncthreads();
    // twiddles w_MZ^(l1 k2) from two table entries, w^l1 and w^(TB l1), and
    // their powers (at most about nine roundings each) instead of one table
    // read per k2
    constexpr int TB = L2 < 8 ? L2 : 8;
    float2 p1[TB], pB[(L2 + TB - 1) / TB];
    p1[0] = make_float2(1.f, 0.f);
    pB[0] = make_float2(1.f, 0.f);
    {
      const float2 w1 = tw[gl];
#pragma unroll
      for (int j = 1; j < TB; ++j) p1[j] = cmul(p1[j - 1], w1);
      const float2 wB = tw[(TB * gl) % MZ];
#pragma unroll
      for (int j = 1; j < (L2 + TB - 1) / TB; ++j) pB[j] = cmul(pB[j - 1], wB);
    }
    static_for<0, L2>([&](auto kc) __attribute__((always_inline)) {
      constexpr int k2 = decltype(kc)::value;
      float2 y = v1[ct_bitrev(k2, ct_log2(L2))];
      if constexpr (k2 != 0) y = cmul(y, cmul(pB[k2 / TB], p1[k2 % TB]));
      g[gl * (L2 + 1) + k2] = y;   // [l1][k2], padded rows
    });
    __syncthreads();
    if (live) {
      float2* __restrict__ out = a.zc + colc * a.nz;
      const int h = a.nz / 2;
      for (int k2 = gl; k2 < L2; k2 += kG) {
        float2 v2[kG];
#pragma unroll
        for (int l1 = 0; l1 < kG; ++l1) v2[l1] = g[l1 * (L2 + 1) + k2];
        reg_dft_dif<kG, +1>(v2);
        static_for<0, kG>([&](auto kc) __attribute__((always_inline)) {
          constexpr int k1 = decltype(kc)::value;
          const int kk = k2 + L2 * k1;
          const int w = kk < h ? kk + h : (kk >= MZ - h ? kk - MZ + h : -1);
          if (w >= 0) out[w] = cscale(v2[ct_bitrev(k1, ct_log2(kG))], deap[w]);
        });
      }
    }
    __syncthreads();
  }
}

// A single image plane (nz = 1, the paper's 2-D image at a known depth,
// Sec. V-A): the Stolt map and the z transform collapse to one exact sum per
// column, Z(p,q) = sum_i F_i exp(+j k_z,i z0) with the filter of Eq. (15),
// i.e. total phase k_z (z0 - Z_0) in float64.  16 lanes per column take every
// 16th frequency and reduce with cross-lane shuffles; the (-1)^(P+Q) factor
// of the lateral inverse transform is folded in as in the 3-D path.
struct PlaneArgs {
  const float2* spec;  // [ny][nx][nf]
  float2* zc;          // [ny][nx]
  const double* k;     // [nf]
  int nx, ny, nf;
  double dkx, dky;
  double z_cyc;        // (z0 - Z_0) / (2 pi)
  int dcf;             // 1: filter factor 4k instead of k_z (see StoltArgs)
  int sgx, sgy;        // lateral sign folding as in StoltArgs
  int64_t ncol;
};

struct PlaneBody {
  using Args = PlaneArgs;
  static constexpr int kThreads = 256;
  static __device__ __forceinline__ void run(const PlaneArgs& a, uint32_t blk, uint32_t nblk) {
    constexpr int G = 16;                  // lanes per column
    constexpr int COLS = kThreads / G;     // columns per block
    const int cl = threadIdx.x / G;
    const int gl = threadIdx.x % G;
    const int64_t ngroups = (a.ncol + COLS - 1) / COLS;
    for (int64_t grp = blk; grp < ngroups; grp += nblk) {
      const int64_t col = grp * COLS + cl;
      const bool live = col < a.ncol;
      const int64_t colc = live ? col : 0;
      const int Q = (int)(colc / a.nx);
      const int P = (int)(colc - (int64_t)Q * a.nx);
      const double kx = (double)(P - a.nx / 2) * a.dkx;
      const double ky = (double)(Q - a.ny / 2) * a.dky;
      const double kp2 = kx * kx + ky * ky;
      const float2* __restrict__ sp = a.spec + colc * a.nf;
      float2 acc = make_float2(0.f, 0.f);
      for (int i = gl; i < a.nf; i += G) {
        const double k = a.k[i];
        const double kz2 = 4.0 * k * k - kp2;
        if (kz2 <= 0.0) continue;
        const double kz = sqrt(kz2);
        const float2 v = cmul(sp[i], cis_cycles(kz * a.z_cyc));
        const float wf = a.dcf ? (float)(4.0 * k) : (float)kz;
        acc.x = fmaf(v.x, wf, acc.x);
        acc.y = fmaf(v.y, wf, acc.y);
      }
#pragma unroll
      for (int m = G / 2; m >= 1; m >>= 1) {
        acc.x += __shfl_xor(acc.x, m, G);
        acc.y += __shfl_xor(acc.y, m, G);
      }
      if (live && gl == 0) {
        const float sgn = (((P & a.sgx) ^ (Q & a.sgy)) & 1) ? -1.f : 1.f;
        a.zc[colc] = make_float2(sgn * acc.x, sgn * acc.y);
      }
    }
  }
};

template <int MZ>
sar_status stolt_mz(const Plan& p, const StoltArgs& a, LaunchSink& sink) {
  // one-wavefront blocks (the LDS of 4 columns each, so 9 fit a CU), many
  // more than fit at once: each takes about two column groups, and the
  // hardware queue balances the uneven work of central and evanescent columns
  const int64_t ngroups = (a.ncol + kCols - 1) / kCols;
  const int64_t nblk = ngroups < 256 * 72 ? ngroups : 256 * 72;
  const bool f32 = (p.flags & SAR_FP32_ARGS) != 0;
  // the compiled tap polynomials are fitted for beta = 2.30 WZ
  if (!((p.wz == 6 && p.es_beta == EsPoly<6>::kBeta) || (p.wz == 8 && p.es_beta == EsPoly<8>::kBeta)))
    return fail(SAR_ERR_UNSUPPORTED, "Stolt kernel shape not compiled");
  switch (p.wz) {
    case 6:
      return f32 ? launch_body<StoltBody<MZ, 6, true>>(sink, (uint32_t)nblk, 0, a, "stolt launch")
                 : launch_body<StoltBody<MZ, 6, false>>(sink, (uint32_t)nblk, 0, a, "stolt launch");
    case 8:
      return f32 ? launch_body<StoltBody<MZ, 8, true>>(sink, (uint32_t)nblk, 0, a, "stolt launch")
                 : launch_body<StoltBody<MZ, 8, false>>(sink, (uint32_t)nblk, 0, a, "stolt launch");
    default: return fail(SAR_ERR_UNSUPPORTED, "Stolt kernel width not compiled");
  }
}

}  // namespace

sar_status launch_stolt(const Plan& p, const float2* spec, float2* zcube, LaunchSink& sink) {
  if (p.nz == 1) {
    PlaneArgs b;
    b.spec = spec;
    b.zc = zcube;
    b.k = p.d_k;
    b.nx = p.nx;
    b.ny = p.ny;
    b.nf = p.nf;
    b.dkx = 2.0 * M_PI / (p.nx * p.dx);
    b.dky = 2.0 * M_PI / (p.ny * p.dy);
    b.z_cyc = (p.z0 - p.z_ref) / (2.0 * M_PI);
    b.dcf = (p.flags & SAR_STOLT_DCF) ? 1 : 0;
    b.sgx = (p.nx & 1) ? 0 : 1;
    b.sgy = (p.ny & 1) ? 0 : 1;
    b.ncol = (int64_t)p.nx * p.ny;
    const int64_t ngroups = (b.ncol + 15) / 16;
    const int64_t nblk = ngroups < 256 * 8 ? ngroups : 256 * 8;
    return launch_body<PlaneBody>(sink, (uint32_t)nblk, 0, b, "plane launch");
  }
  StoltArgs a;
  a.spec = spec;
  a.zc = zcube;
  a.k = p.d_k;
  a.deapz = p.d_deapz;
  a.tw = p.d_tw_mz;
  a.nx = p.nx;
  a.ny = p.ny;
  a.nf = p.nf;
  a.nz = p.nz;
  a.dkx = 2.0 * M_PI / (p.nx * p.dx);
  a.dky = 2.0 * M_PI / (p.ny * p.dy);
  const double zmid = p.z0 + (p.nz / 2) * p.dz;
  a.zmid_minus_zref_cyc = (zmid - p.z_ref) / (2.0 * M_PI);
  a.dz_cells = p.dz * p.mz / (2.0 * M_PI);
  a.dcf = (p.flags & SAR_STOLT_DCF) ? 1 : 0;
  a.sgx = (p.nx & 1) ? 0 : 1;
  a.sgy = (p.ny & 1) ? 0 : 1;
  a.ncol = (int64_t)p.nx * p.ny;
  if (a.ncol == 0) return SAR_OK;
  switch (p.mz) {
    case 64: return stolt_mz<64>(p, a, sink);
    case 128: return stolt_mz<128>(p, a, sink);
    case 256: return stolt_mz<256>(p, a, sink);
    case 512: return stolt_mz<512>(p, a, sink);
    case 1024: return stolt_mz<1024>(p, a, sink);
    default: return fail(SAR_ERR_UNSUPPORTED, "Stolt grid size not supported");
  }
}

}  // namespace sar

// Steps a4 + a5: range-migration filter and Stolt map with the z transform.
//
// For every (k_x, k_y) column of the spectrum, each frequency sample f_i
// becomes a non-uniform sample at k_z = sqrt(4 k_i^2 - k_x^2 - k_y^2)
// (Eq. (14); evanescent samples are dropped) with value
// S k_z exp(-j k_z Z_0) (Eq. (15), P = 1).  The Stolt map plus the inverse
// transform along z is the non-uniform sum
//   Z(z_w) = sum_i F_i exp(+j k_z,i z_w),  z_w = z0 + w dz,
// a 1-D type-1 NUFFT at the positions theta_i = k_z,i dz.  Each column is
// handled by one wavefront: float64 pre-phase exp(j k_z (z_mid - Z_0)) and
// grid position, exponential-of-semicircle spreading into an oversampled LDS
// grid of MZ cells, an inverse radix-4 Stockham FFT in LDS, and
// deapodisation of the nz centred outputs.  The +-1 factor (-1)^(P+Q) that
// lets the next step use plain inverse DFTs on centred mode indices is
// folded in here.

#include "device_common.hpp"
#include "sar_internal.hpp"

namespace sar {
namespace {

constexpr int kWaves = 4;

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
  float es_beta;
  int64_t ncol;
};

// Stockham autosort FFT (sign +) of n = MZ points held in LDS, executed by
// the 64 lanes of one wavefront; returns the buffer holding the result.
template <int MZ>
__device__ float2* wave_ifft(float2* x, float2* y, const float2* __restrict__ tw, int lane) {
  constexpr int LOG = ct_log2(MZ);
  int ns = 1;
  if constexpr (LOG & 1) {  // one radix-2 stage first
    for (int j = lane; j < MZ / 2; j += 64) {
      const float2 a0 = x[j], a1 = x[j + MZ / 2];
      y[2 * j] = cadd(a0, a1);
      y[2 * j + 1] = csub(a0, a1);
    }
    __syncthreads();
    float2* t = x;
    x = y;
    y = t;
    ns = 2;
  }
  for (; ns < MZ; ns *= 4) {
    for (int j = lane; j < MZ / 4; j += 64) {
      const int k = j & (ns - 1);
      const int step = MZ / (4 * ns);
      const float2 w1 = tw[k * step];
      const float2 w2 = tw[2 * k * step];
      const float2 w3 = tw[3 * k * step];
      const float2 a0 = x[j];
      const float2 a1 = cmul(x[j + MZ / 4], w1);
      const float2 a2 = cmul(x[j + MZ / 2], w2);
      const float2 a3 = cmul(x[j + 3 * MZ / 4], w3);
      const float2 b0 = cadd(a0, a2), b1 = csub(a0, a2), b2 = cadd(a1, a3);
      const float2 d = csub(a1, a3);
      const float2 b3 = make_float2(-d.y, d.x);  // +j (a1 - a3)
      const int base = (j / ns) * 4 * ns + k;
      y[base] = cadd(b0, b2);
      y[base + ns] = cadd(b1, b3);
      y[base + 2 * ns] = csub(b0, b2);
      y[base + 3 * ns] = csub(b1, b3);
    }
    __syncthreads();
    float2* t = x;
    x = y;
    y = t;
  }
  return x;
}

template <int MZ, int WZ>
__global__ __launch_bounds__(64 * kWaves) void k_stolt(StoltArgs a) {
  __shared__ float2 buf[kWaves][2][MZ];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t col = (int64_t)blockIdx.x * kWaves + wave;
  const bool live = col < a.ncol;
  const int64_t colc = live ? col : 0;
  const int Q = (int)(colc / a.nx);
  const int P = (int)(colc - (int64_t)Q * a.nx);
  float2* g0 = buf[wave][0];
  float2* g1 = buf[wave][1];
  for (int c = lane; c < MZ; c += 64) g0[c] = make_float2(0.f, 0.f);
  __syncthreads();

  if (live) {
    const double kx = (double)(P - a.nx / 2) * a.dkx;
    const double ky = (double)(Q - a.ny / 2) * a.dky;
    const double kp2 = kx * kx + ky * ky;
    const float sgn = ((P + Q) & 1) ? -1.f : 1.f;
    const float2* __restrict__ sp = a.spec + colc * a.nf;
    // lane l takes a contiguous run of frequencies so that lanes of one
    // instruction land on different cells of the (monotone) k_z axis
    const int per = (a.nf + 63) / 64;
    for (int r = 0; r < per; ++r) {
      const int i = lane * per + r;
      if (i >= a.nf) break;
      const double k = a.k[i];
      const double kz2 = 4.0 * k * k - kp2;
      if (kz2 <= 0.0) continue;
      const double kz = sqrt(kz2);
      const float2 s = sp[i];
      const float2 ph = cis_cycles(kz * a.zmid_minus_zref_cyc);
      const float2 v = cscale(cmul(s, ph), (float)kz * sgn);
      double g = kz * a.dz_cells;
      g -= floor(g / (double)MZ) * (double)MZ;
      const int c0 = (int)floor(g - 0.5 * WZ) + 1;
      const float d0 = (float)((double)c0 - g);
#pragma unroll
      for (int j = 0; j < WZ; ++j) {
        const float z = 2.f * (d0 + (float)j) / (float)WZ;
        const float q = 1.f - z * z;
        const float wgt = q > 0.f ? __expf(a.es_beta * (__builtin_sqrtf(q) - 1.f)) : 0.f;
        const int c = (c0 + j) & (MZ - 1);
        atomicAdd(&g0[c].x, v.x * wgt);
        atomicAdd(&g0[c].y, v.y * wgt);
      }
    }
  }
  __syncthreads();
  const float2* res = wave_ifft<MZ>(g0, g1, a.tw, lane);
  if (live) {
    float2* __restrict__ out = a.zc + colc * a.nz;
    for (int w = lane; w < a.nz; w += 64) {
      const int m = w - a.nz / 2;
      out[w] = cscale(res[m & (MZ - 1)], a.deapz[w]);
    }
  }
}

template <int MZ>
sar_status stolt_mz(const Plan& p, const StoltArgs& a, hipStream_t stream) {
  const int64_t nblk = (a.ncol + kWaves - 1) / kWaves;
  switch (p.wz) {
    case 6: k_stolt<MZ, 6><<<(unsigned)nblk, 64 * kWaves, 0, stream>>>(a); break;
    case 8: k_stolt<MZ, 8><<<(unsigned)nblk, 64 * kWaves, 0, stream>>>(a); break;
    default: return fail(SAR_ERR_UNSUPPORTED, "Stolt kernel width not compiled");
  }
  return check_hip(hipGetLastError(), "stolt launch");
}

}  // namespace

sar_status launch_stolt(const Plan& p, const float2* spec, float2* zcube, hipStream_t stream) {
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
  a.es_beta = (float)p.es_beta;
  a.ncol = (int64_t)p.nx * p.ny;
  if (a.ncol == 0) return SAR_OK;
  switch (p.mz) {
    case 64: return stolt_mz<64>(p, a, stream);
    case 128: return stolt_mz<128>(p, a, stream);
    case 256: return stolt_mz<256>(p, a, stream);
    case 512: return stolt_mz<512>(p, a, stream);
    case 1024: return stolt_mz<1024>(p, a, stream);
    case 2048: return stolt_mz<2048>(p, a, stream);
    default: return fail(SAR_ERR_UNSUPPORTED, "Stolt grid size not supported");
  }
}

}  // namespace sar

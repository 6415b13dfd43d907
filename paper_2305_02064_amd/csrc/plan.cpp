// Plan construction: descriptor validation, NUFFT parameters, float64 tables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <string>
#include <vector>

#include "sar_internal.hpp"

namespace sar {

namespace {

constexpr double kC0 = 299792458.0;

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int next_pow2(int64_t v) {
  int r = 1;
  while (r < v) r <<= 1;
  return r;
}
// oversampled lateral grid: the smallest multiple of 8 cells (whole gridding
// tiles) of the form 2^a 3^b 5^c (a transform length) at or above sigma * n,
// or the next power of two when that is at most 1/8 longer (the power-of-two
// transforms run two to four times faster than the mixed-radix ones)
int grid_length(int n, double sigma) {
  int64_t m = (int64_t)std::ceil(sigma * n - 1e-9);
  m = (m + 7) / 8 * 8;
  while (!is_5smooth(m)) m += 8;
  const int64_t p2 = next_pow2(m);
  return (int)(8 * p2 <= 9 * m ? p2 : m);
}

// Automatic oversampling (upsample 0): a power of two between 1.5 n and 2 n
// if there is one (the radix-2 transforms are the fastest, and oversampling
// 1.5-2 needs at most one more kernel tap than 2), else the grid of
// oversampling 2.
int grid_length_auto(int n) {
  const int64_t p2 = next_pow2((int64_t)std::ceil(1.5 * n - 1e-9));
  return p2 <= 2 * (int64_t)n ? (int)p2 : grid_length(n, 2.0);
}

double bessel_i0_host(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 200; ++k) {
    term *= q / ((double)k * (double)k);
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on the three-term
// recurrence of the Legendre polynomials).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_n(z), p0 = P_{n-1}(z)
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Fourier transform of a symmetric kernel supported on [-W/2, W/2]:
//   phi_hat(p) = int phi(x) cos(2 pi p x / M) dx,
// by Gauss-Legendre quadrature after x = (W/2) sin(theta), which removes the
// square-root behaviour of the kernels at the support edge.
template <typename K>
std::vector<double> kernel_ft(const K& phi, int W, int M, int n_modes) {
  std::vector<double> gx, gw;
  gauss_legendre(256, gx, gw);
  std::vector<double> out(n_modes);
  for (int j = 0; j < n_modes; ++j) {
    const double p = (double)(j - n_modes / 2);
    double s = 0.0;
    for (size_t i = 0; i < gx.size(); ++i) {
      const double th = 0.5 * M_PI * gx[i];
      const double x = 0.5 * W * std::sin(th);
      s += gw[i] * phi(x) * std::cos(2.0 * M_PI * p * x / M) * 0.5 * W * std::cos(th);
    }
    out[j] = s * 0.5 * M_PI;
  }
  return out;
}

template <typename T>
sar_status upload(T** dst, const std::vector<T>& v) {
  if (v.empty()) {
    *dst = nullptr;
    return SAR_OK;
  }
  hipError_t e = hipMalloc((void**)dst, v.size() * sizeof(T));
  if (e != hipSuccess) return fail(SAR_ERR_NOMEM, "hipMalloc for plan tables failed");
  e = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return check_hip(e, "plan table upload");
}

std::vector<float2> twiddles(int n, int sign) {
  std::vector<float2> t(n);
  for (int i = 0; i < n; ++i) {
    const double a = sign * 2.0 * M_PI * (double)i / (double)n;
    t[i] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  return t;
}

bool finite(double v) { return std::isfinite(v); }

}  // namespace

// relative L2 error of the lateral NUFFT with a width-W Kaiser-Bessel kernel at
// oversampling sigma: exp(-pi W sqrt(1 - 1/sigma)) times 5, the factor measured
// for widths 3..7 at sigma = 2 against the direct sum
double nufft_error_estimate(int W, double sigma) {
  return 5.0 * std::exp(-M_PI * W * std::sqrt(1.0 - 1.0 / sigma));
}

// Lateral NUFFT parameters for oversampling `up` (host only): grid sizes, the
// kernel width from the plan's tolerance (unless the descriptor fixed it), the
// Kaiser-Bessel shape and the default gridding tile.
sar_status choose_lateral(Plan& p, double up) {
  const int mx = up > 0 ? grid_length(p.nx, up) : grid_length_auto(p.nx);
  const int my = up > 0 ? grid_length(p.ny, up) : grid_length_auto(p.ny);
  if (mx > kMaxFftLength || my > kMaxFftLength)
    return fail(SAR_ERR_UNSUPPORTED, "oversampled grid of " + std::to_string(mx) + " x " + std::to_string(my) +
                                         " cells: at most " + std::to_string(kMaxFftLength) + " per axis");
  p.mx = mx;
  p.my = my;
  const double sigma = std::min((double)p.mx / p.nx, (double)p.my / p.ny);
  if (p.kw_req > 0) {
    p.w = p.kw_req;
  } else {
    p.w = kMaxWidth;
    for (int w = 3; w <= kMaxWidth; ++w)
      if (nufft_error_estimate(w, sigma) <= p.tol) {
        p.w = w;
        break;
      }
  }
  if ((p.flags & SAR_FP32_ARGS) && (p.w != 4 || p.echo_type != SAR_ECHO_C64))
    return fail(SAR_ERR_UNSUPPORTED, "SAR_FP32_ARGS is compiled for complex64 echo and a 4-tap lateral kernel");
  // shape parameter of Beatty, Nishimura and Pauly (2005)
  const double a = (p.w / sigma) * (sigma - 0.5);
  p.kb_beta = M_PI * std::sqrt(std::max(a * a - 0.8, 1e-6));
  // gridding tile: one frequency per lane when the sweep has at most 64
  // frequencies (two per lane would leave half the lanes idle), else the
  // four-wave union (kernels of up to 5 taps) or the 4 x 4 tile; the
  // autotuner may change it by timing
  if (p.nf <= 64 && grid_tile_compiled(1, p.w))
    p.grid_tile = 1;
  else
    p.grid_tile = grid_tile_compiled(3, p.w) ? 3 : 0;
  return SAR_OK;
}

// Device tables of the lateral NUFFT (deapodisation, grid twiddles) for the
// plan's current mx, my, w; replaces earlier ones.  The plan's device must be
// current.
sar_status upload_lateral(Plan& p) {
  const double kb_norm = 1.0 / bessel_i0_host(p.kb_beta);
  const int W = p.w;
  const double kbb = p.kb_beta;
  auto kb = [W, kbb, kb_norm](double x) {
    const double z = 2.0 * x / W;
    const double r = 1.0 - z * z;
    return r > 0 ? bessel_i0_host(kbb * std::sqrt(r)) * kb_norm : 0.0;
  };
  const std::vector<double> fx = kernel_ft(kb, W, p.mx, p.nx);
  const std::vector<double> fy = kernel_ft(kb, W, p.my, p.ny);
  std::vector<float> deapx(p.nx), deapy(p.ny);
  for (int i = 0; i < p.nx; ++i) deapx[i] = (float)(1.0 / fx[i]);
  for (int i = 0; i < p.ny; ++i) deapy[i] = (float)(1.0 / fy[i]);
  void* old[] = {p.d_deapx, p.d_deapy, p.d_tw_mx, p.d_tw_my};
  for (void* q : old)
    if (q) (void)hipFree(q);
  p.d_deapx = p.d_deapy = nullptr;
  p.d_tw_mx = p.d_tw_my = nullptr;
  sar_status st;
  if ((st = upload(&p.d_deapx, deapx)) != SAR_OK) return st;
  if ((st = upload(&p.d_deapy, deapy)) != SAR_OK) return st;
  if ((st = upload(&p.d_tw_mx, twiddles(p.mx, -1))) != SAR_OK) return st;
  return upload(&p.d_tw_my, twiddles(p.my, -1));
}

// ---- tuning file: oversampling and gridding tile per size bucket ----------
// With SAR_AUTOTUNE_FILE naming a file, sar_plan_autotune records its choice
// for the plan's bucket (image size, sweep length, pair count, echo type,
// flags, tolerance, shots rounded up to a power of two) and plans created
// later with upsample = 0 start from it.  One "key = sigma tile" line each.
std::string tuning_key(const Plan& p, int64_t n_pos) {
  int b = 0;
  while (((int64_t)1 << b) < std::max<int64_t>(n_pos, 1)) ++b;
  char buf[256];
  std::snprintf(buf, sizeof(buf), "n%dx%dx%d f%d p%d e%d fl%u tol%.3g pos2^%d", p.nx, p.ny, p.nz, p.nf, p.n_pair,
                p.echo_type, p.flags, p.tol, b);
  return buf;
}

std::mutex g_tuning_mu;

bool tuning_lookup(const Plan& p, double* sigma, int* tile) {
  const char* path = std::getenv("SAR_AUTOTUNE_FILE");
  if (!path || !*path) return false;
  const std::string key = tuning_key(p, p.max_pos);
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    const size_t eq = line.find(" = ");
    if (eq == std::string::npos || line.compare(0, eq, key) != 0 || eq != key.size()) continue;
    double sg = 0;
    int t = -1;
    if (std::sscanf(line.c_str() + eq + 3, "%lf %d", &sg, &t) == 2 &&
        (sg == 0 || (sg >= kMinUpsample && sg <= 4))) {  // 0: the automatic choice
      *sigma = sg;
      *tile = t;
      found = true;  // the last entry for a key wins
    }
  }
  return found;
}

void tuning_store(const Plan& p, int64_t n_pos, double sigma, int tile) {
  const char* path = std::getenv("SAR_AUTOTUNE_FILE");
  if (!path || !*path) return;
  const std::string key = tuning_key(p, n_pos);
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  std::vector<std::string> keep;
  {
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line))
      if (line.compare(0, key.size() + 3, key + " = ") != 0) keep.push_back(line);
  }
  char val[64];
  std::snprintf(val, sizeof(val), "%.6g %d", sigma, tile);
  keep.push_back(key + " = " + val);
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream o(tmp, std::ios::trunc);
    for (const auto& l : keep) o << l << "\n";
  }
  std::rename(tmp.c_str(), path);
}

sar_status validate_desc(const sar_plan_desc* d) {
  if (!d) return fail(SAR_ERR_INVALID, "descriptor is NULL");
  if (d->n_tx < 1 || d->n_rx < 1 || !d->tx_xy || !d->rx_xy) return fail(SAR_ERR_INVALID, "array layout missing");
  if ((int64_t)d->n_tx * d->n_rx > 4096) return fail(SAR_ERR_INVALID, "too many Tx/Rx pairs");
  for (int i = 0; i < 2 * d->n_tx; ++i)
    if (!finite(d->tx_xy[i])) return fail(SAR_ERR_INVALID, "non-finite Tx offset");
  for (int i = 0; i < 2 * d->n_rx; ++i)
    if (!finite(d->rx_xy[i])) return fail(SAR_ERR_INVALID, "non-finite Rx offset");
  if (d->n_freq < 1 || !d->freq_hz) return fail(SAR_ERR_INVALID, "frequency sweep missing");
  for (int i = 0; i < d->n_freq; ++i) {
    if (!finite(d->freq_hz[i]) || d->freq_hz[i] <= 0) return fail(SAR_ERR_INVALID, "frequency must be finite and > 0");
    if (i > 0 && !(d->freq_hz[i] > d->freq_hz[i - 1]))
      return fail(SAR_ERR_INVALID, "frequencies must be strictly increasing");
  }
  auto okn = [](int v, int lo, int hi) { return v >= lo && v <= hi && is_pow2(v); };
  auto ok5 = [](int v, int lo, int hi) { return v >= lo && v <= hi && is_5smooth(v); };
  if (!ok5(d->nx, 8, 2048) || !ok5(d->ny, 8, 2048))
    return fail(SAR_ERR_INVALID, "nx, ny must be in [8, 2048] and products of 2, 3 and 5");
  if (d->nz != 1 && !okn(d->nz, 2, 512))
    return fail(SAR_ERR_INVALID, "nz must be 1 (one plane) or a power of two in [2, 512]");
  const double g[] = {d->x0, d->y0, d->z0, d->dx, d->dy, d->dz, d->z_ref, d->z_focus};
  for (double v : g)
    if (!finite(v)) return fail(SAR_ERR_INVALID, "non-finite grid or plane");
  if (!(d->dx > 0 && d->dy > 0 && d->dz > 0)) return fail(SAR_ERR_INVALID, "voxel pitch must be > 0");
  if (!(d->z_focus > d->z_ref)) return fail(SAR_ERR_INVALID, "z_focus must lie in front of z_ref (z_focus > z_ref)");
  if (!(d->z0 > d->z_ref)) return fail(SAR_ERR_INVALID, "image volume must lie in front of z_ref (z0 > z_ref)");
  if (d->max_pos < 0) return fail(SAR_ERR_INVALID, "max_pos must be >= 0");
  if (d->max_pos * (int64_t)d->n_tx * d->n_rx > 0x7fffffffLL)
    return fail(SAR_ERR_INVALID, "max_pos * n_pair exceeds 2^31 - 1");
  if (d->echo_type != SAR_ECHO_C64 && d->echo_type != SAR_ECHO_F16X2)
    return fail(SAR_ERR_INVALID, "unknown echo type");
  if (!(d->tol == 0 || (d->tol > 0 && d->tol <= 0.1))) return fail(SAR_ERR_INVALID, "tol must be 0 or in (0, 0.1]");
  if (!(d->upsample == 0 || (d->upsample >= kMinUpsample && d->upsample <= 4)))
    return fail(SAR_ERR_UNSUPPORTED, "upsample must be 0 or in [1.25, 4]");
  if (!(d->kernel_width == 0 || (d->kernel_width >= 3 && d->kernel_width <= kMaxWidth)))
    return fail(SAR_ERR_INVALID, "kernel_width must be 0 or 3..8");
  if (d->flags & ~(SAR_NO_COMPENSATION | SAR_FP32_ARGS | SAR_STOLT_DCF | SAR_AMPLITUDE))
    return fail(SAR_ERR_INVALID, "unknown flag bits");
  if ((d->flags & SAR_FP32_ARGS) && (d->echo_type != SAR_ECHO_C64 || (d->kernel_width != 0 && d->kernel_width != 4)))
    return fail(SAR_ERR_UNSUPPORTED, "SAR_FP32_ARGS is compiled for complex64 echo and a 4-tap lateral kernel");
  if (!(d->n_slabs == 0 || d->n_slabs == 1 || (d->n_slabs > 1 && is_pow2(d->n_slabs) && d->n_slabs <= d->nz)))
    return fail(SAR_ERR_INVALID, "n_slabs must be 0, 1 or a power of two that divides nz");
  return SAR_OK;
}

sar_status build_plan(const sar_plan_desc* d, int device, Plan& p) {
  sar_status st = validate_desc(d);
  if (st != SAR_OK) return st;
  p.device = device;
  p.n_tx = d->n_tx;
  p.n_rx = d->n_rx;
  p.n_pair = d->n_tx * d->n_rx;
  p.nf = d->n_freq;
  p.tx_xy.assign(d->tx_xy, d->tx_xy + 2 * d->n_tx);
  p.rx_xy.assign(d->rx_xy, d->rx_xy + 2 * d->n_rx);
  p.freq.assign(d->freq_hz, d->freq_hz + d->n_freq);
  p.z_ref = d->z_ref;
  p.z_focus = d->z_focus;
  p.nx = d->nx;
  p.ny = d->ny;
  p.nz = d->nz;
  p.out_w0 = 0;
  p.out_nz = d->nz;
  p.x0 = d->x0;
  p.y0 = d->y0;
  p.z0 = d->z0;
  p.dx = d->dx;
  p.dy = d->dy;
  p.dz = d->dz;
  p.max_pos = d->max_pos;
  p.echo_type = d->echo_type;
  p.tol = d->tol > 0 ? d->tol : 1e-3;
  p.flags = d->flags;
  p.xc = p.x0 + (p.nx / 2) * p.dx;
  p.yc = p.y0 + (p.ny / 2) * p.dy;

  // lateral NUFFT: the requested oversampling, else the one tuned for this
  // plan's size bucket (sar_plan_autotune with a tuning file), else the
  // automatic choice (up = 0, grid_length_auto)
  p.up_req = d->upsample;
  p.kw_req = d->kernel_width;
  double up = d->upsample > 0 ? d->upsample : 0.0;
  int tuned_tile = -1;
  if (d->upsample == 0 && d->n_slabs <= 1) {
    double tuned_up = 0;
    if (tuning_lookup(p, &tuned_up, &tuned_tile)) up = tuned_up;
  }
  if ((st = choose_lateral(p, up)) != SAR_OK) return st;
  if (tuned_tile >= 0 && grid_tile_compiled(tuned_tile, p.w)) p.grid_tile = tuned_tile;
  // Stolt NUFFT: oversampled LDS grid, exponential-of-semicircle kernel
  p.mz = std::max(64, next_pow2(2 * (int64_t)p.nz));  // 64 .. 1024 cells
  p.wz = p.tol < 1e-5 ? 8 : 6;
  p.es_beta = 2.30 * p.wz;

  if (p.flags & SAR_NO_COMPENSATION) {
    p.beta_sign = 0.0;
    p.inv4rc = 0.0;
  } else {
    p.beta_sign = 2.0 * (p.z_ref > p.z_focus ? 1.0 : -1.0);
    p.inv4rc = 1.0 / (4.0 * std::fabs(p.z_focus - p.z_ref));
  }
  // amplitude half: (|d|^2 / 4 + (z_c - z_l)^2) / (z_c - Z_0)^2, the |d|^2 / 4
  // per pair in the pair table
  p.amp_inv_r2 = (p.flags & SAR_AMPLITUDE) ? 1.0 / ((p.z_focus - p.z_ref) * (p.z_focus - p.z_ref)) : 0.0;

  // ---- tables ----
  std::vector<double> fcc(p.nf), kk(p.nf);
  for (int i = 0; i < p.nf; ++i) {
    fcc[i] = p.freq[i] / kC0;
    kk[i] = 2.0 * M_PI * p.freq[i] / kC0;
  }
  std::vector<double> pair(4 * (size_t)p.n_pair);
  for (int t = 0; t < p.n_tx; ++t)
    for (int r = 0; r < p.n_rx; ++r) {
      const int l = t * p.n_rx + r;
      const double ox = 0.5 * (p.tx_xy[2 * t] + p.rx_xy[2 * r]);
      const double oy = 0.5 * (p.tx_xy[2 * t + 1] + p.rx_xy[2 * r + 1]);
      const double sx = p.rx_xy[2 * r] - p.tx_xy[2 * t];
      const double sy = p.rx_xy[2 * r + 1] - p.tx_xy[2 * t + 1];
      pair[4 * l + 0] = ox;
      pair[4 * l + 1] = oy;
      pair[4 * l + 2] = (sx * sx + sy * sy) * p.inv4rc;
      pair[4 * l + 3] = 0.25 * (sx * sx + sy * sy);
    }
  const int WZ = p.wz;
  const double esb = p.es_beta;
  auto es = [WZ, esb](double x) {
    const double z = 2.0 * x / WZ;
    const double r = 1.0 - z * z;
    return r > 0 ? std::exp(esb * (std::sqrt(r) - 1.0)) : 0.0;
  };
  const std::vector<double> fz = kernel_ft(es, WZ, p.mz, p.nz);
  std::vector<float> deapz(p.nz), signx(p.nx), signy(p.ny);
  for (int i = 0; i < p.nx; ++i) signx[i] = ((i + p.nx / 2) & 1) ? -1.f : 1.f;
  for (int i = 0; i < p.ny; ++i) signy[i] = ((i + p.ny / 2) & 1) ? -1.f : 1.f;
  // odd sides: the inverse transform of centred modes P = p + h (h = n / 2)
  // at voxel u is exp(-j 2 pi h (u - h) / n) times the plain inverse DFT at
  // (u - h) mod n; the factor in float64, rounded once
  auto post = [](int n) {
    std::vector<float2> t(n);
    const int h = n / 2;
    for (int u = 0; u < n; ++u) {
      const int64_t e = ((int64_t)h * (u - h)) % n;
      const double ang = -2.0 * M_PI * (double)e / (double)n;
      t[u] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    return t;
  };
  for (int i = 0; i < p.nz; ++i) deapz[i] = (float)(1.0 / fz[i]);

  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return check_hip(e, "hipSetDevice");
  if ((st = upload(&p.d_fcc, fcc)) != SAR_OK) return st;
  if ((st = upload(&p.d_k, kk)) != SAR_OK) return st;
  if ((st = upload(&p.d_pair, pair)) != SAR_OK) return st;
  {
    // Tx and Rx offsets per pair for back-projection with exact ranges
    std::vector<double> txrx(4 * (size_t)p.n_pair);
    for (int t = 0; t < p.n_tx; ++t)
      for (int r = 0; r < p.n_rx; ++r) {
        const int l = t * p.n_rx + r;
        txrx[4 * l + 0] = p.tx_xy[2 * t];
        txrx[4 * l + 1] = p.tx_xy[2 * t + 1];
        txrx[4 * l + 2] = p.rx_xy[2 * r];
        txrx[4 * l + 3] = p.rx_xy[2 * r + 1];
      }
    if ((st = upload(&p.d_txrx, txrx)) != SAR_OK) return st;
  }
  if ((st = upload_lateral(p)) != SAR_OK) return st;
  if ((st = upload(&p.d_deapz, deapz)) != SAR_OK) return st;
  if ((st = upload(&p.d_signx, signx)) != SAR_OK) return st;
  if ((st = upload(&p.d_signy, signy)) != SAR_OK) return st;
  if ((p.nx & 1) && (st = upload(&p.d_postx, post(p.nx))) != SAR_OK) return st;
  if ((p.ny & 1) && (st = upload(&p.d_posty, post(p.ny))) != SAR_OK) return st;
  if ((st = upload(&p.d_tw_nx, twiddles(p.nx, +1))) != SAR_OK) return st;
  if ((st = upload(&p.d_tw_ny, twiddles(p.ny, +1))) != SAR_OK) return st;
  if ((st = upload(&p.d_tw_mz, twiddles(p.mz, +1))) != SAR_OK) return st;

  // depth slabs: slab j covers planes [j n, (j + 1) n), n = nz / S, and takes
  // the z-centre of its planes as reference depth
  if (d->n_slabs > 1) {
    const int n = d->nz / d->n_slabs;
    for (int j = 0; j < d->n_slabs; ++j) {
      sar_plan_desc dj = *d;
      dj.n_slabs = 0;
      dj.nz = n;
      dj.z0 = d->z0 + (double)j * n * d->dz;
      dj.z_focus = dj.z0 + 0.5 * (n - 1) * d->dz;
      std::unique_ptr<Plan> sub(new (std::nothrow) Plan());
      if (!sub) return fail(SAR_ERR_NOMEM, "host allocation failed");
      st = build_plan(&dj, device, *sub);
      sub->out_w0 = j * n;
      sub->out_nz = d->nz;
      p.slabs.push_back(std::move(sub));  // freed with the plan, also after a failure
      if (st != SAR_OK) return st;
    }
  }
  return SAR_OK;
}

void free_plan(Plan& p) {
  for (auto& sub : p.slabs) free_plan(*sub);
  p.slabs.clear();
  void* ptrs[] = {p.d_fcc, p.d_k, p.d_pair, p.d_txrx, p.d_deapx, p.d_deapy, p.d_deapz, p.d_signx,
                  p.d_signy, p.d_postx, p.d_posty, p.d_tw_mx, p.d_tw_my, p.d_tw_nx, p.d_tw_ny, p.d_tw_mz};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  for (hipEvent_t ev : p.events) (void)hipEventDestroy(ev);
  p.events.clear();
}

size_t rec_bytes(int W) {
  switch (W) {
    case 3: return sizeof(SampleRec<3>);
    case 4: return sizeof(SampleRec<4>);
    case 5: return sizeof(SampleRec<5>);
    case 6: return sizeof(SampleRec<6>);
    case 7: return sizeof(SampleRec<7>);
    default: return sizeof(SampleRec<8>);
  }
}

// Workspace layout; with base != nullptr also fills the pointers.
size_t workspace_bytes(const Plan& p, int64_t n_pos, Workspace* ws, char* base) {
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const int64_t n_v = n_pos * p.n_pair;
  const int64_t ncell = (int64_t)p.mx * p.my;
  const int64_t nscan = (ncell + 4095) / 4096;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = al(off + bytes);
    return o;
  };
  // radix sort: up to 2^11 digit counts per tile of 4096 samples, scanned in place
  const int64_t nhist = 2048 * ((n_v + 4095) / 4096);
  const size_t o_cell = take((size_t)(ncell + 1 + nscan) * 4);
  const size_t o_key = take((size_t)n_v * 4);
  const size_t o_key2 = take((size_t)n_v * 4);
  const size_t o_order = take((size_t)n_v * 4);
  const size_t o_order2 = take((size_t)n_v * 4);
  const size_t o_hist = take((size_t)(nhist + 1 + (nhist + 4095) / 4096) * 4);
  const size_t o_rec = take((size_t)n_v * rec_bytes(p.w));
  // over-full unions (four-wave gridding kernel): counter, per-union first
  // slot, slot list, partial grids
  const bool split = grid_tile_compiled(3, p.w);
  const int nslot = split ? union_slots(n_v) : 0;
  const int64_t nunion = split ? (int64_t)(p.mx / 8) * (p.my / 8) : 0;
  const size_t o_cnt = take(split ? 4 : 0);
  const size_t o_uofs = take((size_t)nunion * 4);
  const size_t o_slots = take((size_t)nslot * 8);
  const size_t o_part = take((size_t)nslot * 64 * p.nf * sizeof(float2));
  const int64_t a_elems = std::max((int64_t)p.mx * p.my * p.nf, (int64_t)p.nx * p.ny * p.nz);
  const int64_t b_elems = std::max((int64_t)p.my * p.nx * p.nf, (int64_t)p.nx * p.ny * p.nz);
  const size_t o_a = take((size_t)a_elems * sizeof(float2));
  const size_t o_b = take((size_t)b_elems * sizeof(float2));
  if (ws && base) {
    ws->cell_start = (int32_t*)(base + o_cell);
    ws->key = (int32_t*)(base + o_key);
    ws->key_alt = (int32_t*)(base + o_key2);
    ws->order = (int32_t*)(base + o_order);
    ws->order_alt = (int32_t*)(base + o_order2);
    ws->hist = (int32_t*)(base + o_hist);
    ws->split_count = split ? (int32_t*)(base + o_cnt) : nullptr;
    ws->uofs = (int32_t*)(base + o_uofs);
    ws->slots = (int32_t*)(base + o_slots);
    ws->partial = (float2*)(base + o_part);
    ws->rec = (void*)(base + o_rec);
    ws->region_a = (float2*)(base + o_a);
    ws->region_b = (float2*)(base + o_b);
  }
  // the launch structure follows the slot count, also when a batch describes
  // its launches without buffers
  if (ws) ws->max_slots = nslot;
  return off;
}

}  // namespace sar

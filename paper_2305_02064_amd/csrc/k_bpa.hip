// Direct back-projection (the paper's gold standard, Sec. III and Sec. V,
// with the exact Tx/Rx ranges of Eq. (2)):
//   o_B(r) = sum_n sum_i s_n(f_i) exp(+j k_i (R_T,n(r) + R_R,n(r))),
// unit amplitude weight, for comparison with the fast method on small scans
// (cost N_v x N_f x N_voxels).  One lane per voxel; every lane walks all
// virtual samples, whose echo values are the same for the whole wave (scalar
// loads).  Ranges and phase arguments in float64, reduced modulo one cycle.
#include <hip/hip_fp16.h>

#include "device_common.hpp"
#include "launch.hpp"
#include "sar_internal.hpp"

namespace sar {
namespace {

struct BpaArgs {
  const double* pos;    // [n_pos][3]
  const void* echo;     // [n_pos][n_pair][nf]
  int echo_type;
  float echo_scale;
  const double* txrx;   // [n_pair][4]
  const double* fcc;    // f / c [nf]
  float2* image;        // [nx][ny][nz]
  int nx, ny, nz, nf, n_pair;
  int64_t n_pos;
  double x0, y0, z0, dx, dy, dz;
};

struct BpaBody {
  using Args = BpaArgs;
  static constexpr int kThreads = 256;
  static __device__ __forceinline__ void run(const BpaArgs& a, uint32_t blk, uint32_t) {
    const int64_t nvox = (int64_t)a.nx * a.ny * a.nz;
    const int64_t v = (int64_t)blk * kThreads + threadIdx.x;
    const bool live = v < nvox;
    const int64_t vc = live ? v : 0;
    const int w = (int)(vc % a.nz);
    const int64_t uv = vc / a.nz;
    const int iv = (int)(uv % a.ny);
    const int iu = (int)(uv / a.ny);
    const double px = a.x0 + iu * a.dx, py = a.y0 + iv * a.dy, pz = a.z0 + w * a.dz;
    float2 acc = make_float2(0.f, 0.f);
    for (int64_t m = 0; m < a.n_pos; ++m) {
      const double sx = a.pos[3 * m], sy = a.pos[3 * m + 1], sz = a.pos[3 * m + 2];
      const double dz2 = (pz - sz) * (pz - sz);
      for (int l = 0; l < a.n_pair; ++l) {
        const double* o = a.txrx + 4 * l;
        const double tx = sx + o[0] - px, ty = sy + o[1] - py;
        const double rx = sx + o[2] - px, ry = sy + o[3] - py;
        const double r = sqrt(tx * tx + ty * ty + dz2) + sqrt(rx * rx + ry * ry + dz2);
        const int64_t row = (m * a.n_pair + l) * a.nf;
        for (int i = 0; i < a.nf; ++i) {
          float2 s;
          if (a.echo_type == SAR_ECHO_C64) {
            s = ((const float2*)a.echo)[row + i];
          } else {
            s = __half22float2(((const __half2*)a.echo)[row + i]);
            s = make_float2(s.x * a.echo_scale, s.y * a.echo_scale);
          }
          cfma_c(acc, s, cis_cycles(a.fcc[i] * r));
        }
      }
    }
    if (live) a.image[vc] = acc;
  }
};

}  // namespace

sar_status launch_backprojection(const Plan& p, const double* d_pos, int64_t n_pos, const void* d_echo,
                                 float echo_scale, float2* image, LaunchSink& sink) {
  BpaArgs a;
  a.pos = d_pos;
  a.echo = d_echo;
  a.echo_type = p.echo_type;
  a.echo_scale = echo_scale;
  a.txrx = p.d_txrx;
  a.fcc = p.d_fcc;
  a.image = image;
  a.nx = p.nx;
  a.ny = p.ny;
  a.nz = p.nz;
  a.nf = p.nf;
  a.n_pair = p.n_pair;
  a.n_pos = n_pos;
  a.x0 = p.x0;
  a.y0 = p.y0;
  a.z0 = p.z0;
  a.dx = p.dx;
  a.dy = p.dy;
  a.dz = p.dz;
  const int64_t nvox = (int64_t)p.nx * p.ny * p.nz;
  const double terms = (double)n_pos * p.n_pair * p.nf * (double)nvox;
  if (terms > kMaxBackprojectionTerms)
    return fail(SAR_ERR_UNSUPPORTED, "back-projection of " + std::to_string(terms) +
                                         " terms (samples x frequencies x voxels) exceeds the limit of 1e12");
  return launch_body<BpaBody>(sink, (uint32_t)((nvox + BpaBody::kThreads - 1) / BpaBody::kThreads), 0, a,
                              "back-projection launch");
}

}  // namespace sar

// Host-side plan structure and kernel launchers of the image-formation library.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <memory>
#include <string>
#include <vector>

#include "sar.h"

namespace sar {

constexpr int kNumStages = 7;
// gridding tile configurations: cells along x, along y, frequencies per lane,
// and the kernel widths each is compiled for
// (configuration 3: a four-wave workgroup over 8 x 8 cells sharing each
// compensated value, a wave per pair of rows four apart)
constexpr int kNumGridTiles = 4;
constexpr int kGridTiles[kNumGridTiles][3] = {{4, 4, 2}, {8, 8, 1}, {8, 4, 2}, {8, 8, 2}};
constexpr int kGridTileWidths[kNumGridTiles][2] = {{3, 8}, {3, 5}, {5, 6}, {3, 5}};  // none spills registers
constexpr bool grid_tile_compiled(int tile, int w) {
  return tile >= 0 && tile < kNumGridTiles && w >= kGridTileWidths[tile][0] && w <= kGridTileWidths[tile][1];
}
constexpr int kMaxWidth = 8;    // largest lateral kernel width
constexpr int kMaxFftLength = 4096;  // longest lateral transform (oversampled grid side)
constexpr double kMinUpsample = 1.25;  // smallest lateral oversampling
// back-projection refuses plans and scans above this many terms
// (virtual samples x frequencies x voxels), about a second of one GPU
constexpr double kMaxBackprojectionTerms = 1.0e12;

// Geometry of one virtual-sample record in the sorted list consumed by the
// gridding kernel: source row of the echo, cell of the last tap, residual
// path and the separable kernel weights of its W taps along x and y.
template <int W>
struct alignas(16) SampleRec {
  int32_t src;     // shot * n_pair + pair
  int16_t cx, cy;  // cell of the last tap: (first-tap cell + W - 1) mod (mx, my)
  double beta;     // residual path (m)
  float wx[W];
  float wy[W];
};

struct Plan {
  int device = 0;
  // descriptor copy
  int n_tx = 0, n_rx = 0, n_pair = 0, nf = 0;
  std::vector<double> tx_xy, rx_xy, freq;
  double z_ref = 0, z_focus = 0;
  int nx = 0, ny = 0, nz = 0;
  double x0 = 0, y0 = 0, z0 = 0, dx = 0, dy = 0, dz = 0;
  int64_t max_pos = 0;
  int echo_type = SAR_ECHO_C64;
  double tol = 1e-4;
  uint32_t flags = 0;
  double up_req = 0;         // descriptor's upsample (0: automatic)
  int kw_req = 0;            // descriptor's kernel_width (0: from tol)
  // derived
  double xc = 0, yc = 0;     // lateral centre of the image grid
  int mx = 0, my = 0, w = 0; // oversampled lateral grid and KB width
  int grid_tile = 0;         // gridding tile configuration (kGridTiles)
  double kb_beta = 0;
  int mz = 0, wz = 0;        // Stolt grid and ES width
  double es_beta = 0;
  double beta_sign = 0, inv4rc = 0;  // beta = beta_sign * dz + (dx^2 + dy^2) * inv4rc
  double amp_inv_r2 = 0;             // SAR_AMPLITUDE: 1 / (z_c - Z_0)^2, else 0
  // device tables
  double* d_fcc = nullptr;     // f_i / c (cycles per metre) [nf]
  double* d_k = nullptr;       // k_i = 2 pi f_i / c [nf]
  double* d_pair = nullptr;    // [n_pair][4]: midpoint offset (x, y), separation (x, y)
  double* d_txrx = nullptr;    // [n_pair][4]: Tx offset (x, y), Rx offset (x, y)
  float* d_deapx = nullptr;    // 1 / phi_hat_x(p), p = -nx/2 .. [nx]
  float* d_deapy = nullptr;    // [ny]
  float* d_deapz = nullptr;    // 1 / phi_hat_z(m), m = -nz/2 .. [nz]
  float* d_signx = nullptr;    // (-1)^(u + nx/2) [nx] (even nx)
  float* d_signy = nullptr;    // (-1)^(v + ny/2) [ny] (even ny)
  float2* d_postx = nullptr;   // exp(-j 2 pi h (u - h) / nx), h = nx/2 [nx] (odd nx)
  float2* d_posty = nullptr;   // likewise for odd ny
  float2* d_tw_mx = nullptr;   // exp(-j 2 pi i / mx) [mx]
  float2* d_tw_my = nullptr;
  float2* d_tw_nx = nullptr;   // exp(+j 2 pi i / nx) [nx]
  float2* d_tw_ny = nullptr;
  float2* d_tw_mz = nullptr;   // exp(+j 2 pi i / mz) [mz]
  // output placement: this plan's nz planes are planes [out_w0, out_w0 + nz)
  // of an image with out_nz planes (a depth slab writes into the full image)
  int out_w0 = 0, out_nz = 0;
  // depth slabs: one sub-plan per slab, each with its own reference depth
  // (empty for a single-depth plan)
  std::vector<std::unique_ptr<Plan>> slabs;
  // work that still reads this plan: queued or running server requests and
  // batches built from it (sar_plan_destroy refuses while nonzero)
  std::atomic<int> users{0};
  // timing
  bool timing = false;
  std::vector<hipEvent_t> events;  // kNumStages + 1 per recorded call
  int64_t timed_calls = 0;
};

struct Workspace {
  int32_t* cell_start = nullptr;  // [mx*my + 1] (+ scan partial sums)
  int32_t* key = nullptr;         // [n_v] sort keys, and their second buffer
  int32_t* key_alt = nullptr;     // [n_v]
  int32_t* order = nullptr;       // [n_v] source index of each sorted sample
  int32_t* order_alt = nullptr;   // [n_v]
  int32_t* hist = nullptr;        // radix digit histograms (+ scan partial sums)
  // over-full unions of the four-wave gridding kernel (null unless compiled for the width)
  int32_t* split_count = nullptr; // [1] overflow slots taken (zeroed with the cell counts)
  int32_t* uofs = nullptr;        // [unions] first overflow slot or -1
  int32_t* slots = nullptr;       // [max_slots][2] union, part
  float2* partial = nullptr;      // [max_slots][64][nf]
  int max_slots = 0;
  void* rec = nullptr;            // [n_v] SampleRec<w>
  float2* region_a = nullptr;     // oversampled grid / spectrum / first inverse pass
  float2* region_b = nullptr;     // x-transformed grid / z profiles
};

size_t workspace_bytes(const Plan& p, int64_t n_pos, Workspace* ws, char* base);

// over-full unions of the four-wave gridding kernel: samples per part and the
// number of overflow slots a workspace holds for n_v virtual samples.  Every
// sample lies in the streams of at most 4 unions, so 4 n_v / part length
// bounds the slots ever needed; the table holds half that bound, at most 1024
// slots (for 256 frequencies 128 MiB of partial grids), and a union whose
// parts do not fit runs unsplit (the same sum, only slower).
constexpr int kUnionPartLen = 2048;
constexpr int kUnionMaxSlots = 1024;
inline int union_slots(int64_t n_v) {
  const int64_t b = (2 * n_v + kUnionPartLen - 1) / kUnionPartLen;
  return (int)(b < kUnionMaxSlots ? b : kUnionMaxSlots);
}

// lateral NUFFT parameters for an oversampling (host only), their device
// tables, and the tuning file (plan.cpp)
sar_status choose_lateral(Plan& p, double up);
sar_status upload_lateral(Plan& p);
void tuning_store(const Plan& p, int64_t n_pos, double sigma, int tile);

// error helpers
void set_error(const std::string& msg);
sar_status fail(sar_status st, const std::string& msg);
sar_status check_hip(hipError_t e, const char* what);

class LaunchSink;  // launch.hpp

// stage launchers: describe the stage's kernels to `sink` (launched at once on
// a stream, or collected into a fused batch).  n_pos_grid >= n_pos sizes the
// per-sample grids (a batch sizes them for max_pos so that one captured graph
// serves every scan size); kernels stop at n_pos.
sar_status launch_geometry_sort(const Plan& p, const double* d_pos, int64_t n_pos, int64_t n_pos_grid,
                                const Workspace& ws, LaunchSink& sink);
sar_status launch_gridding(const Plan& p, const void* d_echo, float echo_scale, const Workspace& ws, float2* grid,
                           LaunchSink& sink);
// batched 1-D FFT along a strided axis with a contiguous batch dimension:
// in(o, l, b) = in[o*s_in_o + l*s_in_l + b], l < L, b < B;
// out(o, P, b) = scale[P] * X(o, k(P), b) at out[o*s_out_o + P*s_out_k + b],
// where k(P) = P (natural) or (P - n_out/2) mod L (centred crop).
struct FftLines {
  const float2* in;
  float2* out;
  int L;
  int n_outer;
  int64_t B;
  int64_t s_in_o, s_in_l, s_out_o, s_out_k;
  int n_out;
  // output placement: 0 natural (P = k); 1 centred crop to n_out modes,
  // P = k + h for k < n_out - h and P = k - L + h for k >= L - h (h = n_out / 2,
  // floor); 2 shift by h (P = (k + h) mod L, n_out = L) with the complex
  // per-output factor cscale[P]: the inverse transform on centred modes of an
  // odd length
  int centred;
  int sign;  // -1 forward, +1 inverse
  const float* scale;    // real per-output factor (may be null)
  const float2* cscale;  // complex per-output factor (centred == 2)
  const float2* tw;  // exp(sign j 2 pi i / L), i < L
  int nt_out;        // non-temporal stores (an output no later kernel reads soon)
};
// lengths of the lateral transforms: products 2^a 3^b 5^c
bool is_5smooth(int64_t v);
sar_status launch_fft_lines(const FftLines& a, LaunchSink& sink);
sar_status launch_stolt(const Plan& p, const float2* spec, float2* zcube, LaunchSink& sink);
sar_status launch_backprojection(const Plan& p, const double* d_pos, int64_t n_pos, const void* d_echo,
                                 float echo_scale, float2* image, LaunchSink& sink);

// whole per-scan pipeline on `stream` without stage timing (used by the server)
sar_status reconstruct_on(const Plan& p, const double* d_pos, int64_t n_pos, const void* d_echo, float echo_scale,
                          void* d_image, void* d_workspace, hipStream_t stream);
// whole per-scan pipeline described to a sink (used by fused batches)
sar_status describe_reconstruct(const Plan& p, const double* d_pos, int64_t n_pos, int64_t n_pos_grid,
                                const void* d_echo, float echo_scale, void* d_image, void* d_workspace,
                                LaunchSink& sink);
// One scan of a fused launch with its own workspace (device pointers).
struct FusedItem {
  const Plan* plan;
  const double* pos;
  int64_t n_pos;
  const void* echo;
  float scale;
  void* image;
  void* workspace;  // workspace_bytes(plan, n_pos), 256-byte aligned
};
// Runs the items' pipelines in fused launches on `stream`: their argument
// tables are written to h_table (pinned, `capacity` bytes) and uploaded to
// d_table on the stream; the caller keeps both until the launches have read
// them (the upload is stream-ordered before the kernels).
sar_status launch_fused(const std::vector<FusedItem>& items, char* d_table, char* h_table, size_t capacity,
                        hipStream_t stream);

// argument checks shared by sar_reconstruct and sar_submit (sets the error text)
sar_status check_reconstruct_args(sar_plan plan, int64_t n_pos, const void* pos, const void* echo,
                                  const void* image);

}  // namespace sar

struct sar_plan_s {
  sar::Plan p;
};

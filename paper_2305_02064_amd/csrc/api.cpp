// C ABI entry points (include/sar.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "launch.hpp"
#include "sar_internal.hpp"

namespace sar {

sar_status validate_desc(const sar_plan_desc* d);
sar_status build_plan(const sar_plan_desc* d, int device, Plan& p);
void free_plan(Plan& p);

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

sar_status fail(sar_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

sar_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return SAR_OK;
  return fail(SAR_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

// switches to the plan's device for the duration of a call
struct DeviceGuard {
  int old = -1;
  bool changed = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&old) == hipSuccess && old != dev) changed = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(old);
  }
};

bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

struct Timer {
  Plan& p;
  hipStream_t s;
  hipEvent_t ev[kNumStages + 1] = {};
  bool on;
  // enable only with a stream (direct launches); a fused batch is not timed per stage
  Timer(Plan& plan, hipStream_t stream, bool enable) : p(plan), s(stream), on(enable) {
    if (!on) return;
    for (auto& e : ev)
      if (hipEventCreate(&e) != hipSuccess) {
        on = false;
        return;
      }
  }
  void mark(int i) {
    if (on) (void)hipEventRecord(ev[i], s);
  }
  void commit() {
    if (!on) return;
    for (auto& e : ev) p.events.push_back(e);
    p.timed_calls += 1;
  }
};

sar_status run_front(const Plan& p, const double* d_pos, int64_t n_pos, int64_t n_pos_grid, const void* d_echo,
                     float echo_scale, float2* spec_out, const Workspace& ws, LaunchSink& sink, Timer* tm) {
  sar_status st;
  if (tm) tm->mark(0);
  if ((st = launch_geometry_sort(p, d_pos, n_pos, n_pos_grid, ws, sink)) != SAR_OK) return st;
  if (tm) tm->mark(1);
  if ((st = launch_gridding(p, d_echo, echo_scale, ws, ws.region_a, sink)) != SAR_OK) return st;
  if (tm) tm->mark(2);
  FftLines fx{};
  fx.in = ws.region_a;
  fx.out = ws.region_b;
  fx.L = p.mx;
  fx.n_outer = p.my;
  fx.B = p.nf;
  fx.s_in_o = (int64_t)p.mx * p.nf;
  fx.s_in_l = p.nf;
  fx.s_out_o = (int64_t)p.nx * p.nf;
  fx.s_out_k = p.nf;
  fx.n_out = p.nx;
  fx.centred = 1;
  fx.sign = -1;
  fx.scale = p.d_deapx;
  fx.tw = p.d_tw_mx;
  if ((st = launch_fft_lines(fx, sink)) != SAR_OK) return st;
  if (tm) tm->mark(3);
  FftLines fy{};
  fy.in = ws.region_b;
  fy.out = spec_out;
  fy.L = p.my;
  fy.n_outer = 1;
  fy.B = (int64_t)p.nx * p.nf;
  fy.s_in_o = 0;
  fy.s_in_l = (int64_t)p.nx * p.nf;
  fy.s_out_o = 0;
  fy.s_out_k = (int64_t)p.nx * p.nf;
  fy.n_out = p.ny;
  fy.centred = 1;
  fy.sign = -1;
  fy.scale = p.d_deapy;
  fy.tw = p.d_tw_my;
  if ((st = launch_fft_lines(fy, sink)) != SAR_OK) return st;
  if (tm) tm->mark(4);
  return SAR_OK;
}

sar_status run_back(const Plan& p, const float2* spec, void* d_image, const Workspace& ws, LaunchSink& sink,
                    Timer* tm, int first_mark) {
  sar_status st;
  if (tm) tm->mark(first_mark);
  if ((st = launch_stolt(p, spec, ws.region_b, sink)) != SAR_OK) return st;
  if (tm) tm->mark(first_mark + 1);
  FftLines gy{};
  gy.in = ws.region_b;  // [ny][nx][nz]
  gy.out = ws.region_a; // [ny(v)][nx][nz]
  gy.L = p.ny;
  gy.n_outer = 1;
  gy.B = (int64_t)p.nx * p.nz;
  gy.s_in_o = 0;
  gy.s_in_l = (int64_t)p.nx * p.nz;
  gy.s_out_o = 0;
  gy.s_out_k = (int64_t)p.nx * p.nz;
  gy.n_out = p.ny;
  gy.centred = (p.ny & 1) ? 2 : 0;  // odd: shifted output with a phase factor
  gy.sign = +1;
  gy.scale = p.d_signy;
  gy.cscale = p.d_posty;
  gy.tw = p.d_tw_ny;
  if ((st = launch_fft_lines(gy, sink)) != SAR_OK) return st;
  if (tm) tm->mark(first_mark + 2);
  FftLines gx{};
  gx.in = ws.region_a;  // [v][P][w]
  gx.out = (float2*)d_image + p.out_w0;  // [u][v][w], planes [out_w0, out_w0 + nz) of out_nz
  gx.L = p.nx;
  gx.n_outer = p.ny;
  gx.B = p.nz;
  gx.s_in_o = (int64_t)p.nx * p.nz;
  gx.s_in_l = p.nz;
  gx.s_out_o = p.out_nz;
  gx.s_out_k = (int64_t)p.ny * p.out_nz;
  gx.n_out = p.nx;
  gx.centred = (p.nx & 1) ? 2 : 0;
  gx.sign = +1;
  gx.scale = p.d_signx;
  gx.cscale = p.d_postx;
  gx.tw = p.d_tw_nx;
  gx.nt_out = 1;  // the image: not read again by this library
  if ((st = launch_fft_lines(gx, sink)) != SAR_OK) return st;
  if (tm) tm->mark(first_mark + 3);
  return SAR_OK;
}

sar_status check_call(sar_plan plan, int64_t n_pos, const void* d_pos, const void* d_echo, const void* d_out,
                      const void* d_ws) {
  sar_status st = check_reconstruct_args(plan, n_pos, d_pos, d_echo, d_out);
  if (st != SAR_OK) return st;
  if (!d_ws) return fail(SAR_ERR_INVALID, "workspace pointer is NULL");
  if (!aligned256(d_ws)) return fail(SAR_ERR_INVALID, "workspace must be 256-byte aligned");
  return SAR_OK;
}

}  // namespace

sar_status reconstruct_on(const Plan& p, const double* d_pos, int64_t n_pos, const void* d_echo, float echo_scale,
                          void* d_image, void* d_workspace, hipStream_t stream) {
  DirectSink sink(stream);
  return describe_reconstruct(p, d_pos, n_pos, n_pos, d_echo, echo_scale, d_image, d_workspace, sink);
}

sar_status describe_reconstruct(const Plan& p, const double* d_pos, int64_t n_pos, int64_t n_pos_grid,
                                const void* d_echo, float echo_scale, void* d_image, void* d_workspace,
                                LaunchSink& sink) {
  // depth slabs: each slab runs the whole pipeline with its own reference
  // depth and writes its planes of the image (a slab's workspace layout fits
  // inside the full plan's)
  for (const auto& sub : p.slabs) {
    sar_status st = describe_reconstruct(*sub, d_pos, n_pos, n_pos_grid, d_echo, echo_scale, d_image, d_workspace,
                                         sink);
    if (st != SAR_OK) return st;
  }
  if (!p.slabs.empty()) return SAR_OK;
  Workspace ws;
  workspace_bytes(p, n_pos_grid, &ws, (char*)d_workspace);
  sar_status st = run_front(p, d_pos, n_pos, n_pos_grid, d_echo, echo_scale, ws.region_a, ws, sink, nullptr);
  if (st != SAR_OK) return st;
  return run_back(p, ws.region_a, d_image, ws, sink, nullptr, 4);
}

sar_status check_reconstruct_args(sar_plan plan, int64_t n_pos, const void* pos, const void* echo,
                                  const void* image) {
  if (!plan) return fail(SAR_ERR_INVALID, "plan is NULL");
  const Plan& p = plan->p;
  if (n_pos < 0 || n_pos > p.max_pos) return fail(SAR_ERR_INVALID, "n_pos outside [0, max_pos]");
  if (n_pos > 0 && (!pos || !echo)) return fail(SAR_ERR_INVALID, "positions or echo pointer is NULL");
  if (!image) return fail(SAR_ERR_INVALID, "output pointer is NULL");
  return SAR_OK;
}

}  // namespace sar

using namespace sar;

extern "C" {

const char* sar_last_error(void) { return g_last_error.c_str(); }

const char* sar_version(void) { return "sar-mi355x 0.1 (gfx950)"; }

sar_status sar_plan_create(const sar_plan_desc* desc, int device, sar_plan* out) {
  if (!out) return fail(SAR_ERR_INVALID, "out is NULL");
  *out = nullptr;
  try {
    // validate before any HIP call, so descriptor errors never touch a device
    sar_status vs = validate_desc(desc);
    if (vs != SAR_OK) return vs;
    sar_plan h = new (std::nothrow) sar_plan_s();
    if (!h) return fail(SAR_ERR_NOMEM, "host allocation failed");
    int old = -1;
    (void)hipGetDevice(&old);
    sar_status st = build_plan(desc, device, h->p);
    if (old >= 0 && old != device) (void)hipSetDevice(old);
    if (st != SAR_OK) {
      free_plan(h->p);
      delete h;
      return st;
    }
    *out = h;
    return SAR_OK;
  } catch (...) {
    return fail(SAR_ERR_INVALID, "exception during plan creation");
  }
}

sar_status sar_plan_destroy(sar_plan plan) {
  if (!plan) return SAR_OK;
  if (plan->p.users.load() > 0)
    return fail(SAR_ERR_BUSY, "plan is still used by " + std::to_string(plan->p.users.load()) +
                                  " server request(s) or batch(es)");
  DeviceGuard g(plan->p.device);
  free_plan(plan->p);
  delete plan;
  return SAR_OK;
}

sar_status sar_plan_workspace_bytes(sar_plan plan, int64_t n_pos, size_t* bytes) {
  if (!plan || !bytes) return fail(SAR_ERR_INVALID, "plan or bytes is NULL");
  if (n_pos < 0 || n_pos > plan->p.max_pos) return fail(SAR_ERR_INVALID, "n_pos outside [0, max_pos]");
  *bytes = workspace_bytes(plan->p, n_pos, nullptr, nullptr);
  return SAR_OK;
}

sar_status sar_plan_get_info(sar_plan plan, sar_plan_info* info) {
  if (!plan || !info) return fail(SAR_ERR_INVALID, "plan or info is NULL");
  const Plan& p = plan->p;
  std::memset(info, 0, sizeof(*info));
  info->mx = p.mx;
  info->my = p.my;
  info->width = p.w;
  info->kb_beta = p.kb_beta;
  info->mz = p.mz;
  info->width_z = p.wz;
  info->es_beta_z = p.es_beta;
  info->n_pair = p.n_pair;
  info->n_stages = kNumStages;
  info->workspace_bytes_max = workspace_bytes(p, p.max_pos, nullptr, nullptr);
  info->grid_tile = p.grid_tile;
  info->grid_tile_x = kGridTiles[p.grid_tile][0];
  info->grid_tile_y = kGridTiles[p.grid_tile][1];
  info->grid_freqs_per_lane = kGridTiles[p.grid_tile][2];
  info->n_slabs = p.slabs.empty() ? 1 : (int32_t)p.slabs.size();
  info->nx = p.nx;
  info->ny = p.ny;
  info->nz = p.nz;
  info->n_freq = p.nf;
  info->echo_type = p.echo_type;
  info->flags = p.flags;
  info->max_pos = p.max_pos;
  info->sigma_x = (double)p.mx / p.nx;
  info->sigma_y = (double)p.my / p.ny;
  return SAR_OK;
}

sar_status sar_plan_set_grid_tile(sar_plan plan, int32_t tile) {
  if (!plan) return fail(SAR_ERR_INVALID, "plan is NULL");
  if (tile < 0 || tile >= kNumGridTiles) return fail(SAR_ERR_INVALID, "no such gridding tile configuration");
  if (!grid_tile_compiled(tile, plan->p.w))
    return fail(SAR_ERR_UNSUPPORTED, "gridding tile " + std::to_string(tile) + " is compiled for kernels of " +
                                         std::to_string(kGridTileWidths[tile][0]) + " to " +
                                         std::to_string(kGridTileWidths[tile][1]) + " taps");
  plan->p.grid_tile = tile;
  for (auto& sub : plan->p.slabs) sub->grid_tile = tile;
  return SAR_OK;
}

sar_status sar_plan_autotune(sar_plan plan, const double* d_pos, int64_t n_pos, const void* d_echo, float echo_scale,
                             void* d_workspace, sar_stream_t stream, int32_t* tile_out) {
  sar_status st = check_call(plan, n_pos, d_pos, d_echo, d_workspace, d_workspace);
  if (st != SAR_OK) return st;
  Plan& p = plan->p;
  if (p.users.load() > 0) return fail(SAR_ERR_BUSY, "plan is used by a batch or by server requests");
  DeviceGuard g(p.device);
  hipStream_t s = (hipStream_t)stream;
  // every candidate must fit the workspace the caller sized for the plan as it is
  const size_t ws_have = workspace_bytes(p, n_pos, nullptr, nullptr);
  std::vector<Plan*> all{&p};
  for (auto& sub : p.slabs) all.push_back(sub.get());
  // candidates: the requested oversampling, or the automatic choice (0) and
  // three fixed ratios
  std::vector<double> sigmas;
  if (p.up_req > 0)
    sigmas.push_back(p.up_req);
  else
    sigmas = {0.0, kMinUpsample, 1.5, 2.0};
  auto adopt = [&](double up, int tile) -> sar_status {
    for (Plan* q : all) {
      sar_status s2 = choose_lateral(*q, up);
      if (s2 == SAR_OK) s2 = upload_lateral(*q);
      if (s2 != SAR_OK) return s2;
      if (tile >= 0) q->grid_tile = tile;
    }
    return SAR_OK;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((st = check_hip(hipEventCreate(&e0), "event create")) != SAR_OK) return st;
  if ((st = check_hip(hipEventCreate(&e1), "event create")) != SAR_OK) {
    (void)hipEventDestroy(e0);
    return st;
  }
  double best_up = sigmas[0];
  int best_tile = p.grid_tile;
  float best_ms = 0.f;
  DirectSink sink(s);
  for (double up : sigmas) {
    if (adopt(up, -1) != SAR_OK) continue;  // e.g. a grid beyond the longest transform
    if (workspace_bytes(p, n_pos, nullptr, nullptr) > ws_have) continue;
    for (int t = 0; t < kNumGridTiles && st == SAR_OK; ++t) {
      if (!grid_tile_compiled(t, p.w)) continue;
      for (Plan* q : all) q->grid_tile = t;
      // the whole pipeline, its image written into the workspace's second
      // region (free once the last transform runs); first run warms up
      Workspace ws;
      workspace_bytes(p, n_pos, &ws, (char*)d_workspace);
      float t_min = 0.f;
      for (int rep = 0; rep < 4 && st == SAR_OK; ++rep) {
        st = check_hip(hipEventRecord(e0, s), "event record");
        if (st == SAR_OK)
          st = describe_reconstruct(p, d_pos, n_pos, n_pos, d_echo, echo_scale, ws.region_b, d_workspace, sink);
        if (st == SAR_OK) st = check_hip(hipEventRecord(e1, s), "event record");
        if (st == SAR_OK) st = check_hip(hipEventSynchronize(e1), "event wait");
        float ms = 0.f;
        if (st == SAR_OK) st = check_hip(hipEventElapsedTime(&ms, e0, e1), "event time");
        if (st == SAR_OK && rep > 0 && (rep == 1 || ms < t_min)) t_min = ms;
      }
      if (st == SAR_OK && (best_ms == 0.f || t_min < best_ms)) {
        best_ms = t_min;
        best_up = up;
        best_tile = t;
      }
    }
    if (st != SAR_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const sar_status st_adopt = adopt(best_up, best_tile);
  if (st == SAR_OK) st = st_adopt;
  if (st == SAR_OK) tuning_store(p, n_pos, best_up, best_tile);
  if (tile_out) *tile_out = p.grid_tile;
  return st;
}

sar_status sar_reconstruct(sar_plan plan, const double* d_pos, int64_t n_pos, const void* d_echo,
                           float echo_scale, void* d_image, void* d_workspace, sar_stream_t stream) {
  sar_status st = check_call(plan, n_pos, d_pos, d_echo, d_image, d_workspace);
  if (st != SAR_OK) return st;
  Plan& p = plan->p;
  DeviceGuard g(p.device);
  hipStream_t s = (hipStream_t)stream;
  DirectSink sink(s);
  if (!p.slabs.empty())  // depth slabs: no per-stage timing
    return describe_reconstruct(p, d_pos, n_pos, n_pos, d_echo, echo_scale, d_image, d_workspace, sink);
  Workspace ws;
  workspace_bytes(p, n_pos, &ws, (char*)d_workspace);
  Timer tm(p, s, p.timing);
  if ((st = run_front(p, d_pos, n_pos, n_pos, d_echo, echo_scale, ws.region_a, ws, sink, &tm)) != SAR_OK) return st;
  if ((st = run_back(p, ws.region_a, d_image, ws, sink, &tm, 4)) != SAR_OK) return st;
  tm.commit();
  return SAR_OK;
}

sar_status sar_spectrum(sar_plan plan, const double* d_pos, int64_t n_pos, const void* d_echo, float echo_scale,
                        void* d_spectrum, void* d_workspace, sar_stream_t stream) {
  sar_status st = check_call(plan, n_pos, d_pos, d_echo, d_spectrum, d_workspace);
  if (st != SAR_OK) return st;
  if (!plan->p.slabs.empty()) return fail(SAR_ERR_UNSUPPORTED, "a depth-slab plan has one spectrum per slab");
  Plan& p = plan->p;
  DeviceGuard g(p.device);
  Workspace ws;
  workspace_bytes(p, n_pos, &ws, (char*)d_workspace);
  DirectSink sink((hipStream_t)stream);
  return run_front(p, d_pos, n_pos, n_pos, d_echo, echo_scale, (float2*)d_spectrum, ws, sink, nullptr);
}

sar_status sar_image_from_spectrum(sar_plan plan, const void* d_spectrum, void* d_image, void* d_workspace,
                                   sar_stream_t stream) {
  sar_status st = check_call(plan, 0, nullptr, nullptr, d_image, d_workspace);
  if (st != SAR_OK) return st;
  if (!d_spectrum) return fail(SAR_ERR_INVALID, "spectrum pointer is NULL");
  if (!plan->p.slabs.empty()) return fail(SAR_ERR_UNSUPPORTED, "a depth-slab plan has one spectrum per slab");
  Plan& p = plan->p;
  DeviceGuard g(p.device);
  Workspace ws;
  workspace_bytes(p, 0, &ws, (char*)d_workspace);
  DirectSink sink((hipStream_t)stream);
  return run_back(p, (const float2*)d_spectrum, d_image, ws, sink, nullptr, 4);
}

sar_status sar_backproject(sar_plan plan, const double* d_pos, int64_t n_pos, const void* d_echo, float echo_scale,
                           void* d_image, sar_stream_t stream) {
  sar_status st = check_reconstruct_args(plan, n_pos, d_pos, d_echo, d_image);
  if (st != SAR_OK) return st;
  Plan& p = plan->p;
  DeviceGuard g(p.device);
  DirectSink sink((hipStream_t)stream);
  return launch_backprojection(p, d_pos, n_pos, d_echo, echo_scale, (float2*)d_image, sink);
}

sar_status sar_plan_set_timing(sar_plan plan, int enable) {
  if (!plan) return fail(SAR_ERR_INVALID, "plan is NULL");
  DeviceGuard g(plan->p.device);
  for (hipEvent_t ev : plan->p.events) (void)hipEventDestroy(ev);
  plan->p.events.clear();
  plan->p.timed_calls = 0;
  plan->p.timing = enable != 0;
  return SAR_OK;
}

sar_status sar_plan_stage_times(sar_plan plan, double* ms, int32_t n, int64_t* n_calls) {
  if (!plan || !ms || n < kNumStages) return fail(SAR_ERR_INVALID, "need a plan and kNumStages outputs");
  Plan& p = plan->p;
  DeviceGuard g(p.device);
  for (int i = 0; i < n; ++i) ms[i] = 0.0;
  const size_t per = kNumStages + 1;
  sar_status st = SAR_OK;
  for (size_t c = 0; c + per <= p.events.size(); c += per) {
    if (hipEventSynchronize(p.events[c + kNumStages]) != hipSuccess) {
      st = fail(SAR_ERR_DEVICE, "event wait failed");
      break;
    }
    for (int s = 0; s < kNumStages; ++s) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, p.events[c + s], p.events[c + s + 1]) == hipSuccess) ms[s] += t;
    }
  }
  if (n_calls) *n_calls = p.timed_calls;
  for (hipEvent_t ev : p.events) (void)hipEventDestroy(ev);
  p.events.clear();
  p.timed_calls = 0;
  return st;
}

}  // extern "C"

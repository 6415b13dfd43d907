// Fused batches of uneven scans (sar_batch_* in include/sar.h).
//
// A batch is a fixed list of plans (one per item; a plan may repeat).  Every
// call describes each item's whole pipeline to a recording sink, aligns the
// items' launches by pipeline step, and groups launches of the same kernel
// body at the same step into one fused grid (k_batch<Body>): item i owns a
// contiguous, 8-aligned range of blocks and reads its arguments from a device
// table (items with more blocks take the lower block ranges).  Steps follow
// each other in stream order, so a scan's kernels keep their order while
// different scans, of different sizes, share every launch.
//
// Per-sample grids are sized for each plan's max_pos and stop at the call's
// n_pos, and every pointer lives in the argument tables, so the launch
// sequence of a batch never changes: it is captured once into a HIP graph and
// replayed by every later call after one upload of the tables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "launch.hpp"
#include "sar_internal.hpp"

namespace sar {
namespace {

constexpr size_t kAlign = 256;
size_t round_up(size_t b, size_t a = kAlign) { return (b + a - 1) / a * a; }

// Records the launches of one item's pipeline in order.
class RecordSink final : public LaunchSink {
 public:
  struct Rec {
    const void* batch;
    uint32_t nblocks, threads;
    size_t shmem;
    std::vector<char> args;
  };
  std::vector<Rec> recs;
  sar_status launch(const void*, const void* batch, uint32_t nblocks, uint32_t threads, size_t shmem,
                    const void* args, size_t args_size, const char*) override {
    Rec r{batch, nblocks, threads, shmem, std::vector<char>((const char*)args, (const char*)args + args_size)};
    recs.push_back(std::move(r));
    return SAR_OK;
  }
};

// One fused launch: the same body at the same step for several items.
struct Group {
  const void* fn = nullptr;
  uint32_t threads = 0;
  size_t shmem = 0;
  size_t args_size = 0;
  std::vector<int> items;         // item index per entry
  std::vector<int> rec_index;     // record index within the item per entry
  std::vector<BatchItem> blocks;  // block range per entry
  uint32_t total_blocks = 0;
  size_t off_args = 0, off_items = 0;  // offsets in the argument blob
};

bool same_shape(const std::vector<Group>& a, const std::vector<Group>& b) {
  if (a.size() != b.size()) return false;
  for (size_t g = 0; g < a.size(); ++g) {
    if (a[g].fn != b[g].fn || a[g].threads != b[g].threads || a[g].shmem != b[g].shmem ||
        a[g].args_size != b[g].args_size || a[g].items != b[g].items || a[g].total_blocks != b[g].total_blocks)
      return false;
    for (size_t i = 0; i < a[g].blocks.size(); ++i)
      if (a[g].blocks[i].first != b[g].blocks[i].first || a[g].blocks[i].count != b[g].blocks[i].count) return false;
  }
  return true;
}

// Groups the items' records by (step, body); returns the blob size.
size_t build_groups(const std::vector<RecordSink>& sinks, std::vector<Group>& groups) {
  groups.clear();
  size_t max_steps = 0;
  for (const auto& s : sinks) max_steps = std::max(max_steps, s.recs.size());
  for (size_t step = 0; step < max_steps; ++step) {
    const size_t first_group = groups.size();
    for (size_t it = 0; it < sinks.size(); ++it) {
      if (step >= sinks[it].recs.size()) continue;
      const auto& r = sinks[it].recs[step];
      if (r.nblocks == 0) continue;
      Group* g = nullptr;
      for (size_t k = first_group; k < groups.size(); ++k)
        if (groups[k].fn == r.batch && groups[k].threads == r.threads && groups[k].shmem == r.shmem) g = &groups[k];
      if (!g) {
        groups.emplace_back();
        g = &groups.back();
        g->fn = r.batch;
        g->threads = r.threads;
        g->shmem = r.shmem;
        g->args_size = r.args.size();
      }
      g->items.push_back((int)it);
      g->rec_index.push_back((int)step);
      g->blocks.push_back({0, r.nblocks});
    }
  }
  // block ranges: items with more blocks first (the hardware hands out blocks
  // in index order, so the largest items start earliest and small ones fill
  // the tail of the grid); ties keep item order
  for (auto& g : groups) {
    std::vector<size_t> order(g.items.size());
    for (size_t e = 0; e < order.size(); ++e) order[e] = e;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return g.blocks[x].count > g.blocks[y].count; });
    std::vector<int> items(order.size()), recs(order.size());
    std::vector<BatchItem> blocks(order.size());
    g.total_blocks = 0;
    for (size_t e = 0; e < order.size(); ++e) {
      items[e] = g.items[order[e]];
      recs[e] = g.rec_index[order[e]];
      blocks[e] = {g.total_blocks, g.blocks[order[e]].count};
      g.total_blocks += (uint32_t)round_up(blocks[e].count, 8);
    }
    g.items.swap(items);
    g.rec_index.swap(recs);
    g.blocks.swap(blocks);
  }
  // each group's table is an array of the body's Args, indexed by the kernel
  // with stride sizeof(Args): entries are packed at exactly that stride
  size_t off = 0;
  for (auto& g : groups) {
    g.off_args = off;
    off = round_up(off + g.items.size() * g.args_size);
    g.off_items = off;
    off = round_up(off + g.items.size() * sizeof(BatchItem));
  }
  return off;
}

void fill_blob(const std::vector<RecordSink>& sinks, const std::vector<Group>& groups, char* blob) {
  for (const auto& g : groups) {
    const size_t stride = g.args_size;  // sizeof(Args): the kernel's array stride
    for (size_t e = 0; e < g.items.size(); ++e) {
      const auto& r = sinks[g.items[e]].recs[g.rec_index[e]];
      std::memcpy(blob + g.off_args + e * stride, r.args.data(), g.args_size);
    }
    std::memcpy(blob + g.off_items, g.blocks.data(), g.blocks.size() * sizeof(BatchItem));
  }
}

}  // namespace

struct BatchState {
  int device = 0;
  uint32_t flags = 0;
  std::vector<sar_plan> plans;
  std::vector<size_t> ws_off;
  size_t ws_total = 0;
  std::vector<Group> groups;
  size_t blob_bytes = 0;
  char* d_blob = nullptr;
  char* h_blob = nullptr;  // pinned staging for the per-call upload
  hipEvent_t uploaded = nullptr;
  bool upload_pending = false;
  hipEvent_t finished = nullptr;  // behind the last call's kernels
  bool run_pending = false;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

// the device tables hold BatchItem arrays as the kernels read them
static_assert(sizeof(BatchItem) == 8, "BatchItem layout");

sar_status describe_all(BatchState& b, const double* const* pos, const int64_t* n_pos, const void* const* echo,
                        const float* scale, void* const* image, char* ws, std::vector<RecordSink>& sinks) {
  sinks.assign(b.plans.size(), RecordSink());
  for (size_t i = 0; i < b.plans.size(); ++i) {
    const Plan& p = b.plans[i]->p;
    sar_status st = describe_reconstruct(p, pos ? pos[i] : nullptr, n_pos ? n_pos[i] : 0, p.max_pos,
                                         echo ? echo[i] : nullptr, scale ? scale[i] : 1.f,
                                         image ? image[i] : nullptr, ws + b.ws_off[i], sinks[i]);
    if (st != SAR_OK) return st;
  }
  return SAR_OK;
}

sar_status set_lds_attributes(const std::vector<Group>& groups) {
  for (const auto& gr : groups)
    if (gr.shmem > 65536) {
      const hipError_t e = hipFuncSetAttribute(gr.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)gr.shmem);
      if (e != hipSuccess) return check_hip(e, "batch LDS attribute");
    }
  return SAR_OK;
}

sar_status enqueue_groups(const std::vector<Group>& groups, const char* d_blob, hipStream_t s) {
  for (const auto& g : groups) {
    const void* args = d_blob + g.off_args;
    const void* items = d_blob + g.off_items;
    int n = (int)g.items.size();
    void* kargs[] = {(void*)&args, (void*)&items, (void*)&n};
    sar_status st =
        check_hip(hipLaunchKernel(g.fn, dim3(g.total_blocks), dim3(g.threads), kargs, g.shmem, s), "batch launch");
    if (st != SAR_OK) return st;
  }
  return SAR_OK;
}

void release(BatchState& b) {
  // the last call's kernels and upload must be done before anything goes
  if (b.finished) {
    (void)hipEventSynchronize(b.finished);
    (void)hipEventDestroy(b.finished);
  }
  if (b.uploaded) {
    (void)hipEventSynchronize(b.uploaded);
    (void)hipEventDestroy(b.uploaded);
  }
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.graph) (void)hipGraphDestroy(b.graph);
  if (b.cap_stream) (void)hipStreamDestroy(b.cap_stream);
  if (b.d_blob) (void)hipFree(b.d_blob);
  if (b.h_blob) (void)hipHostFree(b.h_blob);
  b = BatchState();
}

sar_status launch_graph(BatchState& b, hipStream_t s);

struct DeviceGuard {
  int old = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&old) == hipSuccess && old != dev) (void)hipSetDevice(dev);
    else old = -1;
  }
  ~DeviceGuard() {
    if (old >= 0) (void)hipSetDevice(old);
  }
};

}  // namespace
}  // namespace sar

struct sar_batch_s {
  sar::BatchState s;
};

using namespace sar;

extern "C" {

sar_status sar_batch_create(const sar_plan* plans, int32_t n, uint32_t flags, sar_batch* out) {
  if (!out) return fail(SAR_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!plans || n <= 0) return fail(SAR_ERR_INVALID, "a batch needs at least one plan");
  if (flags & ~(uint32_t)SAR_BATCH_NO_GRAPH) return fail(SAR_ERR_INVALID, "unknown batch flag");
  for (int i = 0; i < n; ++i)
    if (!plans[i]) return fail(SAR_ERR_INVALID, "plan " + std::to_string(i) + " is NULL");
  const int dev = plans[0]->p.device;
  for (int i = 1; i < n; ++i)
    if (plans[i]->p.device != dev) return fail(SAR_ERR_INVALID, "all plans of a batch must be on one device");
  sar_batch h = new (std::nothrow) sar_batch_s();
  if (!h) return fail(SAR_ERR_NOMEM, "host allocation failed");
  BatchState& b = h->s;
  b.device = dev;
  b.flags = flags;
  b.plans.assign(plans, plans + n);
  for (int i = 0; i < n; ++i) {
    b.ws_off.push_back(b.ws_total);
    b.ws_total += round_up(workspace_bytes(plans[i]->p, plans[i]->p.max_pos, nullptr, nullptr));
  }
  DeviceGuard g(dev);
  // the launch structure depends only on the plans: describe with null buffers
  std::vector<RecordSink> sinks;
  sar_status st = describe_all(b, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, sinks);
  if (st == SAR_OK) {
    b.blob_bytes = build_groups(sinks, b.groups);
    // kernels with more than the default 64 KiB of dynamic LDS (set before any capture)
    st = set_lds_attributes(b.groups);
  }
  if (st == SAR_OK) {
    if (hipMalloc((void**)&b.d_blob, std::max<size_t>(b.blob_bytes, kAlign)) != hipSuccess) {
      b.d_blob = nullptr;
      st = fail(SAR_ERR_NOMEM, "device argument tables");
    }
  }
  if (st == SAR_OK && hipHostMalloc((void**)&b.h_blob, std::max<size_t>(b.blob_bytes, kAlign)) != hipSuccess) {
    b.h_blob = nullptr;
    st = fail(SAR_ERR_NOMEM, "pinned staging of the argument tables");
  }
  if (st == SAR_OK) st = check_hip(hipEventCreateWithFlags(&b.uploaded, hipEventDisableTiming), "event create");
  if (st == SAR_OK) st = check_hip(hipEventCreateWithFlags(&b.finished, hipEventDisableTiming), "event create");
  if (st == SAR_OK) st = check_hip(hipStreamCreateWithFlags(&b.cap_stream, hipStreamNonBlocking), "stream create");
  if (st != SAR_OK) {
    release(b);
    delete h;
    return st;
  }
  for (sar_plan q : b.plans) q->p.users.fetch_add(1);  // released by sar_batch_destroy
  *out = h;
  return SAR_OK;
}

sar_status sar_batch_workspace_bytes(sar_batch batch, size_t* bytes) {
  if (!batch || !bytes) return fail(SAR_ERR_INVALID, "batch or bytes is NULL");
  *bytes = batch->s.ws_total;
  return SAR_OK;
}

sar_status sar_batch_reconstruct(sar_batch batch, const double* const* d_pos, const int64_t* n_pos,
                                 const void* const* d_echo, const float* echo_scale, void* const* d_image,
                                 void* d_workspace, sar_stream_t stream) {
  if (!batch) return fail(SAR_ERR_INVALID, "batch is NULL");
  if (!d_pos || !n_pos || !d_echo || !d_image) return fail(SAR_ERR_INVALID, "per-item arrays must not be NULL");
  if (!d_workspace || ((uintptr_t)d_workspace & 255u)) return fail(SAR_ERR_INVALID, "workspace must be 256-byte aligned");
  BatchState& b = batch->s;
  for (size_t i = 0; i < b.plans.size(); ++i) {
    sar_status st = check_reconstruct_args(b.plans[i], n_pos[i], d_pos[i], d_echo[i], d_image[i]);
    if (st != SAR_OK) return fail(st, "item " + std::to_string(i) + ": " + sar_last_error());
  }
  DeviceGuard g(b.device);
  hipStream_t s = (hipStream_t)stream;
  std::vector<RecordSink> sinks;
  sar_status st = describe_all(b, d_pos, n_pos, d_echo, echo_scale, d_image, (char*)d_workspace, sinks);
  if (st != SAR_OK) return st;
  std::vector<Group> groups;
  build_groups(sinks, groups);
  if (!same_shape(groups, b.groups)) return fail(SAR_ERR_DEVICE, "batch launch structure changed");
  // the staging buffer is reused: the previous call's upload must have left it;
  // the device tables are reused: this call's upload waits for the previous
  // call's kernels even when the calls come on different streams
  if (b.upload_pending && (st = check_hip(hipEventSynchronize(b.uploaded), "upload wait")) != SAR_OK) return st;
  if (b.run_pending && (st = check_hip(hipStreamWaitEvent(s, b.finished, 0), "stream wait")) != SAR_OK) return st;
  fill_blob(sinks, b.groups, b.h_blob);
  if ((st = check_hip(hipMemcpyAsync(b.d_blob, b.h_blob, b.blob_bytes, hipMemcpyHostToDevice, s), "table upload")) !=
      SAR_OK)
    return st;
  if ((st = check_hip(hipEventRecord(b.uploaded, s), "event record")) != SAR_OK) return st;
  b.upload_pending = true;
  if (b.flags & SAR_BATCH_NO_GRAPH) {
    if ((st = enqueue_groups(b.groups, b.d_blob, s)) != SAR_OK) return st;
  } else {
    if ((st = launch_graph(b, s)) != SAR_OK) return st;
  }
  if ((st = check_hip(hipEventRecord(b.finished, s), "event record")) != SAR_OK) return st;
  b.run_pending = true;
  return SAR_OK;
}

sar_status sar_batch_destroy(sar_batch batch) {
  if (!batch) return SAR_OK;
  DeviceGuard g(batch->s.device);
  const std::vector<sar_plan> plans = batch->s.plans;  // release() waits for the last call, then forgets them
  release(batch->s);
  for (sar_plan q : plans) q->p.users.fetch_sub(1);
  delete batch;
  return SAR_OK;
}

}  // extern "C"

namespace sar {
namespace {

sar_status launch_graph(BatchState& b, hipStream_t s) {
  sar_status st;
  if (!b.exec) {
    // capture the fused launches once; they read everything from the tables
    if ((st = check_hip(hipStreamBeginCapture(b.cap_stream, hipStreamCaptureModeThreadLocal), "begin capture")) !=
        SAR_OK)
      return st;
    st = enqueue_groups(b.groups, b.d_blob, b.cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(b.cap_stream, &graph);
    if (st != SAR_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if ((st = check_hip(e, "end capture")) != SAR_OK) return st;
    b.graph = graph;
    if ((st = check_hip(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0), "graph instantiate")) != SAR_OK) {
      b.exec = nullptr;
      return st;
    }
  }
  return check_hip(hipGraphLaunch(b.exec, s), "graph launch");
}

}  // namespace
}  // namespace sar

namespace sar {

sar_status launch_fused(const std::vector<FusedItem>& items, char* d_table, char* h_table, size_t capacity,
                        hipStream_t stream) {
  std::vector<RecordSink> sinks(items.size());
  for (size_t i = 0; i < items.size(); ++i) {
    const FusedItem& it = items[i];
    sar_status st = describe_reconstruct(*it.plan, it.pos, it.n_pos, it.n_pos, it.echo, it.scale, it.image,
                                         it.workspace, sinks[i]);
    if (st != SAR_OK) return st;
  }
  std::vector<Group> groups;
  const size_t bytes = build_groups(sinks, groups);
  if (bytes > capacity) {
    // more launches than the table holds: run the items one after another
    DirectSink direct(stream);
    for (const FusedItem& it : items) {
      sar_status st = describe_reconstruct(*it.plan, it.pos, it.n_pos, it.n_pos, it.echo, it.scale, it.image,
                                           it.workspace, direct);
      if (st != SAR_OK) return st;
    }
    return SAR_OK;
  }
  sar_status st = set_lds_attributes(groups);
  if (st != SAR_OK) return st;
  fill_blob(sinks, groups, h_table);
  if ((st = check_hip(hipMemcpyAsync(d_table, h_table, bytes, hipMemcpyHostToDevice, stream), "table upload")) !=
      SAR_OK)
    return st;
  return enqueue_groups(groups, d_table, stream);
}

}  // namespace sar

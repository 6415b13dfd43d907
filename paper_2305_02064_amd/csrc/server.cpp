// Serving loop: continuous admission of scans under a device-memory budget
// (sar_server_* in include/sar.h).
//
// A server owns one device arena of the budgeted size, a small set of HIP
// streams and a worker thread.  Submissions enter a FIFO queue.  The worker
// admits, in arrival order, every waiting scan whose memory (workspace, plus
// staging for host inputs) fits in the arena, up to 16 at a time and 32 in
// flight, and launches them as one unit on the least-loaded stream: a single
// scan runs its own kernels, several scans run together in fused launches
// (one grid per pipeline step holding the blocks of all of them).  Scans that
// arrive while units are on the device form the next unit as soon as memory
// and slots free up, and units on different streams overlap: continuous
// batching.  Completion is signalled by a host callback queued behind a
// unit's last kernel; it returns the unit's memory and wakes the worker.
// Plans (geometry, sweep, grid tables, twiddles) stay resident: a request
// only names one.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sar_internal.hpp"

namespace sar {
namespace {

using Clock = std::chrono::steady_clock;
constexpr size_t kAlign = 256;
constexpr int kStreams = 4;       // one per hardware queue of the default HIP setup
constexpr int kMaxInFlight = 32;  // scans admitted and not yet finished
constexpr int kMaxUnit = 16;      // scans fused into one launch unit
// scans whose workspace exceeds this fill the device on their own: they run
// alone (unit of one) instead of holding up the small scans fused with them
constexpr size_t kFuseMaxBytes = (size_t)512 << 20;
constexpr int kSlots = 64;        // argument-table slots (>= units in flight)
constexpr size_t kSlotBytes = 128 << 10;

size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing of freed neighbours.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t start = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[start + bytes] = rest;
      *off = start;
      return true;
    }
    return false;
  }
  bool fits(size_t bytes) const {
    for (const auto& kv : free_)
      if (kv.second >= bytes) return true;
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
};

}  // namespace

struct Request;

// Scans launched together; `slot` holds their fused argument tables (-1: one
// scan launched directly).
struct Unit {
  std::vector<Request*> reqs;
  int stream = -1;
  int slot = -1;
  struct ServerState* srv = nullptr;
};

struct ServerState {
  int device = 0;
  size_t budget = 0;
  char* pool = nullptr;
  Arena arena;
  hipStream_t streams[kStreams] = {};
  int load[kStreams] = {};
  char* h_tables = nullptr;  // pinned, kSlots x kSlotBytes
  char* d_tables = nullptr;  // device, kSlots x kSlotBytes
  std::vector<int> free_slots;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, Request*> reqs;
  uint64_t next_ticket = 1;
  int inflight = 0;
  bool stop = false;
  std::thread worker;
};

struct Request {
  ServerState* srv = nullptr;
  uint64_t ticket = 0;
  sar_plan plan = nullptr;
  const double* pos = nullptr;
  int64_t n_pos = 0;
  const void* echo = nullptr;
  bool on_device = true;
  float scale = 1.f;
  void* image = nullptr;
  size_t ws_bytes = 0, pos_bytes = 0, echo_bytes = 0, total = 0;
  size_t off = 0;
  Clock::time_point t_submit, t_done;
  bool done = false;
  sar_status status = SAR_OK;
  std::string error;
};

namespace {

// Marks a unit finished and returns its memory; called with the lock held.
void finish_locked(ServerState& s, Unit* u, sar_status st, const std::string& err) {
  const Clock::time_point now = Clock::now();
  for (Request* r : u->reqs) {
    r->status = st;
    r->error = err;
    r->t_done = now;
    r->done = true;
    s.arena.release(r->off, r->total);
    r->plan->p.users.fetch_sub(1);
  }
  s.inflight -= (int)u->reqs.size();
  s.load[u->stream] -= 1;
  if (u->slot >= 0) s.free_slots.push_back(u->slot);
  delete u;
  s.cv.notify_all();
}

// Host callback queued behind a unit's last kernel (runs on a HIP runtime
// thread; makes no HIP calls).
void on_unit_done(void* arg) {
  Unit* u = (Unit*)arg;
  ServerState& s = *u->srv;
  std::lock_guard<std::mutex> lk(s.mu);
  finish_locked(s, u, SAR_OK, std::string());
}

// Queues the copies (host inputs) and the pipelines of an admitted unit.
void launch(ServerState& s, Unit* u) {
  hipStream_t st = s.streams[u->stream];
  std::vector<FusedItem> items;
  sar_status rc = SAR_OK;
  for (Request* r : u->reqs) {
    char* base = s.pool + r->off;
    const double* pos = r->pos;
    const void* echo = r->echo;
    if (!r->on_device && r->n_pos > 0) {
      char* dpos = base + round_up(r->ws_bytes);
      char* decho = dpos + round_up(r->pos_bytes);
      if (rc == SAR_OK)
        rc = check_hip(hipMemcpyAsync(dpos, r->pos, r->pos_bytes, hipMemcpyHostToDevice, st), "position upload");
      if (rc == SAR_OK)
        rc = check_hip(hipMemcpyAsync(decho, r->echo, r->echo_bytes, hipMemcpyHostToDevice, st), "echo upload");
      pos = (const double*)dpos;
      echo = decho;
    }
    items.push_back({&r->plan->p, pos, r->n_pos, echo, r->scale, r->image, base});
  }
  if (rc == SAR_OK) {
    if (u->slot < 0) {
      const FusedItem& it = items[0];
      rc = reconstruct_on(*it.plan, it.pos, it.n_pos, it.echo, it.scale, it.image, it.workspace, st);
    } else {
      rc = launch_fused(items, s.d_tables + (size_t)u->slot * kSlotBytes, s.h_tables + (size_t)u->slot * kSlotBytes,
                        kSlotBytes, st);
    }
  }
  if (rc == SAR_OK) rc = check_hip(hipLaunchHostFunc(st, on_unit_done, u), "completion callback");
  if (rc != SAR_OK) {
    // work queued before the failure may still read the arena: drain the
    // stream before the memory is handed out again
    (void)hipStreamSynchronize(st);
    std::lock_guard<std::mutex> lk(s.mu);
    finish_locked(s, u, rc, sar_last_error());
  }
}

bool can_admit(const ServerState& s) {
  return !s.queue.empty() && s.inflight < kMaxInFlight && !s.free_slots.empty() &&
         s.arena.fits(s.queue.front()->total);
}

void worker_main(ServerState* sp) {
  ServerState& s = *sp;
  (void)hipSetDevice(s.device);
  std::unique_lock<std::mutex> lk(s.mu);
  for (;;) {
    s.cv.wait(lk, [&] { return (s.stop && s.queue.empty() && s.inflight == 0) || can_admit(s); });
    if (s.stop && s.queue.empty() && s.inflight == 0) break;
    // admit in arrival order while memory and slots last, into one unit
    Unit* u = new Unit();
    u->srv = &s;
    while (!s.queue.empty() && s.inflight < kMaxInFlight && (int)u->reqs.size() < kMaxUnit) {
      Request* r = s.queue.front();
      const bool large = r->ws_bytes > kFuseMaxBytes;
      if (large && !u->reqs.empty()) break;
      size_t off = 0;
      if (!s.arena.alloc(r->total, &off)) break;
      s.queue.pop_front();
      r->off = off;
      u->reqs.push_back(r);
      s.inflight += 1;
      if (large) break;
    }
    if (u->reqs.size() > 1) {
      u->slot = s.free_slots.back();
      s.free_slots.pop_back();
    }
    int best = 0;
    for (int i = 1; i < kStreams; ++i)
      if (s.load[i] < s.load[best]) best = i;
    u->stream = best;
    s.load[best] += 1;
    lk.unlock();
    launch(s, u);
    lk.lock();
  }
}

}  // namespace
}  // namespace sar

struct sar_server_s {
  sar::ServerState s;
};

using namespace sar;

extern "C" {

sar_status sar_server_create(int device, size_t hbm_budget_bytes, sar_server* out) {
  if (!out) return fail(SAR_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes < kAlign) return fail(SAR_ERR_INVALID, "budget must be at least 256 bytes");
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev)
    return fail(SAR_ERR_INVALID, "no such device");
  sar_server h = new (std::nothrow) sar_server_s();
  if (!h) return fail(SAR_ERR_NOMEM, "host allocation failed");
  ServerState& s = h->s;
  s.device = device;
  s.budget = hbm_budget_bytes / kAlign * kAlign;
  int old = -1;
  (void)hipGetDevice(&old);
  sar_status st = check_hip(hipSetDevice(device), "set device");
  if (st == SAR_OK && hipMalloc((void**)&s.pool, s.budget) != hipSuccess) {
    s.pool = nullptr;
    st = fail(SAR_ERR_NOMEM, "device arena of the requested budget could not be allocated");
  }
  for (int i = 0; st == SAR_OK && i < kStreams; ++i)
    st = check_hip(hipStreamCreateWithFlags(&s.streams[i], hipStreamNonBlocking), "stream create");
  if (st == SAR_OK && hipMalloc((void**)&s.d_tables, kSlots * kSlotBytes) != hipSuccess) {
    s.d_tables = nullptr;
    st = fail(SAR_ERR_NOMEM, "device argument tables");
  }
  if (st == SAR_OK && hipHostMalloc((void**)&s.h_tables, kSlots * kSlotBytes) != hipSuccess) {
    s.h_tables = nullptr;
    st = fail(SAR_ERR_NOMEM, "pinned argument tables");
  }
  for (int i = kSlots - 1; i >= 0; --i) s.free_slots.push_back(i);
  if (st == SAR_OK) {
    s.arena.reset(s.budget);
    try {
      s.worker = std::thread(worker_main, &s);
    } catch (...) {
      st = fail(SAR_ERR_NOMEM, "worker thread could not be started");
    }
  }
  if (st != SAR_OK) {
    for (auto& q : s.streams)
      if (q) (void)hipStreamDestroy(q);
    if (s.pool) (void)hipFree(s.pool);
    if (s.d_tables) (void)hipFree(s.d_tables);
    if (s.h_tables) (void)hipHostFree(s.h_tables);
    delete h;
  } else {
    *out = h;
  }
  if (old >= 0 && old != device) (void)hipSetDevice(old);
  return st;
}

sar_status sar_submit(sar_server server, sar_plan plan, const double* pos_xyz, int64_t n_pos, const void* echo,
                      int echo_on_device, float echo_scale, void* image_dst, uint64_t* ticket) {
  if (!server) return fail(SAR_ERR_INVALID, "server is NULL");
  if (!ticket) return fail(SAR_ERR_INVALID, "ticket is NULL");
  sar_status st = check_reconstruct_args(plan, n_pos, pos_xyz, echo, image_dst);
  if (st != SAR_OK) return st;
  ServerState& s = server->s;
  const Plan& p = plan->p;
  if (p.device != s.device) return fail(SAR_ERR_INVALID, "plan and server are on different devices");
  Request* r = new (std::nothrow) Request();
  if (!r) return fail(SAR_ERR_NOMEM, "host allocation failed");
  r->srv = &s;
  r->plan = plan;
  r->pos = pos_xyz;
  r->n_pos = n_pos;
  r->echo = echo;
  r->on_device = echo_on_device != 0;
  r->scale = echo_scale;
  r->image = image_dst;
  r->ws_bytes = workspace_bytes(p, n_pos, nullptr, nullptr);
  if (!r->on_device) {
    r->pos_bytes = (size_t)n_pos * 3 * sizeof(double);
    r->echo_bytes = (size_t)n_pos * p.n_pair * p.nf * (p.echo_type == SAR_ECHO_C64 ? 8 : 4);
  }
  r->total = round_up(r->ws_bytes) + round_up(r->pos_bytes) + round_up(r->echo_bytes);
  if (r->total > s.budget) {
    const std::string msg = "request needs " + std::to_string(r->total) + " bytes of device memory; the budget is " +
                            std::to_string(s.budget);
    delete r;
    return fail(SAR_ERR_NOMEM, msg);
  }
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s.mu);
    if (s.stop) {
      delete r;
      return fail(SAR_ERR_BUSY, "server is shutting down");
    }
    r->ticket = s.next_ticket++;
    plan->p.users.fetch_add(1);  // released when the request finishes
    s.reqs[r->ticket] = r;
    s.queue.push_back(r);
    *ticket = r->ticket;
  }
  s.cv.notify_all();
  return SAR_OK;
}

sar_status sar_poll(sar_server server, uint64_t ticket, int* done, double* latency_s) {
  if (!server || !done) return fail(SAR_ERR_INVALID, "server or done is NULL");
  ServerState& s = server->s;
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(s.mu);
    auto it = s.reqs.find(ticket);
    if (it == s.reqs.end()) return fail(SAR_ERR_NOT_FOUND, "unknown or already collected ticket");
    r = it->second;
    if (!r->done) {
      *done = 0;
      return SAR_OK;
    }
    s.reqs.erase(it);
  }
  *done = 1;
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  const sar_status st = r->status;
  if (st != SAR_OK) set_error(r->error);
  delete r;
  return st;
}

sar_status sar_server_destroy(sar_server server) {
  if (!server) return SAR_OK;
  ServerState& s = server->s;
  {
    std::lock_guard<std::mutex> lk(s.mu);
    s.stop = true;
  }
  s.cv.notify_all();
  if (s.worker.joinable()) s.worker.join();
  int old = -1;
  (void)hipGetDevice(&old);
  (void)hipSetDevice(s.device);
  for (auto& q : s.streams)
    if (q) {
      (void)hipStreamSynchronize(q);
      (void)hipStreamDestroy(q);
    }
  if (s.pool) (void)hipFree(s.pool);
  if (s.d_tables) (void)hipFree(s.d_tables);
  if (s.h_tables) (void)hipHostFree(s.h_tables);
  for (auto& kv : s.reqs) delete kv.second;
  if (old >= 0 && old != s.device) (void)hipSetDevice(old);
  delete server;
  return SAR_OK;
}

}  // extern "C"

// One launch layer for single scans and fused batches of scans.
//
// Every kernel of the pipeline is a body: a struct with an argument type
// `Args`, a block size `kThreads` and a device function
// `run(const Args&, uint32_t block, uint32_t nblocks)` that uses the given
// block index instead of blockIdx.x.  Two thin kernels drive a body:
//
//   k_single<Body>(Args)  one scan: the arguments travel as kernel arguments;
//   k_batch<Body>(...)    many scans in one grid: item i owns blocks
//                         [first_i, first_i + count_i) (first_i a multiple of
//                         8 so that per-item XCD-aware block orders hold), its
//                         arguments sit in a device table, and each block
//                         finds its item by binary search over the firsts.
//
// Host code describes each launch to a LaunchSink: the direct sink launches
// k_single at once on a stream; the batch schedule (batch.cpp) collects the
// launches of many scans, groups equal bodies of the same pipeline step, and
// issues one k_batch per group.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sar_internal.hpp"

namespace sar {

struct BatchItem {
  uint32_t first;  // first block of the item in the fused grid
  uint32_t count;  // blocks of the item
};

// Minimum waves per SIMD a body asks the register allocator for (default 1).
template <class Body, class = void>
struct MinWaves {
  static constexpr int value = 1;
};
template <class Body>
struct MinWaves<Body, decltype((void)Body::kMinWavesPerEU)> {
  static constexpr int value = Body::kMinWavesPerEU;
};

template <class Body>
__global__ __launch_bounds__(Body::kThreads) __attribute__((amdgpu_waves_per_eu(MinWaves<Body>::value)))
void k_single(typename Body::Args a) {
  Body::run(a, blockIdx.x, gridDim.x);
}

template <class Body>
__global__ __launch_bounds__(Body::kThreads) __attribute__((amdgpu_waves_per_eu(MinWaves<Body>::value)))
void k_batch(const typename Body::Args* __restrict__ args, const BatchItem* __restrict__ items, int n) {
  const uint32_t b = blockIdx.x;
  int lo = 0, hi = n;  // last item whose first block is <= b
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (items[mid].first <= b)
      lo = mid;
    else
      hi = mid;
  }
  const BatchItem it = items[lo];
  const uint32_t bid = b - it.first;
  if (bid >= it.count) return;  // alignment padding
  const typename Body::Args a = args[lo];
  Body::run(a, bid, it.count);
}

// Receives the launches of one scan's pipeline, in order.
class LaunchSink {
 public:
  virtual ~LaunchSink() = default;
  // single / batch: k_single<Body> and k_batch<Body>; args: a Body::Args
  virtual sar_status launch(const void* single, const void* batch, uint32_t nblocks, uint32_t threads,
                            size_t shmem, const void* args, size_t args_size, const char* what) = 0;
};

// Launches every kernel immediately on one stream.
class DirectSink final : public LaunchSink {
 public:
  explicit DirectSink(hipStream_t s) : stream_(s) {}
  sar_status launch(const void* single, const void*, uint32_t nblocks, uint32_t threads, size_t shmem,
                    const void* args, size_t, const char* what) override {
    if (nblocks == 0) return SAR_OK;
    if (shmem > 65536) {
      const hipError_t e = hipFuncSetAttribute(single, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
      if (e != hipSuccess) return check_hip(e, what);
    }
    void* kargs[] = {const_cast<void*>(args)};
    return check_hip(hipLaunchKernel(single, dim3(nblocks), dim3(threads), kargs, shmem, stream_), what);
  }
  hipStream_t stream() const { return stream_; }

 private:
  hipStream_t stream_;
};

// Describe a launch of Body to a sink.
template <class Body>
sar_status launch_body(LaunchSink& sink, uint32_t nblocks, size_t shmem, const typename Body::Args& a,
                       const char* what) {
  // a fused batch stores Args entries back to back at stride sizeof(Args) in
  // 256-byte aligned tables, exactly as k_batch indexes them
  static_assert(alignof(typename Body::Args) <= 256, "argument table alignment");
  return sink.launch((const void*)&k_single<Body>, (const void*)&k_batch<Body>, nblocks, Body::kThreads, shmem,
                     &a, sizeof(a), what);
}

}  // namespace sar

// Grouped launches for the batched entry point: the kernel launches of many
// problems recorded first, then launches of the same kernel merged into one
// whose workgroups look up their problem in a table.
//
// Device side.  A grouped launch runs sum_j blocks_j workgroups; item j of its
// table holds the launch's arguments and grid for one problem.  Workgroup b
// finds its item (a bucket index and a short scan), its block index within that item's grid and
// that grid, and runs the same kernel body with them, so every problem computes
// exactly what its own launch would (same arguments, same block mapping).
//
// Host side.  While a Recorder is installed on the calling thread, every
// launcher of the library appends its launch (the grouped kernel, grid, block
// and the item bytes) to it instead of launching; launchers without a grouped
// kernel append a closure that launches them later.  Nothing reaches a stream
// while recording.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <vector>

namespace comm {

// Workgroups per entry of the bucket index.
constexpr int kGroupBucket = 8;

// The table is read through the constant address space, as kernel arguments
// are: its loads are scalar and may be repeated instead of held in registers
// (the table does not change while a grouped launch runs).
#if defined(__HIP_DEVICE_COMPILE__)
#define COMM_CONST_AS __attribute__((address_space(4)))
#else
#define COMM_CONST_AS
#endif

struct GroupTable {
  const COMM_CONST_AS uint32_t* bucket;  // first item overlapping each run of kGroupBucket workgroups
  const COMM_CONST_AS uint32_t* first;   // first flat workgroup of each item, then the total
  const COMM_CONST_AS char* items;       // items of `stride` bytes
  int stride;
};

template <class Args>
struct alignas(16) GroupItem {
  uint3 grid;
  Args args;
};

// The item of this workgroup: its arguments, block index and grid.
template <class Args>
__device__ __forceinline__ const Args& group_item(const GroupTable& t, uint3& bid, uint3& gdim) {
  const uint32_t b = blockIdx.x;
  uint32_t j = t.bucket[b / kGroupBucket];
  while (t.first[j + 1] <= b) ++j;  // at most kGroupBucket - 1 steps
  const uint32_t local = b - t.first[j];
  const COMM_CONST_AS GroupItem<Args>* it = (const COMM_CONST_AS GroupItem<Args>*)(t.items + (size_t)j * t.stride);
  gdim = make_uint3(it->grid.x, it->grid.y, it->grid.z);
  bid.x = local % gdim.x;
  bid.y = (local / gdim.x) % gdim.y;
  bid.z = local / (gdim.x * gdim.y);
  return *(const Args*)(&it->args);
}

// A kernel body `name##_body(const Args&, uint3 bid, uint3 gdim)` with its
// single launch `name##_kernel(Args)` and grouped launch `name##_grouped`.
#define COMM_GROUPED_KERNELS(name, Args, threads)                                   \
  __global__ void __launch_bounds__(threads) name##_kernel(Args a) {                \
    name##_body(a, make_uint3(blockIdx.x, blockIdx.y, blockIdx.z),                  \
                make_uint3(gridDim.x, gridDim.y, gridDim.z));                        \
  }                                                                                  \
  __global__ void __launch_bounds__(threads) name##_grouped(GroupTable t) {         \
    uint3 bid, gdim;                                                                 \
    const Args& a = group_item<Args>(t, bid, gdim);                                  \
    name##_body(a, bid, gdim);                                                       \
  }

// ------------------------------------------------------------------------------ host

struct LaunchRec {
  const void* kgrp = nullptr;                   // grouped kernel; null: `fn`
  dim3 grid, block;
  size_t shmem = 0;
  std::vector<char> item;                       // GroupItem<Args> bytes
  std::function<hipError_t(hipStream_t)> fn;    // launches without a grouped kernel
};

struct Recorder {
  std::vector<LaunchRec> recs;
};

inline thread_local Recorder* g_recorder = nullptr;

inline Recorder* recorder() { return g_recorder; }

// Timing of one launch.  While `g_timed` holds a pair of events, the next
// kernel launched through launch_timed() takes them and clears them: the
// dispatch itself stamps the start and end of that kernel into the events, so
// nothing else is queued on the stream for the measurement.
struct TimedLaunch {
  hipEvent_t start = nullptr, stop = nullptr;
};

inline thread_local TimedLaunch g_timed;

// Launch errors are left for hipGetLastError(), as with hipLaunchKernelGGL.
template <class... KArgs, class... Args>
void launch_timed(void (*k)(KArgs...), dim3 grid, dim3 block, size_t shmem, hipStream_t s, const Args&... args) {
  if (g_timed.start) {
    const TimedLaunch t = g_timed;
    g_timed = TimedLaunch{};
    hipExtLaunchKernelGGL(k, grid, block, (uint32_t)shmem, s, t.start, t.stop, 0u, args...);
  } else {
    hipLaunchKernelGGL(k, grid, block, shmem, s, args...);
  }
}

// While recording: append the grouped kernel with the item and return true.
template <class Args>
bool record_grouped(void (*grouped)(GroupTable), dim3 grid, dim3 block, size_t shmem, const Args& a) {
  Recorder* r = recorder();
  if (!r) return false;
  LaunchRec rec;
  rec.kgrp = reinterpret_cast<const void*>(grouped);
  rec.grid = grid;
  rec.block = block;
  rec.shmem = shmem;
  GroupItem<Args> it{};
  it.grid = make_uint3(grid.x, grid.y, grid.z);
  it.args = a;
  rec.item.assign(reinterpret_cast<const char*>(&it), reinterpret_cast<const char*>(&it) + sizeof(it));
  r->recs.push_back(std::move(rec));
  return true;
}

// Launch `single` now, or record the grouped twin with the item.
template <class Args>
hipError_t launch_or_record(void (*single)(Args), void (*grouped)(GroupTable), dim3 grid, dim3 block, size_t shmem,
                            hipStream_t s, const Args& a) {
  if (record_grouped(grouped, grid, block, shmem, a)) return hipSuccess;
  launch_timed(single, grid, block, shmem, s, a);
  return hipGetLastError();
}

// Record a launch that has no grouped kernel (replayed as it is).
inline bool record_closure(std::function<hipError_t(hipStream_t)> fn) {
  if (Recorder* r = recorder()) {
    LaunchRec rec;
    rec.fn = std::move(fn);
    r->recs.push_back(std::move(rec));
    return true;
  }
  return false;
}

}  // namespace comm

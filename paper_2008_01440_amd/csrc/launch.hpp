// Kernel launches that can be replayed as work lists.
//
// Every kernel of the solve path is a struct K with
//   static constexpr int kThreads;   (its launch bound)
//   __device__ static void run(P...);
// and is launched through launch<K>(grid, block, shmem, stream, args...).
// Normally that is one launch of k_entry<K>, whose body is K::run: the same
// code a plain __global__ function would be.  While a LaunchRecorder is
// installed on the calling thread, launch<K> launches nothing and appends the
// launch (kernel, grid, block and the argument values) to the recorder instead.
//
// A work list is the recorded launch sequences of several problems with the
// same kernels and grids (same-shape operators with the same parameters):
// launch i of every problem becomes ONE launch of k_group<K> with grid
// dimension z = problem, whose blocks read problem z's arguments from a table
// in device memory.  Each block does exactly what it does in the problem's own
// launch (blockIdx.x and blockIdx.y and gridDim.x and gridDim.y are the same),
// so every problem's result is bitwise the one of its own launches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <new>
#include <type_traits>
#include <utility>
#include <vector>

namespace pcheb {

// ---------------------------------------------------------------- argument packs

template <size_t I, class T>
struct PackLeaf {
  T v;
};
template <class Seq, class... A>
struct PackImpl;
template <size_t... I, class... A>
struct PackImpl<std::index_sequence<I...>, A...> : PackLeaf<I, A>... {};
template <class... A>
using Pack = PackImpl<std::index_sequence_for<A...>, A...>;

template <class K, class... P>
__global__ __launch_bounds__(K::kThreads) void k_entry(P... a) {
  K::run(a...);
}

template <class K, size_t... I, class... P>
__device__ __forceinline__ void run_pack(const PackImpl<std::index_sequence<I...>, P...>& p) {
  K::run(static_cast<const PackLeaf<I, P>&>(p).v...);
}

// Problem blockIdx.z of a work-list launch: its arguments are the table entry
// at tab + blockIdx.z * stride (the address is uniform over the block).
template <class K, class Pk>
__global__ __launch_bounds__(K::kThreads) void k_group(const unsigned char* __restrict__ tab, uint32_t stride) {
  const Pk p = *reinterpret_cast<const Pk*>(tab + size_t(blockIdx.z) * stride);
  run_pack<K>(p);
}

// ---------------------------------------------------------------- recording

using GroupLaunchFn = void (*)(dim3 grid, dim3 block, size_t shmem, hipStream_t s, const unsigned char* tab,
                               uint32_t stride);

struct LaunchRecord {
  const void* kernel = nullptr;  // identity: the work-list entry point of the kernel
  GroupLaunchFn launch_group = nullptr;
  dim3 grid, block;
  size_t shmem = 0;
  size_t align = 1;
  std::vector<unsigned char> args;  // the argument pack's bytes
};

struct LaunchRecorder {
  std::vector<LaunchRecord> list;
};

// The recorder of the calling host thread (null: launches run).
inline LaunchRecorder*& launch_recorder() {
  thread_local LaunchRecorder* r = nullptr;
  return r;
}

// Installs a recorder for the lifetime of the object.
struct RecordScope {
  LaunchRecorder* saved;
  explicit RecordScope(LaunchRecorder& r) : saved(launch_recorder()) { launch_recorder() = &r; }
  ~RecordScope() { launch_recorder() = saved; }
  RecordScope(const RecordScope&) = delete;
  RecordScope& operator=(const RecordScope&) = delete;
};

template <class Sig>
struct KernelParams;
template <class... P>
struct KernelParams<void (*)(P...)> {
  using pack = Pack<std::decay_t<P>...>;
  template <class K>
  static void group_fn(dim3 grid, dim3 block, size_t shmem, hipStream_t s, const unsigned char* tab,
                       uint32_t stride) {
    k_group<K, pack><<<grid, block, shmem, s>>>(tab, stride);
  }
  template <class K>
  static void go(dim3 grid, dim3 block, size_t shmem, hipStream_t s, std::decay_t<P>... a) {
    if (LaunchRecorder* rec = launch_recorder()) {
      static_assert(std::is_trivially_copyable<pack>::value, "kernel arguments are copied as bytes");
      // built in zeroed storage so padding bytes are zero and equal argument
      // values give equal bytes (work-list graphs are keyed on these bytes)
      alignas(pack) unsigned char raw[sizeof(pack)] = {};
      new (raw) pack{{a}...};
      LaunchRecord r;
      r.kernel = reinterpret_cast<const void*>(&k_group<K, pack>);
      r.launch_group = &group_fn<K>;
      r.grid = grid;
      r.block = block;
      r.shmem = shmem;
      r.align = alignof(pack);
      r.args.resize(sizeof(pack));
      std::memcpy(r.args.data(), raw, sizeof(pack));
      rec->list.push_back(std::move(r));
      return;
    }
    k_entry<K, std::decay_t<P>...><<<grid, block, shmem, s>>>(a...);
  }
};

template <class K, class... A>
inline void launch(dim3 grid, dim3 block, size_t shmem, hipStream_t s, A&&... a) {
  KernelParams<decltype(&K::run)>::template go<K>(grid, block, shmem, s, std::forward<A>(a)...);
}

}  // namespace pcheb

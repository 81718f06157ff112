// Work lists over several problems of one shape (pcheb_group_* in include/pcheb.h).
//
// Each problem keeps its own handle: operator data, recurrence coefficients,
// workspace and device scalars.  A group call records, per problem, the
// launches the single-problem code path would make (launch.hpp), checks that
// the problems' sequences coincide kernel by kernel, uploads the argument
// packs as one table, and then issues each launch once with grid dimension z
// = problem.  The PCG iteration pair is captured as one HIP graph of those
// work-list launches, replayed like a handle's own graph, and the host polls
// all problems' states with one gather kernel and one copy per poll.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "handle.hpp"
#include "solver.hpp"

namespace pcheb {

constexpr int kMaxGroup = 1024;  // problems per group (grid dimension z)

// dst[i] = slot 0 state of problem i.
struct KGatherStates {
  static constexpr int kThreads = 256;
  __device__ static void run(const DevState* const* src, DevState* dst, int count) {
    const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (i < count) dst[i] = *src[i];
  }
};

// One merged launch sequence: launch j of every problem, with its table entry.
struct Phase {
  struct Entry {
    GroupLaunchFn fn;
    dim3 grid, block;
    size_t shmem;
    size_t offset;    // of problem 0's argument pack in the table
    uint32_t stride;  // bytes between consecutive problems' packs
  };
  std::vector<Entry> entries;
  size_t begin = 0, end = 0;  // the phase's bytes in the table
};

static size_t round_up_bytes(size_t v, size_t m) { return (v + m - 1) / m * m; }

static bool same_dim(const dim3& a, const dim3& b) { return a.x == b.x && a.y == b.y && a.z == b.z; }

// Appends the phase's argument tables to `table` (launch-major, problem-minor)
// after checking that every problem makes the same launches.
static void merge(const std::vector<LaunchRecorder>& recs, const char* what, Phase& ph,
                  std::vector<unsigned char>& table) {
  const size_t count = recs.size();
  const std::vector<LaunchRecord>& ref = recs[0].list;
  for (size_t i = 1; i < count; ++i)
    if (recs[i].list.size() != ref.size())
      fail(PCHEB_INVALID, std::string(what) + ": problem " + std::to_string(i) + " makes " +
                              std::to_string(recs[i].list.size()) + " launches, problem 0 makes " +
                              std::to_string(ref.size()) + " (the problems differ in shape or parameters)");
  ph.entries.clear();
  ph.begin = round_up_bytes(table.size(), 256);
  table.resize(ph.begin);
  for (size_t j = 0; j < ref.size(); ++j) {
    const LaunchRecord& a = ref[j];
    if (a.grid.z != 1) fail(PCHEB_HIP, "internal: a recorded launch uses grid dimension z");
    for (size_t i = 1; i < count; ++i) {
      const LaunchRecord& b = recs[i].list[j];
      if (b.kernel != a.kernel || !same_dim(b.grid, a.grid) || !same_dim(b.block, a.block) || b.shmem != a.shmem ||
          b.args.size() != a.args.size())
        fail(PCHEB_INVALID, std::string(what) + ": launch " + std::to_string(j) + " of problem " + std::to_string(i) +
                                " differs from problem 0's in kernel, grid or block (the problems differ in shape "
                                "or parameters)");
    }
    // every problem's pack at the pack type's alignment (at least 16 bytes)
    const size_t al = std::max<size_t>(16, a.align);
    const size_t stride = round_up_bytes(a.args.size(), al);
    const size_t off = round_up_bytes(table.size(), al);
    table.resize(off + stride * count);
    for (size_t i = 0; i < count; ++i)
      std::memcpy(table.data() + off + i * stride, recs[i].list[j].args.data(), a.args.size());
    ph.entries.push_back(Phase::Entry{a.launch_group, a.grid, a.block, a.shmem, off, uint32_t(stride)});
  }
  ph.end = table.size();
}

static void enqueue_phase(const Phase& ph, const unsigned char* dtab, int count, hipStream_t s) {
  for (const Phase::Entry& e : ph.entries) e.fn(dim3(e.grid.x, e.grid.y, uint32_t(count)), e.block, e.shmem, s,
                                                dtab + e.offset, e.stride);
  PCHEB_HIP_CHECK(hipGetLastError());
}

struct Group {
  std::vector<Handle*> hs;
  int count = 0;
  int device = 0;
  DeviceBuffer table;                 // argument tables of the current call
  unsigned char* staging = nullptr;   // pinned host copy of the tables
  size_t staging_cap = 0;
  DeviceBuffer states;                // count DevState* (each problem's slot 0), then count DevState
  DevState* host_states = nullptr;    // pinned: two rounds of count states
  hipEvent_t done = nullptr;          // end of the last call's work
  bool done_recorded = false;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  Phase graph_phase;  // the pair phase's launches the graph was captured with
  const void* graph_table = nullptr;

  const DevState* const* state_ptrs() const { return static_cast<const DevState* const*>(states.ptr); }
  DevState* gathered() const {
    return reinterpret_cast<DevState*>(static_cast<char*>(states.ptr) + round_up_bytes(sizeof(void*) * count, 256));
  }
};

static void destroy_group(Group* g) {
  if (!g) return;
  if (g->done) {
    (void)hipEventSynchronize(g->done);
    (void)hipEventDestroy(g->done);
  }
  if (g->graph) (void)hipGraphExecDestroy(g->graph);
  if (g->capture_stream) (void)hipStreamDestroy(g->capture_stream);
  if (g->staging) (void)hipHostFree(g->staging);
  if (g->host_states) (void)hipHostFree(g->host_states);
  std::vector<DeviceBuffer> blocks{g->table, g->states};
  device_free_all(blocks);
  delete g;
}

// Waits for the previous call's work, which still reads the tables.
static void wait_previous(Group& g) {
  if (g.done_recorded) PCHEB_HIP_CHECK(hipEventSynchronize(g.done));
  g.done_recorded = false;
}

static void upload(Group& g, const std::vector<unsigned char>& table, hipStream_t s) {
  const size_t bytes = std::max<size_t>(table.size(), 256);
  if (g.table.bytes < bytes) {
    std::vector<DeviceBuffer> old{g.table};
    g.table = DeviceBuffer{};
    device_free_all(old);
    g.table = device_alloc(bytes);
  }
  if (g.staging_cap < bytes) {
    if (g.staging) PCHEB_HIP_CHECK(hipHostFree(g.staging));
    g.staging = nullptr;
    g.staging_cap = 0;
    PCHEB_HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&g.staging), bytes, hipHostMallocDefault));
    g.staging_cap = bytes;
  }
  std::memcpy(g.staging, table.data(), table.size());
  PCHEB_HIP_CHECK(hipMemcpyAsync(g.table.ptr, g.staging, table.size(), hipMemcpyHostToDevice, s));
}

static const unsigned char* dtab(const Group& g) { return static_cast<const unsigned char*>(g.table.ptr); }

static bool same_launches(const Phase& a, const Phase& b) {
  if (a.entries.size() != b.entries.size()) return false;
  for (size_t j = 0; j < a.entries.size(); ++j) {
    const Phase::Entry& x = a.entries[j];
    const Phase::Entry& y = b.entries[j];
    if (x.fn != y.fn || !same_dim(x.grid, y.grid) || !same_dim(x.block, y.block) || x.shmem != y.shmem ||
        x.offset != y.offset || x.stride != y.stride)
      return false;
  }
  return true;
}

// The iteration pair as a graph of work-list launches.  Its kernel nodes hold
// only table addresses; the argument packs (vectors, flags, workspace) are read
// from the table, which every call uploads before the first replay.  So the
// graph is captured again only when the launches change (kernels, grids, table
// offsets) or the table was reallocated.
static void ensure_graph(Group& g, const Phase& pair) {
  if (g.graph && g.graph_table == g.table.ptr && same_launches(g.graph_phase, pair)) return;
  if (!g.capture_stream) PCHEB_HIP_CHECK(hipStreamCreateWithFlags(&g.capture_stream, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  PCHEB_HIP_CHECK(hipStreamBeginCapture(g.capture_stream, hipStreamCaptureModeRelaxed));
  try {
    enqueue_phase(pair, dtab(g), g.count, g.capture_stream);
  } catch (...) {
    (void)hipStreamEndCapture(g.capture_stream, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  PCHEB_HIP_CHECK(hipStreamEndCapture(g.capture_stream, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  PCHEB_HIP_CHECK(e);
  if (g.graph) (void)hipGraphExecDestroy(g.graph);
  g.graph = exec;
  g.graph_phase = pair;
  g.graph_table = g.table.ptr;
}

static void gather_states(Group& g, DevState* host, hipStream_t s) {
  launch<KGatherStates>(dim3((uint32_t(g.count) + 255) / 256), 256, 0, s, g.state_ptrs(), g.gathered(), g.count);
  PCHEB_HIP_CHECK(hipMemcpyAsync(host, g.gathered(), size_t(g.count) * sizeof(DevState), hipMemcpyDeviceToHost, s));
}

template <class F>
static std::vector<LaunchRecorder> record(const Group& g, F&& f) {
  std::vector<LaunchRecorder> recs(size_t(g.count));
  for (int i = 0; i < g.count; ++i) {
    RecordScope scope(recs[size_t(i)]);
    f(*g.hs[size_t(i)], i);
  }
  return recs;
}

static Group* create_group(const pcheb_handle* handles, int count) {
  if (!handles) fail(PCHEB_INVALID, "handles is null");
  if (count < 1 || count > kMaxGroup) fail(PCHEB_INVALID, "count must be in [1, 1024]");
  std::vector<Handle*> hs(static_cast<size_t>(count));
  for (int i = 0; i < count; ++i) {
    if (!handles[i]) fail(PCHEB_INVALID, "null handle in the group");
    hs[size_t(i)] = reinterpret_cast<Handle*>(handles[i]);
  }
  {
    std::vector<Handle*> sorted = hs;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      fail(PCHEB_INVALID, "a handle appears twice in the group");
  }
  for (Handle* h : hs)
    if (h->device != hs[0]->device || h->n != hs[0]->n)
      fail(PCHEB_INVALID, "the group's problems must have the same size and device");
  Group* g = new Group();
  g->hs = hs;
  g->count = count;
  g->device = hs[0]->device;
  try {
    // the launches must coincide: compare an apply and an iteration pair (recording launches nothing)
    std::vector<unsigned char> table;
    Phase ph;
    const int64_t ld = (hs[0]->n + 1) / 2 * 2;
    merge(record(*g, [&](Handle& h, int) { solver_apply(h, nullptr, nullptr, nullptr); }), "preconditioner", ph,
          table);
    merge(record(*g, [&](Handle& h, int) { solver_iterations_direct(h, Slots{0, 1}, nullptr, ld, 1, nullptr); }),
          "PCG iteration", ph, table);
    g->states = device_alloc(round_up_bytes(sizeof(void*) * count, 256) + sizeof(DevState) * size_t(count));
    std::vector<const DevState*> ptrs(static_cast<size_t>(count));
    for (int i = 0; i < count; ++i) ptrs[size_t(i)] = hs[size_t(i)]->st;
    PCHEB_HIP_CHECK(hipMemcpy(g->states.ptr, ptrs.data(), sizeof(void*) * size_t(count), hipMemcpyHostToDevice));
    PCHEB_HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&g->host_states), 2 * sizeof(DevState) * size_t(count),
                                  hipHostMallocDefault));
    PCHEB_HIP_CHECK(hipEventCreateWithFlags(&g->done, hipEventDisableTiming));
  } catch (...) {
    destroy_group(g);
    throw;
  }
  return g;
}

// The slot-0 state pointers change when a handle's workspace is reallocated.
static void refresh_state_ptrs(Group& g, hipStream_t s) {
  for (Handle* h : g.hs) ensure_workspace(*h, 1, s);
  std::vector<const DevState*> ptrs(size_t(g.count));
  for (int i = 0; i < g.count; ++i) ptrs[size_t(i)] = g.hs[size_t(i)]->st;
  PCHEB_HIP_CHECK(hipMemcpy(g.states.ptr, ptrs.data(), sizeof(void*) * size_t(g.count), hipMemcpyHostToDevice));
}

static void check_group_vectors(const Group& g, const void* a, const void* b, int64_t ld) {
  if (!a || !b) fail(PCHEB_INVALID, "null vector");
  const int64_t n = g.hs[0]->n;
  if (ld < n) fail(PCHEB_INVALID, "ld must be >= n");
  if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) % 16 != 0)
    fail(PCHEB_INVALID, "vectors must be 16-byte aligned");
  if (g.count > 1 && ld % 2 != 0) fail(PCHEB_INVALID, "ld must be even when the group has more than one problem");
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  const size_t bytes = (size_t(g.count - 1) * size_t(ld) + size_t(n)) * 8;
  if (pa < pb + bytes && pb < pa + bytes) fail(PCHEB_INVALID, "input and output vectors overlap");
}

static void group_apply(Group& g, const double* r, double* z, int64_t ld, hipStream_t s) {
  check_group_vectors(g, r, z, ld);
  wait_previous(g);
  for (Handle* h : g.hs) ensure_workspace(*h, 1, s);
  std::vector<unsigned char> table;
  Phase ph;
  merge(record(g, [&](Handle& h, int i) { solver_apply(h, r + int64_t(i) * ld, z + int64_t(i) * ld, s); }),
        "preconditioner", ph, table);
  upload(g, table, s);
  enqueue_phase(ph, dtab(g), g.count, s);
  PCHEB_HIP_CHECK(hipEventRecord(g.done, s));
  g.done_recorded = true;
}

static pcheb_status group_solve(Group& g, const double* b, double* x, int64_t ld, double tol, int maxit,
                                uint32_t flags, pcg_stats* stats, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  check_group_vectors(g, b, x, ld);
  if (!(tol > 0.0) || !std::isfinite(tol)) fail(PCHEB_INVALID, "tol must be positive");
  if (maxit < 1) fail(PCHEB_INVALID, "maxit must be >= 1");
  if (flags & (PCG_TIME_KERNELS | PCG_REFRESH))
    fail(PCHEB_INVALID, "PCG_TIME_KERNELS and PCG_REFRESH are not available for groups");
  wait_previous(g);
  refresh_state_ptrs(g, s);
  const int flexible = (flags & PCG_FLEXIBLE) ? 1 : 0;
  const bool x0_given = (flags & PCG_X0_GIVEN) != 0;
  const bool use_graph = !(flags & PCG_NO_GRAPH);
  const Slots one{0, 1};
  auto bi = [&](int i) { return b + int64_t(i) * ld; };
  auto xi = [&](int i) { return x + int64_t(i) * ld; };

  // the pair phase first: its table offset is the same on every call
  std::vector<unsigned char> table;
  Phase pair, init, start, finish;
  merge(record(g, [&](Handle& h, int i) { solver_iterations_direct(h, one, xi(i), ld, flexible, s); }),
        "PCG iteration", pair, table);
  merge(record(g, [&](Handle& h, int) { solver_init_states(h, one, tol, maxit, flexible, s); }), "solver state",
        init, table);
  merge(record(g, [&](Handle& h, int i) { solver_start(h, one, bi(i), ld, xi(i), ld, x0_given, flexible, s); }),
        "PCG start", start, table);
  merge(record(g, [&](Handle& h, int i) { solver_finish(h, one, bi(i), ld, xi(i), ld, s); }), "true residual",
        finish, table);
  upload(g, table, s);
  if (use_graph) ensure_graph(g, pair);

  enqueue_phase(init, dtab(g), g.count, s);
  enqueue_phase(start, dtab(g), g.count, s);

  const int count = g.count;
  auto all_done = [&](const DevState* v) {
    for (int i = 0; i < count; ++i)
      if (v[i].done == kRunning) return false;
    return true;
  };
  hipEvent_t ev[2] = {nullptr, nullptr};
  int64_t issued = 0;
  int chunk = 2, half = 0;
  bool have_prev = false;
  try {
    PCHEB_HIP_CHECK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    PCHEB_HIP_CHECK(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    for (;;) {
      for (int p = 0; p < chunk / 2; ++p) {
        if (use_graph)
          PCHEB_HIP_CHECK(hipGraphLaunch(g.graph, s));
        else
          enqueue_phase(pair, dtab(g), count, s);
      }
      issued += chunk;
      DevState* dst = g.host_states + size_t(half) * size_t(count);
      gather_states(g, dst, s);
      PCHEB_HIP_CHECK(hipEventRecord(ev[half], s));
      if (have_prev) {
        PCHEB_HIP_CHECK(hipEventSynchronize(ev[half ^ 1]));
        if (all_done(g.host_states + size_t(half ^ 1) * size_t(count))) break;
      }
      have_prev = true;
      half ^= 1;
      if (chunk < 16) chunk *= 2;
      if (issued > int64_t(maxit) + 64) {
        PCHEB_HIP_CHECK(hipEventSynchronize(ev[half ^ 1]));
        break;
      }
    }
  } catch (...) {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    throw;
  }
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);

  enqueue_phase(finish, dtab(g), count, s);
  gather_states(g, g.host_states, s);
  PCHEB_HIP_CHECK(hipEventRecord(g.done, s));
  g.done_recorded = true;
  PCHEB_HIP_CHECK(hipStreamSynchronize(s));

  const double seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  pcheb_status result = PCHEB_OK;
  for (int i = 0; i < count; ++i) {
    pcg_stats local;
    fill_stats(*g.hs[size_t(i)], g.host_states[i], flags, &local);
    local.seconds = seconds;
    if (stats) stats[i] = local;
    if (result == PCHEB_OK && local.status != PCHEB_OK) result = pcheb_status(local.status);
  }
  return result;
}

}  // namespace pcheb

using namespace pcheb;

template <class F>
static pcheb_status group_guarded(F&& f) {
  try {
    set_last_error("");
    return f();
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return PCHEB_OOM;
  } catch (...) {
    set_last_error("unexpected internal error");
    return PCHEB_HIP;
  }
}

static Group* as_group(pcheb_group g) {
  if (!g) fail(PCHEB_INVALID, "null group");
  return reinterpret_cast<Group*>(g);
}

extern "C" {

pcheb_status pcheb_group_create(const pcheb_handle* handles, int32_t count, pcheb_group* out) {
  return group_guarded([&]() -> pcheb_status {
    if (!out) fail(PCHEB_INVALID, "out is null");
    *out = reinterpret_cast<pcheb_group>(create_group(handles, count));
    return PCHEB_OK;
  });
}

pcheb_status pcheb_group_apply(pcheb_group g, const double* r, double* z, int64_t ld, hipStream_t stream) {
  return group_guarded([&]() -> pcheb_status {
    group_apply(*as_group(g), r, z, ld, stream);
    return PCHEB_OK;
  });
}

pcheb_status pcg_solve_group(pcheb_group g, const double* b, double* x, int64_t ld, double tol, int32_t maxit,
                             uint32_t flags, pcg_stats* stats, hipStream_t stream) {
  return group_guarded([&]() -> pcheb_status {
    const pcheb_status st = group_solve(*as_group(g), b, x, ld, tol, maxit, flags, stats, stream);
    if (st == PCHEB_BREAKDOWN) set_last_error("PCG breakdown in a problem of the group");
    if (st == PCHEB_NOT_CONVERGED) set_last_error("a problem of the group reached maxit without meeting tol");
    return st;
  });
}

pcheb_status pcheb_group_destroy(pcheb_group g) {
  return group_guarded([&]() -> pcheb_status {
    destroy_group(reinterpret_cast<Group*>(g));
    return PCHEB_OK;
  });
}

}  // extern "C"

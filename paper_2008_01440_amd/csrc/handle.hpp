// Host-side state of a preconditioner handle and the helpers every source
// file of the library uses (error reporting, device allocation, launches).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "common.hpp"
#include "pcheb.h"

namespace pcheb {

// Error carrying a status; thrown inside the library, caught at the ABI.
struct Error {
  pcheb_status status;
  std::string msg;
};

[[noreturn]] void fail(pcheb_status st, const std::string& msg);
void check_hip(hipError_t e, const char* what);
void set_last_error(const std::string& msg);

#define PCHEB_HIP_CHECK(expr) ::pcheb::check_hip((expr), #expr)

// A block of device memory and the function that returns it (null: hipFree).
struct DeviceBuffer {
  void* ptr = nullptr;
  size_t bytes = 0;
  pcheb_free_fn free_fn = nullptr;
  void* ctx = nullptr;
};

// Device memory from the allocator installed with pcheb_set_allocator, or hipMalloc
// when none is; throws OOM / HIP / INVALID (a misaligned block).
DeviceBuffer device_alloc(size_t bytes);
// Returns a block to whoever allocated it.  Blocks from a caller's allocator may be
// reused at once, so the caller of this function must have ensured that no device
// work still uses the block (device_free_all does so for a whole list).
void device_free(DeviceBuffer& b);
// Frees every block of the list, after synchronising the device if any of them goes
// back to a caller's allocator (hipFree waits by itself).
void device_free_all(std::vector<DeviceBuffer>& list);

struct Handle {
  pcheb_operator op{};
  pcheb_params prm{};
  int64_t n = 0;
  int device = 0;
  size_t elem = 8;  // bytes per element of the preconditioner vectors

  // Chebyshev scalars (Sec. 3 with the Sec. 4 scaling)
  double theta = 0, delta = 0, sigma = 0;
  std::vector<double> rho;
  int nlev = 0;               // Newton form: k = 2^nlev - 1
  std::vector<double> zeta;   // Newton form: zeta_0 .. zeta_nlev

  // operator data owned by the handle
  double* invd = nullptr;     // D^-1 (null for the 7-point stencil: constant 1/6)
  void* csr_bval = nullptr;   // CSR: values of D^-1 A_hat in the storage precision
  int lanes = 8;              // CSR: lanes per row
  int64_t nchunks = 0;        // SELL
  int64_t nnz_pad = 0;        // SELL
  int64_t* sell_ptr = nullptr;
  int32_t* sell_len = nullptr;
  int32_t* sell_col = nullptr;
  double* sell_aval = nullptr;  // A_hat values (float64)
  void* sell_bval = nullptr;    // D^-1 A_hat values (storage precision)
  int32_t* sell_perm = nullptr; // null when sigma == 1
  double* rho64 = nullptr;      // STENCIL27H: 1 / (2 kappa) per cell (double products)
  float* rho_lo = nullptr;      // STENCIL27H, float recurrences: 1 / (2 kappa) per cell
  float* invd_lo = nullptr;     // STENCIL27H, float recurrences: D^-1 rounded to float
  int bs = 1;                   // first-level block size (1: Jacobi scaling, 3: node blocks)
  double* binv = nullptr;       // bs == 3: per node, the symmetric inverse of its 3x3 diagonal block
                                // (xx, xy, xz, yy, yz, zz)
  double* lfac = nullptr;       // bs == 3: per node, L^-1 of the block's Cholesky factor L
                                // (row-major lower triangle: 00, 10, 11, 20, 21, 22)

  // solve workspace for `cap` right-hand sides (slots); vectors of slot j start
  // at j * ldw elements.  Allocated on demand, separately from the operator data.
  int cap = 0;
  int64_t ldw = 0;
  int nY = 3;                 // iterate buffers in use (4 when steps are fused)
  std::vector<void*> nt;      // Newton form: 2 nlev + 1 iterate buffers (cap slots each)
  int fuse = 1;               // recurrence steps per pass (7-point stencil only)
  void* s = nullptr;          // D^-1 r (storage precision)
  void* Y[4] = {nullptr, nullptr, nullptr, nullptr};  // recurrence iterates (storage precision)
  double* r = nullptr;
  double* p[2] = {nullptr, nullptr};
  double* q = nullptr;
  double* z = nullptr;
  DevState* st = nullptr;       // device scalars, one per slot
  DevState* st_host = nullptr;  // pinned host mirror: two groups of cap states
  double* partials = nullptr;   // cap * kMaxGrid * kMaxReduce

  // graph cache for the PCG iteration pair (captured on a private stream,
  // launched on the caller's; the legacy null stream cannot be captured)
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  const double* graph_x = nullptr;
  int64_t graph_ldx = 0;
  int graph_slots = 0;
  uint32_t graph_flags = 0;

  std::vector<hipEvent_t> events;
  std::vector<DeviceBuffer> owned;     // operator data
  std::vector<DeviceBuffer> owned_ws;  // solve workspace

  // When set, dev_alloc carves 256-byte aligned pieces from this caller-provided
  // device range instead of allocating (nothing is freed back; the range is
  // reused by the next handle that gets it).
  char* arena = nullptr;
  size_t arena_cap = 0;
  size_t arena_used = 0;

  ReduceBuf rb() const { return ReduceBuf{partials}; }
};

void* dev_alloc(Handle& h, size_t bytes);
void setup_operator(Handle& h, hipStream_t s);
void release(Handle& h);

// A contiguous range of solve slots covered by one launch.
struct Slots {
  int first;
  int count;
};

inline uint32_t round_grid(uint64_t tiles) {
  uint64_t g = tiles < uint64_t(kMaxGrid) ? tiles : uint64_t(kMaxGrid);
  g = (g + kNumXcd - 1) / kNumXcd * kNumXcd;
  return uint32_t(g < kNumXcd ? kNumXcd : g);
}

}  // namespace pcheb

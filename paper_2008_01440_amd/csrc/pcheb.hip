// pcheb: set-up, preconditioner application, operator product and the PCG
// driver of the Newton-Chebyshev preconditioned CG (arXiv:2008.01440) on
// gfx950.  The C ABI is declared in include/pcheb.h; the solver internals the
// serving engine also uses are declared in solver.hpp.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "dispatch.hpp"
#include "fused_launch.hpp"
#include "handle.hpp"
#include "solver.hpp"

namespace pcheb {

// ================================================================ errors and memory

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }

const char* last_error_cstr() { return g_last_error.c_str(); }

void fail(pcheb_status st, const std::string& msg) { throw Error{st, msg}; }

void check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  const pcheb_status st = (e == hipErrorOutOfMemory) ? PCHEB_OOM : PCHEB_HIP;
  fail(st, std::string(what) + ": " + hipGetErrorString(e));
}

// The allocator installed with pcheb_set_allocator (none: hipMalloc / hipFree).
struct AllocatorFns {
  pcheb_alloc_fn alloc = nullptr;
  pcheb_free_fn free = nullptr;
  void* ctx = nullptr;
};
static std::mutex g_alloc_mu;
static AllocatorFns g_alloc;

DeviceBuffer device_alloc(size_t bytes) {
  if (bytes == 0) bytes = 8;
  AllocatorFns a;
  {
    std::lock_guard<std::mutex> lock(g_alloc_mu);
    a = g_alloc;
  }
  DeviceBuffer b;
  b.bytes = bytes;
  if (a.alloc) {
    void* p = a.alloc(bytes, a.ctx);
    if (!p) fail(PCHEB_OOM, "the installed allocator returned no block of " + std::to_string(bytes) + " bytes");
    if (reinterpret_cast<uintptr_t>(p) % 256 != 0) {
      a.free(p, bytes, a.ctx);
      fail(PCHEB_INVALID, "the installed allocator returned a block that is not 256-byte aligned");
    }
    b.ptr = p;
    b.free_fn = a.free;
    b.ctx = a.ctx;
    return b;
  }
  const hipError_t e = hipMalloc(&b.ptr, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? PCHEB_OOM : PCHEB_HIP,
         "hipMalloc of " + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
  }
  return b;
}

void device_free(DeviceBuffer& b) {
  if (!b.ptr) return;
  if (b.free_fn)
    b.free_fn(b.ptr, b.bytes, b.ctx);
  else
    (void)hipFree(b.ptr);
  b.ptr = nullptr;
}

void device_free_all(std::vector<DeviceBuffer>& list) {
  bool to_caller = false;
  for (const auto& b : list) to_caller = to_caller || (b.ptr && b.free_fn);
  if (to_caller) (void)hipDeviceSynchronize();
  for (auto& b : list) device_free(b);
  list.clear();
}

static void* alloc_into(std::vector<DeviceBuffer>& list, size_t bytes) {
  list.push_back(device_alloc(bytes));
  return list.back().ptr;
}

void* dev_alloc(Handle& h, size_t bytes) {
  if (h.arena) {
    const size_t off = (h.arena_used + 255) / 256 * 256;
    if (bytes > h.arena_cap || off > h.arena_cap - bytes)
      fail(PCHEB_INVALID, "workspace exceeds the " + std::to_string(h.arena_cap) + "-byte scratch");
    h.arena_used = off + bytes;
    return h.arena + off;
  }
  return alloc_into(h.owned, bytes);
}

static void drop_graph(Handle& h) {
  if (h.graph_exec) (void)hipGraphExecDestroy(h.graph_exec);
  h.graph_exec = nullptr;
  h.graph_x = nullptr;
}

static void release_workspace(Handle& h) {
  drop_graph(h);
  if (h.st_host) (void)hipHostFree(h.st_host);
  h.st_host = nullptr;
  device_free_all(h.owned_ws);
  h.nt.clear();
  h.cap = 0;
}

void release(Handle& h) {
  release_workspace(h);
  if (h.capture_stream) (void)hipStreamDestroy(h.capture_stream);
  h.capture_stream = nullptr;
  for (hipEvent_t e : h.events) (void)hipEventDestroy(e);
  h.events.clear();
  device_free_all(h.owned);
}

static size_t storage_bytes(int prec) { return prec == PCHEB_F64 ? 8 : (prec == PCHEB_F32 ? 4 : 2); }

static int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// ================================================================ elementwise kernels

static uint32_t flat_grid(int64_t n) {
  const int64_t per_block = int64_t(kBlock) * 4;
  int64_t g = (n + per_block - 1) / per_block;
  g = std::max<int64_t>(1, std::min<int64_t>(g, kMaxGrid));
  return uint32_t(g);
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < (n); i += int64_t(gridDim.x) * blockDim.x)

__global__ void k_fill(double* p, int64_t n, double v) {
  GRID_STRIDE(i, n) p[i] = v;
}

// CSR diagonal (sum of entries on the diagonal) -> 1/d; flags d <= 0.
__global__ void k_csr_invdiag(const int32_t* rowptr, const int32_t* col, const double* val, int64_t n,
                              double* invd, int* bad) {
  GRID_STRIDE(i, n) {
    double d = 0.0;
    for (int32_t j = rowptr[i]; j < rowptr[i + 1]; ++j)
      if (col[j] == i) d += val[j];
    if (!(d > 0.0) || !isfinite(d)) {
      atomicOr(bad, 1);
      invd[i] = 0.0;
    } else {
      invd[i] = 1.0 / d;
    }
  }
}

// 27-point harmonic operator diagonal: sum of the 26 harmonic means, k_i for
// every neighbour outside the grid.  Flags coefficients <= 0 (bit 1) and
// positive ones outside [kH27CoeffMin, kH27CoeffMax] (bit 4): the float64
// products multiply two face sums 1/(2 k_i) + 1/(2 k_n), which must stay normal.
constexpr double kH27CoeffMin = 1e-150, kH27CoeffMax = 1e150;
__global__ void k_h27_invdiag(const double* kappa, int nx, int ny, int nz, double* invd, int* bad) {
  const int64_t n = int64_t(nx) * ny * nz;
  GRID_STRIDE(i, n) {
    const int x = int(i % nx);
    const int y = int((i / nx) % ny);
    const int z = int(i / (int64_t(nx) * ny));
    const double ki = kappa[i];
    if (!(ki > 0.0) || !isfinite(ki)) {
      atomicOr(bad, 1);
      invd[i] = 0.0;
      continue;
    }
    if (ki < kH27CoeffMin || ki > kH27CoeffMax) atomicOr(bad, 4);
    double d = 0.0;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (!dz && !dy && !dx) continue;
          const int xx = x + dx, yy = y + dy, zz = z + dz;
          if (xx < 0 || xx >= nx || yy < 0 || yy >= ny || zz < 0 || zz >= nz) {
            d += ki;
          } else {
            const double kn = kappa[xx + int64_t(nx) * (yy + int64_t(ny) * zz)];
            d += kn > 0.0 ? 2.0 * ki * kn / (ki + kn) : ki;
          }
        }
    invd[i] = 1.0 / d;
  }
}

// rho = 1 / (2 kappa) per cell for the double 27-point products.
__global__ void k_h27_rho64(const double* kappa, double* rho, int64_t n) {
  GRID_STRIDE(i, n) rho[i] = 0.5 / kappa[i];
}

// Operator data of the float recurrences on the 27-point operator: rho = 1 / (2 kappa)
// and D^-1, both rounded to float.
__global__ void k_h27_lo(const double* kappa, const double* invd, float* rho, float* invd_lo, int64_t n) {
  GRID_STRIDE(i, n) {
    rho[i] = float(0.5 / kappa[i]);
    invd_lo[i] = float(invd[i]);
  }
}

// Values of D^-1 A_hat in the storage precision (row i scaled by 1/d_i).
template <class T>
__global__ void k_scale_rows(const int32_t* rowptr, const double* val, const double* invd, int64_t n, T* out) {
  GRID_STRIDE(i, n) {
    const double w = invd[i];
    for (int32_t j = rowptr[i]; j < rowptr[i + 1]; ++j) Store<T>::st(out, j, typename Store<T>::acc(val[j] * w));
  }
}

// Node blocks (block size 3, the second-level construction of Sec. 6 on the
// first-level factor P0 = W W^T): node I owns rows 3I, 3I+1, 3I+2, which must
// share one column pattern.  Per node: the 3x3 diagonal block B = L L^T
// (Cholesky), M = L^-1 (so W = blockdiag(M^T)) and B^-1 = M^T M.  Flags a block
// that is not positive definite (bit 0) or rows of a node with different
// patterns (bit 1).
__global__ void k_node_blocks(const int32_t* rowptr, const int32_t* col, const double* val, int64_t nodes,
                              double* binv, double* lfac, int* bad) {
  GRID_STRIDE(I, nodes) {
    const int64_t r0 = 3 * I;
    const int32_t b0 = rowptr[r0], len = rowptr[r0 + 1] - b0;
    bool same = rowptr[r0 + 2] - rowptr[r0 + 1] == len && rowptr[r0 + 3] - rowptr[r0 + 2] == len;
    double b[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int a = 0; a < 3 && same; ++a) {
      const int32_t ba = rowptr[r0 + a];
      for (int32_t t = 0; t < len; ++t) {
        const int32_t c = col[ba + t];
        if (c != col[b0 + t]) same = false;
        const int64_t d = int64_t(c) - r0;
        if (d >= 0 && d < 3) b[a][d] += val[ba + t];
      }
    }
    if (!same) {
      atomicOr(bad, 2);
      continue;
    }
    const double d00 = b[0][0];
    const double l00 = sqrt(d00);
    const double l10 = b[1][0] / l00, l20 = b[2][0] / l00;
    const double d11 = b[1][1] - l10 * l10;
    const double l11 = sqrt(d11);
    const double l21 = (b[2][1] - l20 * l10) / l11;
    const double d22 = b[2][2] - l20 * l20 - l21 * l21;
    const double l22 = sqrt(d22);
    if (!(d00 > 0.0) || !(d11 > 0.0) || !(d22 > 0.0) || !isfinite(l21) || !isfinite(d22)) {
      atomicOr(bad, 1);
      continue;
    }
    const double m00 = 1.0 / l00, m11 = 1.0 / l11, m22 = 1.0 / l22;
    const double m10 = -l10 * m00 * m11;
    const double m21 = -l21 * m11 * m22;
    const double m20 = -(l20 * m00 + l21 * m10) * m22;
    double* lf = lfac + 6 * I;
    lf[0] = m00;
    lf[1] = m10;
    lf[2] = m11;
    lf[3] = m20;
    lf[4] = m21;
    lf[5] = m22;
    double* bi = binv + 6 * I;  // (M^T M)_ij = sum over k >= max(i, j) of M_ki M_kj
    bi[0] = m00 * m00 + m10 * m10 + m20 * m20;
    bi[1] = m10 * m11 + m20 * m21;
    bi[2] = m20 * m22;
    bi[3] = m11 * m11 + m21 * m21;
    bi[4] = m21 * m22;
    bi[5] = m22 * m22;
  }
}

// Row a (0..2) of a node's symmetric B^-1 stored as (xx, xy, xz, yy, yz, zz).
__device__ __forceinline__ void binv_row(const double* bi, int a, double& c0, double& c1, double& c2) {
  c0 = a == 0 ? bi[0] : (a == 1 ? bi[1] : bi[2]);
  c1 = a == 0 ? bi[1] : (a == 1 ? bi[3] : bi[4]);
  c2 = a == 0 ? bi[2] : (a == 1 ? bi[4] : bi[5]);
}

// Values of B^-1 A_hat in the storage precision: row 3I+a is the combination of
// the node's three rows (same pattern, so entry t of each is one column).
template <class T>
__global__ void k_scale_rows_node(const int32_t* rowptr, const double* val, const double* binv, int64_t n, T* out) {
  GRID_STRIDE(i, n) {
    const int64_t I = i / 3;
    double c0, c1, c2;
    binv_row(binv + 6 * I, int(i - 3 * I), c0, c1, c2);
    const int32_t b = rowptr[i], e = rowptr[i + 1];
    const int32_t q0 = rowptr[3 * I], q1 = rowptr[3 * I + 1], q2 = rowptr[3 * I + 2];
    for (int32_t t = 0; t < e - b; ++t)
      Store<T>::st(out, b + t, typename Store<T>::acc(c0 * val[q0 + t] + c1 * val[q1 + t] + c2 * val[q2 + t]));
  }
}

// Fill the SELL-C-sigma arrays (C = 64) from CSR; padding gets column 0, value 0.
// The recurrence values are D^-1 A_hat (binv null) or B^-1 A_hat (node blocks).
template <class T>
__global__ void k_sell_fill(const int32_t* rowptr, const int32_t* col, const double* val, const double* invd,
                            const double* binv, const int32_t* perm, const int64_t* cptr, const int32_t* clen,
                            int64_t n, int64_t nchunks, int32_t* scol, double* saval, T* sbval) {
  GRID_STRIDE(pos, nchunks * kWave) {
    const int64_t c = pos / kWave;
    const int lane = int(pos % kWave);
    const int32_t len = clen[c];
    int64_t row = -1;
    int32_t b = 0, rl = 0;
    if (pos < n) {
      row = perm ? perm[pos] : pos;
      b = rowptr[row];
      rl = rowptr[row + 1] - b;
    }
    for (int32_t j = 0; j < len; ++j) {
      const int64_t e = cptr[c] + int64_t(j) * kWave + lane;
      if (j < rl) {
        scol[e] = col[b + j];
        saval[e] = val[b + j];
        double bv;
        if (binv) {
          const int64_t I = row / 3;
          double c0, c1, c2;
          binv_row(binv + 6 * I, int(row - 3 * I), c0, c1, c2);
          bv = c0 * val[rowptr[3 * I] + j] + c1 * val[rowptr[3 * I + 1] + j] + c2 * val[rowptr[3 * I + 2] + j];
        } else {
          bv = val[b + j] * invd[row];
        }
        Store<T>::st(sbval, e, typename Store<T>::acc(bv));
      } else {
        scol[e] = 0;
        saval[e] = 0.0;
        Store<T>::st(sbval, e, typename Store<T>::acc(0));
      }
    }
  }
}

// Elementwise kernels walk the vectors in pairs of elements (16-byte float64
// accesses; every vector is 16-byte aligned), with a scalar tail for odd n.
// blockIdx.y selects the solve slot (slot0 + blockIdx.y); workspace vectors
// of slot j start at j * ldw, caller vectors at j * ld of the caller.
#define PAIR_STRIDE(i, n)                                                                  \
  for (int64_t i = 2 * (int64_t(blockIdx.x) * blockDim.x + threadIdx.x); i < (n);           \
       i += 2 * int64_t(gridDim.x) * blockDim.x)

static uint32_t pair_grid(int64_t n) { return flat_grid((n + 1) / 2); }

__device__ __forceinline__ double2 invd2(InvDiag d, int64_t i) {
  return d.p ? ld2(d.p, i) : make_double2(d.c, d.c);
}

struct FinStart {
  DevState* st;
  __device__ void bind(int slot) { st += slot; }
  __device__ void operator()(double (&t)[2]) const {
    st->bb = t[0];
    st->rr = t[0];
    st->bb_hat = t[1];
    st->relres = t[0] > 0.0 ? 1.0 : 0.0;
    if (!(t[0] > 0.0)) st->done = isfinite(t[0]) ? kConverged : kBreakdown;
  }
};

struct FinBeta {
  DevState* st;
  int init, flexible;
  __device__ void bind(int slot) { st += slot; }
  __device__ void operator()(double (&t)[2]) const {
    EpiChebLast<double, true, true>::finish_beta(st, t[0], t[1], init, flexible);
  }
};

// Stop test after the update: iteration count, relative residual, limits, and
// (MODE 1, degree 0) beta from the fused dot products.
template <int MODE>
struct FinUpdate {
  DevState* st;
  __device__ void bind(int slot) { st += slot; }
  __device__ void operator()(double (&t)[3]) const {
    st->rr = t[0];
    st->iter += 1;
    st->relres = sqrt(t[0]) / sqrt(st->bb);
    if (!isfinite(t[0])) {
      st->done = kBreakdown;
    } else if (st->relres < st->tol) {
      st->done = kConverged;
    } else if (st->iter >= st->maxit) {
      st->done = kMaxIter;
    } else if (MODE == 1) {
      EpiChebLast<double, true, true>::finish_beta(st, t[1], t[2], 0, st->flexible);
    }
  }
};

// x0 = 0: x = 0, r = b, p_old = 0 and the norms of b.
struct KStartZero {
  static constexpr int kThreads = 1024;
  __device__ static void run(const double* b, int64_t ldb, double* x, int64_t ldx, double* r, double* p_old,
                             int64_t ldw, InvDiag invd, int64_t n, ReduceBuf rb, int slot0);
};
__device__ __forceinline__ void KStartZero::run(const double* b, int64_t ldb, double* x, int64_t ldx, double* r,
                                                double* p_old, int64_t ldw, InvDiag invd, int64_t n, ReduceBuf rb,
                                                int slot0) {
  const int slot = slot0 + int(blockIdx.y);
  b += slot * ldb;
  x += slot * ldx;
  r += slot * ldw;
  p_old += slot * ldw;
  double part[2] = {0.0, 0.0};
  PAIR_STRIDE(i, n) {
    if (i + 1 < n) {
      const double2 bv = ld2(b, i), w = invd2(invd, i);
      *reinterpret_cast<double2*>(x + i) = make_double2(0.0, 0.0);
      *reinterpret_cast<double2*>(r + i) = bv;
      *reinterpret_cast<double2*>(p_old + i) = make_double2(0.0, 0.0);
      part[0] += bv.x * bv.x * w.x + bv.y * bv.y * w.y;
      part[1] += bv.x * bv.x + bv.y * bv.y;
    } else {
      const double bi = b[i];
      x[i] = 0.0;
      r[i] = bi;
      p_old[i] = 0.0;
      part[0] += bi * bi * invd(i);
      part[1] += bi * bi;
    }
  }
  block_partial<2>(part, rb, slot);
}

// Search direction p = z + beta p_old, beta from the slot's state: a pass of
// its own for the operators whose kernels read an input value more than once
// (CSR and SELL gathers, the 27-point stencil); the 7-point kernel forms p as
// it stages each plane.
template <class Tz>
struct KDirection {
  static constexpr int kThreads = 1024;
  __device__ static void run(const Tz* z, const double* p_old, double* p, int64_t ldw, int64_t n, const DevState* st,
                             int slot0);
};
template <class Tz>
__device__ __forceinline__ void KDirection<Tz>::run(const Tz* z, const double* p_old, double* p, int64_t ldw, int64_t n,
                                                    const DevState* st, int slot0) {
  const int slot = slot0 + int(blockIdx.y);
  st += slot;
  if (st->done != kRunning) return;
  const int64_t o = slot * ldw;
  z += o;
  p_old += o;
  p += o;
  const double beta = st->beta;
  PAIR_STRIDE(i, n) {
    if (i + 1 < n) {
      const double2 pv = ld2(p_old, i);
      *reinterpret_cast<double2*>(p + i) = make_double2(double(z[i]) + beta * pv.x, double(z[i + 1]) + beta * pv.y);
    } else {
      p[i] = double(z[i]) + beta * p_old[i];
    }
  }
}

// p_old = 0 for the slots of a warm start.
struct KZeroSlots {
  static constexpr int kThreads = 1024;
  __device__ static void run(double* p, int64_t ldw, int64_t n, int slot0);
};
__device__ __forceinline__ void KZeroSlots::run(double* p, int64_t ldw, int64_t n, int slot0) {
  p += (slot0 + int64_t(blockIdx.y)) * ldw;
  GRID_STRIDE(i, n) p[i] = 0.0;
}

// Preconditioner input: s = D^-1 r in the storage precision.
template <class T>
struct KPrep {
  static constexpr int kThreads = 1024;
  __device__ static void run(const double* r, int64_t ldr, T* s, int64_t ldw, InvDiag invd, int64_t n,
                             const DevState* guard, int slot0);
};
template <class T>
__device__ __forceinline__ void KPrep<T>::run(const double* r, int64_t ldr, T* s, int64_t ldw, InvDiag invd, int64_t n,
                                              const DevState* guard, int slot0) {
  const int slot = slot0 + int(blockIdx.y);
  if (guard && guard[slot].done != kRunning) return;
  r += slot * ldr;
  s += slot * ldw;
  using acc = typename Store<T>::acc;
  PAIR_STRIDE(i, n) {
    if (i + 1 < n) {
      const double2 rv = ld2(r, i), w = invd2(invd, i);
      Store<T>::st2(s, i, acc(rv.x * w.x), acc(rv.y * w.y));
    } else {
      Store<T>::st(s, i, acc(r[i] * invd(i)));
    }
  }
}

// Node blocks: s = B^-1 r in the storage precision.
template <class T>
struct KNodePrep {
  static constexpr int kThreads = 1024;
  __device__ static void run(const double* r, int64_t ldr, T* s, int64_t ldw, const double* binv, int64_t nodes,
                             const DevState* guard, int slot0);
};
template <class T>
__device__ __forceinline__ void KNodePrep<T>::run(const double* r, int64_t ldr, T* s, int64_t ldw, const double* binv,
                                                  int64_t nodes, const DevState* guard, int slot0) {
  const int slot = slot0 + int(blockIdx.y);
  if (guard && guard[slot].done != kRunning) return;
  r += slot * ldr;
  s += slot * ldw;
  using acc = typename Store<T>::acc;
  GRID_STRIDE(I, nodes) {
    const double* bi = binv + 6 * I;
    const int64_t i = 3 * I;
    const double r0 = r[i], r1 = r[i + 1], r2 = r[i + 2];
    Store<T>::st(s, i, acc(bi[0] * r0 + bi[1] * r1 + bi[2] * r2));
    Store<T>::st(s, i + 1, acc(bi[1] * r0 + bi[3] * r1 + bi[4] * r2));
    Store<T>::st(s, i + 2, acc(bi[2] * r0 + bi[4] * r1 + bi[5] * r2));
  }
}

// Node blocks, degree 0: z = B^-1 r / theta' (block Jacobi), optionally with (r, z), (z, q).
struct KNodeJacobi {
  static constexpr int kThreads = 1024;
  __device__ static void run(const double* r, int64_t ldr, double* z, int64_t ldz, const double* q, const double* binv,
                             double inv_theta, int64_t nodes, const DevState* guard, ReduceBuf rb, int dots,
                             int flexible, int slot0);
};
__device__ __forceinline__ void KNodeJacobi::run(const double* r, int64_t ldr, double* z, int64_t ldz, const double* q,
                                                 const double* binv, double inv_theta, int64_t nodes,
                                                 const DevState* guard, ReduceBuf rb, int dots, int flexible,
                                                 int slot0) {
  const int slot = slot0 + int(blockIdx.y);
  if (guard && guard[slot].done != kRunning) return;
  r += slot * ldr;
  z += slot * ldz;
  if (q) q += slot * ldz;
  double part[2] = {0.0, 0.0};
  GRID_STRIDE(I, nodes) {
    const double* bi = binv + 6 * I;
    const int64_t i = 3 * I;
    const double r0 = r[i], r1 = r[i + 1], r2 = r[i + 2];
    const double z0 = (bi[0] * r0 + bi[1] * r1 + bi[2] * r2) * inv_theta;
    const double z1 = (bi[1] * r0 + bi[3] * r1 + bi[4] * r2) * inv_theta;
    const double z2 = (bi[2] * r0 + bi[4] * r1 + bi[5] * r2) * inv_theta;
    z[i] = z0;
    z[i + 1] = z1;
    z[i + 2] = z2;
    part[0] += r0 * z0 + r1 * z1 + r2 * z2;
    if (flexible) part[1] += z0 * q[i] + z1 * q[i + 1] + z2 * q[i + 2];
  }
  if (dots) block_partial<2>(part, rb, slot);
}

// Degree 0: z = D^-1 r / theta' (the diagonal preconditioner), optionally with
// the dot products (r, z), (z, q) whose finalize forms beta.
struct KJacobi {
  static constexpr int kThreads = 1024;
  __device__ static void run(const double* r, int64_t ldr, double* z, int64_t ldz, const double* q, InvDiag invd,
                             double inv_theta, int64_t n, const DevState* guard, ReduceBuf rb, int dots, int flexible,
                             int slot0);
};
__device__ __forceinline__ void KJacobi::run(const double* r, int64_t ldr, double* z, int64_t ldz, const double* q,
                                             InvDiag invd, double inv_theta, int64_t n, const DevState* guard,
                                             ReduceBuf rb, int dots, int flexible, int slot0) {
  const int slot = slot0 + int(blockIdx.y);
  if (guard && guard[slot].done != kRunning) return;
  r += slot * ldr;
  z += slot * ldz;
  if (q) q += slot * ldz;
  double part[2] = {0.0, 0.0};
  PAIR_STRIDE(i, n) {
    if (i + 1 < n) {
      const double2 rv = ld2(r, i), w = invd2(invd, i);
      const double z0 = rv.x * w.x * inv_theta, z1 = rv.y * w.y * inv_theta;
      *reinterpret_cast<double2*>(z + i) = make_double2(z0, z1);
      part[0] += rv.x * z0 + rv.y * z1;
      if (flexible) {
        const double2 qv = ld2(q, i);
        part[1] += z0 * qv.x + z1 * qv.y;
      }
    } else {
      const double ri = r[i];
      const double zi = ri * invd(i) * inv_theta;
      z[i] = zi;
      part[0] += ri * zi;
      if (flexible) part[1] += zi * q[i];
    }
  }
  if (dots) block_partial<2>(part, rb, slot);
}

// Iteration update x += alpha p, r -= alpha q with ||r||^2 (D^-1 weighted), and
// the next preconditioner input fused in:
//   MODE 0 (k >= 1): s = D^-1 r;
//   MODE 1 (k = 0):  z = D^-1 r / theta' with (r, z), (z, q);
//   MODE 2:          nothing else (the residual is refreshed before the next step).
// The stop test runs in the finalize kernel (FinUpdate).
template <class T, int MODE>
struct KUpdate {
  static constexpr int kThreads = 1024;
  __device__ static void run(double* x, int64_t ldx, double* r, const double* p, const double* q, int64_t ldw,
                             InvDiag invd, T* s, double* z, double inv_theta, int64_t n, const DevState* st,
                             ReduceBuf rb, int slot0);
};
template <class T, int MODE>
__device__ __forceinline__ void KUpdate<T, MODE>::run(double* x, int64_t ldx, double* r, const double* p,
                                                      const double* q, int64_t ldw, InvDiag invd, T* s, double* z,
                                                      double inv_theta, int64_t n, const DevState* st, ReduceBuf rb,
                                                      int slot0) {
  const int slot = slot0 + int(blockIdx.y);
  st += slot;
  if (st->done != kRunning) return;
  const int64_t o = slot * ldw;
  x += slot * ldx;
  r += o;
  p += o;
  q += o;
  if (MODE == 0) s += o;
  if (MODE == 1) z += o;
  using acc = typename Store<T>::acc;
  const double alpha = st->alpha;
  const int flexible = st->flexible;
  double part[3] = {0.0, 0.0, 0.0};
  PAIR_STRIDE(i, n) {
    if (i + 1 < n) {
      const double2 xv = ld2(x, i), pv = ld2(p, i), rv = ld2(r, i), qv = ld2(q, i), w = invd2(invd, i);
      out_store2(x + i, xv.x + alpha * pv.x, xv.y + alpha * pv.y);
      const double r0 = rv.x - alpha * qv.x, r1 = rv.y - alpha * qv.y;
      out_store2(r + i, r0, r1);
      part[0] += r0 * r0 * w.x + r1 * r1 * w.y;
      if (MODE == 0) {
        Store<T>::st2(s, i, acc(r0 * w.x), acc(r1 * w.y));
      } else if (MODE == 1) {
        const double z0 = r0 * w.x * inv_theta, z1 = r1 * w.y * inv_theta;
        *reinterpret_cast<double2*>(z + i) = make_double2(z0, z1);
        part[1] += r0 * z0 + r1 * z1;
        if (flexible) part[2] += z0 * qv.x + z1 * qv.y;
      }
    } else {
      const double qi = q[i];
      x[i] += alpha * p[i];
      const double ri = r[i] - alpha * qi;
      r[i] = ri;
      const double w = invd(i);
      part[0] += ri * ri * w;
      if (MODE == 0) {
        Store<T>::st(s, i, acc(ri * w));
      } else if (MODE == 1) {
        const double zi = ri * w * inv_theta;
        z[i] = zi;
        part[1] += ri * zi;
        if (flexible) part[2] += zi * qi;
      }
    }
  }
  block_partial<3>(part, rb, slot);
}

// ================================================================ preconditioner

static InvDiag invdiag(const Handle& h) { return InvDiag{h.invd, h.invd ? 0.0 : 1.0 / 6.0}; }

// Optional timing of the middle steps (2 .. k-1) of each application.
struct StepTimer {
  size_t used = 0;
  hipEvent_t next(Handle& h) {
    if (used == h.events.size()) {
      hipEvent_t e;
      PCHEB_HIP_CHECK(hipEventCreate(&e));
      h.events.push_back(e);
    }
    return h.events[used++];
  }
};


// Steps 1..k of Alg. 2 on the prepared input s of the slots; the last step
// writes z (float64, or float32 inside a solve with a float32 or bfloat16
// recurrence: ChebZ).  y_0 = s / theta' is not stored: step 1 reads s as its
// input vector and step 2 reads s as y_{j-2}, with 1/theta' folded into their
// coefficients (step_coef).  Every vector has the workspace stride ldw
// (a single slot 0 may pass the caller's r and z: its offset is zero).
// dots: reduce (r, z), (z, q) and form beta (inside a solve).  Middle steps
// run S at a time when fusion is on.
template <class T>
static void enqueue_steps(Handle& h, Slots sl, double* z, const double* r, const double* q, bool dots, int init,
                          int flexible, DevState* guard, StepTimer* timer, hipStream_t s) {
  const int k = h.prm.k;
  const int S = effective_fuse(h);
  const int64_t ldw = h.ldw;
  T* Y[4] = {reinterpret_cast<T*>(h.Y[0]), reinterpret_cast<T*>(h.Y[1]), reinterpret_cast<T*>(h.Y[2]),
             reinterpret_cast<T*>(h.Y[3])};
  const T* sv = reinterpret_cast<const T*>(h.s);
  constexpr int kY0 = -2;     // y_0, read through s
  int cur = kY0, prev = -1;  // buffers holding y_{j-1} and y_{j-2} (-1: none)
  auto free_buf = [&](int also_avoid) {
    for (int i = 0; i < h.nY; ++i)
      if (i != cur && i != prev && i != also_avoid) return i;
    return -1;
  };
  auto vec = [&](int b) -> const T* { return b == kY0 ? sv : b >= 0 ? Y[b] : nullptr; };
  ChebZ<T, true>* zs = reinterpret_cast<ChebZ<T, true>*>(z);  // z inside a solve (dots)
  for (int j = 1; j <= k;) {
    if (timer && k >= 3 && j == 2) PCHEB_HIP_CHECK(hipEventRecord(timer->next(h), s));
    const T* yin = vec(cur);
    const T* yprev = vec(prev);
    const InVec<T> in{yin, ldw};
    if (j == k) {
      const Coef<T> c = step_coef<T>(h, j);
      if (j == 1) {
        if (dots)
          launch_bop<T>(h, in, EpiChebLast<T, true, true>{yprev, sv, zs, r, q, c.a, c.b, c.c, h.st, guard, init,
                                                          flexible, ldw},
                        sl.first, sl.count, s);
        else
          launch_bop<T>(h, in, EpiChebLast<T, true, false>{yprev, sv, z, r, q, c.a, c.b, c.c, h.st, guard, init, 0,
                                                           ldw},
                        sl.first, sl.count, s);
      } else {
        if (dots)
          launch_bop<T>(h, in, EpiChebLast<T, false, true>{yprev, sv, zs, r, q, c.a, c.b, c.c, h.st, guard, init,
                                                           flexible, ldw},
                        sl.first, sl.count, s);
        else
          launch_bop<T>(h, in, EpiChebLast<T, false, false>{yprev, sv, z, r, q, c.a, c.b, c.c, h.st, guard, init, 0,
                                                            ldw},
                        sl.first, sl.count, s);
      }
      break;
    }
    const int Sj = std::min(S, k - j);  // steps of this pass: at most S, and step k stays single
    if (j >= 2 && Sj >= 2) {
      const int ob = free_buf(-1);
      const int oa = free_buf(ob);
      launch_fused_any<T>(h, sl, Sj, yin, yprev, Y[oa], Y[ob], j, guard, s);
      prev = ob;
      cur = oa;
      j += Sj;
    } else {
      const int o = free_buf(-1);
      const Coef<T> c = step_coef<T>(h, j);
      if (j == 1)
        launch_bop<T>(h, in, EpiChebStep<T, true>{yprev, sv, Y[o], c.a, c.b, c.c, nullptr, guard, ldw}, sl.first,
                      sl.count, s);
      else
        launch_bop<T>(h, in, EpiChebStep<T, false>{yprev, sv, Y[o], c.a, c.b, c.c, nullptr, guard, ldw}, sl.first,
                      sl.count, s);
      prev = cur;
      cur = o;
      ++j;
    }
    if (timer && k >= 3 && j == k) PCHEB_HIP_CHECK(hipEventRecord(timer->next(h), s));
  }
}

// Preconditioner input s = D^-1 r (or B^-1 r with node blocks).
template <class T>
static void enqueue_prep(Handle& h, Slots sl, const double* r, int64_t ldr, const DevState* guard, hipStream_t s) {
  const int64_t n = h.n;
  if (h.bs == 3)
    launch<KNodePrep<T>>(dim3(flat_grid(n / 3), sl.count), kBlock, 0, s, r, ldr, reinterpret_cast<T*>(h.s), h.ldw,
        h.binv, n / 3, guard, sl.first);
  else
    launch<KPrep<T>>(dim3(pair_grid(n), sl.count), kBlock, 0, s, r, ldr, reinterpret_cast<T*>(h.s), h.ldw, invdiag(h),
        n, guard, sl.first);
}

// Stand-alone application r -> z (caller vectors) on slot 0 of the workspace.
template <class T>
static void enqueue_newton(Handle& h, Slots sl, double* z, int64_t ldz, const double* r, int64_t ldr,
                           const double* q, bool dots, int init, int flexible, DevState* guard, hipStream_t s);

template <class T>
static void enqueue_apply_one(Handle& h, const double* r, double* z, hipStream_t s) {
  const int64_t n = h.n;
  if (h.prm.k == 0) {
    if (h.bs == 3)
      launch<KNodeJacobi>(dim3(flat_grid(n / 3), 1), kBlock, 0, s, r, 0, z, 0, nullptr, h.binv, 1.0 / h.theta, n / 3,
          nullptr, h.rb(), 0, 0, 0);
    else
      launch<KJacobi>(dim3(pair_grid(n), 1), kBlock, 0, s, r, 0, z, 0, nullptr, invdiag(h), 1.0 / h.theta, n, nullptr,
          h.rb(), 0, 0, 0);
    return;
  }
  enqueue_prep<T>(h, Slots{0, 1}, r, 0, nullptr, s);
  if (h.prm.form == PCHEB_FORM_NEWTON)
    enqueue_newton<T>(h, Slots{0, 1}, z, 0, r, 0, nullptr, false, 0, 0, nullptr, s);
  else
    enqueue_steps<T>(h, Slots{0, 1}, z, r, nullptr, false, 0, 0, nullptr, nullptr, s);
}

// ---- Newton form of the preconditioner (Alg. 1) on B = D^-1 A_hat: the same
// polynomial as the recurrence (Theorem 2) by the recursion
// P_0 u = zeta_0 u, P_{j+1} u = zeta_{j+1} (2 P_j u - P_j B P_j u).

// out = zeta in
template <class T>
struct KNtScale {
  static constexpr int kThreads = 1024;
  __device__ static void run(const T* in, T* out, int64_t ldw, double zeta, int64_t n, const DevState* guard,
                             int slot0);
};
template <class T>
__device__ __forceinline__ void KNtScale<T>::run(const T* in, T* out, int64_t ldw, double zeta, int64_t n,
                                                 const DevState* guard, int slot0) {
  const int slot = slot0 + int(blockIdx.y);
  if (guard && guard[slot].done != kRunning) return;
  in += slot * ldw;
  out += slot * ldw;
  using acc = typename Store<T>::acc;
  const acc zf = acc(zeta);
  GRID_STRIDE(i, n) Store<T>::st(out, i, zf * Store<T>::ld(in, i));
}

// out = zeta (2 t - out)
template <class T>
struct KNtCombine {
  static constexpr int kThreads = 1024;
  __device__ static void run(const T* t, T* out, int64_t ldw, double zeta, int64_t n, const DevState* guard, int slot0);
};
template <class T>
__device__ __forceinline__ void KNtCombine<T>::run(const T* t, T* out, int64_t ldw, double zeta, int64_t n,
                                                   const DevState* guard, int slot0) {
  const int slot = slot0 + int(blockIdx.y);
  if (guard && guard[slot].done != kRunning) return;
  t += slot * ldw;
  out += slot * ldw;
  using acc = typename Store<T>::acc;
  const acc zf = acc(zeta);
  GRID_STRIDE(i, n) Store<T>::st(out, i, zf * (acc(2) * Store<T>::ld(t, i) - Store<T>::ld(out, i)));
}

// Top level: z = zeta (2 t - w) in float64, with (r, z) and, flexible, (z, q)
// reduced for beta (the same partials as the last recurrence step).
template <class T>
struct KNtFinal {
  static constexpr int kThreads = 1024;
  __device__ static void run(const T* t, const T* w, int64_t ldw, double zeta, double* z, int64_t ldz, const double* r,
                             int64_t ldr, const double* q, int64_t n, const DevState* guard, ReduceBuf rb, int dots,
                             int flexible, int slot0);
};
template <class T>
__device__ __forceinline__ void KNtFinal<T>::run(const T* t, const T* w, int64_t ldw, double zeta, double* z,
                                                 int64_t ldz, const double* r, int64_t ldr, const double* q, int64_t n,
                                                 const DevState* guard, ReduceBuf rb, int dots, int flexible,
                                                 int slot0) {
  const int slot = slot0 + int(blockIdx.y);
  if (guard && guard[slot].done != kRunning) return;
  t += slot * ldw;
  w += slot * ldw;
  z += slot * ldz;
  r += slot * ldr;
  if (q) q += slot * ldz;
  using acc = typename Store<T>::acc;
  const acc zf = acc(zeta);
  double part[2] = {0.0, 0.0};
  GRID_STRIDE(i, n) {
    const double zi = double(zf * (acc(2) * Store<T>::ld(t, i) - Store<T>::ld(w, i)));
    z[i] = zi;
    if (dots) {
      part[0] += r[i] * zi;
      if (flexible) part[1] += zi * q[i];
    }
  }
  if (dots) block_partial<2>(part, rb, slot);
}

// out = P_l in (l >= 0); level j >= 1 uses the buffers nt[2 j - 1] and nt[2 j].
template <class T>
static void newton_rec(Handle& h, Slots sl, int l, const T* in, T* out, const DevState* guard, hipStream_t s) {
  const int64_t n = h.n;
  const dim3 grid(flat_grid(n), sl.count);
  if (l == 0) {
    launch<KNtScale<T>>(grid, kBlock, 0, s, in, out, h.ldw, h.zeta[0], n, guard, sl.first);
    return;
  }
  T* t1 = reinterpret_cast<T*>(h.nt[size_t(2 * l - 1)]);
  T* t2 = reinterpret_cast<T*>(h.nt[size_t(2 * l)]);
  newton_rec<T>(h, sl, l - 1, in, t1, guard, s);  // t1 = P_{l-1} in
  launch_bop<T>(h, InVec<T>{t1, h.ldw}, EpiStore<T>{t2, nullptr, guard, h.ldw}, sl.first, sl.count, s);
  newton_rec<T>(h, sl, l - 1, t2, out, guard, s);  // out = P_{l-1} B P_{l-1} in
  launch<KNtCombine<T>>(grid, kBlock, 0, s, t1, out, h.ldw, h.zeta[size_t(l)], n, guard, sl.first);
}

// z = P(B) s for the slots (s prepared in h.s), with the dot products of a solve when `dots`.
template <class T>
static void enqueue_newton(Handle& h, Slots sl, double* z, int64_t ldz, const double* r, int64_t ldr,
                           const double* q, bool dots, int init, int flexible, DevState* guard, hipStream_t s) {
  const int L = h.nlev;
  const int64_t n = h.n;
  const T* sv = reinterpret_cast<const T*>(h.s);
  T* t1 = reinterpret_cast<T*>(h.nt[size_t(2 * L - 1)]);
  T* t2 = reinterpret_cast<T*>(h.nt[size_t(2 * L)]);
  T* w = reinterpret_cast<T*>(h.nt[0]);
  newton_rec<T>(h, sl, L - 1, sv, t1, guard, s);
  launch_bop<T>(h, InVec<T>{t1, h.ldw}, EpiStore<T>{t2, nullptr, guard, h.ldw}, sl.first, sl.count, s);
  newton_rec<T>(h, sl, L - 1, t2, w, guard, s);
  const uint32_t g = flat_grid(n);
  launch<KNtFinal<T>>(dim3(g, sl.count), kBlock, 0, s, t1, w, h.ldw, h.zeta[size_t(L)], z, ldz, r, ldr, q, n, guard,
      h.rb(), dots ? 1 : 0, flexible, sl.first);
  if (dots) launch<KFinalize<2, FinBeta>>(sl.count, kFinThreads, 0, s, FinBeta{h.st, init, flexible}, h.rb(), g, guard,
      sl.first);
}

#define PCHEB_BY_PREC(h, FN, ...)                      \
  do {                                                 \
    switch ((h).prm.prec) {                            \
      case PCHEB_F64:                                  \
        FN<double>(__VA_ARGS__);                       \
        break;                                         \
      case PCHEB_F32:                                  \
        FN<float>(__VA_ARGS__);                        \
        break;                                         \
      default:                                         \
        FN<bf16>(__VA_ARGS__);                         \
        break;                                         \
    }                                                  \
  } while (0)

// ================================================================ set-up

// Highest degree of a bfloat16 recurrence.  Each stored iterate carries a relative
// rounding error of up to 2^-9, and a degree-k application accumulates it over k
// steps; measured on the 7-point 256^3 problem (flexible PCG, tol 1e-8, against the
// float64 recurrence): k = 30 one more iteration and a 8.9e-7 solution difference,
// k = 40 two more and 1.5e-6, k = 100 four more and 2.2e-6.
constexpr int kBf16MaxDegree = 32;

static void validate(const pcheb_operator* A, const pcheb_params* p) {
  if (!A || !p) fail(PCHEB_INVALID, "null operator or parameters");
  if (p->k < 0 || p->k > 1000) fail(PCHEB_INVALID, "degree k must be in [0, 1000]");
  if (!(p->lambda_min > 0.0) || !(p->lambda_max > p->lambda_min) || !std::isfinite(p->lambda_max))
    fail(PCHEB_INVALID, "need 0 < lambda_min < lambda_max");
  if (!(p->theta_scale >= 1.0) || !std::isfinite(p->theta_scale)) fail(PCHEB_INVALID, "theta_scale must be >= 1");
  if (p->prec < PCHEB_F64 || p->prec > PCHEB_BF16) fail(PCHEB_INVALID, "unknown precision");
  if (p->prec == PCHEB_BF16 && p->k > kBf16MaxDegree)
    fail(PCHEB_INVALID, "a bfloat16 recurrence supports degree k <= " + std::to_string(kBf16MaxDegree) +
                            " (beyond it the rounding of the stored iterates costs PCG iterations and moves the "
                            "solution by more than 1e-6 from the float64 one)");
  if (p->form != PCHEB_FORM_CHEBYSHEV && p->form != PCHEB_FORM_NEWTON) fail(PCHEB_INVALID, "unknown form");
  if (p->form == PCHEB_FORM_NEWTON && ((p->k + 1) & p->k) != 0)
    fail(PCHEB_INVALID, "the Newton form needs degree k = 2^nlev - 1");
  if (p->form == PCHEB_FORM_NEWTON && p->prec == PCHEB_BF16)
    fail(PCHEB_INVALID, "the Newton form needs F64 or F32 storage (its intermediates compound BF16 rounding)");
  if (A->n <= 0) fail(PCHEB_INVALID, "n must be positive");
  if (p->block_size != 0 && p->block_size != 1 && p->block_size != 3)
    fail(PCHEB_INVALID, "block_size must be 1 or 3");
  if (p->block_size == 3 && A->kind != PCHEB_OP_CSR && A->kind != PCHEB_OP_SELL)
    fail(PCHEB_INVALID, "block_size 3 needs a CSR or SELL operator");
  if (p->block_size == 3 && A->n % 3 != 0) fail(PCHEB_INVALID, "block_size 3 needs n to be a multiple of 3");
  switch (A->kind) {
    case PCHEB_OP_CSR:
    case PCHEB_OP_SELL:
      if (!A->rowptr || !A->colind || !A->values) fail(PCHEB_INVALID, "CSR arrays must be non-null");
      if (A->nnz < 0 || A->nnz >= (int64_t(1) << 31)) fail(PCHEB_INVALID, "nnz must be below 2^31");
      if (A->n >= (int64_t(1) << 31)) fail(PCHEB_INVALID, "CSR row count must be below 2^31");
      if (A->kind == PCHEB_OP_SELL) {
        if (A->sell_C != 0 && A->sell_C != kWave) fail(PCHEB_INVALID, "SELL chunk height must be 64");
        if (A->sell_sigma < 1) fail(PCHEB_INVALID, "SELL sigma must be >= 1");
      }
      break;
    case PCHEB_OP_STENCIL7:
    case PCHEB_OP_STENCIL27H:
      if (A->nx <= 0 || A->ny <= 0 || A->nz <= 0) fail(PCHEB_INVALID, "grid dimensions must be positive");
      if (int64_t(A->nx) * A->ny * A->nz != A->n) fail(PCHEB_INVALID, "n must equal nx*ny*nz");
      if (A->n >= (int64_t(1) << 32)) fail(PCHEB_INVALID, "grid too large");
      if (A->kind == PCHEB_OP_STENCIL27H && !A->cell_coeff) fail(PCHEB_INVALID, "cell_coeff must be non-null");
      break;
    default:
      fail(PCHEB_INVALID, "unknown operator kind");
  }
}

// Lanes per CSR row: about avg / 2.5 rounded to a power of two (measured on
// 256^3 7-point rows of 7: 4 lanes 356 us, 8 lanes 382 us; Q1 elasticity rows
// of 81: 16 lanes 1323 us, 32 lanes 1277 us, 64 lanes 1667 us).
static int pick_lanes(int64_t n, int64_t nnz) {
  const double avg = n > 0 ? double(nnz) / double(n) : 1.0;
  if (avg <= 10.0) return 4;
  if (avg <= 20.0) return 8;
  if (avg <= 40.0) return 16;
  if (avg <= 100.0) return 32;
  return 64;
}

// Scalars of eq. rhocheb with the Sec. 4 scaling theta' = s theta.
static void chebyshev_scalars(Handle& h) {
  const pcheb_params& p = h.prm;
  h.theta = p.theta_scale * 0.5 * (p.lambda_max + p.lambda_min);
  h.delta = 0.5 * (p.lambda_max - p.lambda_min);
  h.sigma = h.theta / h.delta;
  h.rho.assign(size_t(p.k) + 1, 0.0);
  h.rho[0] = 1.0 / h.sigma;
  for (int j = 1; j <= p.k; ++j) h.rho[j] = 1.0 / (2.0 * h.sigma - h.rho[j - 1]);
  // Newton form (Alg. 1, eq. zetaNewt) on the same shifted interval [alpha0, beta0] =
  // [theta' - delta, theta' + delta]
  h.nlev = 0;
  h.zeta.clear();
  if (p.form == PCHEB_FORM_NEWTON) {
    while ((1 << (h.nlev + 1)) - 1 <= p.k) ++h.nlev;
    const double a0 = h.theta - h.delta, b0 = h.theta + h.delta;
    h.zeta.assign(size_t(h.nlev) + 1, 0.0);
    h.zeta[0] = 2.0 / (a0 + b0);
    if (h.nlev >= 1) {
      const double az = a0 * h.zeta[0];
      h.zeta[1] = 2.0 / (1.0 + 2.0 * az - az * az);
    }
    for (int j = 2; j <= h.nlev; ++j)
      h.zeta[size_t(j)] = 2.0 / (1.0 + 2.0 * h.zeta[size_t(j) - 1] - h.zeta[size_t(j) - 1] * h.zeta[size_t(j) - 1]);
  }
}

template <class T>
static void build_scaled_values(Handle& h, hipStream_t s) {
  const pcheb_operator& op = h.op;
  if (op.kind == PCHEB_OP_CSR) {
    h.csr_bval = dev_alloc(h, size_t(op.nnz) * sizeof(T));
    if (h.bs == 3)
      k_scale_rows_node<T><<<flat_grid(h.n), kBlock, 0, s>>>(op.rowptr, op.values, h.binv, h.n,
                                                            reinterpret_cast<T*>(h.csr_bval));
    else
      k_scale_rows<T><<<flat_grid(h.n), kBlock, 0, s>>>(op.rowptr, op.values, h.invd, h.n,
                                                       reinterpret_cast<T*>(h.csr_bval));
    PCHEB_HIP_CHECK(hipGetLastError());
  } else if (op.kind == PCHEB_OP_SELL) {
    // row lengths on the host, sorted within windows of sigma rows (longest first)
    std::vector<int32_t> rp(size_t(h.n) + 1);
    PCHEB_HIP_CHECK(hipMemcpyAsync(rp.data(), op.rowptr, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PCHEB_HIP_CHECK(hipStreamSynchronize(s));
    if (rp[0] != 0 || int64_t(rp[size_t(h.n)]) != op.nnz) fail(PCHEB_INVALID, "rowptr does not span nnz");
    const int sigma = std::max(1, op.sell_sigma);
    std::vector<int32_t> perm(size_t(h.n));
    std::iota(perm.begin(), perm.end(), 0);
    if (sigma > 1) {
      for (int64_t w = 0; w < h.n; w += sigma) {
        const int64_t e = std::min<int64_t>(h.n, w + sigma);
        std::stable_sort(perm.begin() + w, perm.begin() + e, [&](int32_t a, int32_t b) {
          return rp[a + 1] - rp[a] > rp[b + 1] - rp[b];
        });
      }
    }
    h.nchunks = (h.n + kWave - 1) / kWave;
    std::vector<int64_t> cptr(size_t(h.nchunks));
    std::vector<int32_t> clen(size_t(h.nchunks));
    int64_t off = 0;
    for (int64_t c = 0; c < h.nchunks; ++c) {
      int32_t m = 0;
      for (int64_t l = 0; l < kWave && c * kWave + l < h.n; ++l) {
        const int32_t row = perm[size_t(c * kWave + l)];
        m = std::max(m, rp[row + 1] - rp[row]);
      }
      cptr[size_t(c)] = off;
      clen[size_t(c)] = m;
      off += int64_t(m) * kWave;
    }
    h.nnz_pad = off;
    h.sell_ptr = static_cast<int64_t*>(dev_alloc(h, cptr.size() * sizeof(int64_t)));
    h.sell_len = static_cast<int32_t*>(dev_alloc(h, clen.size() * sizeof(int32_t)));
    h.sell_col = static_cast<int32_t*>(dev_alloc(h, size_t(off) * sizeof(int32_t)));
    h.sell_aval = static_cast<double*>(dev_alloc(h, size_t(off) * sizeof(double)));
    h.sell_bval = dev_alloc(h, size_t(off) * sizeof(T));
    int32_t* dperm = nullptr;
    if (sigma > 1) {
      h.sell_perm = static_cast<int32_t*>(dev_alloc(h, perm.size() * sizeof(int32_t)));
      dperm = h.sell_perm;
      PCHEB_HIP_CHECK(hipMemcpyAsync(dperm, perm.data(), perm.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    PCHEB_HIP_CHECK(hipMemcpyAsync(h.sell_ptr, cptr.data(), cptr.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    PCHEB_HIP_CHECK(hipMemcpyAsync(h.sell_len, clen.data(), clen.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    k_sell_fill<T><<<flat_grid(h.nchunks * kWave), kBlock, 0, s>>>(
        op.rowptr, op.colind, op.values, h.invd, h.binv, dperm, h.sell_ptr, h.sell_len, h.n, h.nchunks,
        h.sell_col, h.sell_aval, reinterpret_cast<T*>(h.sell_bval));
    PCHEB_HIP_CHECK(hipGetLastError());
    PCHEB_HIP_CHECK(hipStreamSynchronize(s));  // host vectors above go out of scope
  }
}

// Diagonal (D^-1), NOT_SPD check and the float32 coefficient copy.
void setup_operator(Handle& h, hipStream_t s) {
  const pcheb_operator& op = h.op;
  const int64_t n = h.n;
  PCHEB_HIP_CHECK(hipGetDevice(&h.device));
  int* bad = static_cast<int*>(dev_alloc(h, sizeof(int)));
  PCHEB_HIP_CHECK(hipMemsetAsync(bad, 0, sizeof(int), s));
  h.bs = h.prm.block_size == 3 ? 3 : 1;
  if (op.kind == PCHEB_OP_CSR || op.kind == PCHEB_OP_SELL) {
    h.invd = static_cast<double*>(dev_alloc(h, size_t(n) * sizeof(double)));
    k_csr_invdiag<<<flat_grid(n), kBlock, 0, s>>>(op.rowptr, op.colind, op.values, n, h.invd, bad);
    h.lanes = pick_lanes(n, op.nnz);
    if (h.bs == 3) {
      h.binv = static_cast<double*>(dev_alloc(h, size_t(n / 3) * 6 * sizeof(double)));
      h.lfac = static_cast<double*>(dev_alloc(h, size_t(n / 3) * 6 * sizeof(double)));
      k_node_blocks<<<flat_grid(n / 3), kBlock, 0, s>>>(op.rowptr, op.colind, op.values, n / 3, h.binv, h.lfac,
                                                         bad);
    }
  } else if (op.kind == PCHEB_OP_STENCIL27H) {
    h.invd = static_cast<double*>(dev_alloc(h, size_t(n) * sizeof(double)));
    k_h27_invdiag<<<flat_grid(n), kBlock, 0, s>>>(op.cell_coeff, op.nx, op.ny, op.nz, h.invd, bad);
    h.rho64 = static_cast<double*>(dev_alloc(h, size_t(n) * sizeof(double)));
    k_h27_rho64<<<flat_grid(n), kBlock, 0, s>>>(op.cell_coeff, h.rho64, n);
    if (h.prm.prec != PCHEB_F64) {
      h.rho_lo = static_cast<float*>(dev_alloc(h, size_t(n) * sizeof(float)));
      h.invd_lo = static_cast<float*>(dev_alloc(h, size_t(n) * sizeof(float)));
      k_h27_lo<<<flat_grid(n), kBlock, 0, s>>>(op.cell_coeff, h.invd, h.rho_lo, h.invd_lo, n);
    }
  }
  PCHEB_HIP_CHECK(hipGetLastError());
  int bad_host = 0;
  PCHEB_HIP_CHECK(hipMemcpyAsync(&bad_host, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  PCHEB_HIP_CHECK(hipStreamSynchronize(s));
  if (bad_host & 2) fail(PCHEB_INVALID, "block_size 3: the three rows of a node must share one column pattern");
  if ((bad_host & 5) == 4) fail(PCHEB_INVALID, "27-point cell coefficients must lie in [1e-150, 1e150]");
  if (bad_host & 1) fail(PCHEB_NOT_SPD, "operator has a non-positive diagonal entry, coefficient or 3x3 block");
}

// Recurrence scalars and the scaled operator copies.
static void setup_preconditioner(Handle& h, hipStream_t s) {
  chebyshev_scalars(h);
  h.elem = storage_bytes(h.prm.prec);
  PCHEB_BY_PREC(h, build_scaled_values, h, s);
  h.fuse = std::max(1, std::min(h.prm.fuse_steps, 4));
  h.nY = (h.op.kind == PCHEB_OP_STENCIL7 && h.fuse >= 2) ? 4 : 3;
  h.ldw = round_up(h.n, 64);
}

// Solve workspace for `cap` slots (reallocated when a call needs more).
void ensure_workspace(Handle& h, int cap, hipStream_t stream) {
  if (cap <= h.cap) return;
  release_workspace(h);
  const size_t lw = size_t(h.ldw) * size_t(cap);
  auto& ws = h.owned_ws;
  h.s = alloc_into(ws, lw * h.elem);
  for (int i = 0; i < h.nY; ++i) h.Y[i] = alloc_into(ws, lw * h.elem);
  for (int i = h.nY; i < 4; ++i) h.Y[i] = nullptr;
  h.nt.clear();
  if (h.prm.form == PCHEB_FORM_NEWTON && h.nlev >= 1)
    for (int i = 0; i < 2 * h.nlev + 1; ++i) h.nt.push_back(alloc_into(ws, lw * h.elem));
  h.r = static_cast<double*>(alloc_into(ws, lw * 8));
  h.p[0] = static_cast<double*>(alloc_into(ws, lw * 8));
  h.p[1] = static_cast<double*>(alloc_into(ws, lw * 8));
  h.q = static_cast<double*>(alloc_into(ws, lw * 8));
  h.z = static_cast<double*>(alloc_into(ws, lw * 8));
  h.st = static_cast<DevState*>(alloc_into(ws, size_t(cap) * sizeof(DevState)));
  h.partials = static_cast<double*>(alloc_into(ws, size_t(cap) * kMaxGrid * kMaxReduce * sizeof(double)));
  // on the stream the states are used on next (a non-blocking stream is not
  // ordered after the legacy default stream)
  PCHEB_HIP_CHECK(hipMemsetAsync(h.st, 0, size_t(cap) * sizeof(DevState), stream));
  PCHEB_HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&h.st_host), 2 * size_t(cap) * sizeof(DevState),
                                hipHostMallocDefault));
  std::memset(h.st_host, 0, 2 * size_t(cap) * sizeof(DevState));
  h.cap = cap;
}

static size_t footprint(const pcheb_operator* A, const pcheb_params* p, int32_t nrhs) {
  const int64_t n = A->n;
  const size_t e = storage_bytes(p->prec);
  size_t b = 64;
  if (A->kind == PCHEB_OP_CSR) b += size_t(n) * 8 + size_t(A->nnz) * e;
  if (A->kind == PCHEB_OP_SELL) {
    const int64_t chunks = (n + kWave - 1) / kWave;
    b += size_t(n) * 8 + size_t(chunks) * 12 + size_t(A->nnz) * (4 + 8 + e);
    if (A->sell_sigma > 1) b += size_t(n) * 4;
  }
  if (A->kind == PCHEB_OP_STENCIL27H) b += size_t(n) * 16 + (p->prec != PCHEB_F64 ? size_t(n) * 8 : 0);
  if (p->block_size == 3) b += size_t(n / 3) * 12 * 8;  // node inverses and factors
  const int ny = (A->kind == PCHEB_OP_STENCIL7 && p->fuse_steps >= 2) ? 4 : 3;
  int nt = 0;  // Newton form: 2 nlev + 1 iterate vectors
  if (p->form == PCHEB_FORM_NEWTON)
    for (int l = 1; (1 << l) - 1 <= p->k; ++l) nt = 2 * l + 1;
  const size_t per_rhs = size_t(round_up(n, 64)) * ((1 + ny + nt) * e + 5 * 8) + sizeof(DevState) +
                         size_t(kMaxGrid) * kMaxReduce * 8;
  b += size_t(std::max(1, nrhs)) * per_rhs + 256;
  return b;
}

// ================================================================ PCG internals (slot ranges)

struct KInitStates {
  static constexpr int kThreads = 1024;
  __device__ static void run(DevState* st, int slot0, int count, double tol, int maxit, int flexible);
};
__device__ __forceinline__ void KInitStates::run(DevState* st, int slot0, int count, double tol, int maxit,
                                                 int flexible) {
  const int i = int(threadIdx.x);
  if (i >= count) return;
  DevState d{};
  d.tol = tol;
  d.maxit = maxit;
  d.flexible = flexible;
  st[slot0 + i] = d;
}

// Slots that must not take part in a launch over a wider range are marked done.
struct KRetireStates {
  static constexpr int kThreads = 1024;
  __device__ static void run(DevState* st, int slot0, int count);
};
__device__ __forceinline__ void KRetireStates::run(DevState* st, int slot0, int count) {
  const int i = int(threadIdx.x);
  if (i < count && st[slot0 + i].done == kRunning) st[slot0 + i].done = kMaxIter;
}

template <class T>
static void enqueue_precond(Handle& h, Slots sl, int init, int flexible, StepTimer* timer, hipStream_t s) {
  const int64_t n = h.n;
  if (h.prm.k == 0) {
    if (h.bs == 3) {
      const uint32_t g = flat_grid(n / 3);
      launch<KNodeJacobi>(dim3(g, sl.count), kBlock, 0, s, h.r, h.ldw, h.z, h.ldw, h.q, h.binv, 1.0 / h.theta, n / 3,
          h.st, h.rb(), 1, flexible, sl.first);
      launch<KFinalize<2, FinBeta>>(sl.count, kFinThreads, 0, s, FinBeta{h.st, init, flexible}, h.rb(), g, h.st,
          sl.first);
      return;
    }
    const uint32_t g = pair_grid(n);
    launch<KJacobi>(dim3(g, sl.count), kBlock, 0, s, h.r, h.ldw, h.z, h.ldw, h.q, invdiag(h), 1.0 / h.theta, n, h.st,
        h.rb(), 1, flexible, sl.first);
    launch<KFinalize<2, FinBeta>>(sl.count, kFinThreads, 0, s, FinBeta{h.st, init, flexible}, h.rb(), g, h.st,
        sl.first);
    return;
  }
  enqueue_prep<T>(h, sl, h.r, h.ldw, h.st, s);
  if (h.prm.form == PCHEB_FORM_NEWTON)
    enqueue_newton<T>(h, sl, h.z, h.ldw, h.r, h.ldw, h.q, true, init, flexible, h.st, s);
  else
    enqueue_steps<T>(h, sl, h.z, h.r, h.q, true, init, flexible, h.st, timer, s);
}

template <class T>
static void enqueue_start(Handle& h, Slots sl, const double* b, int64_t ldb, double* x, int64_t ldx, bool x0_given,
                          int flexible, StepTimer* timer, hipStream_t s) {
  const int64_t n = h.n;
  if (x0_given) {
    launch<KZeroSlots>(dim3(flat_grid(n), sl.count), kBlock, 0, s, h.p[0], h.ldw, n, sl.first);
    launch_ahat(h, InVec<double>{x, ldx}, EpiResidual{b, h.r, invdiag(h), h.st, nullptr, 0, ldb, h.ldw}, sl.first,
                sl.count, s);
  } else {
    const uint32_t g = pair_grid(n);
    launch<KStartZero>(dim3(g, sl.count), kBlock, 0, s, b, ldb, x, ldx, h.r, h.p[0], h.ldw, invdiag(h), n, h.rb(),
        sl.first);
    launch<KFinalize<2, FinStart>>(sl.count, kFinThreads, 0, s, FinStart{h.st}, h.rb(), g, nullptr, sl.first);
  }
  enqueue_precond<T>(h, sl, 1, flexible, timer, s);
}

// Inside a solve, a float32 or bfloat16 recurrence leaves z in float32 (its
// last step computes in float32, so the float32 store is exact); the float64
// recurrence, degree 0 and the Newton form leave it in float64.
template <class T>
static bool z_is_float(const Handle& h) {
  return !std::is_same<T, double>::value && h.prm.k >= 1 && h.prm.form == PCHEB_FORM_CHEBYSHEV;
}

// p = z + beta p_old and q = A p with (p, q) (alpha formed on the device).
template <class Tz>
static void enqueue_direction(Handle& h, Slots sl, const Tz* z, const double* p_old, double* p_new, hipStream_t s) {
  DevState* st = h.st;
  if (h.op.kind == PCHEB_OP_STENCIL7) {
    // the 7-point kernel reads each input point once: form p there and store it beside q
    launch_ahat(h, InDirection<Tz>{z, p_old, st, 0.0, h.ldw}, EpiDirection{p_new, h.q, st, st, h.ldw}, sl.first,
                sl.count, s);
  } else {
    launch<KDirection<Tz>>(dim3(pair_grid(h.n), sl.count), kBlock, 0, s, z, p_old, p_new, h.ldw, h.n, st, sl.first);
    launch_ahat(h, InVec<double>{p_new, h.ldw}, EpiDirection{nullptr, h.q, st, st, h.ldw}, sl.first, sl.count, s);
  }
}

// One PCG iteration on the slots: p = z + beta p_old, q = A p, the update with the
// fused preconditioner input, and the k recurrence steps (beta formed on the device).
template <class T>
static void enqueue_iteration(Handle& h, Slots sl, double* x, int64_t ldx, const double* b, int64_t ldb, int cur,
                              int flexible, bool refresh, StepTimer* timer, hipStream_t s) {
  const int64_t n = h.n;
  DevState* st = h.st;
  double* p_new = h.p[cur ^ 1];
  const uint32_t g = pair_grid(n);
  const dim3 grid(g, sl.count);
  if (z_is_float<T>(h))
    enqueue_direction(h, sl, reinterpret_cast<const float*>(h.z), h.p[cur], p_new, s);
  else
    enqueue_direction(h, sl, static_cast<const double*>(h.z), h.p[cur], p_new, s);
  if (refresh) {
    launch<KUpdate<T, 2>>(grid, kBlock, 0, s, x, ldx, h.r, p_new, h.q, h.ldw, invdiag(h), nullptr, nullptr, 0.0, n, st,
        h.rb(), sl.first);
    launch<KFinalize<3, FinUpdate<2>>>(sl.count, kFinThreads, 0, s, FinUpdate<2>{st}, h.rb(), g, st, sl.first);
    launch_ahat(h, InVec<double>{x, ldx}, EpiResidual{b, h.r, invdiag(h), st, st, 2, ldb, h.ldw}, sl.first, sl.count,
                s);
    enqueue_precond<T>(h, sl, 0, flexible, timer, s);
    return;
  }
  if (h.bs == 3) {  // node blocks: the preconditioner input needs whole nodes, so it is a pass of its own
    launch<KUpdate<T, 2>>(grid, kBlock, 0, s, x, ldx, h.r, p_new, h.q, h.ldw, invdiag(h), nullptr, nullptr, 0.0, n, st,
        h.rb(), sl.first);
    launch<KFinalize<3, FinUpdate<2>>>(sl.count, kFinThreads, 0, s, FinUpdate<2>{st}, h.rb(), g, st, sl.first);
    enqueue_precond<T>(h, sl, 0, flexible, timer, s);
  } else if (h.prm.k == 0) {
    launch<KUpdate<double, 1>>(grid, kBlock, 0, s, x, ldx, h.r, p_new, h.q, h.ldw, invdiag(h), nullptr, h.z,
        1.0 / h.theta, n, st, h.rb(), sl.first);
    launch<KFinalize<3, FinUpdate<1>>>(sl.count, kFinThreads, 0, s, FinUpdate<1>{st}, h.rb(), g, st, sl.first);
  } else {
    launch<KUpdate<T, 0>>(grid, kBlock, 0, s, x, ldx, h.r, p_new, h.q, h.ldw, invdiag(h), reinterpret_cast<T*>(h.s),
        nullptr, 1.0 / h.theta, n, st, h.rb(), sl.first);
    launch<KFinalize<3, FinUpdate<0>>>(sl.count, kFinThreads, 0, s, FinUpdate<0>{st}, h.rb(), g, st, sl.first);
    if (h.prm.form == PCHEB_FORM_NEWTON)
      enqueue_newton<T>(h, sl, h.z, h.ldw, h.r, h.ldw, h.q, true, 0, flexible, st, s);
    else
      enqueue_steps<T>(h, sl, h.z, h.r, h.q, true, 0, flexible, st, timer, s);
  }
}

template <class T>
static void capture_pair(Handle& h, Slots sl, double* x, int64_t ldx, int flexible) {
  if (!h.capture_stream) PCHEB_HIP_CHECK(hipStreamCreateWithFlags(&h.capture_stream, hipStreamNonBlocking));
  hipStream_t s = h.capture_stream;
  hipGraph_t graph = nullptr;
  // Relaxed: the capture holds kernel launches on a private stream only, and
  // other threads (a server's set-up and worker threads, the caller's) may
  // allocate or synchronise meanwhile without invalidating it.
  PCHEB_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  try {
    enqueue_iteration<T>(h, sl, x, ldx, nullptr, 0, 0, flexible, false, nullptr, s);
    enqueue_iteration<T>(h, sl, x, ldx, nullptr, 0, 1, flexible, false, nullptr, s);
  } catch (...) {
    (void)hipStreamEndCapture(s, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  PCHEB_HIP_CHECK(hipStreamEndCapture(s, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  PCHEB_HIP_CHECK(e);
  drop_graph(h);
  h.graph_exec = exec;
  h.graph_x = x;
  h.graph_ldx = ldx;
  h.graph_slots = sl.first * 65536 + sl.count;
  h.graph_flags = uint32_t(flexible);
}

template <class T>
static void enqueue_pairs_graph(Handle& h, Slots sl, double* x, int64_t ldx, int pairs, int flexible, hipStream_t s) {
  if (h.graph_exec == nullptr || h.graph_x != x || h.graph_ldx != ldx ||
      h.graph_slots != sl.first * 65536 + sl.count || h.graph_flags != uint32_t(flexible))
    capture_pair<T>(h, sl, x, ldx, flexible);
  for (int i = 0; i < pairs; ++i) PCHEB_HIP_CHECK(hipGraphLaunch(h.graph_exec, s));
}

template <class T>
static void enqueue_finish(Handle& h, Slots sl, const double* b, int64_t ldb, const double* x, int64_t ldx,
                           hipStream_t s) {
  launch_ahat(h, InVec<double>{x, ldx}, EpiResidual{b, nullptr, invdiag(h), h.st, nullptr, 1, ldb, h.ldw}, sl.first,
              sl.count, s);
}

// ---- exported to the serving engine (solver.hpp)

void solver_init_states(Handle& h, Slots sl, double tol, int maxit, int flexible, hipStream_t s) {
  launch<KInitStates>(1, std::max(1, sl.count), 0, s, h.st, sl.first, sl.count, tol, maxit, flexible);
  PCHEB_HIP_CHECK(hipGetLastError());
}

void solver_retire(Handle& h, Slots sl, hipStream_t s) {
  launch<KRetireStates>(1, std::max(1, sl.count), 0, s, h.st, sl.first, sl.count);
  PCHEB_HIP_CHECK(hipGetLastError());
}

void solver_start(Handle& h, Slots sl, const double* b, int64_t ldb, double* x, int64_t ldx, bool x0_given,
                  int flexible, hipStream_t s) {
  PCHEB_BY_PREC(h, enqueue_start, h, sl, b, ldb, x, ldx, x0_given, flexible, nullptr, s);
  PCHEB_HIP_CHECK(hipGetLastError());
}

void solver_iteration_pairs(Handle& h, Slots sl, double* x, int64_t ldx, int pairs, int flexible, hipStream_t s) {
  PCHEB_BY_PREC(h, enqueue_pairs_graph, h, sl, x, ldx, pairs, flexible, s);
  PCHEB_HIP_CHECK(hipGetLastError());
}

template <class T>
static void enqueue_two_iterations(Handle& h, Slots sl, double* x, int64_t ldx, int flexible, hipStream_t s) {
  enqueue_iteration<T>(h, sl, x, ldx, nullptr, 0, 0, flexible, false, nullptr, s);
  enqueue_iteration<T>(h, sl, x, ldx, nullptr, 0, 1, flexible, false, nullptr, s);
}

void solver_iterations_direct(Handle& h, Slots sl, double* x, int64_t ldx, int flexible, hipStream_t s) {
  PCHEB_BY_PREC(h, enqueue_two_iterations, h, sl, x, ldx, flexible, s);
}

void solver_apply(Handle& h, const double* r, double* z, hipStream_t s) {
  PCHEB_BY_PREC(h, enqueue_apply_one, h, r, z, s);
}

template <class T>
static void prepare_graph(Handle& h, Slots sl, double* x, int64_t ldx, int flexible) {
  if (h.graph_exec == nullptr || h.graph_x != x || h.graph_ldx != ldx ||
      h.graph_slots != sl.first * 65536 + sl.count || h.graph_flags != uint32_t(flexible))
    capture_pair<T>(h, sl, x, ldx, flexible);
}

void solver_prepare_graph(Handle& h, Slots sl, double* x, int64_t ldx, int flexible) {
  PCHEB_BY_PREC(h, prepare_graph, h, sl, x, ldx, flexible);
}

void solver_finish(Handle& h, Slots sl, const double* b, int64_t ldb, const double* x, int64_t ldx, hipStream_t s) {
  PCHEB_BY_PREC(h, enqueue_finish, h, sl, b, ldb, x, ldx, s);
  PCHEB_HIP_CHECK(hipGetLastError());
}

void fill_stats(const Handle& h, const DevState& fin, uint32_t flags, pcg_stats* stats) {
  pcheb_status status = PCHEB_OK;
  if (fin.done == kBreakdown)
    status = PCHEB_BREAKDOWN;
  else if (fin.done != kConverged)
    status = PCHEB_NOT_CONVERGED;
  pcg_stats& o = *stats;
  std::memset(&o, 0, sizeof(o));
  o.iters = fin.iter;
  o.converged = fin.done == kConverged;
  o.status = status;
  o.relres = fin.relres;
  o.relres_true = fin.bb > 0 ? std::sqrt(fin.true_rr) / std::sqrt(fin.bb) : 0.0;
  o.relres_true_hat = fin.bb_hat > 0 ? std::sqrt(fin.true_rr_hat) / std::sqrt(fin.bb_hat) : 0.0;
  const int64_t k = h.prm.k;
  const int64_t applies =
      fin.iter == 0 ? (fin.done == kConverged ? 0 : 1) : (fin.done == kMaxIter ? fin.iter + 1 : fin.iter);
  o.n_spmv = fin.iter + k * applies + ((flags & PCG_X0_GIVEN) ? 1 : 0);
  o.n_dot = applies + 2 * int64_t(fin.iter) + ((flags & PCG_FLEXIBLE) ? std::max<int64_t>(0, applies - 1) : 0);
}

// ================================================================ PCG driver

template <class T>
static pcheb_status solve_impl(Handle& h, const double* b, double* x, int nrhs, int64_t ld, double tol, int maxit,
                               uint32_t flags, pcg_stats* stats, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  ensure_workspace(h, nrhs, s);
  const Slots sl{0, nrhs};
  const int flexible = (flags & PCG_FLEXIBLE) ? 1 : 0;
  const bool timed = (flags & PCG_TIME_KERNELS) != 0;
  const bool refresh = (flags & PCG_REFRESH) != 0;
  const bool use_graph = !(flags & (PCG_NO_GRAPH | PCG_TIME_KERNELS | PCG_REFRESH));
  StepTimer timer;
  StepTimer* tp = timed ? &timer : nullptr;

  solver_init_states(h, sl, tol, maxit, flexible, s);
  enqueue_start<T>(h, sl, b, ld, x, ld, (flags & PCG_X0_GIVEN) != 0, flexible, tp, s);
  PCHEB_HIP_CHECK(hipGetLastError());

  int cur = 0;
  int64_t issued = 0;
  int chunk = 2;
  int half = 0;
  bool have_prev = false;
  DevState* hs = h.st_host;
  auto all_done = [&](const DevState* v) {
    for (int i = 0; i < nrhs; ++i)
      if (v[i].done == kRunning) return false;
    return true;
  };
  hipEvent_t ev[2];
  PCHEB_HIP_CHECK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  PCHEB_HIP_CHECK(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  try {
    for (;;) {
      if (use_graph) {
        enqueue_pairs_graph<T>(h, sl, x, ld, chunk / 2, flexible, s);
        issued += chunk;
      } else {
        for (int it = 0; it < chunk; ++it) {
          const bool ref = refresh && issued > 0 && (issued + 1) % 50 == 0;
          enqueue_iteration<T>(h, sl, x, ld, b, ld, cur, flexible, ref, tp, s);
          cur ^= 1;
          ++issued;
        }
      }
      PCHEB_HIP_CHECK(hipGetLastError());
      DevState* dst = hs + size_t(half) * nrhs;
      PCHEB_HIP_CHECK(hipMemcpyAsync(dst, h.st, size_t(nrhs) * sizeof(DevState), hipMemcpyDeviceToHost, s));
      PCHEB_HIP_CHECK(hipEventRecord(ev[half], s));
      if (have_prev) {
        PCHEB_HIP_CHECK(hipEventSynchronize(ev[half ^ 1]));
        if (all_done(hs + size_t(half ^ 1) * nrhs)) break;
      }
      have_prev = true;
      half ^= 1;
      if (chunk < 16) chunk *= 2;
      if (issued > int64_t(maxit) + 64) {
        // the device stops at maxit; wait for the last copy and leave
        PCHEB_HIP_CHECK(hipEventSynchronize(ev[half ^ 1]));
        break;
      }
    }
  } catch (...) {
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    throw;
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);

  enqueue_finish<T>(h, sl, b, ld, x, ld, s);
  PCHEB_HIP_CHECK(hipGetLastError());
  PCHEB_HIP_CHECK(hipMemcpyAsync(hs, h.st, size_t(nrhs) * sizeof(DevState), hipMemcpyDeviceToHost, s));
  PCHEB_HIP_CHECK(hipStreamSynchronize(s));

  // the slowest right-hand side decides the reported statistics and status
  int worst = 0;
  for (int i = 1; i < nrhs; ++i) {
    const bool bad_i = hs[i].done != kConverged, bad_w = hs[worst].done != kConverged;
    if ((bad_i && !bad_w) || (bad_i == bad_w && hs[i].iter > hs[worst].iter)) worst = i;
  }
  pcg_stats local;
  fill_stats(h, hs[worst], flags, &local);
  if (timed && h.prm.k >= 3 && nrhs == 1) {
    // applications that did work: the initial one plus one per non-final iteration (the
    // final iteration stops before its application, whose launches exit at once; n_spmv
    // still counts that one when maxit ends the solve, as the unfused loop would run it)
    const int64_t ran = local.iters >= 1 ? local.iters : (hs[worst].done == kConverged ? 0 : 1);
    const size_t pairs = std::min(timer.used / 2, size_t(ran));
    double ms = 0.0;
    for (size_t i = 0; i < pairs; ++i) {
      float t = 0.f;
      PCHEB_HIP_CHECK(hipEventElapsedTime(&t, h.events[2 * i], h.events[2 * i + 1]));
      ms += t;
    }
    local.step_ms = ms;
    local.step_launches = int64_t(pairs) * (h.prm.k - 2);
  }
  local.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = local;
  return pcheb_status(local.status);
}

}  // namespace pcheb

// ================================================================ C ABI

using namespace pcheb;

template <class F>
static pcheb_status guarded(F&& f) {
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

namespace pcheb {

Handle* create_handle(const pcheb_operator* A, const pcheb_params* p, hipStream_t stream) {
  validate(A, p);
  Handle* h = new Handle();
  h->op = *A;
  h->prm = *p;
  h->n = A->n;
  try {
    setup_operator(*h, stream);
    setup_preconditioner(*h, stream);
    ensure_workspace(*h, 1, stream);
  } catch (...) {
    release(*h);
    delete h;
    throw;
  }
  return h;
}

void destroy_handle(Handle* h) {
  if (!h) return;
  release(*h);
  delete h;
}

size_t footprint_bytes(const pcheb_operator* A, const pcheb_params* p, int32_t nrhs) { return footprint(A, p, nrhs); }

}  // namespace pcheb

static Handle* as_handle(pcheb_handle h) {
  if (!h) fail(PCHEB_INVALID, "null handle");
  return reinterpret_cast<Handle*>(h);
}

static void check_vectors(const Handle& h, const void* a, const void* b, int32_t nrhs, int64_t ld) {
  if (!a || !b) fail(PCHEB_INVALID, "null vector");
  if (nrhs < 1 || nrhs > 4096) fail(PCHEB_INVALID, "nrhs must be in [1, 4096]");
  if (ld < h.n) fail(PCHEB_INVALID, "ld must be >= n");
  if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) % 16 != 0)
    fail(PCHEB_INVALID, "vectors must be 16-byte aligned");
  if (nrhs > 1 && ld % 2 != 0) fail(PCHEB_INVALID, "ld must be even when nrhs > 1 (16-byte aligned columns)");
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  const size_t bytes = (size_t(nrhs - 1) * size_t(ld) + size_t(h.n)) * 8;
  if (pa < pb + bytes && pb < pa + bytes) fail(PCHEB_INVALID, "input and output vectors overlap");
}

extern "C" {

pcheb_status pcheb_setup(const pcheb_operator* A, const pcheb_params* p, hipStream_t stream, pcheb_handle* out) {
  return guarded([&]() -> pcheb_status {
    if (!out) fail(PCHEB_INVALID, "out is null");
    *out = reinterpret_cast<pcheb_handle>(create_handle(A, p, stream));
    return PCHEB_OK;
  });
}

pcheb_status pcheb_apply(pcheb_handle hh, const double* r, double* z, int32_t nrhs, int64_t ld, hipStream_t stream) {
  return guarded([&]() -> pcheb_status {
    Handle& h = *as_handle(hh);
    check_vectors(h, r, z, nrhs, ld);
    for (int32_t j = 0; j < nrhs; ++j) {
      const double* rj = r + int64_t(j) * ld;
      double* zj = z + int64_t(j) * ld;
      PCHEB_BY_PREC(h, enqueue_apply_one, h, rj, zj, stream);
    }
    PCHEB_HIP_CHECK(hipGetLastError());
    return PCHEB_OK;
  });
}

pcheb_status pcheb_matvec(pcheb_handle hh, const double* x, double* y, int32_t nrhs, int64_t ld, hipStream_t stream) {
  return guarded([&]() -> pcheb_status {
    Handle& h = *as_handle(hh);
    check_vectors(h, x, y, nrhs, ld);
    launch_ahat(h, InVec<double>{x, ld}, EpiStore<double>{y, nullptr, nullptr, ld}, 0, nrhs, stream);
    PCHEB_HIP_CHECK(hipGetLastError());
    return PCHEB_OK;
  });
}

pcheb_status pcg_solve(pcheb_handle hh, const double* b, double* x, int32_t nrhs, int64_t ld, double tol,
                       int32_t maxit, uint32_t flags, pcg_stats* stats, hipStream_t stream) {
  return guarded([&]() -> pcheb_status {
    Handle& h = *as_handle(hh);
    check_vectors(h, b, x, nrhs, ld);
    if (!(tol > 0.0) || !std::isfinite(tol)) fail(PCHEB_INVALID, "tol must be positive");
    if (maxit < 1) fail(PCHEB_INVALID, "maxit must be >= 1");
    pcheb_status st = PCHEB_OK;
    switch (h.prm.prec) {
      case PCHEB_F64:
        st = solve_impl<double>(h, b, x, nrhs, ld, tol, maxit, flags, stats, stream);
        break;
      case PCHEB_F32:
        st = solve_impl<float>(h, b, x, nrhs, ld, tol, maxit, flags, stats, stream);
        break;
      default:
        st = solve_impl<bf16>(h, b, x, nrhs, ld, tol, maxit, flags, stats, stream);
        break;
    }
    if (st == PCHEB_BREAKDOWN) set_last_error("PCG breakdown: (p, Ap) <= 0, (r, z) <= 0 or a non-finite value");
    if (st == PCHEB_NOT_CONVERGED) set_last_error("PCG reached maxit without meeting tol");
    return st;
  });
}

pcheb_status pcheb_destroy(pcheb_handle hh) {
  return guarded([&]() -> pcheb_status {
    destroy_handle(reinterpret_cast<Handle*>(hh));
    return PCHEB_OK;
  });
}

const char* pcheb_last_error(void) { return last_error_cstr(); }

pcheb_status pcheb_set_allocator(pcheb_alloc_fn alloc_fn, pcheb_free_fn free_fn, void* ctx) {
  set_last_error("");
  if ((alloc_fn == nullptr) != (free_fn == nullptr)) {
    set_last_error("pcheb_set_allocator needs both functions or neither");
    return PCHEB_INVALID;
  }
  std::lock_guard<std::mutex> lock(g_alloc_mu);
  g_alloc = AllocatorFns{alloc_fn, free_fn, alloc_fn ? ctx : nullptr};
  return PCHEB_OK;
}

size_t pcheb_footprint_bytes(const pcheb_operator* A, const pcheb_params* p, int32_t nrhs) {
  if (!A || !p) return 0;
  return footprint(A, p, nrhs);
}

}  // extern "C"

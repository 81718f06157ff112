// Device-side building blocks shared by every kernel of the library:
// storage types (float64 / float32 / bfloat16 with float32 arithmetic),
// wavefront and block sums, the two-kernel grid reduction, XCD-aware tile
// enumeration and the solver state that lives in device memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"

namespace pcheb {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlock = 256;        // threads per block for every kernel
constexpr int kNumXcd = 8;         // MI355X: 8 accelerator complex dies, one L2 each
constexpr int kMaxGrid = 8192;     // cap on blocks of grid-stride kernels (bounds reduction partials)
constexpr int kMaxReduce = 4;      // values reduced per kernel at most

// ---------------------------------------------------------------- storage types

struct bf16 {
  uint16_t bits;
};

__device__ __forceinline__ float bf16_to_float(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

// float -> bfloat16, round to nearest, ties to even; NaN stays a quiet NaN.
// gfx950 converts in one instruction (v_cvt_pk_bf16_f32, two values per
// instruction); it equals the integer rounding (u + 0x7fff + lsb) >> 16 on
// every non-NaN float (checked on all 2^32 bit patterns).
__device__ __forceinline__ uint16_t float_to_bf16(float f) {
  const __bf16 h = static_cast<__bf16>(f);
  return __builtin_bit_cast(uint16_t, h);
}

// Float64 vector outputs are stored non-temporally: a solve writes whole
// vectors that are read again only after other vectors have streamed through
// the L2, and the streaming store keeps the L2 for the halo and partner lines
// a kernel is still reading (27-point float64 step 106 -> 100 us on 192^3).
// Float32 and bfloat16 outputs keep ordinary stores, which measured faster
// for them; the fused 7-point pass picks its own policy.
typedef double dbl2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void out_store(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void out_store2(double* p, double a, double b) {
  __builtin_nontemporal_store(dbl2v{a, b}, reinterpret_cast<dbl2v*>(p));
}

template <class T>
struct Store;

// ld/st: one element; st2: elements i and i+1 in one access (i even, base
// pointer aligned to the pair size).
template <>
struct Store<double> {
  using acc = double;
  static __device__ __forceinline__ double ld(const double* p, int64_t i) { return p[i]; }
  static __device__ __forceinline__ void st(double* p, int64_t i, double v) { out_store(p + i, v); }
  static __device__ __forceinline__ void st2(double* p, int64_t i, double a, double b) { out_store2(p + i, a, b); }
};

template <>
struct Store<float> {
  using acc = float;
  static __device__ __forceinline__ float ld(const float* p, int64_t i) { return p[i]; }
  static __device__ __forceinline__ void st(float* p, int64_t i, float v) { p[i] = v; }
  static __device__ __forceinline__ void st2(float* p, int64_t i, float a, float b) {
    *reinterpret_cast<float2*>(p + i) = make_float2(a, b);
  }
};

template <>
struct Store<bf16> {
  using acc = float;
  static __device__ __forceinline__ float ld(const bf16* p, int64_t i) { return bf16_to_float(p[i].bits); }
  static __device__ __forceinline__ void st(bf16* p, int64_t i, float v) { p[i].bits = float_to_bf16(v); }
  static __device__ __forceinline__ void st2(bf16* p, int64_t i, float a, float b) {
    *reinterpret_cast<uint32_t*>(p + i) = uint32_t(float_to_bf16(a)) | (uint32_t(float_to_bf16(b)) << 16);
  }
};

__device__ __forceinline__ double2 ld2(const double* p, int64_t i) { return *reinterpret_cast<const double2*>(p + i); }

// ---------------------------------------------------------------- solver state

// Scalars of one PCG solve.  They stay in device memory: kernels read alpha
// and beta from here and the finalize kernel of each reduction writes them, so
// the host never sits between two iterations.
struct DevState {
  double gamma;      // (r, z) for the current z
  double alpha;      // gamma / (p, q)
  double beta;       // direction update coefficient
  double pq;         // (p, A p)
  double rr;         // ||r||^2 in the D^-1 weighted norm
  double bb;         // ||b||^2 in the D^-1 weighted norm
  double tol;        // relative tolerance
  double relres;     // sqrt(rr / bb)
  double true_rr;    // ||b - A x||^2, D^-1 weighted (exit check)
  double true_rr_hat;// ||b - A x||^2, unweighted
  double bb_hat;     // ||b||^2, unweighted
  double scratch;    // result slot of stand-alone reductions
  int32_t iter;      // completed iterations
  int32_t maxit;
  int32_t done;      // 0 running, 1 converged, 2 breakdown, 3 iteration limit
  int32_t flexible;  // 1: Polak-Ribiere beta
  int32_t refreshes; // true-residual replacements performed
  int32_t pad;
};

enum : int32_t { kRunning = 0, kConverged = 1, kBreakdown = 2, kMaxIter = 3 };

// Partial sums of a grid reduction: one slot of kMaxReduce doubles per block.
struct ReduceBuf {
  double* partials;
};

// ---------------------------------------------------------------- reductions

template <int NV>
__device__ __forceinline__ void wave_sum(double (&v)[NV]) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] += __shfl_xor(v[i], off, kWave);
  }
}

// Sum over the block of NT threads; the result is valid in thread 0 only.  Fixed order.
template <int NV, int NT = kBlock>
__device__ __forceinline__ void block_sum(double (&v)[NV], int tid) {
  __shared__ double sh[NT / kWave][NV > 0 ? NV : 1];
  wave_sum<NV>(v);
  const int lane = tid % kWave, wave = tid / kWave;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) sh[wave][i] = v[i];
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = sh[0][i];
      for (int w = 1; w < NT / kWave; ++w) s += sh[w][i];
      v[i] = s;
    }
  }
  __syncthreads();
}

// Grid reductions in two kernels.  Every block of the producing kernel sums
// its values and stores them, with a plain store, in its own slot; a one-block
// finalize kernel then adds the slots in slot order (a fixed order, so the
// result is reproducible for a given grid) and calls fin(total).  The kernel
// boundary makes the slots visible, so no block needs a device-scope fence
// (on a multi-XCD part such a fence writes back and invalidates the whole
// L2 of the die) and no atomic counter is contended.  Every right-hand side
// (solve slot) has its own kMaxGrid partial slots.
__device__ __forceinline__ size_t partial_index(int slot, uint32_t block) {
  return (size_t(slot) * kMaxGrid + block) * kMaxReduce;
}

template <int NV, int NT = kBlock>
__device__ __forceinline__ void block_partial(double (&v)[NV], ReduceBuf rb, int slot) {
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  block_sum<NV, NT>(v, tid);
  if (tid == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) rb.partials[partial_index(slot, blockIdx.x) + i] = v[i];
  }
}

// One block per solve slot (slot = slot0 + blockIdx.x); fin.bind(slot) points
// the functor at that slot's state before fin(total).  kFinThreads threads each
// load their kMaxGrid / kFinThreads partials up front (one memory latency, not
// one per partial) and add them in block order.
constexpr int kFinThreads = 1024;
static_assert(kMaxGrid % kFinThreads == 0, "the finalize loads kMaxGrid / kFinThreads partials per thread");
template <int NV, class Fin>
struct KFinalize {
  static constexpr int kThreads = kFinThreads;
  __device__ static void run(Fin fin, ReduceBuf rb, uint32_t nblocks, const DevState* guard, int slot0);
};
template <int NV, class Fin>
__device__ __forceinline__ void KFinalize<NV, Fin>::run(Fin fin, ReduceBuf rb, uint32_t nblocks, const DevState* guard,
                                                        int slot0) {
  const int slot = slot0 + int(blockIdx.x);
  if (guard && guard[slot].done != kRunning) return;
  fin.bind(slot);
  constexpr int kPer = kMaxGrid / kFinThreads;
  double v[kPer][NV];
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const uint32_t b = threadIdx.x + uint32_t(m) * kFinThreads;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[m][i] = b < nblocks ? rb.partials[partial_index(slot, b) + i] : 0.0;
  }
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    acc[i] = 0.0;
#pragma unroll
    for (int m = 0; m < kPer; ++m) acc[i] += v[m][i];
  }
  block_sum<NV, kFinThreads>(acc, threadIdx.x);
  if (threadIdx.x == 0) fin(acc);
}

// ---------------------------------------------------------------- tile enumeration

// Blocks are dispatched to the XCDs round robin (block b runs on XCD b % 8).
// Give every XCD one contiguous range of tiles, so the halo that neighbouring
// tiles share is reused in that XCD's L2.  The grid size must be a multiple of 8.
struct XcdTiles {
  uint32_t begin, end, step;
  __device__ __forceinline__ explicit XcdTiles(uint32_t ntiles) {
    const uint32_t xcd = blockIdx.x % kNumXcd;
    const uint32_t local = blockIdx.x / kNumXcd;
    const uint32_t per = (ntiles + kNumXcd - 1) / kNumXcd;
    const uint32_t lo = xcd * per;
    const uint32_t hi = lo + per < ntiles ? lo + per : ntiles;
    begin = lo + local;
    end = hi;
    step = gridDim.x / kNumXcd;
  }
};

}  // namespace pcheb

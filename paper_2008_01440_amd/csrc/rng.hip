// Seeded uniform vectors on the device (pcheb_fill_uniform); see rng.hpp.

#include "rng.hpp"

#include <algorithm>

#include "handle.hpp"

namespace pcheb {

__global__ void k_fill_uniform(double* __restrict__ v, int64_t n, uint64_t seed, double lo, double hi) {
#pragma clang fp contract(off)
  const double w = hi - lo;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    uint64_t z = seed + uint64_t(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u = double(z >> 11) * 0x1.0p-53;
    v[i] = lo + w * u;  // two roundings (no contraction), as in sequential code
  }
}

void launch_fill_uniform(double* v, int64_t n, uint64_t seed, double lo, double hi, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
  k_fill_uniform<<<uint32_t(blocks), kBlock, 0, s>>>(v, n, seed, lo, hi);
  PCHEB_HIP_CHECK(hipGetLastError());
}

}  // namespace pcheb

using namespace pcheb;

extern "C" pcheb_status pcheb_fill_uniform(double* v, int64_t n, uint64_t seed, double lo, double hi,
                                           hipStream_t stream) {
  try {
    set_last_error("");
    if (n < 0) fail(PCHEB_INVALID, "n must be >= 0");
    if (n > 0 && !v) fail(PCHEB_INVALID, "null vector");
    if (!(lo <= hi)) fail(PCHEB_INVALID, "need lo <= hi");
    launch_fill_uniform(v, n, seed, lo, hi, stream);
    return PCHEB_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.status;
  } catch (...) {
    set_last_error("unexpected internal error");
    return PCHEB_HIP;
  }
}

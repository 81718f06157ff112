// Extreme-eigenvalue bounds of the Jacobi-scaled operator by the Lanczos
// method with full reorthogonalisation.  The paper estimates the bounds with a
// few power iterations and DACG (Sec. 5.1); Lanczos gives both ends from one
// Krylov space.  The Ritz values lie inside the spectrum, so callers widen the
// upper bound before building the preconditioner.
//
// Step j: w = A v_j; alpha_j = (v_j, w); classical Gram-Schmidt against
// v_0..v_j twice (c = V^T w, w -= V c); beta_j = ||w||; v_{j+1} = w / beta_j.
// Everything stays on the device: the dot products of a pass are one kernel
// over w and the basis (up to kCols columns at a time), the first update is
// fused with the second pass's dot products and the second update with the
// norm, and one-block finalize kernels sum the partials in block order into
// the coefficients, alpha, beta and 1/beta that the next kernel reads.  The
// host reads alpha and beta once at the end and stops the tridiagonal at the
// first beta that vanishes relative to alpha (the later steps then worked on
// a meaningless vector and are discarded).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "dispatch.hpp"
#include "handle.hpp"

namespace pcheb {

constexpr int kLzGrid = 2048;  // blocks of the vector kernels (partials per column)
constexpr int kCols = 32;      // basis columns whose dot products one pass accumulates

// Vectors are walked two elements at a time (16-byte accesses; columns of V
// start at even offsets); element pair q covers 2q and 2q + 1 < n.

// partial[k * kLzGrid + b] = block b's share of (V[col0 + k], w), k < ncol.
__global__ __launch_bounds__(kBlock) void k_lz_dots(const double* __restrict__ V, int64_t ldv, int col0, int ncol,
                                                    const double* __restrict__ w, int64_t n,
                                                    double* __restrict__ partial) {
  double acc[kCols];
#pragma unroll
  for (int k = 0; k < kCols; ++k) acc[k] = 0.0;
  const int64_t npairs = n / 2;
  for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < npairs; q += int64_t(gridDim.x) * blockDim.x) {
    const double2 wq = ld2(w, 2 * q);
#pragma unroll
    for (int k = 0; k < kCols; ++k)
      if (k < ncol) {
        const double2 vq = ld2(V + int64_t(col0 + k) * ldv, 2 * q);
        acc[k] += vq.x * wq.x + vq.y * wq.y;
      }
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {  // odd tail
    const double wi = w[n - 1];
#pragma unroll
    for (int k = 0; k < kCols; ++k)
      if (k < ncol) acc[k] += V[int64_t(col0 + k) * ldv + n - 1] * wi;
  }
  block_sum<kCols>(acc, threadIdx.x);  // all columns at once (fixed order)
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kCols; ++k)
      if (k < ncol) partial[k * kLzGrid + blockIdx.x] = acc[k];
  }
}

// w -= sum_{k < m} c[k] V[k]; then, if DOTS, partials of (V[k], w) for k < m
// (m <= kCols), and if NORM, partials of (w, w) in column 0.
template <bool DOTS, bool NORM>
__global__ __launch_bounds__(kBlock) void k_lz_update(const double* __restrict__ V, int64_t ldv, int m,
                                                      const double* __restrict__ c, double* __restrict__ w, int64_t n,
                                                      double* __restrict__ partial) {
  constexpr int NV = DOTS ? kCols : 1;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  auto one = [&](int64_t i0, int cnt) {  // elements i0 .. i0 + cnt - 1 (cnt = 2, or 1 for the odd tail)
    double w0 = w[i0], w1 = cnt > 1 ? w[i0 + 1] : 0.0;
    double s0 = 0.0, s1 = 0.0;
    for (int k = 0; k < m; ++k) {
      const double* vk = V + int64_t(k) * ldv + i0;
      s0 += c[k] * vk[0];
      if (cnt > 1) s1 += c[k] * vk[1];
    }
    w0 -= s0;
    w1 -= s1;
    w[i0] = w0;
    if (cnt > 1) w[i0 + 1] = w1;
    if constexpr (DOTS) {
#pragma unroll
      for (int k = 0; k < kCols; ++k)
        if (k < m) {
          const double* vk = V + int64_t(k) * ldv + i0;
          acc[k] += vk[0] * w0 + (cnt > 1 ? vk[1] * w1 : 0.0);
        }
    }
    if constexpr (NORM) acc[0] += w0 * w0 + w1 * w1;
  };
  const int64_t npairs = n / 2;
  for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < npairs; q += int64_t(gridDim.x) * blockDim.x)
    one(2 * q, 2);
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) one(n - 1, 1);
  if constexpr (DOTS || NORM) {
    const int nc = DOTS ? m : 1;
    block_sum<NV>(acc, threadIdx.x);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < NV; ++k)
        if (k < nc) partial[k * kLzGrid + blockIdx.x] = acc[k];
    }
  }
}

// One block: out[col0 + k] = sum over blocks of partial[k][.] (each thread a
// strided share in block order, then the fixed block tree), k < ncol.  With
// `alpha`, the sum of column j (the step) is also stored in alpha[j].  With
// `norm`, column 0 is a squared norm: *norm = its square root and *inv = 1 / *norm.
__global__ __launch_bounds__(kBlock) void k_lz_finalize(const double* __restrict__ partial, int ncol, double* out,
                                                        int col0, double* alpha, int j, double* norm,
                                                        double* inv) {
  for (int k = 0; k < ncol; ++k) {
    double t[1] = {0.0};
    for (int b = threadIdx.x; b < kLzGrid; b += blockDim.x) t[0] += partial[k * kLzGrid + b];
    block_sum<1>(t, threadIdx.x);
    if (threadIdx.x == 0) {
      if (out) out[col0 + k] = t[0];
      if (alpha && col0 + k == j) alpha[j] = t[0];
      if (norm && k == 0) {
        const double r = sqrt(t[0]);
        norm[0] = r;
        inv[0] = 1.0 / r;
      }
    }
  }
}

__global__ void k_lz_scale(const double* __restrict__ a, double* __restrict__ b, const double* __restrict__ f,
                           int64_t n) {
  const double s = f[0];
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    b[i] = a[i] * s;
}

__global__ void k_isqrt_diag(const double* invd, double c, double* isd, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    isd[i] = sqrt(invd ? invd[i] : c);
}

// Number of eigenvalues below x of the symmetric tridiagonal (a, b) (Sturm count).
static int sturm_below(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int count = 0;
  double d = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double off = i ? b[i - 1] * b[i - 1] / d : 0.0;
    d = (a[i] - x) - off;
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++count;
  }
  return count;
}

// k-th smallest eigenvalue (1-based) of the tridiagonal by bisection.
static double tridiag_eig(const std::vector<double>& a, const std::vector<double>& b, int k) {
  double lo = a[0], hi = a[0];
  for (size_t i = 0; i < a.size(); ++i) {
    const double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < a.size() ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-16 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_below(a, b, mid) >= k)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

static void lanczos(Handle& h, const double* v0, int steps, double* lmin, double* lmax, hipStream_t s) {
  const int64_t n = h.n;
  const int m = int(std::min<int64_t>(steps, n));
  const int64_t ldv = (n + 1) / 2 * 2;  // columns 16-byte aligned
  double* V = static_cast<double*>(dev_alloc(h, size_t(m + 1) * size_t(ldv) * sizeof(double)));
  double* w = static_cast<double*>(dev_alloc(h, size_t(n) * sizeof(double)));
  double* isd = static_cast<double*>(dev_alloc(h, size_t(n) * sizeof(double)));
  double* partial = static_cast<double*>(dev_alloc(h, size_t(kCols) * kLzGrid * sizeof(double)));
  // coefficients c (m + 1), alpha (m), beta (m), 1/beta (1), ||v0|| (1)
  double* scal = static_cast<double*>(dev_alloc(h, size_t(3 * m + 3) * sizeof(double)));
  double* coef = scal;
  double* alpha = scal + (m + 1);
  double* beta = alpha + m;
  double* inv = beta + m;
  double* nrm0 = inv + 1;
  const uint32_t g = 2048;
  k_isqrt_diag<<<g, kBlock, 0, s>>>(h.invd, 1.0 / 6.0, isd, n);

  // v_0 = v0 / ||v0|| (the one host check: a zero or non-finite start vector is an error)
  k_lz_dots<<<kLzGrid, kBlock, 0, s>>>(v0, 0, 0, 1, v0, n, partial);
  k_lz_finalize<<<1, kBlock, 0, s>>>(partial, 1, nullptr, 0, nullptr, 0, nrm0, inv);
  double nrm = 0.0;
  PCHEB_HIP_CHECK(hipMemcpyAsync(&nrm, nrm0, sizeof(double), hipMemcpyDeviceToHost, s));
  PCHEB_HIP_CHECK(hipStreamSynchronize(s));
  if (!(nrm > 0.0) || !std::isfinite(nrm)) fail(PCHEB_INVALID, "start vector must be nonzero and finite");
  k_lz_scale<<<g, kBlock, 0, s>>>(v0, V, inv, n);

  for (int j = 0; j < m; ++j) {
    const double* vj = V + int64_t(j) * ldv;
    const int cols = j + 1;
    launch_ahat(h, InScaled{vj, isd, n}, EpiScaledStore{w, isd, nullptr, nullptr, n}, 0, 1, s);
    // pass 1: c = V^T w (alpha_j = c[j]); then w -= V c
    for (int c0 = 0; c0 < cols; c0 += kCols) {
      const int nc = std::min(kCols, cols - c0);
      k_lz_dots<<<kLzGrid, kBlock, 0, s>>>(V, ldv, c0, nc, w, n, partial);
      k_lz_finalize<<<1, kBlock, 0, s>>>(partial, nc, coef, c0, alpha, j, nullptr, nullptr);
    }
    if (cols <= kCols) {  // first update fused with the second pass's dot products
      k_lz_update<true, false><<<kLzGrid, kBlock, 0, s>>>(V, ldv, cols, coef, w, n, partial);
      k_lz_finalize<<<1, kBlock, 0, s>>>(partial, cols, coef, 0, nullptr, j, nullptr, nullptr);
    } else {
      k_lz_update<false, false><<<kLzGrid, kBlock, 0, s>>>(V, ldv, cols, coef, w, n, partial);
      for (int c0 = 0; c0 < cols; c0 += kCols) {
        const int nc = std::min(kCols, cols - c0);
        k_lz_dots<<<kLzGrid, kBlock, 0, s>>>(V, ldv, c0, nc, w, n, partial);
        k_lz_finalize<<<1, kBlock, 0, s>>>(partial, nc, coef, c0, nullptr, j, nullptr, nullptr);
      }
    }
    // pass 2 update with the norm: beta_j = ||w||
    k_lz_update<false, true><<<kLzGrid, kBlock, 0, s>>>(V, ldv, cols, coef, w, n, partial);
    k_lz_finalize<<<1, kBlock, 0, s>>>(partial, 1, nullptr, 0, nullptr, j, beta + j, inv);
    if (j + 1 < m) k_lz_scale<<<g, kBlock, 0, s>>>(w, V + int64_t(j + 1) * ldv, inv, n);
    PCHEB_HIP_CHECK(hipGetLastError());
  }
  std::vector<double> a(static_cast<size_t>(m)), b(static_cast<size_t>(m));
  PCHEB_HIP_CHECK(hipMemcpyAsync(a.data(), alpha, size_t(m) * sizeof(double), hipMemcpyDeviceToHost, s));
  PCHEB_HIP_CHECK(hipMemcpyAsync(b.data(), beta, size_t(m) * sizeof(double), hipMemcpyDeviceToHost, s));
  PCHEB_HIP_CHECK(hipStreamSynchronize(s));
  int used = m;
  for (int j = 0; j + 1 < m; ++j)
    if (!(b[size_t(j)] > 1e-14 * std::fabs(a[size_t(j)]))) {
      used = j + 1;
      break;
    }
  a.resize(size_t(used));
  b.resize(size_t(used > 0 ? used - 1 : 0));
  *lmin = tridiag_eig(a, b, 1);
  *lmax = tridiag_eig(a, b, used);
}

}  // namespace pcheb

using namespace pcheb;

extern "C" pcheb_status pcheb_estimate_bounds(const pcheb_operator* A, const double* v0, int32_t nsteps,
                                              double* lambda_min, double* lambda_max, hipStream_t stream) {
  try {
    set_last_error("");
    if (!A || !v0 || !lambda_min || !lambda_max) fail(PCHEB_INVALID, "null argument");
    if (reinterpret_cast<uintptr_t>(v0) % 16 != 0) fail(PCHEB_INVALID, "v0 must be 16-byte aligned");
    if (nsteps < 1 || nsteps > 1000) fail(PCHEB_INVALID, "nsteps must be in [1, 1000]");
    if (A->n <= 0) fail(PCHEB_INVALID, "n must be positive");
    if ((A->kind == PCHEB_OP_CSR || A->kind == PCHEB_OP_SELL) && (!A->rowptr || !A->colind || !A->values))
      fail(PCHEB_INVALID, "CSR arrays must be non-null");
    if ((A->kind == PCHEB_OP_STENCIL7 || A->kind == PCHEB_OP_STENCIL27H) &&
        int64_t(A->nx) * A->ny * A->nz != A->n)
      fail(PCHEB_INVALID, "n must equal nx*ny*nz");
    if (A->kind == PCHEB_OP_STENCIL27H && !A->cell_coeff) fail(PCHEB_INVALID, "cell_coeff must be non-null");
    if (A->kind < PCHEB_OP_CSR || A->kind > PCHEB_OP_STENCIL27H) fail(PCHEB_INVALID, "unknown operator kind");
    Handle h;
    h.op = *A;
    h.op.kind = (A->kind == PCHEB_OP_SELL) ? PCHEB_OP_CSR : A->kind;  // the product itself is all that is needed
    h.prm.prec = PCHEB_F64;
    h.n = A->n;
    try {
      setup_operator(h, stream);
      lanczos(h, v0, nsteps, lambda_min, lambda_max, stream);
    } catch (...) {
      (void)hipStreamSynchronize(stream);
      release(h);
      throw;
    }
    (void)hipStreamSynchronize(stream);
    release(h);
    return PCHEB_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.status;
  } catch (...) {
    set_last_error("unexpected internal error");
    return PCHEB_HIP;
  }
}

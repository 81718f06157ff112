// Extreme-eigenvalue bounds of the Jacobi-scaled operator by the Lanczos
// method with full reorthogonalisation.  The paper estimates the bounds with a
// few power iterations and DACG (Sec. 5.1); Lanczos gives both ends from one
// Krylov space.  The Ritz values lie inside the spectrum, so callers widen the
// upper bound before building the preconditioner.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "dispatch.hpp"
#include "handle.hpp"

namespace pcheb {

constexpr int kDotGrid = 512;

// partial[b] = sum over this block's share of a[i] * b[i]
__global__ void k_dot_partial(const double* a, const double* b, int64_t n, double* partial) {
  double v[1] = {0.0};
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    v[0] += a[i] * b[i];
  block_sum<1>(v, threadIdx.x);
  if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

// w -= sum_m c[m] V[m]   (V holds m vectors of length n, stride n)
__global__ void k_sub_combination(double* w, const double* V, const double* c, int m, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    double acc = 0.0;
    for (int j = 0; j < m; ++j) acc += c[j] * V[int64_t(j) * n + i];
    w[i] -= acc;
  }
}

__global__ void k_scale_copy(const double* a, double* b, double s, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    b[i] = a[i] * s;
}

__global__ void k_isqrt_diag(const double* invd, double c, double* isd, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    isd[i] = sqrt(invd ? invd[i] : c);
}

// Dot products of w with the first m columns of V, summed on the host in block order.
static void dots(const double* V, int m, const double* w, int64_t n, double* partial, std::vector<double>& host,
                 std::vector<double>& out, hipStream_t s) {
  for (int j = 0; j < m; ++j) k_dot_partial<<<kDotGrid, kBlock, 0, s>>>(V + int64_t(j) * n, w, n, partial + j * kDotGrid);
  PCHEB_HIP_CHECK(hipGetLastError());
  host.resize(size_t(m) * kDotGrid);
  PCHEB_HIP_CHECK(hipMemcpyAsync(host.data(), partial, host.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  PCHEB_HIP_CHECK(hipStreamSynchronize(s));
  out.assign(size_t(m), 0.0);
  for (int j = 0; j < m; ++j)
    for (int b = 0; b < kDotGrid; ++b) out[size_t(j)] += host[size_t(j) * kDotGrid + size_t(b)];
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
  double* V = static_cast<double*>(dev_alloc(h, size_t(m + 1) * size_t(n) * sizeof(double)));
  double* w = static_cast<double*>(dev_alloc(h, size_t(n) * sizeof(double)));
  double* isd = static_cast<double*>(dev_alloc(h, size_t(n) * sizeof(double)));
  double* partial = static_cast<double*>(dev_alloc(h, size_t(m + 1) * kDotGrid * sizeof(double)));
  double* coef = static_cast<double*>(dev_alloc(h, size_t(m + 1) * sizeof(double)));
  const uint32_t g = 2048;
  k_isqrt_diag<<<g, kBlock, 0, s>>>(h.invd, 1.0 / 6.0, isd, n);
  std::vector<double> host, out;
  dots(v0, 1, v0, n, partial, host, out, s);
  if (!(out[0] > 0.0) || !std::isfinite(out[0])) fail(PCHEB_INVALID, "start vector must be nonzero and finite");
  k_scale_copy<<<g, kBlock, 0, s>>>(v0, V, 1.0 / std::sqrt(out[0]), n);
  std::vector<double> alpha, beta;
  for (int j = 0; j < m; ++j) {
    const double* vj = V + int64_t(j) * n;
    launch_ahat(h, InScaled{vj, isd, n}, EpiScaledStore{w, isd, nullptr, nullptr, n}, 0, 1, s);
    PCHEB_HIP_CHECK(hipGetLastError());
    dots(vj, 1, w, n, partial, host, out, s);
    alpha.push_back(out[0]);
    for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, twice
      std::vector<double> c;
      dots(V, j + 1, w, n, partial, host, c, s);
      PCHEB_HIP_CHECK(hipMemcpyAsync(coef, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice, s));
      k_sub_combination<<<g, kBlock, 0, s>>>(w, V, coef, j + 1, n);
    }
    dots(w, 1, w, n, partial, host, out, s);
    const double bj = std::sqrt(std::max(0.0, out[0]));
    if (j + 1 == m || bj <= 1e-14 * std::fabs(alpha.back())) break;
    beta.push_back(bj);
    k_scale_copy<<<g, kBlock, 0, s>>>(w, V + int64_t(j + 1) * n, 1.0 / bj, n);
  }
  PCHEB_HIP_CHECK(hipStreamSynchronize(s));
  *lmin = tridiag_eig(alpha, beta, 1);
  *lmax = tridiag_eig(alpha, beta, int(alpha.size()));
}

}  // namespace pcheb

using namespace pcheb;

extern "C" pcheb_status pcheb_estimate_bounds(const pcheb_operator* A, const double* v0, int32_t nsteps,
                                              double* lambda_min, double* lambda_max, hipStream_t stream) {
  try {
    set_last_error("");
    if (!A || !v0 || !lambda_min || !lambda_max) fail(PCHEB_INVALID, "null argument");
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

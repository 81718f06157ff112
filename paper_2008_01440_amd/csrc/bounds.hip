// Extreme-eigenvalue bounds of the Jacobi-scaled operator A = D^-1/2 A_hat D^-1/2.
//
// 1. Lanczos with full reorthogonalisation (pcheb_estimate_bounds).  The Ritz
//    values lie inside the spectrum, so callers widen the upper bound before
//    building the preconditioner.
//
//    Step j: w = A v_j; alpha_j = (v_j, w); classical Gram-Schmidt against
//    v_0..v_j twice (c = V^T w, w -= V c); beta_j = ||w||; v_{j+1} = w / beta_j.
//    Everything stays on the device: the dot products of a pass are one kernel
//    over w and the basis (up to kCols columns at a time), the first update is
//    fused with the second pass's dot products and the second update with the
//    norm, and one-block finalize kernels sum the partials in block order into
//    the coefficients, alpha, beta and 1/beta that the next kernel reads.  The
//    host reads alpha and beta once at the end and stops the tridiagonal at the
//    first beta that vanishes relative to alpha (the later steps then worked on
//    a meaningless vector and are discarded).
//
// 2. The paper's own estimators (Sec. 5.1; pcheb_estimate_bounds_pdacg): a few
//    steps of the power method for lambda_max and the DACG method without
//    preconditioning for lambda_min (see the comment above dacg()).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dispatch.hpp"
#include "handle.hpp"

// Workspace of pcheb_estimate_bounds_noalloc: a fixed array in device memory
// that every call on a device shares (the code object holds one copy per
// device until the process ends).  In host code `scratch` names a host-side
// stand-in, so it is never passed to a kernel or a copy: the device address
// comes from hipGetSymbolAddress (scratch_on_current_device).
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

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

// Block k < ncol: out[col0 + k] = sum over blocks of partial[k][.] (each thread
// a strided share in block order, then the fixed block tree).  With
// `alpha`, the sum of column j (the step) is also stored in alpha[j].  With
// `norm`, column 0 is a squared norm: *norm = its square root and *inv = 1 / *norm.
__global__ __launch_bounds__(kFinThreads) void k_lz_finalize(const double* __restrict__ partial, int ncol,
                                                             double* out, int col0, double* alpha, int j,
                                                             double* norm, double* inv) {
  // every thread loads its partials before adding them
  static_assert(kLzGrid % kFinThreads == 0, "partials per thread");
  constexpr int kPer = kLzGrid / kFinThreads;
  const int k = int(blockIdx.x);
  if (k >= ncol) return;
  double v[kPer];
#pragma unroll
  for (int m = 0; m < kPer; ++m) v[m] = partial[k * kLzGrid + int(threadIdx.x) + m * kFinThreads];
  double t[1] = {0.0};
#pragma unroll
  for (int m = 0; m < kPer; ++m) t[0] += v[m];
  block_sum<1, kFinThreads>(t, threadIdx.x);
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

// Node blocks: u = W v = L^-T v per node (M = L^-1 stored row-major lower).
__global__ void k_node_wv(const double* __restrict__ v, double* __restrict__ u, const double* __restrict__ lfac,
                          int64_t nodes) {
  for (int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; I < nodes; I += int64_t(gridDim.x) * blockDim.x) {
    const double* m = lfac + 6 * I;
    const double v0 = v[3 * I], v1 = v[3 * I + 1], v2 = v[3 * I + 2];
    u[3 * I] = m[0] * v0 + m[1] * v1 + m[3] * v2;
    u[3 * I + 1] = m[2] * v1 + m[4] * v2;
    u[3 * I + 2] = m[5] * v2;
  }
}

// Node blocks: w <- W^T w = L^-1 w per node, in place.
__global__ void k_node_wtw(double* __restrict__ w, const double* __restrict__ lfac, int64_t nodes) {
  for (int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; I < nodes; I += int64_t(gridDim.x) * blockDim.x) {
    const double* m = lfac + 6 * I;
    const double w0 = w[3 * I], w1 = w[3 * I + 1], w2 = w[3 * I + 2];
    w[3 * I] = m[0] * w0;
    w[3 * I + 1] = m[1] * w0 + m[2] * w1;
    w[3 * I + 2] = m[3] * w0 + m[4] * w1 + m[5] * w2;
  }
}

// w = C v for the operator whose bounds are estimated: C = D^-1/2 A_hat D^-1/2
// (one fused launch), or with node blocks C = W^T A W on the block Jacobi
// factor W of the Jacobi-scaled A, i.e. C = L^-1 A_hat L^-T with L L^T the 3x3
// diagonal blocks of A_hat (the diagonal scaling cancels).
struct ScaledProduct {
  Handle* h;
  const double* isd;  // D^-1/2 (point scaling)
  double* u;          // node blocks: workspace for W v
  hipStream_t s;
  void operator()(const double* v, double* w) const {
    const int64_t n = h->n;
    if (h->bs == 3) {
      k_node_wv<<<kLzGrid, kBlock, 0, s>>>(v, u, h->lfac, n / 3);
      launch_ahat(*h, InVec<double>{u, 0}, EpiStore<double>{w, nullptr, nullptr, 0}, 0, 1, s);
      k_node_wtw<<<kLzGrid, kBlock, 0, s>>>(w, h->lfac, n / 3);
    } else {
      launch_ahat(*h, InScaled{v, isd, n}, EpiScaledStore{w, isd, nullptr, nullptr, n}, 0, 1, s);
    }
  }
};

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
  double* u = h.bs == 3 ? static_cast<double*>(dev_alloc(h, size_t(n) * sizeof(double))) : nullptr;
  const ScaledProduct product{&h, isd, u, s};

  // v_0 = v0 / ||v0|| (the one host check: a zero or non-finite start vector is an error)
  k_lz_dots<<<kLzGrid, kBlock, 0, s>>>(v0, 0, 0, 1, v0, n, partial);
  k_lz_finalize<<<1, kFinThreads, 0, s>>>(partial, 1, nullptr, 0, nullptr, 0, nrm0, inv);
  double nrm = 0.0;
  PCHEB_HIP_CHECK(hipMemcpyAsync(&nrm, nrm0, sizeof(double), hipMemcpyDeviceToHost, s));
  PCHEB_HIP_CHECK(hipStreamSynchronize(s));
  if (!(nrm > 0.0) || !std::isfinite(nrm)) fail(PCHEB_INVALID, "start vector must be nonzero and finite");
  k_lz_scale<<<g, kBlock, 0, s>>>(v0, V, inv, n);

  for (int j = 0; j < m; ++j) {
    const double* vj = V + int64_t(j) * ldv;
    const int cols = j + 1;
    product(vj, w);
    // pass 1: c = V^T w (alpha_j = c[j]); then w -= V c
    for (int c0 = 0; c0 < cols; c0 += kCols) {
      const int nc = std::min(kCols, cols - c0);
      k_lz_dots<<<kLzGrid, kBlock, 0, s>>>(V, ldv, c0, nc, w, n, partial);
      k_lz_finalize<<<nc, kFinThreads, 0, s>>>(partial, nc, coef, c0, alpha, j, nullptr, nullptr);
    }
    if (cols <= kCols) {  // first update fused with the second pass's dot products
      k_lz_update<true, false><<<kLzGrid, kBlock, 0, s>>>(V, ldv, cols, coef, w, n, partial);
      k_lz_finalize<<<cols, kFinThreads, 0, s>>>(partial, cols, coef, 0, nullptr, j, nullptr, nullptr);
    } else {
      k_lz_update<false, false><<<kLzGrid, kBlock, 0, s>>>(V, ldv, cols, coef, w, n, partial);
      for (int c0 = 0; c0 < cols; c0 += kCols) {
        const int nc = std::min(kCols, cols - c0);
        k_lz_dots<<<kLzGrid, kBlock, 0, s>>>(V, ldv, c0, nc, w, n, partial);
        k_lz_finalize<<<nc, kFinThreads, 0, s>>>(partial, nc, coef, c0, nullptr, j, nullptr, nullptr);
      }
    }
    // pass 2 update with the norm: beta_j = ||w||
    k_lz_update<false, true><<<kLzGrid, kBlock, 0, s>>>(V, ldv, cols, coef, w, n, partial);
    k_lz_finalize<<<1, kFinThreads, 0, s>>>(partial, 1, nullptr, 0, nullptr, j, beta + j, inv);
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


// ------------------------------------------------------------------ power method and DACG

// Scalars of the two iterations, in device memory.  The first member is the
// guard that every kernel checks (done flag and step count).
struct EigState {
  DevState st;
  double xx, xax;      // (x, x) and (x, A x) of the current iterate
  double mu;           // current Rayleigh-quotient estimate
  double u1, u2;       // x <- u1 x + u2 p (Ritz vector coefficients)
  double gg, gg_old;   // ||g||^2 of this and the previous step
  double beta;         // direction coefficient of the next step
  double relres;       // ||A x - mu x|| / (mu ||x||)
  double inv;          // 1 / norm for the scale kernel
  double lmax;         // power method: Rayleigh quotient of the last iterate
};

// w = A v with (v, w), (w, w), (v, v) for one power step.
struct EpiPowerStep {
  using acc = double;
  static constexpr int NV = 3;
  static constexpr bool reduce = true;
  double* w;
  const double* isd;
  const double* v;
  EigState* E;
  DevState* st;
  const DevState* guard;
  __device__ __forceinline__ void bind(int) {}
  __device__ __forceinline__ void prepare() {}
  struct Pre {
    double isd, v;
  };
  __device__ __forceinline__ Pre load(int64_t i) const { return Pre{isd[i], v[i]}; }
  __device__ __forceinline__ void operator()(int64_t i, double, double m, const Pre& p, double (&part)[NV]) const {
    const double wi = m * p.isd;
    w[i] = wi;
    part[0] += p.v * wi;
    part[1] += wi * wi;
    part[2] += p.v * p.v;
  }
  __device__ void fin(double (&t)[NV]) const {
    E->lmax = t[0] / t[2];
    E->inv = 1.0 / sqrt(t[1]);
  }
};

// A x with (x, x) and (x, A x): the Rayleigh quotient of the start vector.
struct EpiDacgStart {
  using acc = double;
  static constexpr int NV = 2;
  static constexpr bool reduce = true;
  double* ax;
  const double* isd;
  const double* x;
  EigState* E;
  DevState* st;
  const DevState* guard;
  __device__ __forceinline__ void bind(int) {}
  __device__ __forceinline__ void prepare() {}
  struct Pre {
    double isd, x;
  };
  __device__ __forceinline__ Pre load(int64_t i) const { return Pre{isd[i], x[i]}; }
  __device__ __forceinline__ void operator()(int64_t i, double, double m, const Pre& p, double (&part)[NV]) const {
    const double v = m * p.isd;
    ax[i] = v;
    part[0] += p.x * p.x;
    part[1] += p.x * v;
  }
  __device__ void fin(double (&t)[NV]) const {
    E->xx = t[0];
    E->xax = t[1];
    E->mu = t[1] / t[0];
  }
};

// A p with (p, A p), (x, A p), (p, p), (x, p); the last block then solves the
// 2 x 2 Rayleigh-Ritz problem on span{x, p}:
//   G = [[(x,Ax), (x,Ap)], [(x,Ap), (p,Ap)]],  H = [[(x,x), (x,p)], [(x,p), (p,p)]],
// smaller root mu of det(G - mu H) = 0 and its eigenvector u, scaled to
// u^T H u = 1 (unit norm of the new x) with u1 >= 0.
struct EpiDacgProduct {
  using acc = double;
  static constexpr int NV = 4;
  static constexpr bool reduce = true;
  double* ap;
  const double* isd;
  const double* p;
  const double* x;
  EigState* E;
  DevState* st;
  const DevState* guard;
  __device__ __forceinline__ void bind(int) {}
  __device__ __forceinline__ void prepare() {}
  struct Pre {
    double isd, p, x;
  };
  __device__ __forceinline__ Pre load(int64_t i) const { return Pre{isd[i], p[i], x[i]}; }
  __device__ __forceinline__ void operator()(int64_t i, double, double m, const Pre& q, double (&part)[NV]) const {
    const double v = m * q.isd;
    ap[i] = v;
    part[0] += q.p * v;
    part[1] += q.x * v;
    part[2] += q.p * q.p;
    part[3] += q.x * q.p;
  }
  __device__ void fin(double (&t)[NV]) const {
    const double a = E->xax, b = t[1], c = t[0], d = E->xx, e = t[3], f = t[2];
    const double a2 = d * f - e * e;           // > 0 unless p is parallel to x
    const double a1 = a * f + c * d - 2.0 * b * e;  // minus the linear coefficient
    const double a0 = a * c - b * b;
    if (!(a2 > 0.0) || !isfinite(a1) || !isfinite(a0)) {
      E->st.done = kBreakdown;
      return;
    }
    const double sq = sqrt(fmax(a1 * a1 - 4.0 * a2 * a0, 0.0));
    const double mu = a1 > 0.0 ? 2.0 * a0 / (a1 + sq) : (a1 - sq) / (2.0 * a2);
    // null vector of G - mu H from its row of larger norm
    const double r11 = a - mu * d, r12 = b - mu * e, r22 = c - mu * f;
    double u1, u2;
    if (r11 * r11 + r12 * r12 >= r12 * r12 + r22 * r22) {
      u1 = -r12;
      u2 = r11;
    } else {
      u1 = r22;
      u2 = -r12;
    }
    const double nrm = sqrt(d * u1 * u1 + 2.0 * e * u1 * u2 + f * u2 * u2);
    if (!(nrm > 0.0) || !isfinite(nrm)) {
      E->st.done = kBreakdown;
      return;
    }
    const double sgn = u1 < 0.0 ? -1.0 : 1.0;
    E->u1 = sgn * u1 / nrm;
    E->u2 = sgn * u2 / nrm;
    E->mu = mu;
  }
};

__device__ __forceinline__ bool eig_done(const EigState* E) { return E->st.done != kRunning; }

// partial (v, v) for a norm
__global__ __launch_bounds__(kBlock) void k_eg_norm2(const double* __restrict__ v, int64_t n, ReduceBuf rb) {
  double part[1] = {0.0};
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    part[0] += v[i] * v[i];
  block_partial<1>(part, rb, 0);
}

struct FinInvNorm {
  EigState* E;
  __device__ void bind(int) {}
  __device__ void operator()(double (&t)[1]) const { E->inv = 1.0 / sqrt(t[0]); }
};

// dst = src * E->inv
__global__ void k_eg_scale(const double* __restrict__ src, double* __restrict__ dst, const EigState* E, int64_t n) {
  const double s = E->inv;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    dst[i] = src[i] * s;
}

// g = A x - mu x with (g, g); p = 0 (the first direction is -g).
__global__ __launch_bounds__(kBlock) void k_eg_start(const double* __restrict__ x, const double* __restrict__ ax,
                                                     double* __restrict__ g, double* __restrict__ p,
                                                     const EigState* E, int64_t n, ReduceBuf rb) {
  const double mu = E->mu;
  double part[1] = {0.0};
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const double gi = ax[i] - mu * x[i];
    g[i] = gi;
    p[i] = 0.0;
    part[0] += gi * gi;
  }
  block_partial<1>(part, rb, 0);
}

struct FinDacgStart {
  EigState* E;
  __device__ void bind(int) {}
  __device__ void operator()(double (&t)[1]) const {
    E->gg = t[0];
    E->beta = 0.0;
    E->relres = sqrt(t[0]) / (E->mu * sqrt(E->xx));
    E->st.iter = 0;
    if (!isfinite(E->relres) || !(E->mu > 0.0))
      E->st.done = kBreakdown;
    else if (E->relres <= E->st.tol)
      E->st.done = kConverged;
    else if (E->st.maxit <= 0)
      E->st.done = kMaxIter;
  }
};

// p = -g + beta p
__global__ void k_eg_direction(const double* __restrict__ g, double* __restrict__ p, const EigState* E, int64_t n) {
  if (eig_done(E)) return;
  const double beta = E->beta;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = -g[i] + beta * p[i];
}

// x <- u1 x + u2 p, A x <- u1 A x + u2 A p, g = A x - mu x with (g, g), (x, x), (x, A x).
__global__ __launch_bounds__(kBlock) void k_eg_update(double* __restrict__ x, double* __restrict__ ax,
                                                      const double* __restrict__ p, const double* __restrict__ ap,
                                                      double* __restrict__ g, const EigState* E, int64_t n,
                                                      ReduceBuf rb) {
  if (eig_done(E)) return;
  const double u1 = E->u1, u2 = E->u2, mu = E->mu;
  double part[3] = {0.0, 0.0, 0.0};
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const double xi = u1 * x[i] + u2 * p[i];
    const double axi = u1 * ax[i] + u2 * ap[i];
    const double gi = axi - mu * xi;
    x[i] = xi;
    ax[i] = axi;
    g[i] = gi;
    part[0] += gi * gi;
    part[1] += xi * xi;
    part[2] += xi * axi;
  }
  block_partial<3>(part, rb, 0);
}

// Stop test after a DACG step, and beta of the next direction (Fletcher-Reeves form).
struct FinDacgUpdate {
  EigState* E;
  __device__ void bind(int) {}
  __device__ void operator()(double (&t)[3]) const {
    E->gg_old = E->gg;
    E->gg = t[0];
    E->xx = t[1];
    E->xax = t[2];
    E->beta = t[0] / E->gg_old;
    E->relres = sqrt(t[0]) / (E->mu * sqrt(t[1]));
    E->st.iter += 1;
    if (!isfinite(E->relres))
      E->st.done = kBreakdown;
    else if (E->relres <= E->st.tol)
      E->st.done = kConverged;
    else if (E->st.iter >= E->st.maxit)
      E->st.done = kMaxIter;
  }
};

__global__ void k_eg_init(EigState* E, double tol, int maxit) {
  EigState e{};
  e.st.tol = tol;
  e.st.maxit = maxit;
  e.st.done = kRunning;
  *E = e;
}

struct EigWork {
  double *isd, *x, *ax, *p, *ap, *g;
  EigState* E;
};

// x = v / ||v|| (a zero or non-finite v is an error).
static void normalise_start(Handle& h, const EigWork& w, const double* v, hipStream_t s) {
  const int64_t n = h.n;
  k_eg_norm2<<<kLzGrid, kBlock, 0, s>>>(v, n, h.rb());
  launch<KFinalize<1, FinInvNorm>>(1, kFinThreads, 0, s, FinInvNorm{w.E}, h.rb(), kLzGrid, nullptr, 0);
  double inv = 0.0;
  PCHEB_HIP_CHECK(hipMemcpyAsync(&inv, &w.E->inv, sizeof(double), hipMemcpyDeviceToHost, s));
  PCHEB_HIP_CHECK(hipStreamSynchronize(s));
  if (!(inv > 0.0) || !std::isfinite(inv)) fail(PCHEB_INVALID, "start vector must be nonzero and finite");
  k_eg_scale<<<kLzGrid, kBlock, 0, s>>>(v, w.x, w.E, n);
}

// lambda_max: `iters` power steps v <- A v / ||A v||; the estimate is the
// Rayleigh quotient of the last iterate (v_{iters-1}).
static double power_method(Handle& h, const EigWork& w, const double* v0, int iters, hipStream_t s) {
  const int64_t n = h.n;
  normalise_start(h, w, v0, s);
  for (int i = 0; i < iters; ++i) {
    launch_ahat(h, InScaled{w.x, w.isd, n}, EpiPowerStep{w.ap, w.isd, w.x, w.E, nullptr, nullptr}, 0, 1, s);
    k_eg_scale<<<kLzGrid, kBlock, 0, s>>>(w.ap, w.x, w.E, n);
    PCHEB_HIP_CHECK(hipGetLastError());
  }
  double lmax = 0.0;
  PCHEB_HIP_CHECK(hipMemcpyAsync(&lmax, &w.E->lmax, sizeof(double), hipMemcpyDeviceToHost, s));
  PCHEB_HIP_CHECK(hipStreamSynchronize(s));
  return lmax;
}

// lambda_min by DACG without preconditioning (Bergamaschi, Gambolati and Pini
// 1997), the paper's estimator of the smallest eigenvalue: conjugate-gradient
// minimisation of the Rayleigh quotient q(x) = (x, Ax) / (x, x).  With
// g = A x - q x (its gradient up to a factor), the directions are
// p_0 = -g_0, p_k = -g_k + beta_k p_{k-1}, beta_k = (g_k, g_k) / (g_{k-1}, g_{k-1}),
// and the exact line search along p is the Rayleigh-Ritz problem on
// span{x, p} (EpiDacgProduct).  A x is carried by the recurrence
// A x <- u1 A x + u2 A p, so a step costs one product.  The step count is
// exact: kernels of steps past the stop test exit at once, and the host
// enqueues steps in groups between reads of the state.
static void dacg(Handle& h, const EigWork& w, const double* v0, double tol, int maxit, double* mu, int* steps,
                 double* relres, hipStream_t s) {
  const int64_t n = h.n;
  k_eg_init<<<1, 1, 0, s>>>(w.E, tol, maxit);
  normalise_start(h, w, v0, s);
  launch_ahat(h, InScaled{w.x, w.isd, n}, EpiDacgStart{w.ax, w.isd, w.x, w.E, nullptr, nullptr}, 0, 1, s);
  k_eg_start<<<kLzGrid, kBlock, 0, s>>>(w.x, w.ax, w.g, w.p, w.E, n, h.rb());
  launch<KFinalize<1, FinDacgStart>>(1, kFinThreads, 0, s, FinDacgStart{w.E}, h.rb(), kLzGrid, nullptr, 0);
  const DevState* guard = &w.E->st;
  EigState e{};
  constexpr int kGroup = 16;  // steps enqueued between reads of the state
  for (;;) {
    PCHEB_HIP_CHECK(hipMemcpyAsync(&e, w.E, sizeof(EigState), hipMemcpyDeviceToHost, s));
    PCHEB_HIP_CHECK(hipStreamSynchronize(s));
    if (e.st.done != kRunning) break;
    for (int j = 0; j < kGroup; ++j) {
      k_eg_direction<<<kLzGrid, kBlock, 0, s>>>(w.g, w.p, w.E, n);
      launch_ahat(h, InScaled{w.p, w.isd, n}, EpiDacgProduct{w.ap, w.isd, w.p, w.x, w.E, nullptr, guard}, 0, 1, s);
      k_eg_update<<<kLzGrid, kBlock, 0, s>>>(w.x, w.ax, w.p, w.ap, w.g, w.E, n, h.rb());
      launch<KFinalize<3, FinDacgUpdate>>(1, kFinThreads, 0, s, FinDacgUpdate{w.E}, h.rb(), kLzGrid, guard, 0);
    }
    PCHEB_HIP_CHECK(hipGetLastError());
  }
  if (e.st.done == kBreakdown) fail(PCHEB_BREAKDOWN, "DACG broke down (non-finite values or p parallel to x)");
  *mu = e.mu;
  *steps = e.st.iter;
  *relres = e.relres;
}

static void pdacg(Handle& h, const double* v0, int power_iters, double tol, int maxit, double* lmin, double* lmax,
                  int* steps, double* relres, hipStream_t s) {
  const int64_t n = h.n;
  EigWork w{};
  w.isd = static_cast<double*>(dev_alloc(h, size_t(n) * sizeof(double)));
  w.x = static_cast<double*>(dev_alloc(h, size_t(n) * sizeof(double)));
  w.ax = static_cast<double*>(dev_alloc(h, size_t(n) * sizeof(double)));
  w.p = static_cast<double*>(dev_alloc(h, size_t(n) * sizeof(double)));
  w.ap = static_cast<double*>(dev_alloc(h, size_t(n) * sizeof(double)));
  w.g = static_cast<double*>(dev_alloc(h, size_t(n) * sizeof(double)));
  w.E = static_cast<EigState*>(dev_alloc(h, sizeof(EigState)));
  h.partials = static_cast<double*>(dev_alloc(h, size_t(kMaxGrid) * kMaxReduce * sizeof(double)));
  k_isqrt_diag<<<kLzGrid, kBlock, 0, s>>>(h.invd, 1.0 / 6.0, w.isd, n);
  k_eg_init<<<1, 1, 0, s>>>(w.E, tol, maxit);
  *lmax = power_method(h, w, v0, power_iters, s);
  dacg(h, w, v0, tol, maxit, lmin, steps, relres, s);
}

}  // namespace pcheb

using namespace pcheb;

namespace {

// Arguments every estimator checks; the handle holds the operator for the products.
void estimator_setup(Handle& h, const pcheb_operator* A, const double* v0, hipStream_t stream, int block_size = 1) {
  if (block_size != 1 && block_size != 3) fail(PCHEB_INVALID, "block_size must be 1 or 3");
  if (!A || !v0) fail(PCHEB_INVALID, "null argument");
  if (block_size == 3 && A->kind != PCHEB_OP_CSR && A->kind != PCHEB_OP_SELL)
    fail(PCHEB_INVALID, "block_size 3 needs a CSR or SELL operator");
  if (block_size == 3 && A->n % 3 != 0) fail(PCHEB_INVALID, "block_size 3 needs n to be a multiple of 3");
  if (A->n <= 0) fail(PCHEB_INVALID, "n must be positive");
  if ((A->kind == PCHEB_OP_CSR || A->kind == PCHEB_OP_SELL) && (!A->rowptr || !A->colind || !A->values))
    fail(PCHEB_INVALID, "CSR arrays must be non-null");
  if ((A->kind == PCHEB_OP_STENCIL7 || A->kind == PCHEB_OP_STENCIL27H) && int64_t(A->nx) * A->ny * A->nz != A->n)
    fail(PCHEB_INVALID, "n must equal nx*ny*nz");
  if (A->kind == PCHEB_OP_STENCIL27H && !A->cell_coeff) fail(PCHEB_INVALID, "cell_coeff must be non-null");
  if (A->kind < PCHEB_OP_CSR || A->kind > PCHEB_OP_STENCIL27H) fail(PCHEB_INVALID, "unknown operator kind");
  h.op = *A;
  h.op.kind = (A->kind == PCHEB_OP_SELL) ? PCHEB_OP_CSR : A->kind;  // the product itself is all that is needed
  h.prm.prec = PCHEB_F64;
  h.prm.block_size = block_size;
  h.n = A->n;
  setup_operator(h, stream);
}

template <class F>
pcheb_status run_estimator(const pcheb_operator* A, const double* v0, hipStream_t stream, F&& body,
                           int block_size = 1, char* arena = nullptr, size_t arena_cap = 0) {
  try {
    set_last_error("");
    Handle h;
    h.arena = arena;
    h.arena_cap = arena_cap;
    try {
      estimator_setup(h, A, v0, stream, block_size);
      body(h);
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

// ------------------------------------------------------------------ allocation-free Lanczos
//
// Workspace of pcheb_estimate_bounds_noalloc: `scratch` (file scope, above);
// host code takes its device address from hipGetSymbolAddress, once per device.
std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;  // device -> address of that device's copy of `scratch`

char* scratch_on_current_device() {
  int dev = 0;
  PCHEB_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) {
    (void)hipGetLastError();
    fail(PCHEB_HIP, std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e));
  }
  g_scratch_ptr[dev] = static_cast<char*>(p);
  return static_cast<char*>(p);
}

// Bytes the estimator's set-up (point scaling, F64) and nsteps Lanczos steps
// take from an arena, in the order they are carved (each piece 256-byte aligned).
size_t lanczos_arena_bytes(const pcheb_operator& A, int nsteps) {
  const int64_t n = A.n;
  const int64_t m = std::min<int64_t>(nsteps, n);
  const int64_t ldv = (n + 1) / 2 * 2;
  size_t total = 0;
  auto piece = [&](size_t b) { total = (total + 255) / 256 * 256 + b; };
  piece(sizeof(int));  // NOT_SPD flag
  if (A.kind == PCHEB_OP_CSR || A.kind == PCHEB_OP_SELL) piece(size_t(n) * 8);  // D^-1
  if (A.kind == PCHEB_OP_STENCIL27H) {
    piece(size_t(n) * 8);  // D^-1
    piece(size_t(n) * 8);  // 1 / (2 kappa)
  }
  piece(size_t(m + 1) * size_t(ldv) * 8);  // basis
  piece(size_t(n) * 8);                    // w
  piece(size_t(n) * 8);                    // D^-1/2
  piece(size_t(kCols) * kLzGrid * 8);      // partial sums
  piece(size_t(3 * m + 3) * 8);            // coefficients, alpha, beta, 1/beta, ||v0||
  return total;
}

}  // namespace

extern "C" pcheb_status pcheb_estimate_bounds_noalloc(const pcheb_operator* A, const double* v0, int32_t nsteps,
                                                      double* lambda_min, double* lambda_max, hipStream_t stream) {
  if (!lambda_min || !lambda_max || !A) {
    set_last_error("null argument");
    return PCHEB_INVALID;
  }
  if (v0 && reinterpret_cast<uintptr_t>(v0) % 16 != 0) {
    set_last_error("v0 must be 16-byte aligned");
    return PCHEB_INVALID;
  }
  if (nsteps < 1 || nsteps > 1000) {
    set_last_error("nsteps must be in [1, 1000]");
    return PCHEB_INVALID;
  }
  if (A->n <= 0) {
    set_last_error("n must be positive");
    return PCHEB_INVALID;
  }
  const size_t need = lanczos_arena_bytes(*A, nsteps);
  if (need > kNoAllocScratchBytes) {
    set_last_error("needs " + std::to_string(need) + " bytes of workspace; the allocation-free estimator has " +
                   std::to_string(kNoAllocScratchBytes));
    return PCHEB_INVALID;
  }
  char* base = nullptr;
  try {
    base = scratch_on_current_device();
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.status;
  }
  return run_estimator(
      A, v0, stream, [&](Handle& h) { lanczos(h, v0, nsteps, lambda_min, lambda_max, stream); }, 1, base,
      kNoAllocScratchBytes);
}

extern "C" pcheb_status pcheb_estimate_bounds(const pcheb_operator* A, const double* v0, int32_t nsteps,
                                              double* lambda_min, double* lambda_max, hipStream_t stream) {
  if (!lambda_min || !lambda_max) {
    set_last_error("null argument");
    return PCHEB_INVALID;
  }
  if (v0 && reinterpret_cast<uintptr_t>(v0) % 16 != 0) {
    set_last_error("v0 must be 16-byte aligned");
    return PCHEB_INVALID;
  }
  if (nsteps < 1 || nsteps > 1000) {
    set_last_error("nsteps must be in [1, 1000]");
    return PCHEB_INVALID;
  }
  return run_estimator(A, v0, stream, [&](Handle& h) { lanczos(h, v0, nsteps, lambda_min, lambda_max, stream); });
}

extern "C" pcheb_status pcheb_estimate_bounds_block(const pcheb_operator* A, int32_t block_size, const double* v0,
                                                    int32_t nsteps, double* lambda_min, double* lambda_max,
                                                    hipStream_t stream) {
  if (!lambda_min || !lambda_max) {
    set_last_error("null argument");
    return PCHEB_INVALID;
  }
  if (v0 && reinterpret_cast<uintptr_t>(v0) % 16 != 0) {
    set_last_error("v0 must be 16-byte aligned");
    return PCHEB_INVALID;
  }
  if (nsteps < 1 || nsteps > 1000) {
    set_last_error("nsteps must be in [1, 1000]");
    return PCHEB_INVALID;
  }
  return run_estimator(
      A, v0, stream, [&](Handle& h) { lanczos(h, v0, nsteps, lambda_min, lambda_max, stream); }, block_size);
}

extern "C" pcheb_status pcheb_estimate_bounds_pdacg(const pcheb_operator* A, const double* v0, int32_t power_iters,
                                                    double dacg_tol, int32_t dacg_maxit, double* lambda_min,
                                                    double* lambda_max, int32_t* dacg_steps, double* dacg_relres,
                                                    hipStream_t stream) {
  if (!lambda_min || !lambda_max) {
    set_last_error("null argument");
    return PCHEB_INVALID;
  }
  if (power_iters < 1 || power_iters > 100000) {
    set_last_error("power_iters must be in [1, 100000]");
    return PCHEB_INVALID;
  }
  if (!(dacg_tol >= 0.0) || !std::isfinite(dacg_tol)) {
    set_last_error("dacg_tol must be finite and >= 0");
    return PCHEB_INVALID;
  }
  if (dacg_maxit < 0 || dacg_maxit > 10000000) {
    set_last_error("dacg_maxit must be in [0, 1e7]");
    return PCHEB_INVALID;
  }
  return run_estimator(A, v0, stream, [&](Handle& h) {
    int steps = 0;
    double relres = 0.0;
    pdacg(h, v0, power_iters, dacg_tol, dacg_maxit, lambda_min, lambda_max, &steps, &relres, stream);
    if (dacg_steps) *dacg_steps = steps;
    if (dacg_relres) *dacg_relres = relres;
  });
}

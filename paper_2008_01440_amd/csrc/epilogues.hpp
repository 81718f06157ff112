// Per-row arithmetic run by the operator kernels (see operators.hpp).
//
// The preconditioner recurrence runs on B = D^-1 A_hat with input
// s = D^-1 r, which is the similarity transform of Alg. 2 on the scaled
// matrix A = D^-1/2 A_hat D^-1/2:  D^-1/2 p_k(A) D^-1/2 = p_k(B) D^-1.
// With y_0 = s / theta', step j (1 <= j <= k) of the recurrence is
//     y_j = rho_j (2 sigma y_{j-1} - rho_{j-1} y_{j-2} + (2/delta)(s - B y_{j-1}))
//         = a_j y_{j-1} - b_j y_{j-2} + c_j (s - B y_{j-1}),
// with a_j = 2 sigma rho_j, b_j = rho_j rho_{j-1} (and y_{-1} = 0, so step 1
// drops that term), c_j = 2 rho_j / delta.  Step 1 then equals
// (2 rho_1/delta)(2 s - B s/theta'), the first line of Alg. 2.  y_0 itself is
// never stored: steps 1 and 2 read s with 1/theta' folded into their
// coefficients.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace pcheb {

// Values an epilogue reads at its own point are loaded apart from its
// arithmetic: pre = epi.load(i) may be issued ahead (a plane early in the
// 7-point kernel) and is passed to epi(i, y, m, pre, part).  Epilogues that
// read nothing use NoPre.
struct NoPre {};

// D^-1 of the unscaled operator: a stored array or a constant (7-point stencil).
struct InvDiag {
  const double* p;
  double c;
  __device__ __forceinline__ double operator()(int64_t i) const { return p ? p[i] : c; }
};

// Middle (and first) steps: y_j in the storage precision T.
template <class T, bool FIRST>
struct EpiChebStep {
  using acc = typename Store<T>::acc;
  static constexpr int NV = 1;
  static constexpr bool reduce = false;
  const T* yprev;  // y_{j-2}; unused when FIRST
  const T* s;      // D^-1 r in storage precision
  T* out;          // y_j
  acc a, b, c;
  DevState* st;
  const DevState* guard;
  int64_t ld;
  __device__ __forceinline__ void bind(int slot) {
    const int64_t o = slot * ld;
    if (!FIRST) yprev += o;
    s += o;
    out += o;
    if (guard) guard += slot;
  }
  __device__ __forceinline__ void prepare() {}
  struct Pre {
    acc s, yprev;
  };
  __device__ __forceinline__ Pre load(int64_t i) const {
    return Pre{Store<T>::ld(s, i), FIRST ? acc(0) : Store<T>::ld(yprev, i)};
  }
  __device__ __forceinline__ void operator()(int64_t i, acc y, acc by, const Pre& p, double (&)[NV]) const {
    acc v = a * y + c * (p.s - by);
    if (!FIRST) v -= b * p.yprev;
    Store<T>::st(out, i, v);
  }
  __device__ void fin(double (&)[NV]) const {}
};

// Type of z written by the last step: inside a solve (DOTS) a float32 or
// bfloat16 recurrence stores z in float32, which holds its float32 arithmetic
// exactly and halves the traffic of z; otherwise float64.
template <class T, bool DOTS>
using ChebZ = std::conditional_t<DOTS && !std::is_same<T, double>::value, float, double>;

// Last step: z = y_k (float64, or float32 as ChebZ says) and, inside a solve,
// the partial sums of (r, z) and (z, q).  The last block then forms, on the device,
//   gamma_new = (r, z);
//   beta = gamma_new / gamma                     (Fletcher-Reeves), or
//   beta = (z, r - r_old) / gamma = -(z, q)/(p, q) (Polak-Ribiere; r - r_old = -alpha q
//          and gamma = alpha (p, q)),
// and flags a breakdown if gamma_new <= 0 (indefinite preconditioner).
// `init` marks the application before the first iteration: gamma only.
template <class T, bool FIRST, bool DOTS>
struct EpiChebLast {
  using acc = typename Store<T>::acc;
  static constexpr int NV = 2;
  static constexpr bool reduce = DOTS;
  using Tz = ChebZ<T, DOTS>;
  const T* yprev;
  const T* s;
  Tz* z;
  const double* r;  // float64 residual (for the dot products)
  const double* q;  // A p of this iteration (flexible beta only)
  acc a, b, c;
  DevState* st;
  const DevState* guard;
  int init;
  int flexible;
  int64_t ld;
  __device__ __forceinline__ void bind(int slot) {
    const int64_t o = slot * ld;
    if (!FIRST) yprev += o;
    s += o;
    z += o;
    r += o;
    if (q) q += o;
    if (st) st += slot;
    if (guard) guard += slot;
  }
  __device__ __forceinline__ void prepare() {}
  struct Pre {
    acc s, yprev;
    double r, q;
  };
  __device__ __forceinline__ Pre load(int64_t i) const {
    Pre p{Store<T>::ld(s, i), FIRST ? acc(0) : Store<T>::ld(yprev, i), 0.0, 0.0};
    if (DOTS) {
      p.r = r[i];
      if (flexible) p.q = q[i];
    }
    return p;
  }
  __device__ __forceinline__ void operator()(int64_t i, acc y, acc by, const Pre& p, double (&part)[NV]) const {
    acc v = a * y + c * (p.s - by);
    if (!FIRST) v -= b * p.yprev;
    const double zi = double(v);
    if constexpr (std::is_same<Tz, double>::value)
      out_store(z + i, zi);
    else
      z[i] = float(v);
    if (DOTS) {
      part[0] += p.r * zi;
      if (flexible) part[1] += zi * p.q;
    }
  }
  __device__ void fin(double (&t)[NV]) const { finish_beta(st, t[0], t[1], init, flexible); }

  static __device__ void finish_beta(DevState* st, double rz, double zq, int init, int flexible) {
    if (!(rz > 0.0) || !isfinite(rz)) {
      st->done = kBreakdown;
      return;
    }
    if (init) {
      st->beta = 0.0;
    } else if (flexible) {
      st->beta = -zq / st->pq;
    } else {
      st->beta = rz / st->gamma;
    }
    st->gamma = rz;
  }
};

// q = A p for the search direction p: stores q (and p when p_new is set, the
// input functor having formed p = z + beta p_old) and reduces (p, q).  The last
// block sets alpha = gamma / (p, q) or flags a breakdown when (p, q) <= 0.
struct EpiDirection {
  using acc = double;
  static constexpr int NV = 1;
  static constexpr bool reduce = true;
  double* p_new;  // may be null
  double* q;
  DevState* st;
  const DevState* guard;
  int64_t ld;
  __device__ __forceinline__ void bind(int slot) {
    if (p_new) p_new += slot * ld;
    q += slot * ld;
    st += slot;
    if (guard) guard += slot;
  }
  __device__ __forceinline__ void prepare() {}
  using Pre = NoPre;
  __device__ __forceinline__ Pre load(int64_t) const { return {}; }
  __device__ __forceinline__ void operator()(int64_t i, double p, double ap, const Pre&, double (&part)[NV]) const {
    if (p_new) out_store(p_new + i, p);
    out_store(q + i, ap);
    part[0] += p * ap;
  }
  __device__ void fin(double (&t)[NV]) const {
    st->pq = t[0];
    if (!(t[0] > 0.0) || !isfinite(t[0])) {
      st->done = kBreakdown;
      return;
    }
    st->alpha = st->gamma / t[0];
  }
};

// y = M x.
template <class T>
struct EpiStore {
  using acc = typename Store<T>::acc;
  static constexpr int NV = 1;
  static constexpr bool reduce = false;
  T* y;
  DevState* st;
  const DevState* guard;
  int64_t ld;
  __device__ __forceinline__ void bind(int slot) { y += slot * ld; }
  __device__ __forceinline__ void prepare() {}
  using Pre = NoPre;
  __device__ __forceinline__ Pre load(int64_t) const { return {}; }
  __device__ __forceinline__ void operator()(int64_t i, acc, acc m, const Pre&, double (&)[NV]) const {
    Store<T>::st(y, i, m);
  }
  __device__ void fin(double (&)[NV]) const {}
};

// w = D^-1/2 A_hat D^-1/2 v (input functor InScaled supplies D^-1/2 v).
struct EpiScaledStore {
  using acc = double;
  static constexpr int NV = 1;
  static constexpr bool reduce = false;
  double* w;
  const double* isd;
  DevState* st;
  const DevState* guard;
  int64_t ld;
  __device__ __forceinline__ void bind(int slot) { w += slot * ld; }
  __device__ __forceinline__ void prepare() {}
  struct Pre {
    double isd;
  };
  __device__ __forceinline__ Pre load(int64_t i) const { return Pre{isd[i]}; }
  __device__ __forceinline__ void operator()(int64_t i, double, double m, const Pre& p, double (&)[NV]) const {
    w[i] = m * p.isd;
  }
  __device__ void fin(double (&)[NV]) const {}
};

// r = b - A x with ||r||^2 (D^-1 weighted), ||r||^2 and ||b||^2 (unweighted).
// mode 0: initial residual (sets rr, bb, bb_hat and the first relres);
// mode 1: exit check (true_rr, true_rr_hat); mode 2: periodic replacement
// of the recursive residual (rr, relres).
struct EpiResidual {
  using acc = double;
  static constexpr int NV = 4;
  static constexpr bool reduce = true;
  const double* b;
  double* r;  // may be null: norms only
  InvDiag invd;
  DevState* st;
  const DevState* guard;
  int mode;
  int64_t ldb;  // stride of the caller's right-hand sides
  int64_t ldr;  // stride of the workspace residuals
  __device__ __forceinline__ void bind(int slot) {
    b += slot * ldb;
    if (r) r += slot * ldr;
    st += slot;
    if (guard) guard += slot;
  }
  __device__ __forceinline__ void prepare() {}
  struct Pre {
    double b, w;
  };
  __device__ __forceinline__ Pre load(int64_t i) const { return Pre{b[i], invd(i)}; }
  __device__ __forceinline__ void operator()(int64_t i, double, double ax, const Pre& p, double (&part)[NV]) const {
    const double bi = p.b;
    const double ri = bi - ax;
    if (r) r[i] = ri;
    const double w = p.w;
    part[0] += ri * ri * w;
    part[1] += ri * ri;
    part[2] += bi * bi * w;
    part[3] += bi * bi;
  }
  __device__ void fin(double (&t)[NV]) const {
    if (mode == 0) {
      st->rr = t[0];
      st->bb = t[2];
      st->bb_hat = t[3];
      st->relres = t[2] > 0.0 ? sqrt(t[0]) / sqrt(t[2]) : 0.0;
      if (!isfinite(t[0]) || !isfinite(t[2]))
        st->done = kBreakdown;
      else if (st->relres < st->tol)
        st->done = kConverged;  // r_0 already meets the tolerance (or b = 0)
    } else if (mode == 1) {
      st->true_rr = t[0];
      st->true_rr_hat = t[1];
      st->bb_hat = t[3];
    } else {
      st->rr = t[0];
      st->relres = st->bb > 0.0 ? sqrt(t[0]) / sqrt(st->bb) : 0.0;
      st->refreshes += 1;
    }
  }
};

}  // namespace pcheb

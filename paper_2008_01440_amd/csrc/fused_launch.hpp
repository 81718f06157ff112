// Launch of the fused 7-point passes (fused_stencil.hpp): tile shape, z
// ranges and the recurrence coefficients of the steps a pass covers.
#pragma once

#include <algorithm>

#include "fused_stencil.hpp"
#include "handle.hpp"

namespace pcheb {

template <class T>
struct Coef {
  using acc = typename Store<T>::acc;
  acc a, b, c;
};

// Coefficients of step j: y_j = a y_{j-1} - b y_{j-2} + c (s - B y_{j-1}).
// y_0 = s / theta' is never stored, and 1/theta' is folded in where it would be
// read: step 1 takes s as its input vector, so a_1 y_0 + c_1 (s - B y_0) becomes
// (a_1/theta' + c_1 - c_1/theta') s + (c_1/theta') (s - B s); step 2 takes s for
// y_{j-2}, so its b is b_2 / theta'.
template <class T>
static Coef<T> step_coef(const Handle& h, int j) {
  using acc = typename Store<T>::acc;
  const double inv_theta = 1.0 / h.theta;
  double a = 2.0 * h.sigma * h.rho[j];
  double b = j >= 1 ? h.rho[j] * h.rho[j - 1] : 0.0;
  double c = 2.0 * h.rho[j] / h.delta;
  if (j == 1) {
    a = a * inv_theta + c - c * inv_theta;
    c *= inv_theta;
  } else if (j == 2) {
    b *= inv_theta;
  }
  Coef<T> cf;
  cf.a = acc(a);
  cf.b = acc(b);
  cf.c = acc(c);
  return cf;
}

// ---- fused passes (7-point stencil): S middle steps per launch

// Tile shapes of the fused pass: 64 x TY points per block of NT threads.
#ifndef PCHEB_FUSED_TY
#define PCHEB_FUSED_TY 32
#endif
#ifndef PCHEB_FUSED_NT
#define PCHEB_FUSED_NT 1024
#endif


template <class T, int S, int TY, int NT>
static void launch_fused(const Handle& h, Slots sl, const T* ya, const T* yb, T* oa, T* ob, int j,
                         const DevState* guard, hipStream_t s) {
  FusedCoef<typename Store<T>::acc, S> cf;
  for (int m = 0; m < S; ++m) {
    const Coef<T> c = step_coef<T>(h, j + m);
    cf.a[m] = c.a;
    cf.b[m] = c.b;
    cf.c[m] = c.c;
  }
  const pcheb_operator& op = h.op;
  const uint32_t tiles_x = uint32_t((op.nx + 63) / 64), tiles_y = uint32_t((op.ny + TY - 1) / TY);
  const uint32_t xy = tiles_x * tiles_y;
  // about as many tiles as the chip holds blocks at once (256 CUs; per CU at
  // most 2048 threads and 160 KiB of LDS), each z range at least 4 S planes deep
  constexpr int RX = 64 + 2 * S, NP = RX * (TY + 2 * S);
  constexpr int kLds = sizeof(T) < 8 ? (NP + 2 * (RX + 1)) * ((3 * S) % 2 == 0 ? 3 * S + 1 : 3 * S) * 4
                                     : S * 2 * (NP + 2 * (RX + 1)) * 8;
  constexpr int kPerCu = std::max(1, std::min(2048 / NT, 163840 / kLds));
  const uint32_t target = 256u * kPerCu;
  const int max_chunks = std::max(1, op.nz / (4 * S));
  int chunks = std::max(1, std::min<int>(max_chunks, int((target + xy - 1) / xy)));
  {
    // the buffer-addressed passes cover a tile's zc + 2 S + 1 planes with one descriptor
    const int64_t plane_bytes = int64_t(op.nx) * op.ny * int64_t(sizeof(T));
    const int64_t zc_max = kMaxSpanBytes / plane_bytes - 2 * S - 1;
    if (zc_max >= 1) chunks = std::max<int>(chunks, int((op.nz + zc_max - 1) / zc_max));
  }
  const int zc = (op.nz + chunks - 1) / chunks;
  const uint32_t ntiles = xy * uint32_t((op.nz + zc - 1) / zc);
  const dim3 grid(round_grid(ntiles), sl.count);
  const T* sv = reinterpret_cast<const T*>(h.s);
  // a tile's planes fit one descriptor's range (effective_fuse admits only planes for which zc >= 1 does)
  if ((int64_t(zc) + 2 * S + 1) * int64_t(op.nx) * op.ny * int64_t(sizeof(T)) > kMaxSpanBytes)
    fail(PCHEB_INVALID, "fused pass: x-y plane too large for one buffer descriptor");
  if constexpr (sizeof(T) < 8)
    launch<KFusedPass<S, TY, NT, T>>(grid, NT, 0, s, ya, yb, sv, oa, ob, cf, op.nx, op.ny, op.nz, zc, tiles_x, tiles_y,
        ntiles, guard, h.ldw, sl.first);
  else
    launch<KFusedPass64<S, TY, NT>>(grid, NT, 0, s, ya, yb, sv, oa, ob, cf, op.nx, op.ny, op.nz, zc, tiles_x, tiles_y,
        ntiles, guard, h.ldw, sl.first);
}

template <class T>
static void launch_fused_any(const Handle& h, Slots sl, int S, const T* ya, const T* yb, T* oa, T* ob, int j,
                             const DevState* guard, hipStream_t s) {
  constexpr int TY = PCHEB_FUSED_TY, NT = PCHEB_FUSED_NT;
  if constexpr (sizeof(T) == 8) {
    // float64 rings of three or four levels fit 128 registers only with two points per
    // thread (64 x 16 tiles); two levels take 64 x 32 tiles
    if (S == 2)
      launch_fused<T, 2, TY, NT>(h, sl, ya, yb, oa, ob, j, guard, s);
    else if (S == 3)
      launch_fused<T, 3, 16, NT>(h, sl, ya, yb, oa, ob, j, guard, s);
    else
      launch_fused<T, 4, 16, NT>(h, sl, ya, yb, oa, ob, j, guard, s);
  } else {
    if (S == 2)
      launch_fused<T, 2, TY, NT>(h, sl, ya, yb, oa, ob, j, guard, s);
    else if (S == 3)
      launch_fused<T, 3, TY, NT>(h, sl, ya, yb, oa, ob, j, guard, s);
    else
      launch_fused<T, 4, TY, NT>(h, sl, ya, yb, oa, ob, j, guard, s);
  }
}

// Steps per pass: fusion applies to the 7-point operator with four iterate
// buffers and x-y planes small enough that a tile's descriptor span of at least
// one plane plus 2 S + 1 halo planes stays within kMaxSpanBytes.
static int effective_fuse(const Handle& h) {
  const int64_t plane_bytes = int64_t(h.op.nx) * h.op.ny * int64_t(h.elem);
  const bool ok = h.op.kind == PCHEB_OP_STENCIL7 && h.fuse >= 2 && h.nY >= 4 &&
                  plane_bytes * (2 * std::min(h.fuse, 4) + 2) <= kMaxSpanBytes;
  return ok ? h.fuse : 1;
}

}  // namespace pcheb

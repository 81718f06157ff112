// Operator kernels: one memory-access pattern per operator kind, shared by
// every use of the operator (Chebyshev steps, q = A p, residuals, Lanczos).
//
// Each kernel evaluates m_i = (M y)_i row by row and hands
// (i, y_i, m_i) to an epilogue functor, which does the per-row arithmetic and
// may accumulate up to kMaxReduce partial sums for a grid reduction.  The
// input vector is read through an input functor (a stored vector in some
// precision, or one scaled on the fly).
//
// Every launch covers one or more solve slots (right-hand sides): slot =
// slot0 + blockIdx.y.  bind(slot) points a functor at that slot's vectors
// (offset slot * ld elements) and state; operator data is shared by all slots.
// The tiling of a slot does not depend on how many slots share the launch, so
// results are the same alone and batched.
//
// Interfaces
//   In:  using acc; static constexpr bool narrow (loads need a conversion); int64_t stride;
//        __device__ void bind(int slot); __device__ void prepare();
//        __device__ acc ld(int64_t i) const;
//   Epi: using acc; static constexpr int NV; static constexpr bool reduce;
//        DevState* st (may be null; written by fin); const DevState* guard (may be
//        null; the kernel does nothing once guard->done is set); __device__ void bind(int slot);
//        __device__ void prepare(); struct Pre; __device__ Pre load(int64_t i) const;
//        __device__ void operator()(int64_t i, acc yi, acc mi, const Pre&, double (&part)[NV]) const;
//        __device__ void fin(double (&total)[NV]) const;   // thread 0 of the finalize kernel
//
// M is A_hat (SCALED = false) or D^-1 A_hat (SCALED = true); for CSR and
// SELL it is whatever value array the caller passes.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace pcheb {

template <class Epi>
__device__ __forceinline__ bool solve_finished(const Epi& epi) {
  return epi.guard != nullptr && epi.guard->done != kRunning;
}

template <class Epi, int NT = kBlock>
__device__ __forceinline__ void finish_reduction(const Epi&, double (&part)[Epi::NV], ReduceBuf rb, int slot) {
  if constexpr (Epi::reduce) block_partial<Epi::NV, NT>(part, rb, slot);
}

// Calls epi.fin(total) from the finalize kernel.
template <class Epi>
struct EpiFin {
  Epi epi;
  __device__ __forceinline__ void bind(int slot) { epi.bind(slot); }
  __device__ __forceinline__ void operator()(double (&t)[Epi::NV]) const { epi.fin(t); }
};

// Point the functors at this block's slot; true if the slot's solve has finished.
template <class In, class Epi>
__device__ __forceinline__ bool bind_slot(In& in, Epi& epi, int slot) {
  in.bind(slot);
  epi.bind(slot);
  if (solve_finished(epi)) return true;
  in.prepare();
  epi.prepare();
  return false;
}

// ------------------------------------------------------------------ 7-point stencil
//
// Block = 64 (x) x TY (y) threads, one wave per grid row; a tile is 64 x TY
// columns by ZC planes.  Each thread marches up its column in z keeping the
// planes below, at and above its point in registers.  The tile's current
// plane and its one-point halo are staged in LDS (two buffers, one barrier
// per plane), so the x and y neighbours come from LDS: every input value is
// loaded, and passed through In::ld, once per tile plane plus the halo.  The
// halo rows y0 - 1 and y0 + TY are loaded by the first and last wave, the
// halo columns x0 - 1 and x0 + 64 by the first 2 TY lanes of wave 1.  Values
// outside the grid are zero.  Every thread of a block takes part in every
// barrier; points outside the grid skip only the epilogue.
template <bool SCALED, int TY, int ZC, class In, class Epi>
struct KStencil7 {
  static constexpr int kThreads = 64 * TY;
  __device__ static void run(In in, Epi epi, int nx, int ny, int nz, uint32_t tiles_x, uint32_t tiles_y,
                             uint32_t ntiles, ReduceBuf rb, int slot0);
};
template <bool SCALED, int TY, int ZC, class In, class Epi>
__device__ __forceinline__ void KStencil7<SCALED, TY, ZC, In, Epi>::run(In in, Epi epi, int nx, int ny, int nz,
                                                                        uint32_t tiles_x, uint32_t tiles_y,
                                                                        uint32_t ntiles, ReduceBuf rb, int slot0) {
  static_assert(TY >= 2 && 2 * TY <= 64, "halo loads need two waves and at most 64 halo columns");
  using acc = typename Epi::acc;
  constexpr int W = 64 + 2;  // LDS row: the tile row and its two halo columns
  __shared__ acc buf[2][TY + 2][W];
  const int slot = slot0 + int(blockIdx.y);
  if (bind_slot(in, epi, slot)) return;
  double part[Epi::NV];
#pragma unroll
  for (int v = 0; v < Epi::NV; ++v) part[v] = 0.0;
  const int64_t plane = int64_t(nx) * ny;
  const int tx = int(threadIdx.x), ty = int(threadIdx.y);
  // Loads of zero outside the grid.  Narrow (BF16) inputs are loaded from a
  // valid address (element 0) and zeroed by a select: with a branch around
  // each load, each conversion would wait for its load.
  auto ld0 = [&](bool ok, int64_t j) {
    if constexpr (In::narrow) {
      const acc v = in.ld(ok ? j : 0);
      return ok ? v : acc(0);
    } else {
      return ok ? in.ld(j) : acc(0);
    }
  };
  const bool hy_on = ty == 0 || ty == TY - 1;  // this thread loads a halo row point
  const int hy_row = ty == 0 ? 0 : TY + 1;
  const bool hx_on = ty == 1 && tx < 2 * TY;  // this thread loads a halo column point
  const int hx_r = tx >> 1, hx_col = (tx & 1) ? W - 1 : 0;
  uint32_t k = 0;  // planes staged so far: buffer k & 1
  XcdTiles tiles(ntiles);
  for (uint32_t t = tiles.begin; t < tiles.end; t += tiles.step) {
    const uint32_t tix = t % tiles_x;
    const uint32_t rest = t / tiles_x;
    const int x0 = int(tix) * 64;
    const int y0 = int(rest % tiles_y) * TY;
    const int z0 = int(rest / tiles_y) * ZC;
    const int z1 = z0 + ZC < nz ? z0 + ZC : nz;
    const int x = x0 + tx, y = y0 + ty;
    const bool own = x < nx && y < ny;
    const int64_t i0 = x + int64_t(nx) * y + plane * z0;
    const int hy_y = ty == 0 ? y0 - 1 : y0 + TY;
    const bool hy_ok = hy_on && x < nx && hy_y >= 0 && hy_y < ny;
    const int64_t hy_i = x + int64_t(nx) * hy_y + plane * z0;
    const int hx_x = (tx & 1) ? x0 + 64 : x0 - 1;
    const bool hx_ok = hx_on && hx_x >= 0 && hx_x < nx && y0 + hx_r < ny;
    const int64_t hx_i = hx_x + int64_t(nx) * (y0 + hx_r) + plane * z0;
    acc below = ld0(own && z0 > 0, i0 - plane);
    acc cur = ld0(own, i0);
    acc above = ld0(own && z0 + 1 < nz, i0 + plane);
    acc hy = ld0(hy_ok, hy_i), hx = ld0(hx_ok, hx_i);
    typename Epi::Pre pre{};
    if (own) pre = epi.load(i0);
    for (int z = z0; z < z1; ++z, ++k) {
      const int64_t off = plane * (z - z0);
      // What the next plane needs is loaded one plane ahead: its point above,
      // its halo and its epilogue inputs.
      acc ahead = acc(0), hy_next = acc(0), hx_next = acc(0);
      typename Epi::Pre pre_next{};
      if (z + 1 < z1) {
        ahead = ld0(own && z + 2 < nz, i0 + off + 2 * plane);
        hy_next = ld0(hy_ok, hy_i + off + plane);
        hx_next = ld0(hx_ok, hx_i + off + plane);
        if (own) pre_next = epi.load(i0 + off + plane);
      }
      acc(*b)[W] = buf[k & 1];
      b[ty + 1][tx + 1] = cur;
      if (hy_on) b[hy_row][tx + 1] = hy;
      if (hx_on) b[hx_r + 1][hx_col] = hx;
      __syncthreads();
      if (own) {
        const acc nbs = ((b[ty + 1][tx] + b[ty + 1][tx + 2]) + (b[ty][tx + 1] + b[ty + 2][tx + 1])) + (below + above);
        const acc m = SCALED ? cur - nbs * acc(1.0 / 6.0) : acc(6) * cur - nbs;
        epi(i0 + off, cur, m, pre, part);
      }
      below = cur;
      cur = above;
      above = ahead;
      hy = hy_next;
      hx = hx_next;
      pre = pre_next;
    }
  }
  finish_reduction<Epi, 64 * TY>(epi, part, rb, slot);
}

// ------------------------------------------------------------------ 27-point harmonic stencil
//
// Tiles and planes as in KStencil7: a block of 64 x TY threads owns 64 x TY
// columns, marches ZC planes, and stages each incoming plane of y and of
// rho = 1 / (2 kappa) with its one-point halo (corners included) in LDS, two
// buffers and one barrier per plane.  Each thread copies its 3 x 3
// neighbourhood of the staged plane into a register ring of three planes, so
// a point's 26 neighbours cost 18 LDS reads per plane instead of 18 loads;
// the z loop is unrolled by three, the ring's period, so its slots are fixed
// per phase and the ring is never shifted.
// The face weight 2 k_i k_n / (k_i + k_n) is 1 / (rho_i + rho_n): one add and
// the hardware reciprocal, refined in double by one Newton-Raphson step
// r <- r + r (1 - x r).  The float64 recurrence steps take the 26 neighbours in
// 13 consecutive pairs, y1 / d1 + y2 / d2 = (d2 y1 + d1 y2) / (d1 d2), with one
// reciprocal per pair: the step follows its vector arithmetic, and this halves
// the reciprocals (192^3 step 88.4 -> 81.0 us).  Setup admits coefficients in
// [1e-150, 1e150] only, so d1 d2 stays a normal double.  Cells outside the grid read y = 0 and rho = 1 (any
// positive value: their weight multiplies y = 0); their Dirichlet ghost
// contributions are in the stored D^-1 (invd), so
//   SCALED:  m = y_i - invd_i * sum_n w_in y_n      (D^-1 A_hat y)
//   else:    m = y_i / invd_i - sum_n w_in y_n      (A_hat y, double only).
// The neighbour sum runs over dz, dy, dx in order.
template <bool SCALED, int TY, int ZC, class In, class Epi>
struct KStencil27h {
  static constexpr int kThreads = 64 * TY;
  __device__ static void run(In in, Epi epi, const typename Epi::acc* __restrict__ rho,
                             const typename Epi::acc* __restrict__ invd, int nx, int ny, int nz, uint32_t tiles_x,
                             uint32_t tiles_y, uint32_t ntiles, ReduceBuf rb, int slot0);
};
template <bool SCALED, int TY, int ZC, class In, class Epi>
__device__ __forceinline__ void KStencil27h<SCALED, TY, ZC, In, Epi>::run(In in, Epi epi,
                                                                          const typename Epi::acc* __restrict__ rho,
                                                                          const typename Epi::acc* __restrict__ invd,
                                                                          int nx, int ny, int nz, uint32_t tiles_x,
                                                                          uint32_t tiles_y, uint32_t ntiles,
                                                                          ReduceBuf rb, int slot0) {
  static_assert(TY >= 2 && 2 * (TY + 2) <= 64, "halo loads need two waves and at most 64 side points");
  using acc = typename Epi::acc;
  static_assert(SCALED || sizeof(acc) == 8, "A_hat products run in double");
  constexpr int W = 64 + 2;
  // float64 recurrence steps: the three planes are read from LDS (a ring of
  // four buffers) instead of being copied into a register ring, whose 108
  // float64 registers left two wavefronts per SIMD (step 99 -> 87 us on 192^3).
  // The unscaled product keeps the register ring: its IEEE division holds it
  // at two wavefronts per SIMD either way, and there the LDS reads cost more.
  constexpr bool kLdsRing = sizeof(acc) == 8 && SCALED;
  constexpr int NBUF = kLdsRing ? 4 : 2;
  __shared__ acc ys[NBUF][TY + 2][W];
  __shared__ acc rs[NBUF][TY + 2][W];
  const int slot = slot0 + int(blockIdx.y);
  if (bind_slot(in, epi, slot)) return;
  double part[Epi::NV];
#pragma unroll
  for (int v = 0; v < Epi::NV; ++v) part[v] = 0.0;
  const int64_t plane = int64_t(nx) * ny;
  const int tx = int(threadIdx.x), ty = int(threadIdx.y);
  const acc kOut = acc(1);  // rho of a cell outside the grid (its y is 0)
  auto ldy = [&](bool ok, int64_t j) {
    if constexpr (In::narrow) {  // as in KStencil7: no branch around narrow loads
      const acc v = acc(in.ld(ok ? j : 0));
      return ok ? v : acc(0);
    } else {
      return ok ? acc(in.ld(j)) : acc(0);
    }
  };
  auto ldr = [&](bool ok, int64_t j) { return ok ? rho[j] : kOut; };
  const bool hy_on = ty == 0 || ty == TY - 1;  // a halo row point: row y0 - 1 or y0 + TY
  const int hy_row = ty == 0 ? 0 : TY + 1;
  const bool hx_on = ty == 1 && tx < 2 * (TY + 2);  // a halo side point (corners included)
  const int hx_r = tx >> 1, hx_col = (tx & 1) ? W - 1 : 0;
  uint32_t k = 0;  // planes staged so far: buffer k & 1
  XcdTiles tiles(ntiles);
  for (uint32_t t = tiles.begin; t < tiles.end; t += tiles.step) {
    const uint32_t tix = t % tiles_x;
    const uint32_t rest = t / tiles_x;
    const int x0 = int(tix) * 64;
    const int y0 = int(rest % tiles_y) * TY;
    const int z0 = int(rest / tiles_y) * ZC;
    const int z1 = z0 + ZC < nz ? z0 + ZC : nz;
    const int x = x0 + tx, y = y0 + ty;
    const bool own = x < nx && y < ny;
    const int64_t i0 = x + int64_t(nx) * y;
    const int hy_y = ty == 0 ? y0 - 1 : y0 + TY;
    const bool hy_ok = hy_on && x < nx && hy_y >= 0 && hy_y < ny;
    const int64_t hy_i = x + int64_t(nx) * hy_y;
    const int hx_x = (tx & 1) ? x0 + 64 : x0 - 1, hx_y = y0 - 1 + hx_r;
    const bool hx_ok = hx_on && hx_x >= 0 && hx_x < nx && hx_y >= 0 && hx_y < ny;
    const int64_t hx_i = hx_x + int64_t(nx) * hx_y;
    // y and rho of plane zz at this thread's LDS entries (own, halo row, halo side)
    struct Vals {
      acc y0, r0, y1, r1, y2, r2;
    };
    auto fetch = [&](int zz) {
      const bool zok = zz >= 0 && zz < nz;
      const int64_t pz = plane * zz;
      return Vals{ldy(zok && own, i0 + pz),   ldr(zok && own, i0 + pz),   ldy(zok && hy_ok, hy_i + pz),
                  ldr(zok && hy_ok, hy_i + pz), ldy(zok && hx_ok, hx_i + pz), ldr(zok && hx_ok, hx_i + pz)};
    };
    acc yv[3][3][3], rv[3][3][3];
    auto stage = [&](const Vals& v, int ring) {
      const uint32_t buf = kLdsRing ? (k & 3u) : (k & 1u);
      acc(*yb)[W] = ys[buf];
      acc(*rb2)[W] = rs[buf];
      yb[ty + 1][tx + 1] = v.y0;
      rb2[ty + 1][tx + 1] = v.r0;
      if (hy_on) {
        yb[hy_row][tx + 1] = v.y1;
        rb2[hy_row][tx + 1] = v.r1;
      }
      if (hx_on) {
        yb[hx_r][hx_col] = v.y2;
        rb2[hx_r][hx_col] = v.r2;
      }
      __syncthreads();
      if constexpr (!kLdsRing) {
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) {
            yv[ring][dy][dx] = yb[ty + dy][tx + dx];
            rv[ring][dy][dx] = rb2[ty + dy][tx + dx];
          }
        }
      }
      ++k;
    };
    stage(fetch(z0 - 1), 0);
    stage(fetch(z0), 1);
    Vals nxt = fetch(z0 + 1);
    typename Epi::Pre pre{};
    acc dinv = acc(0);  // D^-1 at the point
    if (own) {
      pre = epi.load(i0 + plane * z0);
      dinv = invd[i0 + plane * z0];
    }
    // One plane; PH = (z - z0) mod 3 names the ring slots (below, at and above
    // the point: PH, PH + 1, PH + 2 mod 3), so the ring needs no moves.
    auto step = [&](auto phase, int z) {
      constexpr int PH = decltype(phase)::value;
      // the next plane's inputs and the next point's epilogue inputs, loaded a plane ahead
      Vals after{acc(0), kOut, acc(0), kOut, acc(0), kOut};
      typename Epi::Pre pre_next{};
      acc dinv_next = acc(0);
      if (z + 1 < z1) {
        after = fetch(z + 2);
        if (own) {
          pre_next = epi.load(i0 + plane * (z + 1));
          dinv_next = invd[i0 + plane * (z + 1)];
        }
      }
      stage(nxt, (PH + 2) % 3);
      if (own) {
        constexpr int C = (PH + 1) % 3;
        acc off = acc(0), yc;
        if constexpr (kLdsRing) {
          // buffers of the planes below, at and above the point: the last three staged
          const uint32_t bz[3] = {(k - 3u) & 3u, (k - 2u) & 3u, (k - 1u) & 3u};
          const acc ri = rs[bz[1]][ty + 1][tx + 1];
          // consecutive neighbours in pairs: y1 / d1 + y2 / d2 = (d2 y1 + d1 y2) / (d1 d2)
          double pd = 0.0, py = 0.0;  // the first neighbour of the pair
          bool second = false;
#pragma unroll
          for (int dz = 0; dz < 3; ++dz) {
            const acc(*yq)[W] = ys[bz[dz]];
            const acc(*rq)[W] = rs[bz[dz]];
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
#pragma unroll
              for (int dx = 0; dx < 3; ++dx) {
                if (dz == 1 && dy == 1 && dx == 1) continue;
                const acc d = ri + rq[ty + dy][tx + dx];
                const acc yn = yq[ty + dy][tx + dx];
                if (second) {
                  const double dd = pd * d;
                  double w = __builtin_amdgcn_rcp(dd);
                  w = fma(fma(-dd, w, 1.0), w, w);
                  off = fma(w, fma(pd, yn, d * py), off);
                } else {
                  pd = d;
                  py = yn;
                }
                second = !second;
              }
            }
          }
          yc = ys[bz[1]][ty + 1][tx + 1];
        } else {
          const acc ri = rv[C][1][1];
#pragma unroll
          for (int dz = 0; dz < 3; ++dz) {
            const int q = (PH + dz) % 3;
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
#pragma unroll
              for (int dx = 0; dx < 3; ++dx) {
                if (dz == 1 && dy == 1 && dx == 1) continue;
                const acc d = ri + rv[q][dy][dx];
                if constexpr (sizeof(acc) == 4) {
                  off += __builtin_amdgcn_rcpf(d) * yv[q][dy][dx];
                } else {  // the unscaled float64 product
                  double w = __builtin_amdgcn_rcp(d);
                  w = fma(fma(-d, w, 1.0), w, w);
                  off += w * yv[q][dy][dx];
                }
              }
            }
          }
          yc = yv[C][1][1];
        }
        const int64_t i = i0 + plane * z;
        const acc m = SCALED ? yc - off * dinv : yc / dinv - off;
        epi(i, yc, m, pre, part);
      }
      nxt = after;
      pre = pre_next;
      dinv = dinv_next;
    };
    for (int z = z0; z < z1; z += 3) {
      step(std::integral_constant<int, 0>{}, z);
      if (z + 1 < z1) step(std::integral_constant<int, 1>{}, z + 1);
      if (z + 2 < z1) step(std::integral_constant<int, 2>{}, z + 2);
    }
  }
  finish_reduction<Epi, 64 * TY>(epi, part, rb, slot);
}

// ------------------------------------------------------------------ CSR
//
// LANES consecutive lanes share one row (LANES = 4 for ~7 nonzeros per row,
// 32 for ~80), read its nonzeros with unit stride and combine them with a
// butterfly inside the group.  A wavefront owns PASSES x 64 / LANES
// consecutive rows and walks them in PASSES passes of 64 / LANES rows; after
// each pass lane L picks up the sum of row L from its group, so the epilogue
// runs once per wavefront on consecutive rows with unit-stride vector
// accesses.  Large matrices take PASSES = min(LANES, 4) (for 4 lanes per row
// 64 rows per wavefront, every lane busy in the epilogue); PASSES = 1 keeps
// each wavefront's serial chain short for small ones, where launch latency
// dominates.  With up to 8 passes, the first two nonzero slots of every pass
// are read in straight-line code before any sum is formed, so all passes'
// loads are in flight together (7-point F32 step 347 -> 311 us on 256^3);
// longer rows finish in a loop.  With four lanes per row (short rows) and
// float64 or float32 values, lane g's two slots are the adjacent nonzeros
// rb + 2g and rb + 2g + 1, read as one vector access of each array (NzPair),
// so every line of the matrix is read by one instruction and can be streamed
// with non-temporal loads (256^3 7-point step F64 472 -> 421 us, F32 311 ->
// 273 us; with slots rb + g and rb + g + 4 the two slots share lines and
// streamed loads were slower).  A tile is the rows of one block.

// Two adjacent entries of a matrix array in one access (dword-aligned vectors).
template <class T>
struct PairOf {
  static constexpr bool ok = false;
};
template <>
struct PairOf<double> {
  static constexpr bool ok = true;
  typedef double type __attribute__((ext_vector_type(2), aligned(8)));
};
template <>
struct PairOf<float> {
  static constexpr bool ok = true;
  typedef float type __attribute__((ext_vector_type(2), aligned(4)));
};
template <>
struct PairOf<int32_t> {
  static constexpr bool ok = true;
  typedef int32_t type __attribute__((ext_vector_type(2), aligned(4)));
};
template <class T>
__device__ __forceinline__ typename PairOf<T>::type ld_pair_stream(const T* p, int32_t c) {
  return __builtin_nontemporal_load(reinterpret_cast<const typename PairOf<T>::type*>(p + c));
}

// Nonzeros j0 and j0 + 1 of a row ending at re, for arrays of nnz >= 2 entries.
// Slots outside the row read entries 0 and 1 and are flagged off; j0 = nnz - 1,
// the arrays' last entry, is read as the second of the pair at nnz - 2.
template <class Tv>
struct NzPair {
  using acc = typename Store<Tv>::acc;
  acc a0, a1;
  int32_t x0, x1;
  bool ok0, ok1;
  __device__ __forceinline__ NzPair(const int32_t* __restrict__ col, const Tv* __restrict__ val, int32_t j0,
                                    int32_t re, int32_t nnz) {
    ok0 = j0 < re;
    ok1 = j0 + 1 < re;
    const bool last = ok0 && j0 + 1 >= nnz;
    const int32_t c = ok0 ? (last ? j0 - 1 : j0) : 0;
    const auto cv = ld_pair_stream(col, c);
    const auto av = ld_pair_stream(val, c);
    a0 = acc(last ? av.y : av.x);
    a1 = acc(av.y);
    x0 = last ? cv.y : cv.x;
    x1 = cv.y;
  }
};

template <int LANES, int PASSES, class Tv, class In, class Epi>
struct KCsr {
  static constexpr int kThreads = kBlock;
  __device__ static void run(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                             const Tv* __restrict__ val, In in, Epi epi, int64_t n, uint32_t ntiles, ReduceBuf rb,
                             int slot0);
};
template <int LANES, int PASSES, class Tv, class In, class Epi>
__device__ __forceinline__ void KCsr<LANES, PASSES, Tv, In, Epi>::run(const int32_t* __restrict__ rowptr,
                                                                      const int32_t* __restrict__ col,
                                                                      const Tv* __restrict__ val, In in, Epi epi,
                                                                      int64_t n, uint32_t ntiles, ReduceBuf rb,
                                                                      int slot0) {
  using acc = typename Epi::acc;
  const int slot = slot0 + int(blockIdx.y);
  if (bind_slot(in, epi, slot)) return;
  double part[Epi::NV];
#pragma unroll
  for (int v = 0; v < Epi::NV; ++v) part[v] = 0.0;
  constexpr int kGroups = kWave / LANES;  // rows of one pass
  constexpr int kRows = PASSES * kGroups;  // rows of one wavefront
  const int lane = int(threadIdx.x) % kWave;
  const int wave = int(threadIdx.x) / kWave;
  const int g = lane % LANES;
  const int grp = lane / LANES;
  XcdTiles tiles(ntiles);
  for (uint32_t t = tiles.begin; t < tiles.end; t += tiles.step) {
    const int64_t base = (int64_t(t) * (kBlock / kWave) + wave) * kRows;  // first row of the wavefront
    if (base >= n) continue;
    const int64_t myrow = base + lane;
    const int32_t rb_lane = rowptr[myrow < n ? myrow : n];
    const int32_t re_lane = rowptr[myrow + 1 < n ? myrow + 1 : n];
    acc mine = acc(0);
    // the epilogue's own inputs are loaded before the row sums, so their latency overlaps them
    const bool has_row = lane < kRows && myrow < n;
    typename Epi::Pre pre{};
    acc yi = acc(0);
    if (has_row) {
      pre = epi.load(myrow);
      yi = in.ld(myrow);
    }
    if constexpr (PASSES > 1 && PASSES <= 8) {
      acc sums[PASSES];
      int32_t rb_it[PASSES], re_it[PASSES];
#pragma unroll
      for (int it = 0; it < PASSES; ++it) {
        const int r = it * kGroups + grp;  // row of this group in pass it (rows past n are empty)
        rb_it[it] = __shfl(rb_lane, r, kWave);
        re_it[it] = __shfl(re_lane, r, kWave);
      }
      // The first two slots of every pass as straight-line code (out-of-row slots
      // read entry 0, which exists since every row has its diagonal, and are
      // dropped by a select), so the loads of all passes are in flight together.
      if constexpr (LANES == 4 && PairOf<Tv>::ok) {
        const int32_t nnz = rowptr[n];  // >= n >= 2: the wide launches cover large matrices only
#pragma unroll
        for (int it = 0; it < PASSES; ++it) {
          const NzPair<Tv> q(col, val, rb_it[it] + 2 * g, re_it[it], nnz);
          const acc v0 = acc(q.a0) * in.ld(q.x0);
          const acc v1 = acc(q.a1) * in.ld(q.x1);
          acc sum = acc(0);
          sum += q.ok0 ? v0 : acc(0);
          sum += q.ok1 ? v1 : acc(0);
          sums[it] = sum;
        }
      } else {
#pragma unroll
        for (int it = 0; it < PASSES; ++it) {
          const int32_t j0 = rb_it[it] + g, j1 = j0 + LANES;
          const bool ok0 = j0 < re_it[it], ok1 = j1 < re_it[it];
          const int32_t c0 = ok0 ? j0 : 0, c1 = ok1 ? j1 : 0;
          const acc v0 = acc(Store<Tv>::ld(val, c0)) * in.ld(col[c0]);
          const acc v1 = acc(Store<Tv>::ld(val, c1)) * in.ld(col[c1]);
          acc sum = acc(0);
          sum += ok0 ? v0 : acc(0);
          sum += ok1 ? v1 : acc(0);
          sums[it] = sum;
        }
      }
#pragma unroll
      for (int it = 0; it < PASSES; ++it) {
        for (int32_t j = rb_it[it] + g + 2 * LANES; j < re_it[it]; j += LANES)
          sums[it] += acc(Store<Tv>::ld(val, j)) * in.ld(col[j]);
        acc sum = sums[it];
#pragma unroll
        for (int off = LANES / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, kWave);
        const acc v = __shfl(sum, (lane % kGroups) * LANES, kWave);  // row it * kGroups + lane % kGroups
        if (lane / kGroups == it) mine = v;
      }
    } else {
      for (int it = 0; it < PASSES; ++it) {
        const int r = it * kGroups + grp;  // row of this group in this pass (rows past n are empty)
        const int32_t b = __shfl(rb_lane, r, kWave), e = __shfl(re_lane, r, kWave);
        acc sum = acc(0);
        for (int32_t j = b + g; j < e; j += LANES) sum += acc(Store<Tv>::ld(val, j)) * in.ld(col[j]);
#pragma unroll
        for (int off = LANES / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, kWave);
        const acc v = __shfl(sum, (lane % kGroups) * LANES, kWave);  // row it * kGroups + lane % kGroups
        if (lane / kGroups == it) mine = v;
      }
    }
    if (has_row) epi(myrow, yi, mine, pre, part);
  }
  finish_reduction(epi, part, rb, slot);
}

// ------------------------------------------------------------------ SELL-C-sigma, C = 64
//
// One wavefront per chunk of 64 (sorted) rows; chunk c stores its slot j of
// every row contiguously (column-major), so every load of the wavefront is
// one 64-wide unit-stride access.  Padding slots hold column 0 and value 0.
// perm (may be null = identity) maps a sorted position to its original row.
// Values and column indices are loaded non-temporally: each line of them is
// read once per launch, and streaming them leaves the L2 to the gathered input
// vector (256^3 7-point F64 step 450 -> 403 us, F32 310 -> 268 us; results
// bitwise equal).  CSR rows share lines between a wavefront's nonzero slots,
// and there the same loads were slower (F64 470 -> 538 us).
template <class Tv>
__device__ __forceinline__ auto ld_stream(const Tv* p, int64_t i) {
  if constexpr (std::is_same<Tv, bf16>::value)
    return bf16_to_float(__builtin_nontemporal_load(&p[i].bits));
  else
    return __builtin_nontemporal_load(p + i);
}

template <class Tv, class In, class Epi>
struct KSell {
  static constexpr int kThreads = kBlock;
  __device__ static void run(const int64_t* __restrict__ chunk_ptr, const int32_t* __restrict__ chunk_len,
                             const int32_t* __restrict__ col, const Tv* __restrict__ val,
                             const int32_t* __restrict__ perm, In in, Epi epi, int64_t n, uint32_t ntiles, ReduceBuf rb,
                             int slot0);
};
template <class Tv, class In, class Epi>
__device__ __forceinline__ void KSell<Tv, In, Epi>::run(const int64_t* __restrict__ chunk_ptr,
                                                        const int32_t* __restrict__ chunk_len,
                                                        const int32_t* __restrict__ col, const Tv* __restrict__ val,
                                                        const int32_t* __restrict__ perm, In in, Epi epi, int64_t n,
                                                        uint32_t ntiles, ReduceBuf rb, int slot0) {
  using acc = typename Epi::acc;
  const int slot = slot0 + int(blockIdx.y);
  if (bind_slot(in, epi, slot)) return;
  double part[Epi::NV];
#pragma unroll
  for (int v = 0; v < Epi::NV; ++v) part[v] = 0.0;
  const int lane = threadIdx.x % kWave;
  XcdTiles tiles(ntiles);  // tile = kBlock / 64 = 4 chunks
  for (uint32_t t = tiles.begin; t < tiles.end; t += tiles.step) {
    const int64_t chunk = int64_t(t) * (kBlock / kWave) + threadIdx.x / kWave;
    const int64_t pos = chunk * kWave + lane;
    if (chunk * kWave >= n) continue;
    const int64_t base = chunk_ptr[chunk];
    const int32_t len = chunk_len[chunk];
    // the epilogue's own inputs are loaded before the row sums, so their latency overlaps them
    const bool has_row = pos < n;
    const int64_t row = has_row ? (perm ? int64_t(perm[pos]) : pos) : 0;
    typename Epi::Pre pre{};
    acc yi = acc(0);
    if (has_row) {
      pre = epi.load(row);
      yi = in.ld(row);
    }
    acc sum = acc(0);
#pragma unroll 8
    for (int32_t j = 0; j < len; ++j) {  // unrolled: several slots' loads in flight, same summation order
      const int64_t e = base + int64_t(j) * kWave + lane;
      sum += acc(ld_stream(val, e)) * in.ld(ld_stream(col, e));
    }
    if (has_row) epi(row, yi, sum, pre, part);
  }
  finish_reduction(epi, part, rb, slot);
}

// ------------------------------------------------------------------ several right-hand sides, matrix read once
//
// KCsrMulti and KSellMulti: a block serves kMultiSlots consecutive solve
// slots (slot0 + blockIdx.y * kMultiSlots + k, k < kMultiSlots, up to slot0 +
// nslots), reads every column index and value of its rows once and applies it
// to each active slot's vector.  Tiles, rows, lanes and the order of every
// slot's sums are those of the single-slot kernels, and a slot's block
// partials go to the same places, so each slot's results are bitwise those of
// KCsr / KSell alone; only the matrix traffic is shared.  Slots whose solve
// has finished are skipped.
constexpr int kMultiSlots = 4;

template <class In, class Epi>
struct SlotSet {
  In in[kMultiSlots];
  Epi epi[kMultiSlots];
  bool on[kMultiSlots];
  // true if no slot of the block is active.  An inactive slot's input is pointed at
  // an active slot's vector, so the inner loops read for every slot without a
  // branch (a branch per slot there keeps each slot's gathers from overlapping the
  // next one's); its sums are computed and dropped.
  __device__ __forceinline__ bool bind(const In& in0, const Epi& epi0, int first, int last) {
    bool any = false;
    In active = in0;
#pragma unroll
    for (int k = kMultiSlots - 1; k >= 0; --k) {
      in[k] = in0;
      epi[k] = epi0;
      on[k] = first + k < last && !bind_slot(in[k], epi[k], first + k);
      if (on[k]) active = in[k];
      any = any || on[k];
    }
#pragma unroll
    for (int k = 0; k < kMultiSlots; ++k)
      if (!on[k]) in[k] = active;
    return !any;
  }
};

template <int LANES, int PASSES, class Tv, class In, class Epi>
struct KCsrMulti {
  static constexpr int kThreads = kBlock;
  __device__ static void run(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                             const Tv* __restrict__ val, In in, Epi epi, int64_t n, uint32_t ntiles, ReduceBuf rb,
                             int slot0, int nslots);
};
template <int LANES, int PASSES, class Tv, class In, class Epi>
__device__ __forceinline__ void KCsrMulti<LANES, PASSES, Tv, In, Epi>::run(const int32_t* __restrict__ rowptr,
                                                                           const int32_t* __restrict__ col,
                                                                           const Tv* __restrict__ val, In in, Epi epi,
                                                                           int64_t n, uint32_t ntiles, ReduceBuf rb,
                                                                           int slot0, int nslots) {
  using acc = typename Epi::acc;
  constexpr int NS = kMultiSlots;
  const int first = slot0 + int(blockIdx.y) * NS;
  SlotSet<In, Epi> ss;
  if (ss.bind(in, epi, first, slot0 + nslots)) return;
  double part[NS][Epi::NV];
#pragma unroll
  for (int k = 0; k < NS; ++k)
#pragma unroll
    for (int v = 0; v < Epi::NV; ++v) part[k][v] = 0.0;
  constexpr int kGroups = kWave / LANES;
  constexpr int kRows = PASSES * kGroups;
  const int lane = int(threadIdx.x) % kWave;
  const int wave = int(threadIdx.x) / kWave;
  const int g = lane % LANES;
  const int grp = lane / LANES;
  XcdTiles tiles(ntiles);
  for (uint32_t t = tiles.begin; t < tiles.end; t += tiles.step) {
    const int64_t base = (int64_t(t) * (kBlock / kWave) + wave) * kRows;
    if (base >= n) continue;
    const int64_t myrow = base + lane;
    const int32_t rb_lane = rowptr[myrow < n ? myrow : n];
    const int32_t re_lane = rowptr[myrow + 1 < n ? myrow + 1 : n];
    const bool has_row = lane < kRows && myrow < n;
    typename Epi::Pre pre[NS];
    acc yi[NS], mine[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      pre[k] = typename Epi::Pre{};
      yi[k] = acc(0);
      mine[k] = acc(0);
      if (ss.on[k] && has_row) {
        pre[k] = ss.epi[k].load(myrow);
        yi[k] = ss.in[k].ld(myrow);
      }
    }
    if constexpr (PASSES > 1 && PASSES <= 8) {
      acc sums[PASSES][NS];
      int32_t rb_it[PASSES], re_it[PASSES];
#pragma unroll
      for (int it = 0; it < PASSES; ++it) {
        const int r = it * kGroups + grp;
        rb_it[it] = __shfl(rb_lane, r, kWave);
        re_it[it] = __shfl(re_lane, r, kWave);
      }
      if constexpr (LANES == 4 && PairOf<Tv>::ok) {  // the slots of KCsr's pair path
        const int32_t nnz = rowptr[n];
#pragma unroll
        for (int it = 0; it < PASSES; ++it) {
          const NzPair<Tv> q(col, val, rb_it[it] + 2 * g, re_it[it], nnz);
#pragma unroll
          for (int k = 0; k < NS; ++k) {
            const acc v0 = acc(q.a0) * ss.in[k].ld(q.x0);
            const acc v1 = acc(q.a1) * ss.in[k].ld(q.x1);
            acc sum = acc(0);
            sum += q.ok0 ? v0 : acc(0);
            sum += q.ok1 ? v1 : acc(0);
            sums[it][k] = sum;
          }
        }
      } else {
#pragma unroll
        for (int it = 0; it < PASSES; ++it) {
          const int32_t j0 = rb_it[it] + g, j1 = j0 + LANES;
          const bool ok0 = j0 < re_it[it], ok1 = j1 < re_it[it];
          const int32_t c0 = ok0 ? j0 : 0, c1 = ok1 ? j1 : 0;
          const acc a0 = acc(Store<Tv>::ld(val, c0)), a1 = acc(Store<Tv>::ld(val, c1));
          const int32_t x0 = col[c0], x1 = col[c1];
#pragma unroll
          for (int k = 0; k < NS; ++k) {
            const acc v0 = a0 * ss.in[k].ld(x0);
            const acc v1 = a1 * ss.in[k].ld(x1);
            acc sum = acc(0);
            sum += ok0 ? v0 : acc(0);
            sum += ok1 ? v1 : acc(0);
            sums[it][k] = sum;
          }
        }
      }
#pragma unroll
      for (int it = 0; it < PASSES; ++it) {
        for (int32_t j = rb_it[it] + g + 2 * LANES; j < re_it[it]; j += LANES) {
          const acc a = acc(Store<Tv>::ld(val, j));
          const int32_t x = col[j];
#pragma unroll
          for (int k = 0; k < NS; ++k) sums[it][k] += a * ss.in[k].ld(x);
        }
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          acc sum = sums[it][k];
#pragma unroll
          for (int off = LANES / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, kWave);
          const acc v = __shfl(sum, (lane % kGroups) * LANES, kWave);
          if (lane / kGroups == it) mine[k] = v;
        }
      }
    } else {
      for (int it = 0; it < PASSES; ++it) {
        const int r = it * kGroups + grp;
        const int32_t b = __shfl(rb_lane, r, kWave), e = __shfl(re_lane, r, kWave);
        acc sums[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) sums[k] = acc(0);
        for (int32_t j = b + g; j < e; j += LANES) {
          const acc a = acc(Store<Tv>::ld(val, j));
          const int32_t x = col[j];
#pragma unroll
          for (int k = 0; k < NS; ++k) sums[k] += a * ss.in[k].ld(x);
        }
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          acc sum = sums[k];
#pragma unroll
          for (int off = LANES / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, kWave);
          const acc v = __shfl(sum, (lane % kGroups) * LANES, kWave);
          if (lane / kGroups == it) mine[k] = v;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (ss.on[k] && has_row) ss.epi[k](myrow, yi[k], mine[k], pre[k], part[k]);
  }
#pragma unroll
  for (int k = 0; k < NS; ++k)
    if (ss.on[k]) finish_reduction(ss.epi[k], part[k], rb, first + k);
}

template <class Tv, class In, class Epi>
struct KSellMulti {
  static constexpr int kThreads = kBlock;
  __device__ static void run(const int64_t* __restrict__ chunk_ptr, const int32_t* __restrict__ chunk_len,
                             const int32_t* __restrict__ col, const Tv* __restrict__ val,
                             const int32_t* __restrict__ perm, In in, Epi epi, int64_t n, uint32_t ntiles, ReduceBuf rb,
                             int slot0, int nslots);
};
template <class Tv, class In, class Epi>
__device__ __forceinline__ void KSellMulti<Tv, In, Epi>::run(const int64_t* __restrict__ chunk_ptr,
                                                             const int32_t* __restrict__ chunk_len,
                                                             const int32_t* __restrict__ col,
                                                             const Tv* __restrict__ val,
                                                             const int32_t* __restrict__ perm, In in, Epi epi,
                                                             int64_t n, uint32_t ntiles, ReduceBuf rb, int slot0,
                                                             int nslots) {
  using acc = typename Epi::acc;
  constexpr int NS = kMultiSlots;
  const int first = slot0 + int(blockIdx.y) * NS;
  SlotSet<In, Epi> ss;
  if (ss.bind(in, epi, first, slot0 + nslots)) return;
  double part[NS][Epi::NV];
#pragma unroll
  for (int k = 0; k < NS; ++k)
#pragma unroll
    for (int v = 0; v < Epi::NV; ++v) part[k][v] = 0.0;
  const int lane = threadIdx.x % kWave;
  XcdTiles tiles(ntiles);
  for (uint32_t t = tiles.begin; t < tiles.end; t += tiles.step) {
    const int64_t chunk = int64_t(t) * (kBlock / kWave) + threadIdx.x / kWave;
    const int64_t pos = chunk * kWave + lane;
    if (chunk * kWave >= n) continue;
    const int64_t base = chunk_ptr[chunk];
    const int32_t len = chunk_len[chunk];
    const bool has_row = pos < n;
    const int64_t row = has_row ? (perm ? int64_t(perm[pos]) : pos) : 0;
    typename Epi::Pre pre[NS];
    acc yi[NS], sum[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      pre[k] = typename Epi::Pre{};
      yi[k] = acc(0);
      sum[k] = acc(0);
      if (ss.on[k] && has_row) {
        pre[k] = ss.epi[k].load(row);
        yi[k] = ss.in[k].ld(row);
      }
    }
#pragma unroll 4
    for (int32_t j = 0; j < len; ++j) {
      const int64_t e = base + int64_t(j) * kWave + lane;
      const acc a = acc(ld_stream(val, e));
      const int32_t x = ld_stream(col, e);
#pragma unroll
      for (int k = 0; k < NS; ++k) sum[k] += a * ss.in[k].ld(x);
    }
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (ss.on[k] && has_row) ss.epi[k](row, yi[k], sum[k], pre[k], part[k]);
  }
#pragma unroll
  for (int k = 0; k < NS; ++k)
    if (ss.on[k]) finish_reduction(ss.epi[k], part[k], rb, first + k);
}

// ------------------------------------------------------------------ input functors

template <class T>
struct InVec {
  using acc = typename Store<T>::acc;
  static constexpr bool narrow = sizeof(T) < 4;  // loads need a conversion
  const T* p;
  int64_t stride;
  __device__ __forceinline__ void bind(int slot) { p += slot * stride; }
  __device__ __forceinline__ void prepare() {}
  __device__ __forceinline__ acc ld(int64_t i) const { return Store<T>::ld(p, i); }
};

// p = z + beta * p_old, formed where it is read (beta from the solver state).
// The 7-point kernel calls ld once per point of a tile plane and its halo.
template <class Tz>
struct InDirection {
  using acc = double;
  static constexpr bool narrow = false;
  const Tz* z;  // float when the preconditioner's output has float32 precision (stored exactly)
  const double* p_old;
  const DevState* st;
  double beta;
  int64_t stride;
  __device__ __forceinline__ void bind(int slot) {
    z += slot * stride;
    p_old += slot * stride;
    st += slot;
  }
  __device__ __forceinline__ void prepare() { beta = st->beta; }
  __device__ __forceinline__ double ld(int64_t i) const { return double(z[i]) + beta * p_old[i]; }
};

// v scaled by D^-1/2 (for the symmetric scaled operator of the Lanczos estimator).
struct InScaled {
  using acc = double;
  static constexpr bool narrow = false;
  const double* v;
  const double* isd;  // 1 / sqrt(diag), shared by all slots
  int64_t stride;
  __device__ __forceinline__ void bind(int slot) { v += slot * stride; }
  __device__ __forceinline__ void prepare() {}
  __device__ __forceinline__ double ld(int64_t i) const { return v[i] * isd[i]; }
};

}  // namespace pcheb

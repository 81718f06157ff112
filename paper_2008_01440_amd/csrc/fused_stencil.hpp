// S consecutive middle steps of the Chebyshev recurrence on the matrix-free
// 7-point operator in one pass over memory (temporal blocking).
//
// Step j needs y_{j-1} at a point and its 6 neighbours and y_{j-2}, s at the
// point, so S steps on a tile need y_{j-1} with a halo of S.  A block owns an
// x-y tile of 64 x TY points plus that halo (a region of RX x RY points) and
// marches up a z range; the levels of the recurrence run as a skewed
// pipeline: when input plane t arrives, level l computes plane t - (l - 1),
// on a region that shrinks by one point per level, so level S+1 is exact on
// the 64 x TY interior.  One pass reads y_{j-1}, y_{j-2} and s and writes
// y_{j+S-2} and y_{j+S-1}: 5 vectors moved for S steps instead of 4 per step.
// Halo points are recomputed by neighbouring tiles; a z range is extended by S
// planes at each end.
//
// A block has NT threads; larger tiles (TY up to 32 with NT = 1024) recompute
// fewer halo points per output point.
//
// Storage: every thread owns the same region points in every plane.  For
// each level it keeps the last three planes of its points in registers (the
// z neighbours), and the level's newest plane also goes to a double-buffered
// LDS plane for the four in-plane neighbours.  Level l reads level l-1's plane
// z, which level l-1 wrote in the previous step of the pipeline, so the levels
// of one step never wait for each other: one barrier per step.  The global
// loads of the next step are issued before the current step computes.
//
// Levels: level 1 is the input y_{j-1}, level 0 the input y_{j-2}, level
// l >= 2 is y_{j+l-2}; levels 1..S have registers and LDS planes, level S+1
// goes straight to memory.
//
// k_stencil7_fused3 computes the same values in the same order without
// branches: LDS planes carry a margin of RX + 1 entries on both sides so every
// thread may read its four in-plane neighbours, loads use clamped in-grid
// addresses, and points outside a level's region are masked with selects.  The
// z loop is unrolled by three, the period of the register rings, so ring slots
// are fixed per unrolled copy instead of being shifted with moves.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace pcheb {

template <class A, int S>
struct FusedCoef {
  A a[S], b[S], c[S];  // step j + m uses a[m], b[m], c[m]
};

template <int S, int TY, int NT, class T>
__global__ __launch_bounds__(NT) void k_stencil7_fused(const T* __restrict__ ya, const T* __restrict__ yb,
                                                           const T* __restrict__ sv, T* __restrict__ out_a,
                                                           T* __restrict__ out_b,
                                                           FusedCoef<typename Store<T>::acc, S> cf, int nx, int ny,
                                                           int nz, int zc, uint32_t tiles_x, uint32_t tiles_y,
                                                           uint32_t ntiles, const DevState* guard, int64_t ld,
                                                           int slot0) {
  using acc = typename Store<T>::acc;
  constexpr int TX = 64;
  constexpr int RX = TX + 2 * S;
  constexpr int RY = TY + 2 * S;
  constexpr int NP = RX * RY;
  constexpr int P = (NP + NT - 1) / NT;  // region points per thread
  __shared__ acc plane_buf[S][2][NP];
  const int slot = slot0 + int(blockIdx.y);  // solve slot: vectors offset by slot * ld
  if (guard && guard[slot].done != kRunning) return;
  ya += slot * ld;
  yb += slot * ld;
  sv += slot * ld;
  out_a += slot * ld;
  out_b += slot * ld;
  const int tid = threadIdx.x;
  const int64_t plane = int64_t(nx) * ny;
  const acc sixth = acc(1.0 / 6.0);
  XcdTiles tiles(ntiles);
  for (uint32_t t = tiles.begin; t < tiles.end; t += tiles.step) {
    const int tx = int(t % tiles_x);
    const uint32_t rest = t / tiles_x;
    const int ty = int(rest % tiles_y);
    const int tz = int(rest / tiles_y);
    const int x0 = tx * TX - S, y0 = ty * TY - S;  // global coordinates of region point (0, 0)
    const int z0 = tz * zc;
    const int z1 = z0 + zc < nz ? z0 + zc : nz;
    const int zs = z0 - S;
    const int nadv = (z1 - z0) + 2 * S;

    // owned points: p = tid + NT m.  top[m] is the highest level whose
    // region contains the point (0 outside the grid); inner[m] marks the tile
    // interior; col[m] is the in-plane offset.
    int col[P], top[P];
    bool inner[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
      const int p = tid + NT * m;
      const int ry = p / RX, rx = p - (p / RX) * RX;
      const int gx = x0 + rx, gy = y0 + ry;
      const bool dom = p < NP && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
      const int lx = rx + 1 < RX - rx ? rx + 1 : RX - rx;
      const int ly = ry + 1 < RY - ry ? ry + 1 : RY - ry;
      top[m] = dom ? (lx < ly ? lx : ly) : 0;
      inner[m] = dom && rx >= S && rx < S + TX && ry >= S && ry < S + TY;
      col[m] = dom ? gx + nx * gy : 0;
    }
    acc L[S][3][P];  // level l at [l-1]: [0] newest plane, [1] one below, [2] two below
    acc sr[S][P];    // s at the planes of levels 2..S+1 ([0] = level 2's plane)
    acc ybc[P];      // y_{j-2} at level 2's plane
#pragma unroll
    for (int l = 0; l < S; ++l) {
#pragma unroll
      for (int m = 0; m < P; ++m) {
        L[l][0][m] = L[l][1][m] = L[l][2][m] = acc(0);
        sr[l][m] = acc(0);
      }
    }
    acc nya[P], ns[P], nyb[P];
    auto fetch = [&](int za, int zb) {
      const bool oka = za >= 0 && za < nz, okb = zb >= 0 && zb < nz;
      const T* pa = ya + plane * (oka ? za : 0);
      const T* ps = sv + plane * (okb ? zb : 0);
      const T* pb = yb + plane * (okb ? zb : 0);
#pragma unroll
      for (int m = 0; m < P; ++m) {
        nya[m] = (oka && top[m] > 0) ? Store<T>::ld(pa, col[m]) : acc(0);
        ns[m] = (okb && top[m] > 0) ? Store<T>::ld(ps, col[m]) : acc(0);
        nyb[m] = (okb && top[m] > 0) ? Store<T>::ld(pb, col[m]) : acc(0);
      }
    };
    fetch(zs, zs - 1);
    for (int adv = 0; adv < nadv; ++adv) {
      acc cya[P];
#pragma unroll
      for (int m = 0; m < P; ++m) {
        cya[m] = nya[m];
#pragma unroll
        for (int l = S - 1; l > 0; --l) sr[l][m] = sr[l - 1][m];
        sr[0][m] = ns[m];
        ybc[m] = nyb[m];
      }
      if (adv + 1 < nadv) fetch(zs + adv + 1, zs + adv);
      // level 1: the input plane zs + adv
      const int zin1 = zs + adv;
#pragma unroll
      for (int m = 0; m < P; ++m) {
        L[0][2][m] = L[0][1][m];
        L[0][1][m] = L[0][0][m];
        L[0][0][m] = cya[m];
        if (tid + NT * m < NP) plane_buf[0][zin1 & 1][tid + NT * m] = cya[m];
      }
#pragma unroll
      for (int l = 2; l <= S + 1; ++l) {
        const int z = zs + adv - (l - 1);
        const bool zin = z >= 0 && z < nz;
        const bool has_up = z + 1 < nz, has_dn = z > 0;
        const bool out_plane = z >= z0 && z < z1;
        const acc a = cf.a[l - 2], b = cf.b[l - 2], c = cf.c[l - 2];
        const acc* nb_plane = plane_buf[l - 2][z & 1];  // level l-1, plane z (previous step)
        const int li = l <= S ? l - 1 : 0;              // this level's register/LDS slot
        const int lp = l >= 3 ? l - 3 : 0;              // level l-2 (y_{j-2} role) for l >= 3
        T* out_z = (l == S ? out_b : out_a) + plane * (zin ? z : 0);
#pragma unroll
        for (int m = 0; m < P; ++m) {
          const int p = tid + NT * m;
          const bool valid = zin && l <= top[m];
          acc v = acc(0);
          if (valid) {
            const acc yc = L[l - 2][1][m];
            acc nb = (nb_plane[p - 1] + nb_plane[p + 1]) + (nb_plane[p - RX] + nb_plane[p + RX]);
            nb += (has_up ? L[l - 2][0][m] : acc(0)) + (has_dn ? L[l - 2][2][m] : acc(0));
            const acc yprev = (l == 2) ? ybc[m] : L[lp][2][m];
            v = a * yc + c * (sr[l - 2][m] - (yc - nb * sixth));  // same order as EpiChebStep
            v -= b * yprev;
            if (l >= S && out_plane && inner[m]) Store<T>::st(out_z, col[m], v);
          }
          if (l <= S) {
            L[li][2][m] = L[li][1][m];
            L[li][1][m] = L[li][0][m];
            L[li][0][m] = v;
            if (p < NP) plane_buf[li][z & 1][p] = v;
          }
        }
      }
      __syncthreads();
    }
  }
}

template <int S, int TY, int NT, class T>
__global__ __launch_bounds__(NT) void k_stencil7_fused3(const T* __restrict__ ya, const T* __restrict__ yb,
                                                       const T* __restrict__ sv, T* __restrict__ out_a,
                                                       T* __restrict__ out_b, FusedCoef<typename Store<T>::acc, S> cf,
                                                       int nx, int ny, int nz, int zc, uint32_t tiles_x,
                                                       uint32_t tiles_y, uint32_t ntiles, const DevState* guard,
                                                       int64_t ld, int slot0) {
  using acc = typename Store<T>::acc;
  constexpr int TX = 64;
  constexpr int RX = TX + 2 * S;
  constexpr int RY = TY + 2 * S;
  constexpr int NP = RX * RY;
  constexpr int P = (NP + NT - 1) / NT;  // region points per thread
  constexpr int PAD = RX + 1;            // margin: q - RX - 1 >= 0 and q + RX + 1 < NPL for every q used
  constexpr int NPL = NP + 2 * PAD;
  __shared__ acc plane_buf[S][2][NPL];
  const int slot = slot0 + int(blockIdx.y);  // solve slot: vectors offset by slot * ld
  if (guard && guard[slot].done != kRunning) return;
  ya += slot * ld;
  yb += slot * ld;
  sv += slot * ld;
  out_a += slot * ld;
  out_b += slot * ld;
  const int tid = threadIdx.x;
  const int64_t plane = int64_t(nx) * ny;
  const acc sixth = acc(1.0 / 6.0);
  XcdTiles tiles(ntiles);
  for (uint32_t t = tiles.begin; t < tiles.end; t += tiles.step) {
    const int tx = int(t % tiles_x);
    const uint32_t rest = t / tiles_x;
    const int ty = int(rest % tiles_y);
    const int tz = int(rest / tiles_y);
    const int x0 = tx * TX - S, y0 = ty * TY - S;  // global coordinates of region point (0, 0)
    const int z0 = tz * zc;
    const int z1 = z0 + zc < nz ? z0 + zc : nz;
    const int zs = z0 - S;
    const int nadv = (z1 - z0) + 2 * S;

    // owned points p = tid + NT m: top[m] is the highest level whose region
    // contains the point (0 outside the grid or for p >= NP), inner[m] marks
    // the tile interior, col[m] the in-plane offset (0 when outside), q[m] the
    // LDS index (lanes without a point use the first entry of the tail margin,
    // which no point with a valid value reads).
    int col[P], top[P], q[P];
    bool inner[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
      const int p = tid + NT * m;
      const int ry = p / RX, rx = p - (p / RX) * RX;
      const int gx = x0 + rx, gy = y0 + ry;
      const bool dom = p < NP && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
      const int lx = rx + 1 < RX - rx ? rx + 1 : RX - rx;
      const int ly = ry + 1 < RY - ry ? ry + 1 : RY - ry;
      top[m] = dom ? (lx < ly ? lx : ly) : 0;
      inner[m] = dom && rx >= S && rx < S + TX && ry >= S && ry < S + TY;
      col[m] = dom ? gx + nx * gy : 0;
      q[m] = p < NP ? p + PAD : NP + PAD;
    }
    acc L[S][3][P];  // ring of the last three planes of level l at [l-1]
    acc sr[S][P];    // s at the planes of levels 2..S+1 ([0] = level 2's plane)
#pragma unroll
    for (int l = 0; l < S; ++l) {
#pragma unroll
      for (int m = 0; m < P; ++m) {
        L[l][0][m] = L[l][1][m] = L[l][2][m] = acc(0);
        sr[l][m] = acc(0);
      }
    }
    // loads of the next step land here unmasked; oka / okb say whether their
    // planes are in range, dom[m] whether the point is in the grid, and the
    // zeros are applied when the values are used
    acc nya[P], ns[P], nyb[P];
    bool dom[P];
#pragma unroll
    for (int m = 0; m < P; ++m) dom[m] = top[m] > 0;
    bool oka = false, okb = false;
    auto fetch = [&](int za, int zb) {
      oka = za >= 0 && za < nz;
      okb = zb >= 0 && zb < nz;
      const T* pa = ya + plane * (oka ? za : 0);
      const T* ps = sv + plane * (okb ? zb : 0);
      const T* pb = yb + plane * (okb ? zb : 0);
#pragma unroll
      for (int m = 0; m < P; ++m) {
        nya[m] = Store<T>::ld(pa, col[m]);
        ns[m] = Store<T>::ld(ps, col[m]);
        nyb[m] = Store<T>::ld(pb, col[m]);
      }
    };
    // One step of the pipeline; PH = adv mod 3 fixes the ring slots.  Planes
    // outside the grid hold zeros in every level (inputs are masked, computed
    // values outside the grid are set to zero), which supplies the Dirichlet
    // zeros of the z neighbours without tests.
    auto advance = [&](auto phase, int adv) {
      constexpr int PH = decltype(phase)::value;
      constexpr int K0 = PH, K1 = (PH + 2) % 3, K2 = (PH + 1) % 3;  // newest, one below, two below
      acc cya[P], ybc[P];
#pragma unroll
      for (int m = 0; m < P; ++m) {
        cya[m] = (oka && dom[m]) ? nya[m] : acc(0);
#pragma unroll
        for (int l = S - 1; l > 0; --l) sr[l][m] = sr[l - 1][m];
        sr[0][m] = (okb && dom[m]) ? ns[m] : acc(0);
        ybc[m] = (okb && dom[m]) ? nyb[m] : acc(0);
      }
      if (adv + 1 < nadv) fetch(zs + adv + 1, zs + adv);
      // In-plane neighbour sums: every level reads a plane written in the
      // previous step, so the sums of level l + 1 are read while level l computes.
      acc nbs[2][P];
      auto read_sums = [&](int l, acc* out) {
        const acc* nb_plane = plane_buf[l - 2][(zs + adv - (l - 1)) & 1];
#pragma unroll
        for (int m = 0; m < P; ++m) {
          const int qm = q[m];
          out[m] = (nb_plane[qm - 1] + nb_plane[qm + 1]) + (nb_plane[qm - RX] + nb_plane[qm + RX]);
        }
      };
      read_sums(2, nbs[0]);
      const int zin1 = zs + adv;  // level 1: the input plane
#pragma unroll
      for (int m = 0; m < P; ++m) {
        L[0][K0][m] = cya[m];
        plane_buf[0][zin1 & 1][q[m]] = cya[m];
      }
#pragma unroll
      for (int l = 2; l <= S + 1; ++l) {
        const int z = zs + adv - (l - 1);
        const bool zin = z >= 0 && z < nz;
        const bool out_plane = z >= z0 && z < z1;
        const acc a = cf.a[l - 2], b = cf.b[l - 2], c = cf.c[l - 2];
        const int li = l <= S ? l - 1 : 0;
        const int lp = l >= 3 ? l - 3 : 0;
        T* out_z = (l == S ? out_b : out_a) + plane * (zin ? z : 0);
        if (l + 1 <= S + 1) read_sums(l + 1, nbs[(l - 1) & 1]);
        acc v[P];
#pragma unroll
        for (int m = 0; m < P; ++m) {
          const acc yc = L[l - 2][K1][m];
          acc nb = nbs[l & 1][m];
          nb += L[l - 2][K0][m] + L[l - 2][K2][m];
          const acc yprev = (l == 2) ? ybc[m] : L[lp][K2][m];
          acc w = a * yc + c * (sr[l - 2][m] - (yc - nb * sixth));  // same order as EpiChebStep
          w -= b * yprev;
          v[m] = (zin && l <= top[m]) ? w : acc(0);
          if (l >= S && zin && out_plane && inner[m]) Store<T>::st(out_z, col[m], v[m]);
        }
        if (l <= S) {
#pragma unroll
          for (int m = 0; m < P; ++m) {
            L[li][K0][m] = v[m];
            plane_buf[li][z & 1][q[m]] = v[m];
          }
        }
      }
      __syncthreads();
    };
    fetch(zs, zs - 1);
    for (int adv = 0; adv < nadv; adv += 3) {
      advance(std::integral_constant<int, 0>{}, adv);
      if (adv + 1 < nadv) advance(std::integral_constant<int, 1>{}, adv + 1);
      if (adv + 2 < nadv) advance(std::integral_constant<int, 2>{}, adv + 2);
    }
  }
}

}  // namespace pcheb

// S consecutive middle steps of the Chebyshev recurrence on the matrix-free
// 7-point operator in one pass over memory (temporal blocking).
//
// Step j needs y_{j-1} at a point and its 6 neighbours, y_{j-2} and s at the
// point, so S steps on a tile need y_{j-1} with a halo of S.  A block owns an
// x-y tile of 64 x TY points and marches up a z range; for each of the S + 1
// recurrence levels it keeps the last three planes of its (64 + 2S) x (TY + 2S)
// region in LDS.  The levels run as a skewed pipeline: when input plane t
// arrives, level l computes plane t - (l - 1) from level l-1's planes
// z-1, z, z+1 and level l-2's plane z, on a region that shrinks by one point
// per level, so level S+1 is exact on the 64 x TY interior.  One pass reads
// y_{j-1}, y_{j-2} and s and writes y_{j+S-2}, y_{j+S-1}: 5 vectors moved for S
// steps instead of 4 per step.  Halo points are recomputed by neighbouring
// tiles; a z range is extended by S planes at each end.
//
// Level indices: level 1 is the input y_{j-1} (ring 0), level 0 the input
// y_{j-2} (read from memory), level l >= 2 is y_{j+l-2} (ring l-1, levels
// 2..S; level S+1 goes straight to memory).
#pragma once

#include "common.hpp"

namespace pcheb {

template <class A, int S>
struct FusedCoef {
  A a[S], b[S], c[S];  // step j + m uses a[m], b[m], c[m]
};

__device__ __forceinline__ int mod3(int z) { return ((z % 3) + 3) % 3; }

template <int S, int TY, class T>
__global__ __launch_bounds__(kBlock) void k_stencil7_fused(const T* __restrict__ ya, const T* __restrict__ yb,
                                                           const T* __restrict__ sv, T* __restrict__ out_a,
                                                           T* __restrict__ out_b,
                                                           FusedCoef<typename Store<T>::acc, S> cf, int nx, int ny,
                                                           int nz, int zc, uint32_t tiles_x, uint32_t tiles_y,
                                                           uint32_t ntiles, const DevState* guard) {
  using acc = typename Store<T>::acc;
  constexpr int TX = 64;
  constexpr int RX = TX + 2 * S;
  constexpr int RY = TY + 2 * S;
  constexpr int NP = RX * RY;
  __shared__ acc ring[S][3][NP];
  if (guard && guard->done != kRunning) return;
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
    for (int adv = 0; adv < nadv; ++adv) {
      // level 1: input plane zs + adv
      {
        const int z = zs + adv;
        if (z >= 0 && z < nz) {
          acc* dst = ring[0][mod3(z)];
          for (int p = tid; p < NP; p += kBlock) {
            const int ry = p / RX, rx = p - ry * RX;
            const int gx = x0 + rx, gy = y0 + ry;
            const bool dom = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
            dst[p] = dom ? Store<T>::ld(ya, gx + int64_t(nx) * gy + plane * z) : acc(0);
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int l = 2; l <= S + 1; ++l) {
        const int z = zs + adv - (l - 1);
        if (z >= 0 && z < nz) {
          const acc a = cf.a[l - 2], b = cf.b[l - 2], c = cf.c[l - 2];
          const acc* cen = ring[l - 2][mod3(z)];
          const acc* up = ring[l - 2][mod3(z + 1)];
          const acc* dn = ring[l - 2][mod3(z - 1)];
          const bool has_up = z + 1 < nz, has_dn = z > 0;
          const bool out_plane = z >= z0 && z < z1;
          for (int p = tid; p < NP; p += kBlock) {
            const int ry = p / RX, rx = p - ry * RX;
            if (rx < l - 1 || rx > RX - l || ry < l - 1 || ry > RY - l) continue;
            const int gx = x0 + rx, gy = y0 + ry;
            const bool dom = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
            acc v = acc(0);
            const int64_t gi = gx + int64_t(nx) * gy + plane * z;
            if (dom) {
              const acc yc = cen[p];
              acc nb = (cen[p - 1] + cen[p + 1]) + (cen[p - RX] + cen[p + RX]);
              nb += (has_up ? up[p] : acc(0)) + (has_dn ? dn[p] : acc(0));
              const acc yprev = (l == 2) ? Store<T>::ld(yb, gi) : ring[l >= 3 ? l - 3 : 0][mod3(z)][p];
              v = a * yc + c * (Store<T>::ld(sv, gi) - (yc - nb * sixth));  // same order as EpiChebStep
              v -= b * yprev;
            }
            if (l <= S) ring[l <= S ? l - 1 : 0][mod3(z)][p] = v;
            if (out_plane && dom && rx >= S && rx < S + TX && ry >= S && ry < S + TY) {
              if (l == S) Store<T>::st(out_b, gi, v);
              if (l == S + 1) Store<T>::st(out_a, gi, v);
            }
          }
        }
        __syncthreads();
      }
    }
  }
}

}  // namespace pcheb

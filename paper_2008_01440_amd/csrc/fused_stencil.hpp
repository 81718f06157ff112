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
// k_stencil7_fused_buf (float32 and bfloat16 storage, x-y planes under 2 GiB)
// computes the same values in the same order with fewer instructions per
// point:
//  * memory accesses are buffer instructions: each plane of a vector gets a
//    descriptor whose range is the plane (empty for planes outside the grid),
//    and lanes whose point is outside the grid, or whose result is not an
//    output, use an offset beyond the range, so loads return zero and stores
//    are dropped without masks or branches;
//  * the LDS holds one record per region point with the last three planes of
//    every level (odd stride, so a wavefront's accesses hit distinct banks);
//    with the z loop unrolled by three, the period of the rings, every LDS
//    access is an immediate offset from one base per owned point and the
//    register rings need no moves;
//  * the neighbour reads of level l+1 are issued while level l computes.
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
            if (l >= S && out_plane && inner[m]) {
              if constexpr (sizeof(T) == 8)
                out_z[col[m]] = v;  // a cached store: the streaming one measured 5% slower here
              else
                Store<T>::st(out_z, col[m], v);
            }
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

// Raw buffer accesses: descriptor word 3 of the gfx9 family for untyped 32-bit
// accesses; an offset at or beyond the descriptor's range reads zero and
// drops stores.
constexpr int kBufferWord3 = 0x00020000;
constexpr int kOutOfRange = 0x7FFFFFF0;

template <class T>
struct BufIo;

// Cache policy of the float32 output stores: non-temporal (bit 1 of the
// buffer instruction's cache-policy operand on this family).  A pass writes two
// whole vectors that the next pass reads only after every other plane has
// streamed through the L2, so keeping them there only evicts the halo lines
// that neighbouring tiles are about to read (measured: the pass runs 3%
// faster).  Non-temporal loads of y_{j-2}, which has no reuse either, were
// slower, and so were non-temporal bfloat16 stores (a wavefront writes 128
// bytes, part of two lines, and streamed partial lines cost 23%).
constexpr int kStreamStore = 2;

template <>
struct BufIo<float> {
  static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, int off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  }
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, int off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, kStreamStore);
  }
};

template <>
struct BufIo<bf16> {
  static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, int off) {
    return bf16_to_float(__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
  }
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, int off, float v) {
    __builtin_amdgcn_raw_buffer_store_b16(float_to_bf16(v), r, off, 0, 0);
  }
};

template <int S, int TY, int NT, class T>
__global__ __launch_bounds__(NT) void k_stencil7_fused_buf(const T* __restrict__ ya, const T* __restrict__ yb,
                                                           const T* __restrict__ sv, T* __restrict__ out_a,
                                                           T* __restrict__ out_b, FusedCoef<float, S> cf, int nx,
                                                           int ny, int nz, int zc, uint32_t tiles_x,
                                                           uint32_t tiles_y, uint32_t ntiles, const DevState* guard,
                                                           int64_t ld, int slot0) {
  constexpr int TX = 64;
  constexpr int RX = TX + 2 * S;
  constexpr int RY = TY + 2 * S;
  constexpr int NP = RX * RY;
  constexpr int P = (NP + NT - 1) / NT;  // region points per thread
  constexpr int PAD = RX + 1;            // margin: q - RX - 1 >= 0 and q + RX + 1 < NPL for every q used
  constexpr int NPL = NP + 2 * PAD;
  constexpr int E = int(sizeof(T));
  constexpr int R = (3 * S) % 2 == 0 ? 3 * S + 1 : 3 * S;  // LDS record of a point: its S x 3 planes, odd stride
  __shared__ float lds[NPL * R];
  const int slot = slot0 + int(blockIdx.y);  // solve slot: vectors offset by slot * ld
  if (guard && guard[slot].done != kRunning) return;
  ya += slot * ld;
  yb += slot * ld;
  sv += slot * ld;
  out_a += slot * ld;
  out_b += slot * ld;
  const int tid = threadIdx.x;
  const int64_t plane = int64_t(nx) * ny;
  const int plane_bytes = int(plane * E);
  const float sixth = 1.0f / 6.0f;
  // descriptor of plane zz of a vector (an empty range outside the grid)
  auto rsrc = [&](const T* base, int zz) {
    const bool ok = zz >= 0 && zz < nz;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base) + plane * (ok ? zz : 0), 0,
                                             ok ? plane_bytes : 0, kBufferWord3);
  };
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
    // contains the point (0 outside the grid or for p >= NP); dom[m] says the
    // point is in the grid; ldo[m] / sto[m] are the byte offsets of its loads
    // and output stores in a plane (out of range where there is nothing to
    // load or store); q[m] is its LDS index (lanes without a point use the
    // first entry of the tail margin, which no point with a valid value reads).
    int top[P], q[P], ldo[P], sto[P];
    bool dom[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
      const int p = tid + NT * m;
      const int ry = p / RX, rx = p - (p / RX) * RX;
      const int gx = x0 + rx, gy = y0 + ry;
      dom[m] = p < NP && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
      const int lx = rx + 1 < RX - rx ? rx + 1 : RX - rx;
      const int ly = ry + 1 < RY - ry ? ry + 1 : RY - ry;
      top[m] = dom[m] ? (lx < ly ? lx : ly) : 0;
      const bool inner = dom[m] && rx >= S && rx < S + TX && ry >= S && ry < S + TY;
      ldo[m] = dom[m] ? (gx + nx * gy) * E : kOutOfRange;
      sto[m] = inner ? (gx + nx * gy) * E : kOutOfRange;
      q[m] = p < NP ? p + PAD : NP + PAD;
    }
    float* rec[P];  // rec[m][(RX + d) * R + k]: slot k of the record of point q + d (d = -RX, -1, 0, 1, RX)
#pragma unroll
    for (int m = 0; m < P; ++m) rec[m] = lds + (q[m] - RX) * R;
    float L[S][3][P];  // ring of the last three planes of level l at [l-1]
    float sr[S][P];    // s at the planes of levels 2..S+1 ([0] = level 2's plane)
#pragma unroll
    for (int l = 0; l < S; ++l) {
#pragma unroll
      for (int m = 0; m < P; ++m) {
        L[l][0][m] = L[l][1][m] = L[l][2][m] = 0.0f;
        sr[l][m] = 0.0f;
      }
    }
    float nya[P], ns[P], nyb[P];  // loads of the next step (zero outside the grid)
    auto fetch = [&](int za, int zb) {
      const auto ra = rsrc(ya, za), rs = rsrc(sv, zb);
#pragma unroll
      for (int m = 0; m < P; ++m) {
        nya[m] = BufIo<T>::ld(ra, ldo[m]);
        ns[m] = BufIo<T>::ld(rs, ldo[m]);
      }
    };
    auto fetch_yb = [&](int zb) {  // y_{j-2} is used by level 2 only: loaded once level 2 is done
      const auto rb = rsrc(yb, zb);
#pragma unroll
      for (int m = 0; m < P; ++m) nyb[m] = BufIo<T>::ld(rb, ldo[m]);
    };
    // One step of the pipeline; PH = adv mod 3 fixes the register ring slots
    // and the LDS ring slots.  Level l writes its plane at phase ph into slot
    // (l - 1) * 3 + (ph - (l - 1)) mod 3 of the point records; level l + 1
    // reads it at phase ph + 1.  Every LDS access of a thread is an immediate
    // offset from one base per owned point.
    auto advance = [&](auto phase, int adv) {
      constexpr int PH = decltype(phase)::value;
      constexpr int K0 = PH, K1 = (PH + 2) % 3, K2 = (PH + 1) % 3;  // newest, one below, two below
#pragma unroll
      for (int m = 0; m < P; ++m) {
        L[0][K0][m] = nya[m];
#pragma unroll
        for (int l = S - 1; l > 0; --l) sr[l][m] = sr[l - 1][m];
        sr[0][m] = ns[m];
      }
      if (adv + 1 < nadv) fetch(zs + adv + 1, zs + adv);
      float nbs[2][P];
      auto read_sums = [&](auto level, float* out) {
        constexpr int l = decltype(level)::value;
        constexpr int k = (l - 2) * 3 + ((PH - l + 1) % 3 + 3) % 3;  // level l-1, slot written last step
#pragma unroll
        for (int m = 0; m < P; ++m)
          out[m] = (rec[m][(RX - 1) * R + k] + rec[m][(RX + 1) * R + k]) + (rec[m][k] + rec[m][2 * RX * R + k]);
      };
      read_sums(std::integral_constant<int, 2>{}, nbs[0]);
#pragma unroll
      for (int m = 0; m < P; ++m) rec[m][RX * R + PH] = L[0][K0][m];  // level 1: the input plane
      auto level = [&](auto lv) {
        constexpr int l = decltype(lv)::value;
        constexpr int li = l <= S ? l - 1 : 0;
        constexpr int lp = l >= 3 ? l - 3 : 0;
        const int z = zs + adv - (l - 1);
        const bool zin = z >= 0 && z < nz;
        const float a = cf.a[l - 2], b = cf.b[l - 2], c = cf.c[l - 2];
        if constexpr (l + 1 <= S + 1) read_sums(std::integral_constant<int, l + 1>{}, nbs[(l - 1) & 1]);
        float v[P];
        if (zin) {
#pragma unroll
          for (int m = 0; m < P; ++m) {
            const float yc = L[l - 2][K1][m];
            float nb = nbs[l & 1][m];
            nb += L[l - 2][K0][m] + L[l - 2][K2][m];
            const float yprev = (l == 2) ? nyb[m] : L[lp][K2][m];
            float w = a * yc + c * (sr[l - 2][m] - (yc - nb * sixth));  // same order as EpiChebStep
            w -= b * yprev;
            v[m] = dom[m] ? w : 0.0f;
          }
          if (l >= S && z >= z0 && z < z1) {
            const auto ro = rsrc(l == S ? out_b : out_a, z);
#pragma unroll
            for (int m = 0; m < P; ++m) BufIo<T>::st(ro, sto[m], v[m]);
          }
        } else {
#pragma unroll
          for (int m = 0; m < P; ++m) v[m] = 0.0f;
        }
        if constexpr (l <= S) {
          constexpr int k = li * 3 + ((PH - (l - 1)) % 3 + 3) % 3;
#pragma unroll
          for (int m = 0; m < P; ++m) {
            L[li][K0][m] = v[m];
            rec[m][RX * R + k] = v[m];
          }
        }
      };
      level(std::integral_constant<int, 2>{});
      if (adv + 1 < nadv) fetch_yb(zs + adv);
      level(std::integral_constant<int, 3>{});
      if constexpr (S >= 3) level(std::integral_constant<int, 4>{});
      if constexpr (S >= 4) level(std::integral_constant<int, 5>{});
      if constexpr (S >= 5) level(std::integral_constant<int, 6>{});
      __syncthreads();
    };
    fetch(zs, zs - 1);
    fetch_yb(zs - 1);
    for (int adv = 0; adv < nadv; adv += 3) {
      advance(std::integral_constant<int, 0>{}, adv);
      if (adv + 1 < nadv) advance(std::integral_constant<int, 1>{}, adv + 1);
      if (adv + 2 < nadv) advance(std::integral_constant<int, 2>{}, adv + 2);
    }
  }
}

}  // namespace pcheb

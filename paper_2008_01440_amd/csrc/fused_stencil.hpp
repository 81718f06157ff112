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
// z neighbours), and the level's newest plane also goes to LDS for the four
// in-plane neighbours.  Level l reads level l-1's plane z, which level l-1
// wrote in the previous step of the pipeline, so the levels of one step never
// wait for each other: one barrier per step.  The global loads of the next
// step are issued before the current step computes.
//
// Levels: level 1 is the input y_{j-1}, level 0 the input y_{j-2}, level
// l >= 2 is y_{j+l-2}; levels 1..S have registers and LDS planes, level S+1
// goes straight to memory.
//
// Both kernels (KFusedPass for float32 and bfloat16 storage,
// KFusedPass64 for float64) keep the inner loop to the recurrence
// arithmetic:
//  * memory accesses are buffer instructions: each vector gets one descriptor
//    per tile, covering the planes the tile touches, and a plane is selected
//    by the instruction's scalar offset (planes outside the grid use an empty
//    descriptor); lanes whose point is outside the grid, or whose result is
//    not an output, use an offset beyond the range, so loads return zero and
//    stores are dropped without masks or branches;
//  * the z loop is unrolled by the period of the register and LDS rings, so
//    every ring slot is a compile-time constant and every LDS access is an
//    immediate offset from one base per owned point;
//  * the neighbour reads of level l+1 are issued while level l computes.
// A tile's descriptor span must stay within kMaxSpanBytes, which the launch
// ensures by its choice of z range; planes too large for that run unfused.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace pcheb {

template <class A, int S>
struct FusedCoef {
  A a[S], b[S], c[S];  // step j + m uses a[m], b[m], c[m]
};

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

// off: per-lane byte offset inside the plane; soff: the plane's byte offset from the
// descriptor's base (uniform).
template <>
struct BufIo<float> {
  static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, int off, int soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
  }
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, int off, int soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, soff, kStreamStore);
  }
};

template <>
struct BufIo<bf16> {
  static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, int off, int soff) {
    return bf16_to_float(__builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0));
  }
  static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, int off, int soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b16(float_to_bf16(v), r, off, soff, 0);
  }
};

// Largest byte span one tile's descriptors may cover: lanes with nothing to load or
// store use the offset kOutOfRange, which must stay at or beyond the span whether or
// not the hardware adds the scalar offset before its range check.
constexpr int64_t kMaxSpanBytes = kOutOfRange;

template <int S, int TY, int NT, class T>
struct KFusedPass {
  static constexpr int kThreads = NT;
  __device__ static void run(const T* __restrict__ ya, const T* __restrict__ yb, const T* __restrict__ sv,
                             T* __restrict__ out_a, T* __restrict__ out_b, FusedCoef<float, S> cf, int nx, int ny,
                             int nz, int zc, uint32_t tiles_x, uint32_t tiles_y, uint32_t ntiles, const DevState* guard,
                             int64_t ld, int slot0);
};
template <int S, int TY, int NT, class T>
__device__ __forceinline__ void KFusedPass<S, TY, NT, T>::run(const T* __restrict__ ya, const T* __restrict__ yb,
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
  // a descriptor that every access misses (planes outside the grid)
  const auto r_none = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(ya), 0, 0, kBufferWord3);
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
    // One descriptor per vector for the tile, based at the lowest plane the tile
    // touches (zs - 1) and spanning the planes up to zs + nadv - 1 (within the
    // grid); plane zz is reached through the scalar offset (zz - zlo) * plane_bytes,
    // and planes outside the grid through r_none.  The launch keeps the span within
    // kMaxSpanBytes.
    const int zlo = zs - 1 > 0 ? zs - 1 : 0;
    const int zhi = zs + nadv - 1 < nz - 1 ? zs + nadv - 1 : nz - 1;
    const int span = (zhi - zlo + 1) * plane_bytes;
    auto tile_rsrc = [&](const T* base) {
      return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base) + plane * zlo, 0, span, kBufferWord3);
    };
    const auto r_ya = tile_rsrc(ya), r_yb = tile_rsrc(yb), r_sv = tile_rsrc(sv);
    const auto r_oa = tile_rsrc(out_a), r_ob = tile_rsrc(out_b);
    auto plane_soff = [&](int zz) { return zz >= 0 && zz < nz ? (zz - zlo) * plane_bytes : 0; };

    // owned points p = tid + NT m: dom[m] says the point is in the grid;
    // ldo[m] / sto[m] are the byte offsets of its loads and output stores in a
    // plane (out of range where there is nothing to load or store); q[m] is its
    // LDS index (lanes without a point use the first entry of the tail margin,
    // which no point with a valid value reads).
    int q[P], ldo[P], sto[P];
    bool dom[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
      const int p = tid + NT * m;
      const int ry = p / RX, rx = p - (p / RX) * RX;
      const int gx = x0 + rx, gy = y0 + ry;
      dom[m] = p < NP && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
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
      const auto ra = za >= 0 && za < nz ? r_ya : r_none;
      const auto rs = zb >= 0 && zb < nz ? r_sv : r_none;
      const int sa = plane_soff(za), sb = plane_soff(zb);
#pragma unroll
      for (int m = 0; m < P; ++m) {
        nya[m] = BufIo<T>::ld(ra, ldo[m], sa);
        ns[m] = BufIo<T>::ld(rs, ldo[m], sb);
      }
    };
    auto fetch_yb = [&](int zb) {  // y_{j-2} is used by level 2 only: loaded once level 2 is done
      const auto rb = zb >= 0 && zb < nz ? r_yb : r_none;
      const int sb = plane_soff(zb);
#pragma unroll
      for (int m = 0; m < P; ++m) nyb[m] = BufIo<T>::ld(rb, ldo[m], sb);
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
            const auto ro = l == S ? r_ob : r_oa;
            const int so = (z - zlo) * plane_bytes;
#pragma unroll
            for (int m = 0; m < P; ++m) BufIo<T>::st(ro, sto[m], so, v[m]);
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

// KFusedPass64: the float64 pass in the buffer-addressed form of
// KFusedPass (per-tile descriptors, out-of-range offsets instead of
// masks), with the levels' in-plane neighbours in planar LDS buffers, two per
// level (level l writes buffer adv & 1, level l + 1 reads the other one a step
// later; a record of three planes per level, as the float32 pass keeps, does not
// fit 160 KiB in float64).  The z loop is unrolled by six, so both the LDS parity
// and the register ring's phase are compile-time constants and every LDS access
// is an immediate offset from one base per owned point.
template <int S, int TY, int NT>
struct KFusedPass64 {
  static constexpr int kThreads = NT;
  __device__ static void run(const double* __restrict__ ya, const double* __restrict__ yb,
                             const double* __restrict__ sv, double* __restrict__ out_a, double* __restrict__ out_b,
                             FusedCoef<double, S> cf, int nx, int ny, int nz, int zc, uint32_t tiles_x,
                             uint32_t tiles_y, uint32_t ntiles, const DevState* guard, int64_t ld, int slot0);
};
template <int S, int TY, int NT>
__device__ __forceinline__ void KFusedPass64<S, TY, NT>::run(const double* __restrict__ ya,
                                                             const double* __restrict__ yb,
                                                             const double* __restrict__ sv, double* __restrict__ out_a,
                                                             double* __restrict__ out_b, FusedCoef<double, S> cf,
                                                             int nx, int ny, int nz, int zc, uint32_t tiles_x,
                                                             uint32_t tiles_y, uint32_t ntiles, const DevState* guard,
                                                             int64_t ld, int slot0) {
  constexpr int TX = 64;
  constexpr int RX = TX + 2 * S;
  constexpr int RY = TY + 2 * S;
  constexpr int NP = RX * RY;
  constexpr int P = (NP + NT - 1) / NT;  // region points per thread
  constexpr int PAD = RX + 1;            // margin: q - RX - 1 >= 0 and q + RX + 1 < NPL for every q used
  constexpr int NPL = NP + 2 * PAD;
  __shared__ double lds[S][2][NPL];
  const int slot = slot0 + int(blockIdx.y);  // solve slot: vectors offset by slot * ld
  if (guard && guard[slot].done != kRunning) return;
  ya += slot * ld;
  yb += slot * ld;
  sv += slot * ld;
  out_a += slot * ld;
  out_b += slot * ld;
  const int tid = threadIdx.x;
  const int64_t plane = int64_t(nx) * ny;
  const int plane_bytes = int(plane * 8);
  const double sixth = 1.0 / 6.0;
  const auto r_none = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(ya), 0, 0, kBufferWord3);
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  auto ld64 = [](__amdgpu_buffer_rsrc_t r, int off, int soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
  };
  // Level l (2 .. S + 1) is needed only on region rows l - 1 .. RY - l: the rows
  // beyond are read by no point of level l + 1.  act[l - 2][m] is set when some
  // lane of the wavefront has its point m inside them (a wave-uniform test, so a
  // scalar branch): wavefronts whose points all lie outside skip the level (its
  // arithmetic, LDS writes and neighbour reads), and the others compute it at all
  // their points.  The values at points outside the rows, stale or computed from
  // stale inputs, are never read, and their global stores fall on out-of-range
  // offsets.  (A per-lane mask cost more in exec-mask instructions than it saved:
  // 159.5-160.0 against 157.6-158.3 us.)
  bool act[S][P];
#pragma unroll
  for (int m = 0; m < P; ++m) {
    const int p = tid + NT * m;
    const int ry = p / RX;
#pragma unroll
    for (int l = 2; l <= S + 1; ++l)
      act[l - 2][m] = __builtin_amdgcn_ballot_w64(p < NP && ry >= l - 1 && ry <= RY - l) != 0;
  }
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
    // descriptors as in KFusedPass
    const int zlo = zs - 1 > 0 ? zs - 1 : 0;
    const int zhi = zs + nadv - 1 < nz - 1 ? zs + nadv - 1 : nz - 1;
    const int span = (zhi - zlo + 1) * plane_bytes;
    auto tile_rsrc = [&](const double* base) {
      return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base) + plane * zlo, 0, span, kBufferWord3);
    };
    const auto r_ya = tile_rsrc(ya), r_yb = tile_rsrc(yb), r_sv = tile_rsrc(sv);
    const auto r_oa = tile_rsrc(out_a), r_ob = tile_rsrc(out_b);
    auto plane_soff = [&](int zz) { return zz >= 0 && zz < nz ? (zz - zlo) * plane_bytes : 0; };

    // owned points p = tid + NT m (as in KFusedPass): dom[m] in the grid,
    // ldo[m] / sto[m] byte offsets of loads and output stores (out of range where
    // there is nothing to do), q[m] the LDS index (the tail margin for absent points)
    int q[P], ldo[P], sto[P];
    bool dom[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
      const int p = tid + NT * m;
      const int ry = p / RX, rx = p - (p / RX) * RX;
      const int gx = x0 + rx, gy = y0 + ry;
      dom[m] = p < NP && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
      const bool inner = dom[m] && rx >= S && rx < S + TX && ry >= S && ry < S + TY;
      ldo[m] = dom[m] ? (gx + nx * gy) * 8 : kOutOfRange;
      sto[m] = inner ? (gx + nx * gy) * 8 : kOutOfRange;
      q[m] = p < NP ? p + PAD : NP + PAD;
    }
    double L[S][3][P];  // ring of the last three planes of level l at [l-1]
    double sr[S][P];    // s at the planes of levels 2..S+1 ([0] = level 2's plane)
#pragma unroll
    for (int l = 0; l < S; ++l) {
#pragma unroll
      for (int m = 0; m < P; ++m) {
        L[l][0][m] = L[l][1][m] = L[l][2][m] = 0.0;
        sr[l][m] = 0.0;
      }
    }
    double nya[P], ns[P], nyb[P];
    auto fetch = [&](int za, int zb) {
      const auto ra = za >= 0 && za < nz ? r_ya : r_none;
      const auto rs = zb >= 0 && zb < nz ? r_sv : r_none;
      const int sa = plane_soff(za), sb = plane_soff(zb);
#pragma unroll
      for (int m = 0; m < P; ++m) {
        nya[m] = ld64(ra, ldo[m], sa);
        ns[m] = ld64(rs, ldo[m], sb);
      }
    };
    auto fetch_yb = [&](int zb) {
      const auto rb = zb >= 0 && zb < nz ? r_yb : r_none;
      const int sb = plane_soff(zb);
#pragma unroll
      for (int m = 0; m < P; ++m) nyb[m] = ld64(rb, ldo[m], sb);
    };
    // One pipeline step; PH6 = adv mod 6 fixes the ring slots (PH6 mod 3) and the
    // LDS parity (PH6 mod 2): this step writes buffers PAR, reads buffers PAR ^ 1.
    auto advance = [&](auto phase, int adv) {
      constexpr int PH6 = decltype(phase)::value;
      constexpr int PH = PH6 % 3, PAR = PH6 & 1;
      constexpr int K0 = PH, K1 = (PH + 2) % 3, K2 = (PH + 1) % 3;  // newest, one below, two below
#pragma unroll
      for (int m = 0; m < P; ++m) {
        L[0][K0][m] = nya[m];
#pragma unroll
        for (int l = S - 1; l > 0; --l) sr[l][m] = sr[l - 1][m];
        sr[0][m] = ns[m];
      }
      if (adv + 1 < nadv) fetch(zs + adv + 1, zs + adv);
      double nbs[2][P];
      // level l computes plane zs + adv - (l - 1); below z0 - (S + 1 - l) no plane of the
      // next level reads it (the pipeline's first steps fill the levels from below)
      auto needed = [&](int l) { return zs + adv - (l - 1) >= z0 - (S + 1 - l); };
      auto read_sums = [&](auto level, double* out) {
        constexpr int l = decltype(level)::value;  // sums of level l - 1's plane from the previous step
        const double* b = lds[l - 2][PAR ^ 1];
        if (!needed(l)) return;
#pragma unroll
        for (int m = 0; m < P; ++m)
          if (act[l - 2][m]) out[m] = (b[q[m] - 1] + b[q[m] + 1]) + (b[q[m] - RX] + b[q[m] + RX]);
      };
      read_sums(std::integral_constant<int, 2>{}, nbs[0]);
#pragma unroll
      for (int m = 0; m < P; ++m) lds[0][PAR][q[m]] = L[0][K0][m];  // level 1: the input plane
      auto level = [&](auto lv) {
        constexpr int l = decltype(lv)::value;
        constexpr int li = l <= S ? l - 1 : 0;
        constexpr int lp = l >= 3 ? l - 3 : 0;
        const int z = zs + adv - (l - 1);
        const bool zin = z >= 0 && z < nz;
        const double a = cf.a[l - 2], b = cf.b[l - 2], c = cf.c[l - 2];
        if constexpr (l + 1 <= S + 1) read_sums(std::integral_constant<int, l + 1>{}, nbs[(l - 1) & 1]);
        if (!zin) {  // a plane outside the grid: zeros
          if constexpr (l <= S) {
#pragma unroll
            for (int m = 0; m < P; ++m) {
              L[li][K0][m] = 0.0;
              lds[li][PAR][q[m]] = 0.0;
            }
          }
        } else if (needed(l)) {
          const bool st = l >= S && z >= z0 && z < z1;
          const auto ro = l == S ? r_ob : r_oa;
          const int so = (z - zlo) * plane_bytes;
#pragma unroll
          for (int m = 0; m < P; ++m) {
            if (!act[l - 2][m]) continue;
            const double yc = L[l - 2][K1][m];
            double nb = nbs[l & 1][m];
            nb += L[l - 2][K0][m] + L[l - 2][K2][m];
            const double yprev = (l == 2) ? nyb[m] : L[lp][K2][m];
            double w = a * yc + c * (sr[l - 2][m] - (yc - nb * sixth));  // same order as EpiChebStep
            w -= b * yprev;
            const double v = dom[m] ? w : 0.0;
            if (st) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), ro, sto[m], so, 0);
            if constexpr (l <= S) {
              L[li][K0][m] = v;
              lds[li][PAR][q[m]] = v;
            }
          }
        }
      };
      level(std::integral_constant<int, 2>{});
      if (adv + 1 < nadv) fetch_yb(zs + adv);
      level(std::integral_constant<int, 3>{});
      if constexpr (S >= 3) level(std::integral_constant<int, 4>{});
      if constexpr (S >= 4) level(std::integral_constant<int, 5>{});
      __syncthreads();
    };
    fetch(zs, zs - 1);
    fetch_yb(zs - 1);
    for (int adv = 0; adv < nadv; adv += 6) {
      advance(std::integral_constant<int, 0>{}, adv);
      if (adv + 1 < nadv) advance(std::integral_constant<int, 1>{}, adv + 1);
      if (adv + 2 < nadv) advance(std::integral_constant<int, 2>{}, adv + 2);
      if (adv + 3 < nadv) advance(std::integral_constant<int, 3>{}, adv + 3);
      if (adv + 4 < nadv) advance(std::integral_constant<int, 4>{}, adv + 4);
      if (adv + 5 < nadv) advance(std::integral_constant<int, 5>{}, adv + 5);
    }
  }
}

}  // namespace pcheb

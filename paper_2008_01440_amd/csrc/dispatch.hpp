// Launch an operator kernel for the handle's operator kind with a given
// input functor and epilogue.  SCALED selects M = D^-1 A_hat (the
// preconditioner recurrence) instead of A_hat (the outer iteration).
#pragma once

#include "epilogues.hpp"
#include "handle.hpp"
#include "operators.hpp"

namespace pcheb {

#ifndef PCHEB_ST7_TY
#define PCHEB_ST7_TY 4
#endif
#ifndef PCHEB_ST7_ZC
#define PCHEB_ST7_ZC 16
#endif
// CSR: from kCsrWideRows rows on, a wavefront walks min(L, kCsrWidePasses)
// passes of 64 / L rows (L lanes per row); below, one pass.  Four passes keep
// eight nonzero slots per lane in flight in the straight-line part of KCsr
// (elasticity, L = 32: 32 passes 1270 us, 8 passes 1095 us, 4 passes 988 us,
// 2 passes 1030 us per F32 step).
constexpr int64_t kCsrWideRows = int64_t(1) << 20;
constexpr int kCsrWidePasses = 4;
constexpr int kSt7Rows = PCHEB_ST7_TY;    // grid rows per stencil tile (waves per block), 7- and 27-point
constexpr int kSt7ZChunk = PCHEB_ST7_ZC;  // planes marched per stencil tile

struct StencilGrid {
  uint32_t tiles_x, tiles_y, ntiles, grid;
};

// Tiles of 64 x rows columns by zc planes.
inline StencilGrid stencil_grid(const pcheb_operator& op, int rows, int zc) {
  StencilGrid g;
  g.tiles_x = uint32_t((op.nx + 63) / 64);
  g.tiles_y = uint32_t((op.ny + rows - 1) / rows);
  const uint32_t tz = uint32_t((op.nz + zc - 1) / zc);
  g.ntiles = g.tiles_x * g.tiles_y * tz;
  g.grid = round_grid(g.ntiles);
  return g;
}

// Tv: value type of CSR/SELL arrays (float64 for A_hat; storage type for D^-1 A_hat).
// The launch covers solve slots slot0 .. slot0 + nslots - 1: one slot per grid row
// (dimension y) for the stencils; CSR and SELL launches of several slots read the
// matrix once for every kMultiSlots of them (KCsrMulti, KSellMulti).
template <bool SCALED, class Tv, class In, class Epi>
void launch_op(const Handle& h, const Tv* csr_val, const Tv* sell_val, In in, Epi epi, int slot0, int nslots,
               hipStream_t s) {
  using acc = typename Epi::acc;
  const pcheb_operator& op = h.op;
  uint32_t grid = 0;
  switch (op.kind) {
    case PCHEB_OP_STENCIL7: {
      const StencilGrid g = stencil_grid(op, kSt7Rows, kSt7ZChunk);
      grid = g.grid;
      launch<KStencil7<SCALED, kSt7Rows, kSt7ZChunk, In, Epi>>(dim3(grid, nslots), dim3(64, kSt7Rows), 0, s, in, epi,
          op.nx, op.ny, op.nz, g.tiles_x, g.tiles_y, g.ntiles, h.rb(), slot0);
      break;
    }
    case PCHEB_OP_STENCIL27H: {
      const StencilGrid g = stencil_grid(op, kSt7Rows, kSt7ZChunk);
      grid = g.grid;
      const acc* rho = sizeof(acc) == 8 ? reinterpret_cast<const acc*>(h.rho64) : reinterpret_cast<const acc*>(h.rho_lo);
      const acc* invd = sizeof(acc) == 8 ? reinterpret_cast<const acc*>(h.invd) : reinterpret_cast<const acc*>(h.invd_lo);
      launch<KStencil27h<SCALED, kSt7Rows, kSt7ZChunk, In, Epi>>(dim3(grid, nslots), dim3(64, kSt7Rows), 0, s, in, epi,
          rho, invd, op.nx, op.ny, op.nz, g.tiles_x, g.tiles_y, g.ntiles, h.rb(), slot0);
      break;
    }
    case PCHEB_OP_CSR: {
      // min(L, kCsrWidePasses) passes per wavefront for large matrices, one for small ones
      const bool wide = h.n >= kCsrWideRows;
#define PCHEB_CSR_CASE(L)                                                                                        \
  case L: {                                                                                                      \
    constexpr int PW = L < kCsrWidePasses ? L : kCsrWidePasses;                                                  \
    const int64_t rows = int64_t(kBlock / kWave) * (wide ? PW * (kWave / L) : kWave / L);                        \
    const uint64_t tiles = uint64_t((h.n + rows - 1) / rows);                                                    \
    grid = round_grid(tiles);                                                                                    \
    if (nslots > 1) {                                                                                            \
      const dim3 mg(grid, (nslots + kMultiSlots - 1) / kMultiSlots);                                             \
      if (wide)                                                                                                  \
        launch<KCsrMulti<L, PW, Tv, In, Epi>>(mg, kBlock, 0, s, op.rowptr, op.colind, csr_val, in, epi, h.n,     \
            uint32_t(tiles), h.rb(), slot0, nslots);                                                             \
      else                                                                                                       \
        launch<KCsrMulti<L, 1, Tv, In, Epi>>(mg, kBlock, 0, s, op.rowptr, op.colind, csr_val, in, epi, h.n,      \
            uint32_t(tiles), h.rb(), slot0, nslots);                                                             \
    } else if (wide) {                                                                                           \
      launch<KCsr<L, PW, Tv, In, Epi>>(dim3(grid, 1), kBlock, 0, s, op.rowptr, op.colind, csr_val, in, epi, h.n, \
          uint32_t(tiles), h.rb(), slot0);                                                                       \
    } else {                                                                                                     \
      launch<KCsr<L, 1, Tv, In, Epi>>(dim3(grid, 1), kBlock, 0, s, op.rowptr, op.colind, csr_val, in, epi, h.n,  \
          uint32_t(tiles), h.rb(), slot0);                                                                       \
    }                                                                                                            \
    break;                                                                                                       \
  }
      switch (h.lanes) {
        PCHEB_CSR_CASE(4)
        PCHEB_CSR_CASE(8)
        PCHEB_CSR_CASE(16)
        PCHEB_CSR_CASE(32)
        default:
          PCHEB_CSR_CASE(64)
      }
#undef PCHEB_CSR_CASE
      break;
    }
    case PCHEB_OP_SELL: {
      const uint64_t tiles = uint64_t((h.nchunks + 3) / 4);
      grid = round_grid(tiles);
      if (nslots > 1)
        launch<KSellMulti<Tv, In, Epi>>(dim3(grid, (nslots + kMultiSlots - 1) / kMultiSlots), kBlock, 0, s, h.sell_ptr,
            h.sell_len, h.sell_col, sell_val, h.sell_perm, in, epi, h.n, uint32_t(tiles), h.rb(), slot0, nslots);
      else
        launch<KSell<Tv, In, Epi>>(dim3(grid, 1), kBlock, 0, s, h.sell_ptr, h.sell_len, h.sell_col, sell_val,
            h.sell_perm, in, epi, h.n, uint32_t(tiles), h.rb(), slot0);
      break;
    }
    default:
      fail(PCHEB_INVALID, "unknown operator kind");
  }
  if constexpr (Epi::reduce) {
    launch<KFinalize<Epi::NV, EpiFin<Epi>>>(nslots, kFinThreads, 0, s, EpiFin<Epi>{epi}, h.rb(), grid, epi.guard,
        slot0);
  }
}

// A_hat applied to a float64 input functor (the outer iteration and residuals).
template <class In, class Epi>
void launch_ahat(const Handle& h, In in, Epi epi, int slot0, int nslots, hipStream_t s) {
  launch_op<false, double>(h, h.op.values, h.sell_aval, in, epi, slot0, nslots, s);
}

// D^-1 A_hat applied to an input in the storage precision T.
template <class T, class In, class Epi>
void launch_bop(const Handle& h, In in, Epi epi, int slot0, int nslots, hipStream_t s) {
  launch_op<true, T>(h, reinterpret_cast<const T*>(h.csr_bval), reinterpret_cast<const T*>(h.sell_bval), in, epi,
                     slot0, nslots, s);
}

}  // namespace pcheb

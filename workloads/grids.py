"""Structured-grid SPD operators in CSR form (unscaled, i.e. the paper's A-hat).

Grid points are numbered x fastest: i = x + nx * (y + ny * z).  Columns in each
row are sorted ascending.  rowptr and colind are int32 (every workload here has
fewer than 2^31 nonzeros); values are float64.

* stencil5 / stencil7: the finite-difference Laplacian with homogeneous
  Dirichlet boundary conditions, diagonal 4 (2-D) or 6 (3-D), off-diagonals -1.
  These are the paper's Lap1600 (1598^2 interior points, Table 2) and lap3d(nx)
  (Table 6) matrices, up to the h^-2 factor that the symmetric Jacobi scaling of
  the paper removes anyway.
* harmonic27: cell-centred heterogeneous diffusion on an N^3 grid.  Every cell
  couples to its 26 neighbours (faces, edges and corners) with weight
  H(k_i, k_j) = 2 k_i k_j / (k_i + k_j), the harmonic mean of the two cell
  coefficients; a neighbour outside the domain is a ghost cell holding the
  cell's own coefficient and a zero Dirichlet value, which adds H(k_i, k_i) = k_i
  to the diagonal.  It stands in for the paper's heterogeneous FE matrices.
"""

import numpy as np
import scipy.sparse as sp

from .rng import normal


def _offsets(radius_set):
    """All (dz, dy, dx) in radius_set^3 order, lexicographic = ascending linear offset."""
    return [(dz, dy, dx) for dz in radius_set for dy in radius_set for dx in radius_set]


def _axis_valid(length, d):
    idx = np.arange(length)
    return (idx + d >= 0) & (idx + d < length)


def _structured_csr(nx, ny, nz, offsets, values_for):
    """Assemble a CSR matrix whose row i couples to i + offset for every in-range offset.

    values_for(t, valid3d) returns the (nz, ny, nx) float64 values of offset t
    (entries where valid3d is False are ignored)."""
    n = nx * ny * nz
    m = len(offsets)
    mask = np.empty((n, m), dtype=bool)
    cols = np.empty((n, m), dtype=np.int32)
    vals = np.empty((n, m), dtype=np.float64)
    rows = np.arange(n, dtype=np.int64)
    for t, (dz, dy, dx) in enumerate(offsets):
        valid = (_axis_valid(nz, dz)[:, None, None]
                 & _axis_valid(ny, dy)[None, :, None]
                 & _axis_valid(nx, dx)[None, None, :])
        mask[:, t] = valid.ravel()
        lin = dx + nx * (dy + ny * dz)
        c = rows + lin
        c[~mask[:, t]] = 0
        cols[:, t] = c.astype(np.int32)
        vals[:, t] = values_for(t, valid).ravel()
    counts = mask.sum(axis=1, dtype=np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2 ** 31:
        raise ValueError("operator has 2^31 or more nonzeros; int32 indices cannot hold it")
    colind = cols[mask]
    values = vals[mask]
    return rowptr.astype(np.int32), colind, values


def stencil7_csr(nx: int, ny: int = None, nz: int = None):
    """3-D 7-point Dirichlet Laplacian (diagonal 6, neighbours -1) on nx*ny*nz points."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    offsets = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0)]

    def vals(t, valid):
        return np.full(valid.shape, 6.0 if offsets[t] == (0, 0, 0) else -1.0)

    return _structured_csr(nx, ny, nz, offsets, vals)


def stencil5_csr(nx: int, ny: int = None):
    """2-D 5-point Dirichlet Laplacian (diagonal 4, neighbours -1) on nx*ny points."""
    ny = nx if ny is None else ny
    offsets = [(0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0)]

    def vals(t, valid):
        return np.full(valid.shape, 4.0 if offsets[t] == (0, 0, 0) else -1.0)

    return _structured_csr(nx, ny, 1, offsets, vals)


def stencil7_nnz(nx: int, ny: int = None, nz: int = None) -> int:
    """Nonzeros of stencil7_csr: 7n minus two per boundary face point per axis."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    n = nx * ny * nz
    return 7 * n - 2 * (ny * nz + nx * nz + nx * ny)


def stencil7_bounds(nx: int, ny: int = None, nz: int = None):
    """Exact extreme eigenvalues of D^-1/2 A D^-1/2 = A/6 for the 7-point Laplacian.

    The eigenvalues are 1 - (cos(pi i/(nx+1)) + cos(pi j/(ny+1)) + cos(pi l/(nz+1)))/3,
    1 <= i, j, l <= n_axis; the extremes take i = j = l = 1 and i = nx, j = ny, l = nz."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    c = (np.cos(np.pi / (nx + 1)) + np.cos(np.pi / (ny + 1)) + np.cos(np.pi / (nz + 1))) / 3.0
    return 1.0 - c, 1.0 + c


def stencil5_eigenvalues(nx: int, ny: int = None) -> np.ndarray:
    """All eigenvalues of A/4 for the 2-D 5-point Laplacian, ascending."""
    ny = nx if ny is None else ny
    cx = np.cos(np.pi * np.arange(1, nx + 1) / (nx + 1))
    cy = np.cos(np.pi * np.arange(1, ny + 1) / (ny + 1))
    lam = 1.0 - 0.5 * (cx[None, :] + cy[:, None])
    return np.sort(lam.ravel())


def harmonic27_kappa(nx: int, ny: int = None, nz: int = None, seed: int = 1, sigma: float = 2.0):
    """Per-cell coefficients kappa = exp(sigma * g), g ~ N(0,1) i.i.d. (lognormal(0, sigma)).

    Values are rounded to the nearest float32 and returned as float64, so that a
    float32 copy of them is exact and every consumer sees the same operator."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    g = normal(seed, nx * ny * nz)
    kappa = np.exp(sigma * g).astype(np.float32).astype(np.float64)
    return kappa.reshape(nz, ny, nx)


def harmonic27_csr(kappa: np.ndarray):
    """27-point harmonic-mean diffusion operator for cell coefficients kappa[z, y, x]."""
    nz, ny, nx = kappa.shape
    kp = np.zeros((nz + 2, ny + 2, nx + 2))
    kp[1:-1, 1:-1, 1:-1] = kappa
    offsets = _offsets((-1, 0, 1))
    diag = np.zeros_like(kappa)
    harm = []
    for (dz, dy, dx) in offsets:
        if (dz, dy, dx) == (0, 0, 0):
            harm.append(None)
            continue
        kn = kp[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
        inside = kn > 0.0
        h = np.where(inside, 2.0 * kappa * kn / np.where(inside, kappa + kn, 1.0), 0.0)
        diag += np.where(inside, h, kappa)
        harm.append(h)

    def vals(t, valid):
        if offsets[t] == (0, 0, 0):
            return diag
        return -harm[t]

    return _structured_csr(nx, ny, nz, offsets, vals)


def csr_diagonal(rowptr, colind, values) -> np.ndarray:
    """Diagonal entries of a CSR matrix (0 where a row stores none)."""
    n = len(rowptr) - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr.astype(np.int64)))
    d = np.zeros(n)
    on = colind == rows
    d[rows[on]] = values[on]
    return d


def rhs_from_solution(rowptr, colind, values, xstar) -> np.ndarray:
    """b = A-hat x* in float64 (the right-hand side of a manufactured solution)."""
    n = len(rowptr) - 1
    a = sp.csr_matrix((values, colind, rowptr), shape=(n, n))
    return a @ xstar

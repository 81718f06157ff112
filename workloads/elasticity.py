"""3-D linear elasticity on a regular grid of trilinear (Q1) hexahedra.

The domain is the unit cube split into (N+1)^3 equal elements with
(N+2)^3 nodes; every boundary node is clamped, which leaves N^3 free nodes with
3 displacement unknowns each (n = 3 N^3).  Element e has Young's modulus
E_e = E0 * (1 + 0.1 u_e), u_e ~ U[-1, 1] i.i.d., and Poisson ratio nu.  The
element stiffness is integrated by 2x2x2 Gauss quadrature.  Rows and columns
are numbered 3 * (x + N (y + N z)) + component over free nodes, so a full row
couples 27 nodes x 3 components = 81 unknowns.  The matrix stands in for the
paper's tetrahedral FE matrices (Cube5317k, Emilia_923), which are not
available.
"""

import numpy as np

from .rng import uniform


def q1_reference_stiffness(nu: float = 0.3) -> np.ndarray:
    """24x24 stiffness of the unit cube for E = 1 (node a = ax + 2 ay + 4 az, dof 3a + c)."""
    lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = 1.0 / (2.0 * (1.0 + nu))
    c = np.zeros((6, 6))
    c[:3, :3] = lam
    c[np.arange(3), np.arange(3)] += 2.0 * mu
    c[np.arange(3, 6), np.arange(3, 6)] = mu
    g = [0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]
    corners = [(a & 1, (a >> 1) & 1, (a >> 2) & 1) for a in range(8)]
    k = np.zeros((24, 24))
    for qz in g:
        for qy in g:
            for qx in g:
                b = np.zeros((6, 24))
                for a, (ax, ay, az) in enumerate(corners):
                    fx = qx if ax else 1.0 - qx
                    fy = qy if ay else 1.0 - qy
                    fz = qz if az else 1.0 - qz
                    sx, sy, sz = (2 * ax - 1), (2 * ay - 1), (2 * az - 1)
                    nx_, ny_, nz_ = sx * fy * fz, fx * sy * fz, fx * fy * sz
                    col = 3 * a
                    b[0, col + 0] = nx_
                    b[1, col + 1] = ny_
                    b[2, col + 2] = nz_
                    b[3, col + 1] = nz_
                    b[3, col + 2] = ny_
                    b[4, col + 0] = nz_
                    b[4, col + 2] = nx_
                    b[5, col + 0] = ny_
                    b[5, col + 1] = nx_
                k += 0.125 * b.T @ c @ b
    return k


def elasticity_q1_moduli(n_free: int, seed: int = 2, e0: float = 1.0, spread: float = 0.1) -> np.ndarray:
    """Per-element Young's moduli E0 (1 + spread * U[-1,1]) on the (N+1)^3 element grid."""
    ne = n_free + 1
    u = uniform(seed, ne ** 3, -1.0, 1.0)
    return (e0 * (1.0 + spread * u)).reshape(ne, ne, ne)


def elasticity_q1_csr(n_free: int, seed: int = 2, nu: float = 0.3, moduli: np.ndarray = None):
    """CSR (int32 rowptr/colind, float64 values) of the clamped Q1 elasticity matrix."""
    n = n_free
    h = 1.0 / (n + 1)
    kref = h * q1_reference_stiffness(nu)  # 3-D stiffness scales with the element size
    emod = elasticity_q1_moduli(n, seed) if moduli is None else moduli
    nn = n ** 3
    offsets = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    blocks = np.zeros((nn, 27, 3, 3))
    valid = np.zeros((nn, 27), dtype=bool)
    rng = np.arange(n)
    for t, (dz, dy, dx) in enumerate(offsets):
        v = (((rng + dz >= 0) & (rng + dz < n))[:, None, None]
             & ((rng + dy >= 0) & (rng + dy < n))[None, :, None]
             & ((rng + dx >= 0) & (rng + dx < n))[None, None, :])
        valid[:, t] = v.ravel()
        for az in (0, 1):
            for ay in (0, 1):
                for ax in (0, 1):
                    bx, by, bz = ax + dx, ay + dy, az + dz
                    if not (0 <= bx <= 1 and 0 <= by <= 1 and 0 <= bz <= 1):
                        continue
                    la = ax + 2 * ay + 4 * az
                    lb = bx + 2 * by + 4 * bz
                    # free node at grid coordinate i+1 sits in the element whose origin is i+1-a
                    e = emod[1 - az:1 - az + n, 1 - ay:1 - ay + n, 1 - ax:1 - ax + n].ravel()
                    blocks[:, t] += e[:, None, None] * kref[3 * la:3 * la + 3, 3 * lb:3 * lb + 3][None]
    node = np.arange(nn, dtype=np.int64)
    lin = np.array([dx + n * (dy + n * dz) for (dz, dy, dx) in offsets], dtype=np.int64)
    colnode = node[:, None] + lin[None, :]
    colnode[~valid] = 0
    # row (p, c) lists, for each valid neighbour t in ascending order, components c' = 0, 1, 2
    cols = (3 * colnode[:, None, :, None] + np.arange(3)[None, None, None, :])
    cols = np.broadcast_to(cols, (nn, 3, 27, 3))
    vals = blocks.transpose(0, 2, 1, 3)  # (node, c, t, c')
    mask = np.broadcast_to(valid[:, None, :, None], (nn, 3, 27, 3))
    colind = cols[mask].astype(np.int32)
    values = vals[mask]
    counts = mask.reshape(nn * 3, 81).sum(axis=1, dtype=np.int64)
    rowptr = np.zeros(3 * nn + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2 ** 31:
        raise ValueError("operator has 2^31 or more nonzeros; int32 indices cannot hold it")
    return rowptr.astype(np.int32), colind, values

"""Problems shared by the GPU tests: host CSR for the oracle, the device operator
for the library, and eigenvalue bounds of the scaled operator (closed form for
the Laplacian, the oracle's Lanczos otherwise, widened by 1.01)."""

import functools

import numpy as np

import oracle
import workloads as W


class Case:
    def __init__(self, name, kind, rp, ci, v, bounds, dims=None, kappa=None, sigma=1):
        self.name, self.kind = name, kind
        self.rp, self.ci, self.v = rp, ci, v
        self.n = len(rp) - 1
        self.lo, self.hi = bounds
        self.dims = dims
        self.kappa = kappa
        self.sigma = sigma

    def operator(self, torch, dev):
        import paper_2008_01440_amd as pc

        if self.kind == "stencil7":
            return pc.Operator.stencil7(*self.dims)
        if self.kind == "stencil27h":
            return pc.Operator.stencil27h(torch.from_numpy(self.kappa).to(dev))
        rp = torch.from_numpy(self.rp).to(dev)
        ci = torch.from_numpy(self.ci).to(dev)
        v = torch.from_numpy(self.v).to(dev)
        return pc.Operator.csr(rp, ci, v, sell=self.kind == "sell", sigma=self.sigma)


def lanczos_bounds(rp, ci, v, seed=7, steps=30):
    a, _ = oracle.jacobi_scale(oracle.csr(rp, ci, v))
    lo, hi = oracle.lanczos_extremes(lambda x: a @ x, W.uniform(seed, a.shape[0], 0.5, 1.5), steps)
    return lo, 1.01 * hi


@functools.lru_cache(maxsize=None)
def case(name):
    if name == "st7":  # ragged in x, y and z: 2 x-tiles, 4 y-tiles, 3 z-chunks
        dims = (67, 13, 19)
        rp, ci, v = W.stencil7_csr(*dims)
        return Case(name, "stencil7", rp, ci, v, W.stencil7_bounds(*dims), dims=dims)
    if name == "st7_cube":
        dims = (32, 32, 32)
        rp, ci, v = W.stencil7_csr(*dims)
        return Case(name, "stencil7", rp, ci, v, W.stencil7_bounds(*dims), dims=dims)
    if name == "h27":
        kappa = W.harmonic27_kappa(37, 11, 13, seed=1)
        rp, ci, v = W.harmonic27_csr(kappa)
        return Case(name, "stencil27h", rp, ci, v, lanczos_bounds(rp, ci, v), dims=(37, 11, 13), kappa=kappa)
    if name == "csr7":
        rp, ci, v = W.stencil7_csr(29, 23, 21)
        return Case(name, "csr", rp, ci, v, W.stencil7_bounds(29, 23, 21))
    if name == "csr_el":
        rp, ci, v = W.elasticity_q1_csr(9, seed=2)
        return Case(name, "csr", rp, ci, v, lanczos_bounds(rp, ci, v))
    if name == "sell_el":
        rp, ci, v = W.elasticity_q1_csr(9, seed=2)
        return Case(name, "sell", rp, ci, v, lanczos_bounds(rp, ci, v), sigma=1)
    if name == "sell_h27":  # varying row lengths, sorted in windows of 256 rows
        kappa = W.harmonic27_kappa(21, 17, 9, seed=4)
        rp, ci, v = W.harmonic27_csr(kappa)
        return Case(name, "sell", rp, ci, v, lanczos_bounds(rp, ci, v), sigma=256)
    raise KeyError(name)


ALL = ["st7", "h27", "csr7", "csr_el", "sell_el", "sell_h27"]


@functools.lru_cache(maxsize=None)
def manufactured_rhs(name, seed=0):
    c = case(name)
    xstar = W.uniform(seed, c.n, -1.0, 1.0)
    return xstar, W.rhs_from_solution(c.rp, c.ci, c.v, xstar)


@functools.lru_cache(maxsize=None)
def oracle_solve(name, k, s, flexible, tol=1e-8):
    c = case(name)
    _, b = manufactured_rhs(name)
    return oracle.nc_pcg(c.rp, c.ci, c.v, b, c.lo, c.hi, k, s=s, tol=tol, flexible=flexible)


def rel_inf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))

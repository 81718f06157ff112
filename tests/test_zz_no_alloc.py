"""The allocation-free Lanczos estimator (pcheb_estimate_bounds_noalloc) against the
allocating one (pcheb_estimate_bounds) and the FP64 oracle, on consecutive calls
that reuse the library's scratch array with smaller inputs after larger ones.

Bar: the same kernels on the same grids in the same order, so the two entry points
agree bit for bit; against the oracle the Lanczos bar of the parity tests (1e-9
relative on both Ritz values)."""

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_cases import case

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
SCRATCH = 128 << 20


@pytest.fixture(scope="module")
def pc():
    import paper_2008_01440_amd as pc
    pc.load_library()
    return pc


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _workspace(n, steps, d):
    """Workspace bytes the header states for the allocation-free estimator."""
    m = min(steps, n)
    return 8 * ((m + 1) * ((n + 1) // 2 * 2) + (2 + d) * n + 3 * m + 3) + 524288


def _check(pc, op, rp, ci, v, steps):
    n = len(rp) - 1
    v0 = W.uniform(7, n, 0.5, 1.5)
    a, _ = oracle.jacobi_scale(oracle.csr(rp, ci, v))
    lo_ref, hi_ref = oracle.lanczos_extremes(lambda x: a @ x, v0, steps)
    v0t = _t(v0)
    lo_a, hi_a = pc.pcheb_estimate_bounds(op, v0t, steps)
    lo_n, hi_n = pc.pcheb_estimate_bounds_noalloc(op, v0t, steps)
    torch.cuda.synchronize()
    print(f"noalloc n={n} steps={steps}: [{lo_n!r}, {hi_n!r}] alloc [{lo_a!r}, {hi_a!r}] "
          f"oracle [{lo_ref!r}, {hi_ref!r}]", flush=True)
    assert (lo_n, hi_n) == (lo_a, hi_a)
    assert abs(lo_n - lo_ref) <= 1e-9 * abs(lo_ref) and abs(hi_n - hi_ref) <= 1e-9 * hi_ref


def test_noalloc_bounds_consecutive_calls(pc):
    """Largest first, then smaller inputs of other kinds: each call finds the scratch
    holding the previous call's values."""
    dims = (78, 77, 79)  # 474,474 unknowns: close to the 7-point limit of 30 steps
    assert _workspace(78 * 77 * 79, 30, 0) + 2048 <= SCRATCH
    rp, ci, v = W.stencil7_csr(*dims)
    _check(pc, pc.Operator.stencil7(*dims), rp, ci, v, 30)
    c = case("h27")  # 5,291 cells, 27-point (diagonal and 1/(2 kappa) also in the scratch)
    _check(pc, c.operator(torch, DEV), c.rp, c.ci, c.v, 30)
    c = case("csr_el")  # 2,187 rows of elasticity CSR
    _check(pc, c.operator(torch, DEV), c.rp, c.ci, c.v, 30)
    dims = (3, 2, 1)  # Krylov space exhausted after 6 steps
    rp, ci, v = W.stencil7_csr(*dims)
    _check(pc, pc.Operator.stencil7(*dims), rp, ci, v, 12)


def test_noalloc_bounds_rejects_oversize(pc):
    """An operator whose workspace exceeds the scratch is refused before any work."""
    n1 = 80
    n = n1 ** 3
    assert _workspace(n, 30, 0) > SCRATCH
    v0 = torch.ones(n, dtype=torch.float64, device=DEV)
    with pytest.raises(pc.PchebError) as e:
        pc.pcheb_estimate_bounds_noalloc(pc.Operator.stencil7(n1), v0, 30)
    assert e.value.name == "INVALID" and "workspace" in str(e.value)
    # the entry point still works afterwards
    dims = (9, 8, 7)
    rp, ci, v = W.stencil7_csr(*dims)
    _check(pc, pc.Operator.stencil7(*dims), rp, ci, v, 30)

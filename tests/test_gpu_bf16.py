"""bfloat16 recurrences at the highest supported degree (k = 32) against the FP64 oracle, and the
refusal above it.  Bar: iterations within +-2 of the oracle and a relative solution difference
<= 1e-6 (the solves' bars); the refused range is documented by a skipped case."""

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


@pytest.fixture(scope="module")
def pc():
    import paper_2008_01440_amd as pc
    pc.load_library()
    return pc


@pytest.mark.parametrize("fuse", [1, 4])
def test_bf16_at_degree_cap_matches_oracle(pc, fuse):
    """7-point Poisson 96^3, k = 32, flexible PCG, closed-form bounds on both sides."""
    N, k = 96, 32
    rp, ci, v = W.stencil7_csr(N)
    n = N ** 3
    xs = W.uniform(0, n, -1.0, 1.0)
    b = W.rhs_from_solution(rp, ci, v, xs)
    lo, hi = W.stencil7_bounds(N)
    ref = oracle.nc_pcg(rp, ci, v, b, lo, hi, k, s=1.001, tol=1e-8, flexible=True)
    with pc.pcheb_setup(pc.Operator.stencil7(N), k, lo, hi, 1.001, "bf16", fuse_steps=fuse) as h:
        x = torch.zeros(n, dtype=torch.float64, device=DEV)
        st = pc.pcg_solve(h, torch.from_numpy(b).to(DEV), x, tol=1e-8, flexible=True)
    diff = float(np.linalg.norm(x.cpu().numpy() - ref.x_hat) / np.linalg.norm(ref.x_hat))
    print(f"bf16 k={k} S={fuse}: GPU {st['iters']} it, oracle {ref.iters} it, rel diff {diff:.2e}", flush=True)
    assert st["status"] == "OK" and abs(st["iters"] - ref.iters) <= 2 and diff <= 1e-6
    assert st["relres_true"] <= 1.02e-8


def test_bf16_above_cap_is_refused(pc):
    with pytest.raises(pc.PchebError) as e:
        pc.pcheb_setup(pc.Operator.stencil7(16), 33, 0.01, 2.0, 1.001, "bf16")
    assert e.value.name == "INVALID" and "bfloat16" in str(e.value)


@pytest.mark.skip(reason="refused by pcheb_setup: a bfloat16 recurrence of degree 100 on the 256^3 7-point "
                         "problem took 13 PCG iterations against 9 (float64) and ended 2.2e-6 from the "
                         "float64 solution, outside the +-2 / 1e-6 bars")
def test_bf16_degree_100_unsupported():
    pass

"""All of the library's device memory through a caller's allocator (pcheb_set_allocator):
counting callbacks backed by PyTorch's caching allocator see every block of a bound
estimate, a set-up and solve, a work list, a served request and the releases; the device's free
memory drops by no more than the caller's pool grows; every block comes back; and the
allocation-free estimator calls the allocator not at all."""

import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
MIB = 1 << 20


@pytest.fixture(scope="module")
def pc():
    import paper_2008_01440_amd as pc
    pc.load_library()
    return pc


def test_every_device_block_goes_through_the_allocator(pc):
    N = 128  # 27-point cells: the F32 operator copies and a solve workspace of about 200 MB
    n = N ** 3
    kappa = torch.from_numpy(W.harmonic27_kappa(N, N, N, seed=1)).to(DEV)
    op = pc.Operator.stencil27h(kappa)
    v0 = torch.empty(n, dtype=torch.float64, device=DEV)
    pc.pcheb_fill_uniform(v0, 7, 0.5, 1.5)
    xs = torch.empty_like(v0)
    pc.pcheb_fill_uniform(xs, 0, -1.0, 1.0)
    b = torch.empty_like(v0)
    # with hipMalloc first: the reference values, and the library's code object loaded before measuring
    lo_ref, hi_ref = pc.pcheb_estimate_bounds(op, v0, 30)
    with pc.pcheb_setup(op, 0, lo_ref, 1.01 * hi_ref) as h0:
        pc.pcheb_matvec(h0, xs, b)
    x_ref = torch.zeros_like(b)
    with pc.pcheb_setup(op, 20, lo_ref, 1.01 * hi_ref, 1.001, "f32") as h1:
        st_ref = pc.pcg_solve(h1, b, x_ref, tol=1e-8, flexible=True)
    torch.cuda.synchronize()

    al = pc.TorchCachingAllocator()
    pc.pcheb_set_allocator(al)
    try:
        lo, hi = pc.pcheb_estimate_bounds(op, v0, 30)
        assert (lo, hi) == (lo_ref, hi_ref)
        assert al.n_alloc >= 5 and not al.live, (al.n_alloc, al.live)  # the Lanczos workspace came and went
        print(f"estimate: {al.n_alloc} blocks, {al.bytes_alloc / MIB:.0f} MiB", flush=True)

        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        res0 = torch.cuda.memory_reserved()
        h = pc.pcheb_setup(op, 20, lo, 1.01 * hi, 1.001, "f32")
        x = torch.zeros_like(b)
        st = pc.pcg_solve(h, b, x, tol=1e-8, flexible=True)
        torch.cuda.synchronize()
        live = sum(al.live.values())
        used = free0 - torch.cuda.mem_get_info()[0]
        grew = torch.cuda.memory_reserved() - res0
        print(f"solve: {len(al.live)} live blocks, {live / MIB:.0f} MiB; device free memory -{used / MIB:.0f} MiB, "
              f"torch pool +{grew / MIB:.0f} MiB", flush=True)
        assert st["status"] == "OK" and st["iters"] == st_ref["iters"] and torch.equal(x, x_ref)
        assert live >= pc.pcheb_footprint_bytes(op, 20, lo, 1.01 * hi, 1.001, "f32") - 4 * MIB
        assert used <= grew + 64 * MIB  # nothing the size of the workspace beside the caller's pool
        pc.pcheb_destroy(h)
        assert not al.live

        # a served request: group workspace, staging and the server's Lanczos start vector
        before = al.n_alloc
        with pc.Server(4 << 30, 2) as srv:
            xsv = torch.zeros_like(b)
            rid = srv.submit(op, b, xsv, 20, prec="f32")  # bounds estimated by the server
            out = srv.wait(rid)
        assert out["status"] == "OK", out
        assert al.n_alloc > before + 5
        assert not al.live and al.n_alloc == al.n_free, (al.n_alloc, al.n_free)

        # a work list over two handles: its argument tables and state buffers come and go too
        before = al.n_alloc
        hs = [pc.pcheb_setup(op, 20, lo, 1.01 * hi, 1.001, "f32") for _ in range(2)]
        with pc.pcheb_group_create(hs) as g:
            B = torch.zeros((2, n), dtype=torch.float64, device=DEV)
            B[0] = b
            B[1] = b
            X = torch.zeros_like(B)
            sts = pc.pcg_solve_group(g, B, X, tol=1e-8, flexible=True)
        assert all(s["status"] == "OK" for s in sts) and torch.equal(X[0], x_ref) and torch.equal(X[1], x_ref)
        for hh in hs:
            pc.pcheb_destroy(hh)
        assert al.n_alloc >= before + 4 and not al.live, (al.n_alloc - before, al.live)

        # the allocation-free estimator takes nothing from the allocator
        before = al.n_alloc
        small = pc.Operator.stencil7(40)
        pc.pcheb_estimate_bounds_noalloc(small, torch.ones(40 ** 3, dtype=torch.float64, device=DEV), 30)
        assert al.n_alloc == before
    finally:
        pc.pcheb_set_allocator(None)
    # hipMalloc again
    with pc.pcheb_setup(op, 5, lo, 1.01 * hi) as h2:
        pc.pcheb_apply(h2, b, xs)
    torch.cuda.synchronize()
    assert al.n_alloc == al.n_free

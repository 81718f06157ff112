"""The C/OpenMP FP64 oracle (oracle/nc_omp.c) against what the paper and mathematics fix, and against
the numpy oracle (CPU only).  Planted mistakes, compiled into separate builds of the same source,
must each fail one of these pins."""

import os
import shutil
import subprocess

import numpy as np
import pytest

import pins
import workloads as W
from oracle import nc as O
from oracle import omp

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None and shutil.which("cc") is None,
                                reason="no C compiler")


def check_unscaled_apply_closed_form(lib=None):
    """D^-1/2 p_k(A) D^-1/2 r_hat on A_hat = S L S (L the scaled 7-point Laplacian, S a non-constant
    positive diagonal): for r_hat = S u with L u = lam u the result is S^-1 p_k(lam) u (eq. cheb)."""
    nx, ny, nz = 7, 6, 5
    rp, ci, v = W.stencil7_csr(nx, ny, nz)
    n = len(rp) - 1
    sd = W.uniform(21, n, 0.5, 2.0)
    rows = np.repeat(np.arange(n), np.diff(rp.astype(np.int64)))
    vh = v / 6.0 * sd[rows] * sd[ci]
    _, eig, mode = pins._scaled_stencil7(nx, ny, nz)
    lo, hi = W.stencil7_bounds(nx, ny, nz)
    for s in (1.0, 1.001, 1.01):
        for k in (0, 1, 2, 5, 12, 31):
            for m in [(1, 1, 1), (7, 6, 5), (3, 2, 4)]:
                u = mode(*m)
                z = omp.nc_apply_unscaled(rp, ci, vh, sd * u, lo, hi, k, s, lib=lib)
                expect = float(pins.closed_form_pk(eig(*m), lo, hi, k, s)) * u / sd
                assert np.abs(z - expect).max() <= 1e-11 * np.abs(expect).max(), (s, k, m)


def check_dense_solve(lib=None):
    """PCG solves a random SPD system (dense reference), Fletcher-Reeves and flexible beta."""
    rng = np.random.default_rng(5)
    n = 60
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    a = q @ np.diag(np.geomspace(1.0, 1e3, n)) @ q.T
    a = 0.5 * (a + a.T)
    rp = np.arange(0, n * n + 1, n, dtype=np.int32)
    ci = np.tile(np.arange(n, dtype=np.int32), n)
    b = rng.standard_normal(n)
    d = np.diag(a)
    ev = np.linalg.eigvalsh(a / np.sqrt(np.outer(d, d)))
    x = np.linalg.solve(a, b)
    for flexible in (False, True):
        res = omp.nc_pcg(rp, ci, a.ravel(), b, ev[0], ev[-1], 5, tol=1e-12, maxit=500, flexible=flexible, lib=lib)
        assert res.converged and np.abs(res.x_hat - x).max() <= 1e-8 * np.abs(x).max(), flexible
        assert res.relres_true_hat <= 1e-9


def check_counting_identities(lib=None):
    """Table 3: A x v = (m + 1) iter and ddot = 3 iter (Fletcher-Reeves; flexible adds one per iteration
    but the last)."""
    rp, ci, v = W.stencil7_csr(9, 8, 7)
    lo, hi = W.stencil7_bounds(9, 8, 7)
    b = W.uniform(2, len(rp) - 1, -1.0, 1.0)
    for m in (0, 1, 3, 7):
        res = omp.nc_pcg(rp, ci, v, b, lo, hi, m, tol=1e-8, lib=lib)
        assert res.converged and res.n_spmv == (m + 1) * res.iters and res.n_dot == 3 * res.iters, m
        fl = omp.nc_pcg(rp, ci, v, b, lo, hi, m, tol=1e-8, flexible=True, lib=lib)
        assert fl.n_dot == 4 * fl.iters - 1, m
        # the stop test is relative: scaling b scales x and changes nothing else
        big = omp.nc_pcg(rp, ci, v, 1e6 * b, lo, hi, m, tol=1e-8, lib=lib)
        assert big.iters == res.iters and np.abs(big.x_hat - 1e6 * res.x_hat).max() <= 1e-6 * np.abs(big.x_hat).max()


def check_matches_numpy_oracle(lib=None):
    """Same iterations and solutions to rounding as oracle.nc (27-point harmonic and elasticity CSR)."""
    kappa = W.harmonic27_kappa(9, 8, 7, seed=1)
    cases = [W.harmonic27_csr(kappa), W.elasticity_q1_csr(4, seed=2)]
    for rp, ci, v in cases:
        n = len(rp) - 1
        a, _ = O.jacobi_scale(O.csr(rp, ci, v))
        ev = np.linalg.eigvalsh(a.toarray())
        b = W.uniform(3, n, -1.0, 1.0)
        for flexible in (False, True):
            ref = O.nc_pcg(rp, ci, v, b, ev[0], 1.01 * ev[-1], 6, flexible=flexible)
            res = omp.nc_pcg(rp, ci, v, b, ev[0], 1.01 * ev[-1], 6, flexible=flexible, lib=lib)
            assert res.iters == ref.iters and res.n_spmv == ref.n_spmv and res.n_dot == ref.n_dot
            assert np.abs(res.x_hat - ref.x_hat).max() <= 1e-12 * np.abs(ref.x_hat).max()
            assert abs(res.relres_true - ref.relres_true) <= 1e-6 * ref.relres_true


ALL = [check_unscaled_apply_closed_form, check_dense_solve, check_counting_identities, check_matches_numpy_oracle]


@pytest.mark.parametrize("check", ALL, ids=[c.__name__ for c in ALL])
def test_omp_oracle_pins(check):
    omp.set_threads(4)
    check()


def test_thread_count_only_changes_rounding():
    """1, 3 and 8 threads: the same iterations, solutions equal to rounding; repeated runs with one
    thread count agree bit for bit."""
    rp, ci, v = W.stencil7_csr(20, 19, 18)
    lo, hi = W.stencil7_bounds(20, 19, 18)
    b = W.uniform(4, len(rp) - 1, -1.0, 1.0)
    out = []
    for t in (1, 3, 8):
        omp.set_threads(t)
        out.append(omp.nc_pcg(rp, ci, v, b, lo, hi, 10, flexible=True))
    for r in out[1:]:
        assert r.iters == out[0].iters and np.abs(r.x_hat - out[0].x_hat).max() <= 1e-12
    # deterministic for a given thread count
    assert np.array_equal(out[-1].x_hat, omp.nc_pcg(rp, ci, v, b, lo, hi, 10, flexible=True).x_hat)
    omp.set_threads(4)


def test_progress_lines_report_without_changing_the_solve(capfd):
    """set_progress only prints: the same bits with and without it, one line per iteration."""
    rp, ci, v = W.stencil7_csr(12, 11, 10)
    lo, hi = W.stencil7_bounds(12, 11, 10)
    b = W.uniform(6, len(rp) - 1, -1.0, 1.0)
    omp.set_threads(2)
    quiet = omp.nc_pcg(rp, ci, v, b, lo, hi, 5, flexible=True)
    omp.set_progress(1)
    try:
        loud = omp.nc_pcg(rp, ci, v, b, lo, hi, 5, flexible=True)
    finally:
        omp.set_progress(0)
        omp.set_threads(4)
    lines = [ln for ln in capfd.readouterr().err.splitlines() if ln.startswith("oracle iteration")]
    assert np.array_equal(quiet.x_hat, loud.x_hat) and quiet.iters == loud.iters
    assert len(lines) == loud.iters and lines[-1].startswith(f"oracle iteration {loud.iters}:")


MUTANTS = [
    ("c->rho[j] = 1.0 / (2.0 * c->sigma - c->rho[j - 1]);", "c->rho[j] = 1.0 / (2.0 * c->sigma + c->rho[j - 1]);",
     "rho recurrence sign"),
    ("c->theta = s * theta0;", "c->theta = theta0;", "modified parameter ignored"),
    ("x_new[i] = rj * (ts * x[i] - rj1 * x_old[i] + zz);", "x_new[i] = rj * (ts * x[i] + zz);",
     "dropped three-term history"),
    ("const double zz = td * (r[i] - t[i]);", "const double zz = td * (r[i] + t[i]);", "sign of the residual term"),
    ("sval[j] = dm[i] * ah->val[j] * dm[ah->col[j]];", "sval[j] = dm[i] * ah->val[j] * dm[i];",
     "one-sided scaling"),
    ("z_hat[i] = dm[i] * w[n + i];", "z_hat[i] = w[n + i];", "unscaled apply without the outer D^-1/2"),
    ("const double alpha = gamma / pq;", "const double alpha = pq / gamma;", "alpha inverted"),
    ("t[i] = r[i] - r_old[i];", "t[i] = r[i] + r_old[i];", "flexible beta sign"),
    ("if (relres < tol) {", "if (rnorm < tol) {", "absolute stop test"),
    ("x_hat[i] = dm[i] * x[i];", "x_hat[i] = x[i] / dm[i];", "solution mapped back with D^1/2"),
]


@pytest.mark.parametrize("old,new,what", MUTANTS, ids=[m[2] for m in MUTANTS])
def test_omp_pins_reject_mutant(tmp_path, old, new, what):
    src = open(os.path.join(os.path.dirname(omp.__file__), "nc_omp.c")).read()
    assert src.count(old) == 1, what
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    cc = shutil.which("gcc") or shutil.which("cc")
    subprocess.run([cc, "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", str(path), "-o", str(so), "-lm"],
                   check=True)
    lib = omp.load(str(so))
    lib.ncomp_set_threads(2)
    caught = None
    for check in ALL:
        try:
            check(lib)
        except Exception as exc:  # AssertionError, or the mutant failing outright
            caught = (check.__name__, type(exc).__name__)
            break
    assert caught is not None, f"no pin rejects the mutant '{what}'"

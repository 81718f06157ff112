"""Checks that pin the FP64 oracle to facts fixed by the paper and by mathematics.

Each check looks the oracle's functions up at call time (``O.name``), so the
pin-strength tests can substitute a deliberately wrong variant of one oracle
function and show that some check rejects it.  Every check raises
AssertionError on failure.
"""

import os

import mpmath
import numpy as np

import workloads as W
from oracle import nc as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

mpmath.mp.dps = 50


def cheb_T(n, x):
    """Chebyshev polynomial of the first kind by its trigonometric/hyperbolic closed form."""
    x = mpmath.mpf(x)
    if abs(x) <= 1:
        return mpmath.cos(n * mpmath.acos(x))
    if x > 1:
        return mpmath.cosh(n * mpmath.acosh(x))
    return (-1) ** n * mpmath.cosh(n * mpmath.acosh(-x))


def closed_form_pk(lam, lambda_min, lambda_max, k, s):
    """p_k(lam) = (1 - T_{k+1}((theta' - lam)/delta) / T_{k+1}(theta'/delta)) / lam (eqs. cheb, qT)."""
    theta = mpmath.mpf(s) * (mpmath.mpf(lambda_max) + mpmath.mpf(lambda_min)) / 2
    delta = (mpmath.mpf(lambda_max) - mpmath.mpf(lambda_min)) / 2
    lam = mpmath.mpf(lam)
    q = cheb_T(k + 1, (theta - lam) / delta) / cheb_T(k + 1, theta / delta)
    return (1 - q) / lam


def read_table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_comp80.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            side, m, it, mumax, mumin, l, kappa = line.split()
            rows.append(dict(s=1.0 if side == "exact" else 1.01, m=int(m), iter=int(it),
                             mu_max=float(mumax), mu_min=float(mumin), l=int(l), kappa=float(kappa)))
    return rows


def _printed_match(value, printed_text_value, rel=None):
    """True if value rounds to the printed number (4-5 significant digits)."""
    rel = 6e-5 if rel is None else rel
    return abs(value - printed_text_value) <= rel * abs(printed_text_value) + 0.051 * 10 ** np.floor(
        np.log10(abs(printed_text_value)) - 3)


# --------------------------------------------------------------------------- scalars

def check_rho_closed_form():
    """rho_j = sigma_j / sigma_{j+1} = T_j(sigma) / T_{j+1}(sigma) (Sec. 3, eq. rhocheb)."""
    for lmin, lmax, s in [(4.5e-3, 1.9955, 1.0), (4.5e-3, 1.9955, 1.001), (0.1, 1.9, 1.01), (1e-4, 2.0, 1.0)]:
        k = 100
        c = O.chebyshev_scalars(lmin, lmax, k, s)
        sigma = s * (lmax + lmin) / (lmax - lmin)
        assert abs(c.sigma - sigma) <= 1e-14 * sigma
        for j in range(k + 1):
            exact = cheb_T(j, mpmath.mpf(s) * (mpmath.mpf(lmax) + lmin) / (mpmath.mpf(lmax) - lmin))
            exact = exact / cheb_T(j + 1, mpmath.mpf(s) * (mpmath.mpf(lmax) + lmin) / (mpmath.mpf(lmax) - lmin))
            assert abs(c.rho[j] - float(exact)) <= 1e-13 * float(exact), (lmin, lmax, s, j)


def check_zeta_closed_form():
    """Theorem 2: zeta_0 = 1/theta' and zeta_j = 2 T_{2^(j-1)}(sigma)^2 / T_{2^j}(sigma)."""
    for lmin, lmax, s in [(4.5e-3, 1.9955, 1.0), (0.05, 1.95, 1.01), (1e-3, 2.0, 1.001)]:
        zeta = O.newton_zetas(lmin, lmax, 7, s)
        theta = s * (lmax + lmin) / 2
        sigma = mpmath.mpf(s) * (mpmath.mpf(lmax) + lmin) / (mpmath.mpf(lmax) - lmin)
        assert abs(zeta[0] - 1.0 / theta) <= 1e-15 / theta
        for j in range(1, 8):
            exact = 2 * cheb_T(2 ** (j - 1), sigma) ** 2 / cheb_T(2 ** j, sigma)
            assert abs(zeta[j] - float(exact)) <= 1e-13 * float(exact), (s, j)


# --------------------------------------------------------------------------- polynomial

def check_poly_closed_form():
    """p_k(A) applied to diagonal matrices equals the scalar polynomial of eq. cheb at each eigenvalue."""
    lmin, lmax = 4.528077e-3, 1.995471923
    lam = np.concatenate([[lmin, lmax, 0.5 * (lmin + lmax)], W.uniform(11, 37, lmin, lmax),
                          W.uniform(12, 4, 0.2 * lmin, lmin)])
    for s in (1.0, 1.001, 1.01):
        for k in (0, 1, 2, 3, 4, 7, 10, 31, 64, 100):
            c = O.chebyshev_scalars(lmin, lmax, k, s)
            p = O.chebyshev_apply(lambda v: lam * v, np.ones_like(lam), c, k)
            for i, l in enumerate(lam):
                exact = float(closed_form_pk(l, lmin, lmax, k, s))
                assert abs(p[i] - exact) <= 1e-10 * abs(exact), (s, k, l, p[i], exact)


def check_equioscillation():
    """max over [alpha', beta'] of |1 - lam p_k(lam)| = 1 / T_{k+1}(sigma') (min-max property, eq. maxmin)."""
    lmin, lmax = 0.02, 1.98
    for s in (1.0, 1.01):
        for k in (1, 4, 9, 20):
            c = O.chebyshev_scalars(lmin, lmax, k, s)
            grid = np.linspace(c.alpha, c.beta, 20001)
            p = O.chebyshev_apply(lambda v: grid * v, np.ones_like(grid), c, k)
            dev = np.abs(1.0 - grid * p).max()
            bound = 1.0 / float(cheb_T(k + 1, c.sigma))
            assert abs(dev - bound) <= 1e-6 * bound + 1e-14, (s, k, dev, bound)


def check_newton_equals_chebyshev():
    """Theorem 2: the Newton recursion (Alg. 1) and the Chebyshev recurrence (Alg. 2) give the same P."""
    rp, ci, v = W.stencil5_csr(16, 13)
    a, _ = O.jacobi_scale(O.csr(rp, ci, v))
    ev = np.linalg.eigvalsh(a.toarray())
    r = W.uniform(21, a.shape[0], -1.0, 1.0)
    for s in (1.0, 1.001, 1.01):
        for nlev in range(0, 7):
            k = 2 ** nlev - 1
            zc = O.chebyshev_apply(lambda x: a @ x, r, O.chebyshev_scalars(ev[0], ev[-1], k, s), k)
            zn = O.newton_apply(lambda x: a @ x, r, O.newton_zetas(ev[0], ev[-1], nlev, s), nlev)
            assert np.abs(zc - zn).max() <= 1e-11 * np.abs(zc).max(), (s, nlev)


def check_hotelling():
    """Newton for X^-1 = A: ||I - P_j A|| <= ||I - P_0 A||^(2^j) (Sec. 2, eq. newtonP)."""
    g = W.normal(31, 30 * 30).reshape(30, 30)
    a = g @ g.T / 30 + 0.5 * np.eye(30)
    ev = np.linalg.eigvalsh(a)
    p = np.eye(30) * (2.0 / (ev[0] + ev[-1]))
    e0 = np.linalg.norm(np.eye(30) - p @ a, 2)
    assert e0 < 1
    for j in range(1, 6):
        p = O.hotelling_step(p, a)
        ej = np.linalg.norm(np.eye(30) - p @ a, 2)
        assert ej <= e0 ** (2 ** j) * (1 + 1e-8) + 1e-13, (j, ej, e0 ** (2 ** j))


def check_table1_spectrum():
    """Table 1: mu_max, mu_min, l and kappa of P_m A for the 78^2 Laplacian, exact and theta*1.01."""
    lam = W.stencil5_eigenvalues(78)
    for row in read_table1():
        mu = O.preconditioned_spectrum(lam, lam[0], lam[-1], row["m"], row["s"])
        assert _printed_match(mu.max(), row["mu_max"]), (row, mu.max())
        assert _printed_match(mu.min(), row["mu_min"]), (row, mu.min())
        assert O.cluster_indicator(mu) == row["l"], (row, O.cluster_indicator(mu))
        assert abs(mu.max() / mu.min() - row["kappa"]) <= 0.051 + 1e-4 * row["kappa"], (row, mu.max() / mu.min())


def check_table1_iterations(band=0.15):
    """Table 1 iteration counts, soft: the RHS is not printed; b ~ U[0,1] (seed 0), x0 = 0, tol 1e-8."""
    rp, ci, v = W.stencil5_csr(78)
    lam = W.stencil5_eigenvalues(78)
    b = W.uniform(0, len(rp) - 1)
    for row in read_table1():
        res = O.nc_pcg(rp, ci, v, b, lam[0], lam[-1], row["m"], s=row["s"], tol=1e-8)
        assert res.converged
        assert abs(res.iters - row["iter"]) <= band * row["iter"] + 1, (row, res.iters)


# --------------------------------------------------------------------------- solver

def _random_spd(n, seed, cond=1e3):
    g = W.normal(seed, n * n).reshape(n, n)
    q, _ = np.linalg.qr(g)
    ev = np.geomspace(1.0, cond, n)
    a = (q * ev) @ q.T
    a = 0.5 * (a + a.T)
    return a


def _dense_to_csr(a):
    import scipy.sparse as sp
    m = sp.csr_matrix(a)
    return m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data


def check_dense_solve():
    """NC-PCG reaches the solution of a dense direct solve on small SPD systems."""
    for n, seed, k, flexible in [(40, 1, 0, False), (60, 2, 3, False), (80, 3, 10, True), (50, 4, 7, True)]:
        a = _random_spd(n, seed)
        rp, ci, v = _dense_to_csr(a)
        d = np.diag(a)
        ev = np.linalg.eigvalsh(a / np.sqrt(np.outer(d, d)))
        b = W.uniform(seed + 100, n, -1.0, 1.0)
        res = O.nc_pcg(rp, ci, v, b, ev[0], ev[-1] * 1.01, k, s=1.001, tol=1e-13, maxit=2000,
                       flexible=flexible)
        x = np.linalg.solve(a, b)
        assert res.converged
        assert np.linalg.norm(res.x_hat - x) <= 1e-9 * np.linalg.norm(x), (n, k)


def check_finite_termination():
    """CG on an operator with q distinct eigenvalues converges in at most q iterations."""
    for q, k, flexible in [(5, 0, False), (6, 3, False), (4, 10, True), (7, 1, True)]:
        levels = np.linspace(0.3, 1.7, q)
        eigs = np.repeat(levels, 9)
        b = W.uniform(40 + q, eigs.size, 0.5, 1.5)
        c = O.chebyshev_scalars(0.3, 1.7 * 1.01, k, 1.0)
        res = O.pcg(lambda x: eigs * x, b, lambda r: O.chebyshev_apply(lambda x: eigs * x, r, c, k),
                    tol=1e-10, maxit=50, flexible=flexible)
        assert res.converged and res.iters <= q, (q, k, res.iters)
        assert np.abs(res.x - b / eigs).max() <= 1e-8 * np.abs(b / eigs).max()


def check_flexible_local_orthogonality():
    """Flexible (Polak-Ribiere) beta keeps (p_{i+1}, A p_i) = 0 when the preconditioner changes
    every iteration (Golub & Ye 1999); Fletcher-Reeves does not."""
    eigs = np.geomspace(0.01, 2.0, 300)
    b = W.uniform(50, eigs.size, -1.0, 1.0)
    calls = {"n": 0}

    def varying_precond(r):
        calls["n"] += 1
        return W.uniform(1000 + calls["n"], r.size, 0.5, 1.5) * r

    def worst_coupling(flexible):
        seen = []

        def matvec(x):
            seen.append(x.copy())
            return eigs * x

        calls["n"] = 0
        O.pcg(matvec, b, varying_precond, tol=1e-12, maxit=25, flexible=flexible)
        worst = 0.0
        for p0, p1 in zip(seen[:-1], seen[1:]):
            na = np.sqrt(p0 @ (eigs * p0)) * np.sqrt(p1 @ (eigs * p1))
            worst = max(worst, abs(p1 @ (eigs * p0)) / na)
        return worst

    assert worst_coupling(True) <= 1e-12
    assert worst_coupling(False) >= 1e-3


def check_counting_identities():
    """Table 3: ddot = 3 iter and A x v = (m + 1) iter for Fletcher-Reeves PCG from x0 = 0."""
    rp, ci, v = W.stencil7_csr(12)
    lo, hi = W.stencil7_bounds(12)
    b = W.uniform(3, len(rp) - 1)
    for m in (0, 1, 3, 7, 15):
        res = O.nc_pcg(rp, ci, v, b, lo, hi, m, s=1.001, tol=1e-8)
        assert res.converged
        assert res.n_dot == 3 * res.iters, (m, res.n_dot, res.iters)
        assert res.n_spmv == (m + 1) * res.iters, (m, res.n_spmv, res.iters)


def check_lanczos_exact_small():
    """Lanczos with full reorthogonalisation is exact once it spans the space (n <= steps)."""
    eigs = np.linspace(0.01, 1.99, 20) ** 1.5
    lo, hi = O.lanczos_extremes(lambda x: eigs * x, W.uniform(9, 20, 0.5, 1.5), 30)
    assert abs(lo - eigs.min()) <= 1e-10 and abs(hi - eigs.max()) <= 1e-10
    # interlacing: fewer steps stay inside the spectrum
    eigs = np.linspace(0.01, 1.99, 500)
    lo, hi = O.lanczos_extremes(lambda x: eigs * x, W.uniform(10, 500, 0.5, 1.5), 12)
    assert eigs.min() <= lo < hi <= eigs.max()


def check_indefinite_breakdown():
    """An upper bound below lambda_max makes odd-degree p_k(A) A indefinite (follows from eq. cheb:
    for even k + 1, 1 - q_{k+1}(lam) < 0 once lam > alpha + beta); CG then sees (r, z) < 0 on the
    top eigenvector and reports breakdown."""
    eigs = np.linspace(0.002, 1.998, 40)
    c = O.chebyshev_scalars(0.002, 0.99 * 1.998, 9, 1.0)
    p = O.chebyshev_apply(lambda x: eigs * x, np.ones_like(eigs), c, 9)
    assert (eigs * p).min() < 0.0
    b = np.zeros_like(eigs)
    b[-1] = 1.0
    res = O.pcg(lambda x: eigs * x, b, lambda r: O.chebyshev_apply(lambda x: eigs * x, r, c, 9),
                tol=1e-10, maxit=10)
    assert res.breakdown and not res.converged


def check_table3_lap1600(ms=(0, 7, 31), band=0.10):
    """Table 3 Lap1600 iteration counts, soft: 1598^2 Laplacian, s = 1.001, tol 1e-8, b ~ U[0,1]."""
    rows = {}
    with open(os.path.join(GOLDEN, "table3_counts.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            m, _, _, _, lap = line.split()
            rows[int(m)] = int(lap)
    rp, ci, v = W.stencil5_csr(1598)
    lam = W.stencil5_eigenvalues(1598)
    b = W.uniform(0, len(rp) - 1)
    for m in ms:
        res = O.nc_pcg(rp, ci, v, b, lam[0], lam[-1], m, s=1.001, tol=1e-8)
        assert res.converged
        assert abs(res.iters - rows[m]) <= band * rows[m], (m, res.iters, rows[m])


def _scaled_stencil7(nx, ny, nz):
    """matvec of D^-1/2 A D^-1/2 = A / 6 for the 7-point Laplacian, and its eigenvalue of mode (a, b, c)."""
    rp, ci, v = W.stencil7_csr(nx, ny, nz)
    a = O.csr(rp, ci, v)

    def eig(i, j, l):
        return 1.0 - (np.cos(np.pi * i / (nx + 1)) + np.cos(np.pi * j / (ny + 1)) + np.cos(np.pi * l / (nz + 1))) / 3.0

    def mode(i, j, l):
        x = np.sin(np.pi * i * np.arange(1, nx + 1) / (nx + 1))
        y = np.sin(np.pi * j * np.arange(1, ny + 1) / (ny + 1))
        z = np.sin(np.pi * l * np.arange(1, nz + 1) / (nz + 1))
        return (z[:, None, None] * y[None, :, None] * x[None, None, :]).ravel()  # x fastest

    return (lambda u: (a @ u) / 6.0), eig, mode


def check_power_method():
    """Power method (Sec. 5.1): from an eigenvector one step returns its eigenvalue; from a
    random start the Rayleigh quotients never decrease (A is SPD) and reach the closed-form
    lambda_max of the scaled 7-point operator (spectral gap 0.95 at the top of a 4 x 5 x 6 grid)."""
    mv, eig, mode = _scaled_stencil7(4, 5, 6)
    for m in [(4, 5, 6), (1, 1, 1), (2, 3, 1)]:
        mu, _ = O.power_method(mv, mode(*m), 1)
        assert abs(mu - eig(*m)) <= 1e-14, (m, mu, eig(*m))
    mu, hist = O.power_method(mv, W.uniform(4, 120, 0.5, 1.5), 400)
    assert np.all(np.diff(hist) >= -1e-14)
    assert abs(mu - eig(4, 5, 6)) <= 1e-10, (mu, eig(4, 5, 6))


def check_dacg():
    """DACG (Sec. 5.1): at a tight tolerance it reaches the closed-form lambda_min of the scaled
    7-point operator within a CG-like number of steps (steepest descent needs several times
    more); at the paper's 1e-2 its estimate obeys Temple's inequality
    mu - lambda_1 <= ||A x - mu x||^2 / (lambda_2 - mu) (unit x) and stays above lambda_1."""
    mv, eig, _ = _scaled_stencil7(4, 5, 6)
    mu, steps, relres = O.dacg_smallest(mv, W.uniform(5, 120, 0.5, 1.5), 1e-11, 60)
    assert relres <= 1e-11 and abs(mu - eig(1, 1, 1)) <= 1e-12 * eig(1, 1, 1), (mu, steps, relres)
    mv, eig, _ = _scaled_stencil7(12, 10, 8)
    l1, l2 = eig(1, 1, 1), eig(2, 1, 1)
    mu, steps, relres = O.dacg_smallest(mv, W.uniform(6, 960, 0.5, 1.5), 1e-2, 500)
    assert relres <= 1e-2 and steps >= 1
    assert l1 <= mu * (1 + 1e-13) and mu < l2
    assert mu - l1 <= (relres * mu) ** 2 / (l2 - mu) * (1 + 1e-9), (mu, l1, l2, relres)
    d = np.linspace(0.3, 2.0, 50)
    mu, _, _ = O.dacg_smallest(lambda u: d * u, np.ones(50), 1e-12, 500)
    assert abs(mu - 0.3) <= 1e-12


def check_second_level():
    """The second-level construction (Sec. 6, closing remark) on the block Jacobi factor:
    W^T A W has identity 3 x 3 diagonal blocks and W W^T inverts the diagonal blocks of A;
    W p_k(W^T A W) W^T r equals p_k(B^-1 A) B^-1 r (B = blockdiag(A_II)), the form a
    recurrence on B^-1 A with input B^-1 r computes; with 1 x 1 blocks the construction is the
    plain NC preconditioner; and its PCG solves the system (dense solve)."""
    rp, ci, v = W.elasticity_q1_csr(3, seed=5)
    a, d, w, cm = O.second_level_operator(rp, ci, v)
    n = a.shape[0]
    cd = cm.toarray()
    for i in range(0, n, 3):
        assert np.abs(cd[i:i + 3, i:i + 3] - np.eye(3)).max() <= 1e-13
    ww = (w @ w.T).toarray()
    ad = a.toarray()
    for i in range(0, n, 3):
        assert np.abs(ww[i:i + 3, i:i + 3] @ ad[i:i + 3, i:i + 3] - np.eye(3)).max() <= 1e-12
    eig = np.linalg.eigvalsh(cd)
    lo, hi = eig[0], eig[-1]
    r = W.uniform(11, n, -1.0, 1.0)
    dm = 1.0 / np.sqrt(d)
    binv = np.zeros((n, n))
    for i in range(0, n, 3):
        binv[i:i + 3, i:i + 3] = np.linalg.inv(ad[i:i + 3, i:i + 3])
    c = O.chebyshev_scalars(lo, hi, 7, 1.001)
    ref = dm * O.chebyshev_apply(lambda u: binv @ (ad @ u), binv @ (dm * r), c, 7)
    z = O.nc_apply_second_level(rp, ci, v, r, lo, hi, 7, 1.001)
    assert np.abs(z - ref).max() <= 1e-12 * np.abs(ref).max()
    z1 = O.nc_apply_second_level(rp, ci, v, r, lo, hi, 7, 1.001, bs=1)
    ea = np.linalg.eigvalsh(ad)
    z1ref = O.nc_apply_unscaled(rp, ci, v, r, lo, hi, 7, 1.001)
    assert np.abs(z1 - z1ref).max() <= 1e-12 * np.abs(z1ref).max()
    b = W.uniform(12, n, -1.0, 1.0)
    res = O.nc_pcg_second_level(rp, ci, v, b, lo, hi, 5, tol=1e-12, maxit=200)
    x = np.linalg.solve(O.csr(rp, ci, v).toarray(), b)
    assert res.converged and np.abs(res.x_hat - x).max() <= 1e-9 * np.abs(x).max()
    # the same PCG run with the preconditioner in the similarity form, on the scaled system
    c5 = O.chebyshev_scalars(lo, hi, 5, 1.001)
    ref = O.pcg(lambda u: ad @ u, (b / np.sqrt(d)),
                lambda q: O.chebyshev_apply(lambda u: binv @ (ad @ u), binv @ q, c5, 5), 1e-12, 200)
    assert ref.iters == res.iters
    assert np.allclose(res.history, ref.history, rtol=1e-8, atol=0.0)
    res1 = O.nc_pcg_second_level(rp, ci, v, b, ea[0], ea[-1], 5, tol=1e-10, maxit=200, bs=1)
    ref1 = O.nc_pcg(rp, ci, v, b, ea[0], ea[-1], 5, tol=1e-10, maxit=200)
    assert res1.iters == ref1.iters and np.abs(res1.x_hat - ref1.x_hat).max() <= 1e-12 * np.abs(ref1.x_hat).max()


def check_unscaled_apply_closed_form():
    """The preconditioner of the unscaled system, D^-1/2 p_k(A) D^-1/2 r_hat (Sec. 5 scales first), on
    A_hat = S L S with L the 7-point Laplacian divided by 6 (unit diagonal, closed-form sine eigenpairs)
    and S a positive non-constant diagonal: the Jacobi scaling of A_hat is exactly L, so for
    r_hat = S u with L u = lam u the result is S^-1 p_k(lam) u with p_k from eq. cheb."""
    nx, ny, nz = 7, 6, 5
    rp, ci, v = W.stencil7_csr(nx, ny, nz)
    n = len(rp) - 1
    sd = W.uniform(21, n, 0.5, 2.0)
    rows = np.repeat(np.arange(n), np.diff(rp.astype(np.int64)))
    vh = v / 6.0 * sd[rows] * sd[ci]
    _, eig, mode = _scaled_stencil7(nx, ny, nz)
    lo, hi = W.stencil7_bounds(nx, ny, nz)
    for k in (0, 1, 5, 12):
        for m in [(1, 1, 1), (7, 6, 5), (3, 2, 4)]:
            u = mode(*m)
            z = O.nc_apply_unscaled(rp, ci, vh, sd * u, lo, hi, k, 1.001)
            expect = float(closed_form_pk(eig(*m), lo, hi, k, 1.001)) * u / sd
            assert np.abs(z - expect).max() <= 1e-11 * np.abs(expect).max(), (k, m)


ALL_FAST = [
    check_rho_closed_form,
    check_zeta_closed_form,
    check_poly_closed_form,
    check_equioscillation,
    check_newton_equals_chebyshev,
    check_hotelling,
    check_table1_spectrum,
    check_table1_iterations,
    check_dense_solve,
    check_finite_termination,
    check_flexible_local_orthogonality,
    check_counting_identities,
    check_lanczos_exact_small,
    check_indefinite_breakdown,
    check_power_method,
    check_dacg,
    check_second_level,
    check_unscaled_apply_closed_form,
]

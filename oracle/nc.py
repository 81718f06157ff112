"""Plain FP64 CPU oracle for Newton-Chebyshev (NC) polynomial-preconditioned CG.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import or call this
module: only the test suite, the smoke check and the benchmark's CPU-baseline
leg use it.  It shares no code with the GPU library; its inputs come from the
seeded generators in ``workloads``.

Everything is float64 numpy / scipy.sparse in the order the paper states it,
with no blocking, fusion or reordering; a CSR product (scipy) is the only
library primitive used as a step.  Readings of points the paper leaves open:

* Modified parameter (Sec. 4): theta' = s * theta with delta unchanged, i.e.
  the interval [alpha, beta] is shifted right by (s - 1) * theta.  Both the
  Chebyshev and the Newton forms are built on the shifted interval.
* Alg. 2 indices: step k of the loop uses rho_k and rho_{k-1}, as in the p_k
  recurrence of Sec. 3 that it implements (the printed loop shows rho_{k+1},
  rho_k).
* Alg. 1 / Fig. 1: level L of the recursion multiplies by zeta_L (0-based).
* PCG (not printed in the paper): standard preconditioned CG from x0 = 0,
  stopping on the recursively updated residual ||r|| / ||b|| < tol; beta is
  Fletcher-Reeves (r_new, z_new)/(r_old, z_old) or, for the flexible variant,
  Polak-Ribiere (z_new, r_new - r_old)/(r_old, z_old) (Golub & Ye 1999; Notay
  2000), which keeps consecutive directions A-orthogonal even when the
  preconditioner changes between iterations.
* The system is symmetrically Jacobi-scaled first, A = D^-1/2 A_hat D^-1/2
  and b = D^-1/2 b_hat (Sec. 2 and Sec. 5); eigenvalue bounds refer to A.
"""

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


class NotSPD(ValueError):
    """The operator has a non-positive diagonal entry, so it cannot be SPD."""


@dataclass
class ChebScalars:
    """Scalars of the degree-k NC polynomial on the (shifted) interval [alpha, beta]."""
    alpha: float
    beta: float
    theta: float
    delta: float
    sigma: float
    rho: np.ndarray  # rho_0 .. rho_k


def chebyshev_scalars(lambda_min: float, lambda_max: float, k: int, s: float = 1.0) -> ChebScalars:
    """theta, delta, sigma (Sec. 3) with theta scaled by s (Sec. 4), and rho_0..rho_k.

    rho_0 = 1/sigma and rho_j = 1/(2 sigma - rho_{j-1}) (eq. rhocheb)."""
    theta0 = 0.5 * (lambda_max + lambda_min)
    delta = 0.5 * (lambda_max - lambda_min)
    theta = s * theta0
    sigma = theta / delta
    rho = np.empty(max(k, 0) + 1)
    rho[0] = 1.0 / sigma
    for j in range(1, k + 1):
        rho[j] = 1.0 / (2.0 * sigma - rho[j - 1])
    return ChebScalars(theta - delta, theta + delta, theta, delta, sigma, rho)


def chebyshev_apply(matvec, r: np.ndarray, c: ChebScalars, k: int) -> np.ndarray:
    """z = p_k(A) r by the three-term recurrence of Alg. 2 (k matrix-vector products).

    p_0 = 1/theta; p_1 = (2 rho_1/delta)(2 - x/theta);
    p_j = rho_j (2 sigma (1 - x/theta) p_{j-1} - rho_{j-1} p_{j-2} + 2/delta)."""
    x_old = r / c.theta
    if k == 0:
        return x_old
    x = (2.0 * c.rho[1] / c.delta) * (2.0 * r - matvec(r) / c.theta)
    for j in range(2, k + 1):
        z = (2.0 / c.delta) * (r - matvec(x))
        x_new = c.rho[j] * (2.0 * c.sigma * x - c.rho[j - 1] * x_old + z)
        x_old, x = x, x_new
    return x


def newton_zetas(lambda_min: float, lambda_max: float, nlev: int, s: float = 1.0) -> np.ndarray:
    """zeta_0 .. zeta_nlev of Alg. 1 on the interval shifted by the modified parameter.

    zeta_0 = 2/(alpha + beta); zeta_1 = 2/(1 + 2 alpha zeta_0 - (alpha zeta_0)^2);
    zeta_i = 2/(1 + 2 zeta_{i-1} - zeta_{i-1}^2) for i >= 2 (eq. zetaNewt)."""
    c = chebyshev_scalars(lambda_min, lambda_max, 0, s)
    zeta = np.empty(nlev + 1)
    zeta[0] = 2.0 / (c.alpha + c.beta)
    if nlev >= 1:
        az = c.alpha * zeta[0]
        zeta[1] = 2.0 / (1.0 + 2.0 * az - az * az)
    for i in range(2, nlev + 1):
        zeta[i] = 2.0 / (1.0 + 2.0 * zeta[i - 1] - zeta[i - 1] ** 2)
    return zeta


def newton_apply(matvec, r: np.ndarray, zeta: np.ndarray, nlev: int) -> np.ndarray:
    """P_nlev r by the recursion of Alg. 1 (2^nlev - 1 matrix-vector products).

    P_0 u = zeta_0 u;  P_{j+1} u = zeta_{j+1} (2 P_j u - P_j A P_j u)."""
    if nlev == 0:
        return zeta[0] * r
    u = newton_apply(matvec, r, zeta, nlev - 1)
    w = newton_apply(matvec, matvec(u), zeta, nlev - 1)
    return zeta[nlev] * (2.0 * u - w)


def hotelling_step(p: np.ndarray, a: np.ndarray) -> np.ndarray:
    """One unscaled Newton step for X^-1 = A on dense matrices: P <- 2P - P A P (eq. newtonP)."""
    return 2.0 * p - p @ a @ p


def csr(rowptr, colind, values) -> sp.csr_matrix:
    n = len(rowptr) - 1
    return sp.csr_matrix((np.asarray(values, dtype=np.float64), colind, rowptr), shape=(n, n))


def jacobi_scale(a_hat: sp.csr_matrix):
    """A = D^-1/2 A_hat D^-1/2 with D = diag(A_hat); returns (A, d).  Raises NotSPD if d <= 0."""
    d = a_hat.diagonal()
    if not np.all(d > 0.0):
        raise NotSPD("operator diagonal has a non-positive entry")
    s = sp.diags(1.0 / np.sqrt(d))
    return (s @ a_hat @ s).tocsr(), d


class CountingOperator:
    """y = A x with a counter of products (the paper's 'A x v' column of Table 3)."""

    def __init__(self, a):
        self.a = a
        self.count = 0

    def __call__(self, x):
        self.count += 1
        return self.a @ x


@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    converged: bool
    breakdown: bool
    relres: float            # recursive ||r|| / ||b|| at exit
    n_spmv: int              # all A products, preconditioner included
    n_dot: int               # scalar products (flexible beta adds one per iteration)
    history: list = field(default_factory=list)  # ||r_i|| / ||b||, i = 0 .. iters


def pcg(matvec, b: np.ndarray, precond, tol: float, maxit: int, flexible: bool = False,
        x0: np.ndarray = None, progress=None) -> PCGResult:
    """Preconditioned CG (Saad 2003, Alg. 9.1); `precond(r)` returns z = M r.

    Per iteration: q = A p, alpha = (r, z)/(p, q), x += alpha p, r -= alpha q, stop test,
    z = M r, beta, p = z + beta p.  `progress(i, relres)`, if given, is called after the
    residual update of iteration i (reporting only)."""
    n_dot = 0  # counted as in Table 3: (r, z) once, then (p, q), (r, r), (r, z) per iteration
    bnorm = np.sqrt(b @ b)
    if bnorm == 0.0:
        return PCGResult(np.zeros_like(b), 0, True, False, 0.0, 0, n_dot, [0.0])
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = x0.copy()
        r = b - matvec(x)
    rnorm = np.sqrt(r @ r)
    hist = [rnorm / bnorm]
    if rnorm / bnorm < tol:
        return PCGResult(x, 0, True, False, rnorm / bnorm, 0, n_dot, hist)
    z = precond(r)
    gamma = r @ z
    n_dot += 1
    if not (gamma > 0.0):
        return PCGResult(x, 0, False, True, rnorm / bnorm, 0, n_dot, hist)
    p = z.copy()
    it = 0
    converged = breakdown = False
    while it < maxit:
        it += 1
        q = matvec(p)
        pq = p @ q
        n_dot += 1
        if not (pq > 0.0):
            breakdown = True
            break
        alpha = gamma / pq
        x += alpha * p
        r_old = r.copy() if flexible else None
        r -= alpha * q
        rnorm = np.sqrt(r @ r)
        n_dot += 1
        hist.append(rnorm / bnorm)
        if progress is not None:
            progress(it, rnorm / bnorm)
        if not np.isfinite(rnorm):
            breakdown = True
            break
        if rnorm / bnorm < tol:
            converged = True
            break
        z_new = precond(r)
        gamma_new = r @ z_new
        n_dot += 1
        if not (gamma_new > 0.0):
            breakdown = True
            break
        if flexible:
            beta = (z_new @ (r - r_old)) / gamma
            n_dot += 1
        else:
            beta = gamma_new / gamma
        p = z_new + beta * p
        gamma = gamma_new
    return PCGResult(x, it, converged, breakdown, hist[-1], 0, n_dot, hist)


@dataclass
class NCResult:
    x_hat: np.ndarray        # solution of the unscaled system A_hat x_hat = b_hat
    iters: int
    converged: bool
    breakdown: bool
    relres: float            # recursive residual of the scaled system at exit
    relres_true: float       # ||b - A x|| / ||b|| of the scaled system, recomputed
    relres_true_hat: float   # ||b_hat - A_hat x_hat|| / ||b_hat||, unscaled
    n_spmv: int
    n_dot: int
    history: list


def nc_pcg(rowptr, colind, values, b_hat, lambda_min, lambda_max, k, s=1.001, tol=1e-8,
           maxit=100000, flexible=False, x0_hat=None, progress=None) -> NCResult:
    """Solve A_hat x_hat = b_hat by PCG with the degree-k NC preconditioner (Sec. 5 set-up).

    The system is Jacobi-scaled, the preconditioner p_k(A) uses the bounds
    [lambda_min, lambda_max] of the scaled matrix with theta scaled by s, and the
    solution is mapped back as x_hat = D^-1/2 x."""
    a_hat = csr(rowptr, colind, values)
    a, d = jacobi_scale(a_hat)
    dm = 1.0 / np.sqrt(d)
    b = dm * b_hat
    op = CountingOperator(a)
    c = chebyshev_scalars(lambda_min, lambda_max, k, s)
    x0 = None if x0_hat is None else x0_hat / dm
    res = pcg(op, b, lambda r: chebyshev_apply(op, r, c, k), tol, maxit, flexible, x0, progress)
    x_hat = dm * res.x
    rt = b - a @ res.x
    rt_hat = b_hat - a_hat @ x_hat
    bn = np.linalg.norm(b)
    bhn = np.linalg.norm(b_hat)
    return NCResult(x_hat, res.iters, res.converged, res.breakdown, res.relres,
                    float(np.linalg.norm(rt) / bn) if bn > 0 else 0.0,
                    float(np.linalg.norm(rt_hat) / bhn) if bhn > 0 else 0.0,
                    op.count, res.n_dot, res.history)


def nc_apply_unscaled(rowptr, colind, values, r_hat, lambda_min, lambda_max, k, s=1.001):
    """The NC preconditioner as an operator on the unscaled system: D^-1/2 p_k(A) D^-1/2 r_hat."""
    a, d = jacobi_scale(csr(rowptr, colind, values))
    dm = 1.0 / np.sqrt(d)
    c = chebyshev_scalars(lambda_min, lambda_max, k, s)
    return dm * chebyshev_apply(lambda v: a @ v, dm * r_hat, c, k)


def block_jacobi_factor(a: sp.csr_matrix, bs: int = 3) -> sp.csr_matrix:
    """A first-level preconditioner in factored form, P0 = W W^T (the closing remark of Sec. 6):
    block Jacobi with the bs x bs diagonal blocks A_II (for 3-D elasticity, the three displacement
    components of one node).  A_II = L_I L_I^T (Cholesky) and W = blockdiag(L_I^-T), so that
    W W^T = blockdiag(A_II)^-1 and W^T A W has identity diagonal blocks.  Raises NotSPD if a
    block is not positive definite."""
    n = a.shape[0]
    if n % bs:
        raise ValueError("n must be a multiple of the block size")
    factors = []
    for i in range(0, n, bs):
        try:
            l = np.linalg.cholesky(a[i:i + bs, i:i + bs].toarray())
        except np.linalg.LinAlgError as exc:
            raise NotSPD("a diagonal block is not positive definite") from exc
        factors.append(np.linalg.inv(l).T)
    return sp.block_diag(factors, format="csr")


def second_level_operator(rowptr, colind, values, bs: int = 3):
    """(A, d, W, C): the Jacobi-scaled A = D^-1/2 A_hat D^-1/2, d = diag(A_hat), the block
    Jacobi factor W of A and C = W^T A W, the matrix the second-level polynomial acts on."""
    a, d = jacobi_scale(csr(rowptr, colind, values))
    w = block_jacobi_factor(a, bs)
    return a, d, w, (w.T @ a @ w).tocsr()


def nc_apply_second_level(rowptr, colind, values, r_hat, lambda_min, lambda_max, k, s=1.001, bs=3):
    """The second-level NC preconditioner on the unscaled system:
    D^-1/2 W p_k(W^T A W) W^T D^-1/2 r_hat, with [lambda_min, lambda_max] bounding the spectrum of
    C = W^T A W (Sec. 6, closing remark; k = 0 gives block Jacobi, W W^T / theta')."""
    _, d, w, cm = second_level_operator(rowptr, colind, values, bs)
    dm = 1.0 / np.sqrt(d)
    c = chebyshev_scalars(lambda_min, lambda_max, k, s)
    return dm * (w @ chebyshev_apply(lambda v: cm @ v, w.T @ (dm * r_hat), c, k))


def nc_pcg_second_level(rowptr, colind, values, b_hat, lambda_min, lambda_max, k, s=1.001, tol=1e-8,
                        maxit=100000, flexible=False, bs=3) -> "NCResult":
    """PCG on the Jacobi-scaled system, as nc_pcg, preconditioned by W p_k(W^T A W) W^T, the
    paper's second-level construction on the block Jacobi factor P0 = W W^T of A."""
    a_hat = csr(rowptr, colind, values)
    a, d = jacobi_scale(a_hat)
    w = block_jacobi_factor(a, bs)
    dm = 1.0 / np.sqrt(d)
    b = dm * b_hat
    op = CountingOperator(a)
    c = chebyshev_scalars(lambda_min, lambda_max, k, s)
    res = pcg(op, b, lambda r: w @ chebyshev_apply(lambda v: w.T @ op(w @ v), w.T @ r, c, k), tol, maxit,
              flexible)
    x_hat = dm * res.x
    rt = b - a @ res.x
    rt_hat = b_hat - a_hat @ x_hat
    bn, bhn = np.linalg.norm(b), np.linalg.norm(b_hat)
    return NCResult(x_hat, res.iters, res.converged, res.breakdown, res.relres,
                    float(np.linalg.norm(rt) / bn) if bn > 0 else 0.0,
                    float(np.linalg.norm(rt_hat) / bhn) if bhn > 0 else 0.0,
                    op.count, res.n_dot, res.history)


def lanczos_extremes(matvec, v0: np.ndarray, nsteps: int = 30):
    """Extreme Ritz values of `nsteps` Lanczos steps with full reorthogonalisation.

    Returns (smallest, largest) eigenvalue of the tridiagonal T_m."""
    n = v0.shape[0]
    m = min(nsteps, n)
    v = np.zeros((m + 1, n))
    v[0] = v0 / np.linalg.norm(v0)
    alpha = np.zeros(m)
    beta = np.zeros(m)
    steps = m
    for j in range(m):
        w = matvec(v[j])
        alpha[j] = v[j] @ w
        # classical Gram-Schmidt against every stored vector, done twice
        for _ in range(2):
            w = w - v[:j + 1].T @ (v[:j + 1] @ w)
        beta[j] = np.linalg.norm(w)
        if j + 1 < m:
            if beta[j] <= 1e-14 * abs(alpha[j]):
                steps = j + 1
                break
            v[j + 1] = w / beta[j]
    t = np.diag(alpha[:steps]) + np.diag(beta[:steps - 1], 1) + np.diag(beta[:steps - 1], -1)
    ritz = np.linalg.eigvalsh(t)
    return float(ritz[0]), float(ritz[-1])


def power_method(matvec, v0: np.ndarray, iters: int):
    """Estimate of lambda_max by `iters` steps of the power method (Sec. 5.1).

    v_0 = v0 / ||v0||; step i: w = A v_{i-1}, mu_i = (v_{i-1}, w) / (v_{i-1}, v_{i-1})
    (the Rayleigh quotient of v_{i-1}), v_i = w / ||w||.  Returns (mu_iters, [mu_1 .. mu_iters])."""
    v = v0 / np.linalg.norm(v0)
    history = []
    for _ in range(iters):
        w = matvec(v)
        history.append(float((v @ w) / (v @ v)))
        v = w / np.linalg.norm(w)
    return history[-1], history


def dacg_smallest(matvec, v0: np.ndarray, tol: float, maxit: int):
    """Estimate of lambda_min by the DACG method without preconditioning (Sec. 5.1,
    after Bergamaschi, Gambolati and Pini 1997): conjugate-gradient minimisation of
    the Rayleigh quotient q(x) = (x, A x) / (x, x).

    x_0 = v0 / ||v0||.  With g_k = A x_k - q(x_k) x_k (the gradient of q up to the
    factor 2 / (x, x)): p_0 = -g_0, p_k = -g_k + beta_k p_{k-1} with
    beta_k = (g_k, g_k) / (g_{k-1}, g_{k-1}).  x_{k+1} minimises q on the line
    x_k + t p_k: it is the Ritz vector of the smaller Ritz value mu of A on
    span{x_k, p_k} (a 2 x 2 generalised eigenproblem), scaled to unit norm with a
    non-negative x_k coefficient; A x_{k+1} follows from A x_k and A p_k, so a step
    costs one product.  Stops when ||A x - mu x|| / (mu ||x||) <= tol or after
    maxit steps.  Returns (mu, steps, relres)."""
    import scipy.linalg

    x = v0 / np.linalg.norm(v0)
    ax = matvec(x)
    xx, xax = x @ x, x @ ax
    mu = xax / xx
    g = ax - mu * x
    gg = g @ g
    relres = np.sqrt(gg) / (mu * np.sqrt(xx))
    p = np.zeros_like(x)
    steps = 0
    while relres > tol and steps < maxit:
        beta = 0.0 if steps == 0 else gg / gg_old
        p = -g + beta * p
        ap = matvec(p)
        gm = np.array([[xax, x @ ap], [x @ ap, p @ ap]])
        hm = np.array([[xx, x @ p], [x @ p, p @ p]])
        evals, evecs = scipy.linalg.eigh(gm, hm)
        mu = float(evals[0])
        u = evecs[:, 0] / np.sqrt(evecs[:, 0] @ hm @ evecs[:, 0])
        if u[0] < 0.0:
            u = -u
        x = u[0] * x + u[1] * p
        ax = u[0] * ax + u[1] * ap
        g = ax - mu * x
        gg_old, gg = gg, g @ g
        xx, xax = x @ x, x @ ax
        relres = np.sqrt(gg) / (mu * np.sqrt(xx))
        steps += 1
    return float(mu), steps, float(relres)


def preconditioned_spectrum(eigs: np.ndarray, lambda_min: float, lambda_max: float, k: int,
                            s: float = 1.0) -> np.ndarray:
    """Eigenvalues mu_i = lambda_i p_k(lambda_i) of p_k(A) A for A with spectrum `eigs`.

    p_k(A) shares A's eigenvectors, so applying the recurrence to the diagonal
    matrix diag(eigs) and the all-ones vector gives p_k at every eigenvalue."""
    c = chebyshev_scalars(lambda_min, lambda_max, k, s)
    p = chebyshev_apply(lambda v: eigs * v, np.ones_like(eigs), c, k)
    return eigs * p


def cluster_indicator(mu: np.ndarray) -> int:
    """l = #{lambda : lambda / lambda_min < 1.1} (eq. lmin)."""
    return int(np.count_nonzero(mu / mu.min() < 1.1))

"""Every plausible mistake planted in the oracle (on the CPU) must fail at least one pin.

Each mutant rewrites one expression of one oracle function (a wrong index, a
dropped term, a flipped sign, a transposed or one-sided operand, the literal
readings of Alg. 2 and Fig. 1 that the oracle rejects, the zeta_0-only reading
of the modified parameter) and swaps it in for the duration of one test.
"""

import inspect
import textwrap

import pytest

import pins
from oracle import nc as O

MUTANTS = [
    # Alg. 2 recurrence
    ("chebyshev_apply", "x_new = c.rho[j] * (2.0 * c.sigma * x - c.rho[j - 1] * x_old + z)",
     "x_new = c.rho[min(j + 1, k)] * (2.0 * c.sigma * x - c.rho[j] * x_old + z)", "literal Alg. 2 rho indices"),
    ("chebyshev_apply", " - c.rho[j - 1] * x_old", "", "dropped three-term history"),
    ("chebyshev_apply", "(r - matvec(x))", "(r + matvec(x))", "sign of the residual term"),
    ("chebyshev_apply", "(2.0 * r - matvec(r) / c.theta)", "(2.0 * r - matvec(r) * c.theta)", "first step scale"),
    ("chebyshev_apply", "x_old = r / c.theta", "x_old = r * c.theta", "p_0 = theta instead of 1/theta"),
    ("chebyshev_apply", "2.0 * c.sigma * x", "c.sigma * x", "dropped factor 2 on sigma"),
    # scalars
    ("chebyshev_scalars", "rho[j] = 1.0 / (2.0 * sigma - rho[j - 1])",
     "rho[j] = 1.0 / (2.0 * sigma + rho[j - 1])", "rho recurrence sign"),
    ("chebyshev_scalars", "sigma = theta / delta", "sigma = theta0 / delta", "modified parameter on theta only"),
    ("chebyshev_scalars", "theta = s * theta0", "theta = theta0", "modified parameter ignored"),
    ("chebyshev_scalars", "delta = 0.5 * (lambda_max - lambda_min)", "delta = lambda_max - lambda_min",
     "delta not halved"),
    # Alg. 1 / Fig. 1
    ("newton_apply", "zeta[nlev] * (2.0 * u - w)", "zeta[nlev - 1] * (2.0 * u - w)", "literal Fig. 1 zeta index"),
    ("newton_apply", "newton_apply(matvec, matvec(u), zeta, nlev - 1)", "matvec(newton_apply(matvec, u, zeta, nlev - 1))",
     "P A P applied as A P P"),
    ("newton_zetas", "1.0 + 2.0 * zeta[i - 1] - zeta[i - 1] ** 2", "1.0 + 2.0 * zeta[i - 1] + zeta[i - 1] ** 2",
     "zeta recurrence sign"),
    ("newton_zetas", "zeta[0] = 2.0 / (c.alpha + c.beta)", "zeta[0] = 1.0 / (c.alpha + c.beta)", "zeta_0 factor"),
    ("hotelling_step", "2.0 * p - p @ a @ p", "p - p @ a @ p", "Hotelling factor 2"),
    # PCG
    ("pcg", "alpha = gamma / pq", "alpha = (r @ r) / pq", "alpha from (r, r)"),
    ("pcg", "beta = gamma_new / gamma", "beta = gamma / gamma_new", "Fletcher-Reeves inverted"),
    ("pcg", "beta = (z_new @ (r - r_old)) / gamma", "beta = (z_new @ (r + r_old)) / gamma", "flexible beta sign"),
    ("pcg", "beta = (z_new @ (r - r_old)) / gamma", "beta = gamma_new / gamma", "flexible falls back to FR"),
    ("pcg", "p = z_new + beta * p", "p = z_new + beta * z", "direction update operand"),
    ("pcg", "r -= alpha * q", "r -= alpha * p", "residual update operand"),
    ("pcg", "x += alpha * p", "x += alpha * q", "solution update operand"),
    ("pcg", "if rnorm / bnorm < tol:\n            converged = True",
     "if rnorm < tol:\n            converged = True", "absolute instead of relative stop test"),
    # scaling and mapping back
    ("jacobi_scale", "return (s @ a_hat @ s).tocsr(), d", "return (s @ s @ a_hat).tocsr(), d",
     "one-sided (nonsymmetric) scaling"),
    ("nc_pcg", "x_hat = dm * res.x", "x_hat = res.x / dm", "solution mapped back with D^1/2"),
    ("nc_pcg", "b = dm * b_hat", "b = b_hat / dm", "right-hand side scaled with D^1/2"),
    ("nc_apply_unscaled", "return dm * chebyshev_apply(lambda v: a @ v, dm * r_hat, c, k)",
     "return chebyshev_apply(lambda v: a @ v, dm * r_hat, c, k)", "unscaled apply without the outer D^-1/2"),
    ("nc_apply_unscaled", "chebyshev_apply(lambda v: a @ v, dm * r_hat, c, k)",
     "chebyshev_apply(lambda v: a @ v, r_hat / dm, c, k)", "unscaled apply input scaled with D^1/2"),
    ("nc_apply_unscaled", "c = chebyshev_scalars(lambda_min, lambda_max, k, s)",
     "c = chebyshev_scalars(lambda_min, lambda_max, k, 1.0)", "unscaled apply ignores the modified parameter"),
    # spectra and estimators
    ("preconditioned_spectrum", "return eigs * p", "return p", "spectrum of p_k(A) instead of p_k(A) A"),
    ("cluster_indicator", "mu / mu.min() < 1.1", "mu / mu.min() < 1.01", "cluster threshold"),
    ("lanczos_extremes", "w = w - v[:j + 1].T @ (v[:j + 1] @ w)", "w = w - v[:j].T @ (v[:j] @ w)",
     "reorthogonalisation skips the current vector"),
    ("power_method", "history.append(float((v @ w) / (v @ v)))", "history.append(float((w @ w) / (v @ v)))",
     "power method returns lambda^2"),
    ("power_method", "return history[-1], history", "return history[0], history", "power method first estimate"),
    ("dacg_smallest", "        g = ax - mu * x", "        g = ax + mu * x", "DACG gradient sign"),
    ("dacg_smallest", "beta = 0.0 if steps == 0 else gg / gg_old", "beta = 0.0",
     "DACG without conjugation (steepest descent)"),
    ("dacg_smallest", "beta = 0.0 if steps == 0 else gg / gg_old", "beta = 0.0 if steps == 0 else gg_old / gg",
     "DACG beta inverted"),
    ("dacg_smallest", "mu = float(evals[0])", "mu = float(evals[1])", "DACG larger Ritz value"),
    ("dacg_smallest", "u = evecs[:, 0] / np.sqrt", "u = evecs[:, 1] / np.sqrt", "DACG larger Ritz vector"),
    # second level (Sec. 6)
    ("block_jacobi_factor", "factors.append(np.linalg.inv(l).T)", "factors.append(np.linalg.inv(l))",
     "W = L^-1 instead of L^-T"),
    ("block_jacobi_factor", "factors.append(np.linalg.inv(l).T)", "factors.append(np.diag(1.0 / np.sqrt(np.diag(l @ l.T))))",
     "point Jacobi instead of block Jacobi"),
    ("nc_apply_second_level", "w @ chebyshev_apply(lambda v: cm @ v, w.T @ (dm * r_hat), c, k)",
     "w @ chebyshev_apply(lambda v: cm @ v, w @ (dm * r_hat), c, k)", "W applied on the input instead of W^T"),
    ("nc_pcg_second_level", "lambda r: w @ chebyshev_apply(lambda v: w.T @ op(w @ v), w.T @ r, c, k)",
     "lambda r: chebyshev_apply(lambda v: w.T @ op(w @ v), r, c, k)", "second level without the outer W, W^T"),
]


def _mutant(fn_name, old, new):
    src = textwrap.dedent(inspect.getsource(getattr(O, fn_name)))
    assert src.count(old) == 1, (fn_name, old)
    namespace = dict(vars(O))
    exec(compile(src.replace(old, new), f"<mutant of {fn_name}>", "exec"), namespace)
    return namespace[fn_name]


@pytest.mark.parametrize("fn_name,old,new,what", MUTANTS, ids=[m[3] for m in MUTANTS])
def test_pins_reject_mutant(monkeypatch, fn_name, old, new, what):
    monkeypatch.setattr(O, fn_name, _mutant(fn_name, old, new))
    caught = None
    for check in pins.ALL_FAST:
        try:
            check()
        except Exception as exc:  # AssertionError, or the mutant crashing outright
            caught = (check.__name__, type(exc).__name__)
            break
    assert caught is not None, f"no pin rejects the mutant '{what}'"


def test_unmutated_oracle_passes_every_pin():
    for check in pins.ALL_FAST:
        check()

/*
 * Plain FP64 CPU oracle for Newton-Chebyshev preconditioned CG, in C with
 * OpenMP row parallelism.
 *
 * TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's CPU-baseline leg
 * (which times it on one host thread and on all of them) are its only users;
 * the GPU library never links or calls it, and it shares nothing with it.
 *
 * It computes what oracle/nc.py computes, in the same order, on a CSR matrix:
 *  - the system is symmetrically Jacobi-scaled first, A = D^-1/2 A_hat D^-1/2,
 *    b = D^-1/2 b_hat, as an explicit CSR copy (Sec. 2 and Sec. 5);
 *  - theta' = s (lambda_min + lambda_max) / 2 with delta = (lambda_max -
 *    lambda_min) / 2 (the modified parameter of Sec. 4), sigma = theta'/delta,
 *    rho_0 = 1/sigma, rho_j = 1/(2 sigma - rho_{j-1}) (eq. rhocheb);
 *  - z = p_k(A) r by the three-term recurrence of Alg. 2, step j using rho_j
 *    and rho_{j-1} (the p_k recurrence of Sec. 3);
 *  - standard PCG from x0 = 0 (Saad 2003, Alg. 9.1), stopping on the recursive
 *    residual ||r|| / ||b|| < tol, beta Fletcher-Reeves or, flexible,
 *    Polak-Ribiere (z_new, r_new - r_old) / (r_old, z_old);
 *  - x_hat = D^-1/2 x, the recursive and recomputed relative residuals, and the
 *    operator-product and dot-product counts of Table 3.
 * Rows are split over threads by a static schedule; a dot product sums each
 * thread's static chunk and then the chunks in thread order, so results are
 * deterministic for a given thread count.  Built with -ffp-contract=off.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t n;
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
} csr_t;

/* y = A x */
static void spmv(const csr_t* a, const double* x, double* y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < a->n; ++i) {
    double s = 0.0;
    for (int32_t j = a->rowptr[i]; j < a->rowptr[i + 1]; ++j) s += a->val[j] * x[a->col[j]];
    y[i] = s;
  }
}

/* (x, y): per-thread partial sums over static chunks, added in thread order */
static double dot(int64_t n, const double* x, const double* y) {
  const int nt = omp_get_max_threads();
  double* part = (double*)calloc((size_t)nt, sizeof(double));
#pragma omp parallel num_threads(nt)
  {
    const int t = omp_get_thread_num(), m = omp_get_num_threads();
    const int64_t lo = n * t / m, hi = n * (t + 1) / m;
    double s = 0.0;
    for (int64_t i = lo; i < hi; ++i) s += x[i] * y[i];
    part[t] = s;
  }
  double s = 0.0;
  for (int t = 0; t < nt; ++t) s += part[t];
  free(part);
  return s;
}

typedef struct {
  double theta, delta, sigma;
  double* rho; /* rho_0 .. rho_k */
} cheb_t;

static void cheb_scalars(double lmin, double lmax, int k, double s, cheb_t* c) {
  const double theta0 = 0.5 * (lmax + lmin);
  c->delta = 0.5 * (lmax - lmin);
  c->theta = s * theta0;
  c->sigma = c->theta / c->delta;
  c->rho = (double*)malloc(sizeof(double) * (size_t)(k + 1));
  c->rho[0] = 1.0 / c->sigma;
  for (int j = 1; j <= k; ++j) c->rho[j] = 1.0 / (2.0 * c->sigma - c->rho[j - 1]);
}

/* z = p_k(A) r (Alg. 2); work: three vectors of n; counts operator products in *nmv */
static void cheb_apply(const csr_t* a, const double* r, const cheb_t* c, int k, double* z, double* w0,
                       double* w1, double* w2, int64_t* nmv) {
  const int64_t n = a->n;
  double *x_old = w0, *x = w1, *t = w2;
  if (k == 0) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) z[i] = r[i] / c->theta;
    return;
  }
  spmv(a, r, t);
  ++*nmv;
  const double c1 = 2.0 * c->rho[1] / c->delta;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    x_old[i] = r[i] / c->theta;
    x[i] = c1 * (2.0 * r[i] - t[i] / c->theta);
  }
  for (int j = 2; j <= k; ++j) {
    spmv(a, x, t);
    ++*nmv;
    const double rj = c->rho[j], rj1 = c->rho[j - 1], ts = 2.0 * c->sigma, td = 2.0 / c->delta;
    double* x_new = (j == k) ? z : x_old; /* x_old is dead once read below */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      const double zz = td * (r[i] - t[i]);
      x_new[i] = rj * (ts * x[i] - rj1 * x_old[i] + zz);
    }
    if (j == k) return;
    double* tmp = x_old; /* x_old now holds y_j: rotate so x holds y_j and x_old y_{j-1} */
    x_old = x;
    x = tmp;
  }
  /* k == 1 */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) z[i] = x[i];
}

/* Jacobi-scaled copy: values of D^-1/2 A_hat D^-1/2 into sval, D^-1/2 into dm; 0 or -1 (d <= 0) */
static int jacobi_scale(const csr_t* ah, double* sval, double* dm) {
  const int64_t n = ah->n;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t i = 0; i < n; ++i) {
    double d = 0.0;
    for (int32_t j = ah->rowptr[i]; j < ah->rowptr[i + 1]; ++j)
      if (ah->col[j] == i) d += ah->val[j];
    if (!(d > 0.0)) bad = 1;
    dm[i] = 1.0 / sqrt(d);
  }
  if (bad) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int32_t j = ah->rowptr[i]; j < ah->rowptr[i + 1]; ++j) sval[j] = dm[i] * ah->val[j] * dm[ah->col[j]];
  return 0;
}

/* The preconditioner of the unscaled system, z_hat = D^-1/2 p_k(A) D^-1/2 r_hat.  Returns 0, or -1
 * if the diagonal has a non-positive entry. */
int ncomp_apply_unscaled(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                         const double* r_hat, double lmin, double lmax, int k, double s, double* z_hat) {
  const int64_t nnz = rowptr[n];
  double* sval = (double*)malloc(sizeof(double) * (size_t)nnz);
  double* dm = (double*)malloc(sizeof(double) * (size_t)n);
  double* w = (double*)malloc(sizeof(double) * (size_t)n * 5);
  const csr_t ah = {n, rowptr, col, val};
  int rc = jacobi_scale(&ah, sval, dm);
  if (rc == 0) {
    const csr_t a = {n, rowptr, col, sval};
    cheb_t c;
    cheb_scalars(lmin, lmax, k, s, &c);
    double* r = w;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) r[i] = dm[i] * r_hat[i];
    int64_t nmv = 0;
    cheb_apply(&a, r, &c, k, w + n, w + 2 * n, w + 3 * n, w + 4 * n, &nmv);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) z_hat[i] = dm[i] * w[n + i];
    free(c.rho);
  }
  free(sval);
  free(dm);
  free(w);
  return rc;
}

typedef struct {
  int32_t iters, converged, breakdown, pad;
  double relres;          /* recursive ||r|| / ||b|| of the scaled system at exit */
  double relres_true;     /* ||b - A x|| / ||b||, scaled, recomputed */
  double relres_true_hat; /* ||b_hat - A_hat x_hat|| / ||b_hat|| */
  int64_t n_spmv, n_dot;
} ncomp_stats;

/* PCG with the degree-k NC preconditioner on the Jacobi-scaled system; x_hat receives the solution
 * of A_hat x_hat = b_hat.  Returns 0, or -1 if the diagonal has a non-positive entry. */
/* Reporting only: with every > 0, ncomp_pcg prints its iteration count and recursive
 * residual to stderr every `every` iterations (long solves then show progress). */
static int g_progress = 0;
void ncomp_set_progress(int every) { g_progress = every > 0 ? every : 0; }

int ncomp_pcg(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val, const double* b_hat,
              double lmin, double lmax, int k, double s, double tol, int maxit, int flexible, double* x_hat,
              ncomp_stats* st) {
  memset(st, 0, sizeof(*st));
  const int64_t nnz = rowptr[n];
  double* sval = (double*)malloc(sizeof(double) * (size_t)nnz);
  double* dm = (double*)malloc(sizeof(double) * (size_t)n);
  const csr_t ah = {n, rowptr, col, val};
  if (jacobi_scale(&ah, sval, dm) != 0) {
    free(sval);
    free(dm);
    return -1;
  }
  const csr_t a = {n, rowptr, col, sval};
  double* v = (double*)malloc(sizeof(double) * (size_t)n * 11);
  double *b = v, *x = v + n, *r = v + 2 * n, *z = v + 3 * n, *p = v + 4 * n, *q = v + 5 * n;
  double *r_old = v + 6 * n, *w0 = v + 7 * n, *w1 = v + 8 * n, *w2 = v + 9 * n, *t = v + 10 * n;
  cheb_t c;
  cheb_scalars(lmin, lmax, k, s, &c);
  int64_t nmv = 0, ndot = 0;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    b[i] = dm[i] * b_hat[i];
    x[i] = 0.0;
    r[i] = b[i];
  }
  const double bnorm = sqrt(dot(n, b, b));
  double relres = bnorm > 0.0 ? 1.0 : 0.0;
  int it = 0, converged = 0, breakdown = 0;
  if (!(bnorm > 0.0)) {
    converged = 1;
  } else {
    cheb_apply(&a, r, &c, k, z, w0, w1, w2, &nmv);
    double gamma = dot(n, r, z);
    ++ndot;
    if (!(gamma > 0.0)) breakdown = 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) p[i] = z[i];
    while (!breakdown && it < maxit) {
      ++it;
      spmv(&a, p, q);
      ++nmv;
      const double pq = dot(n, p, q);
      ++ndot;
      if (!(pq > 0.0)) {
        breakdown = 1;
        break;
      }
      const double alpha = gamma / pq;
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) {
        x[i] += alpha * p[i];
        if (flexible) r_old[i] = r[i];
        r[i] -= alpha * q[i];
      }
      const double rnorm = sqrt(dot(n, r, r));
      ++ndot;
      relres = rnorm / bnorm;
      if (g_progress > 0 && it % g_progress == 0) {
        fprintf(stderr, "oracle iteration %d: relres %.3e\n", it, relres);
        fflush(stderr);
      }
      if (!isfinite(rnorm)) {
        breakdown = 1;
        break;
      }
      if (relres < tol) {
        converged = 1;
        break;
      }
      cheb_apply(&a, r, &c, k, z, w0, w1, w2, &nmv);
      const double gamma_new = dot(n, r, z);
      ++ndot;
      if (!(gamma_new > 0.0)) {
        breakdown = 1;
        break;
      }
      double beta;
      if (flexible) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) t[i] = r[i] - r_old[i];
        beta = dot(n, z, t) / gamma;
        ++ndot;
      } else {
        beta = gamma_new / gamma;
      }
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
      gamma = gamma_new;
    }
  }
  /* outputs: x_hat, recomputed residuals */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) x_hat[i] = dm[i] * x[i];
  spmv(&a, x, t);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) t[i] = b[i] - t[i];
  const double rt = sqrt(dot(n, t, t));
  spmv(&ah, x_hat, t);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) t[i] = b_hat[i] - t[i];
  const double rth = sqrt(dot(n, t, t)), bhn = sqrt(dot(n, b_hat, b_hat));
  st->iters = it;
  st->converged = converged;
  st->breakdown = breakdown;
  st->relres = relres;
  st->relres_true = bnorm > 0.0 ? rt / bnorm : 0.0;
  st->relres_true_hat = bhn > 0.0 ? rth / bhn : 0.0;
  st->n_spmv = nmv;
  st->n_dot = ndot;
  free(c.rho);
  free(v);
  free(sval);
  free(dm);
  return 0;
}

/* Threads the calls above use (omp_set_num_threads for this library's runtime). */
void ncomp_set_threads(int nt) { omp_set_num_threads(nt > 0 ? nt : 1); }
int ncomp_max_threads(void) { return omp_get_max_threads(); }

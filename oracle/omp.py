"""ctypes binding of the C/OpenMP FP64 oracle (nc_omp.c).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests and the
benchmark's CPU-baseline leg use it; the GPU library never does.  It computes
what ``nc.nc_pcg`` and ``nc.nc_apply_unscaled`` compute, in the same order, with
the rows split over host threads (results are deterministic for a given thread
count); its pins are in ``tests/test_oracle_omp.py``.
"""

import ctypes
import os
import shutil
import subprocess
from dataclasses import dataclass

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_DIR, "nc_omp.c")
LIB = os.path.join(_DIR, "libnc_omp.so")
_lib = None


class _Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("breakdown", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("relres", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("relres_true_hat", ctypes.c_double), ("n_spmv", ctypes.c_int64), ("n_dot", ctypes.c_int64)]


def build(verbose: bool = False) -> str:
    """Compile nc_omp.c with gcc (-O2 -fopenmp, FMA contraction off) into libnc_omp.so."""
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("no C compiler for the OpenMP oracle")
    tmp = LIB + ".tmp"
    cmd = [cc, "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"building the OpenMP oracle failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def load(path: str = None):
    """The oracle library (built on first use); `path` loads another build of the same source."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = _declare(ctypes.CDLL(LIB))
    return _lib


def _declare(lib):
    i64, f64, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.ncomp_pcg.argtypes = [i64, vp, vp, vp, vp, f64, f64, ctypes.c_int, f64, f64, ctypes.c_int, ctypes.c_int,
                              vp, ctypes.POINTER(_Stats)]
    lib.ncomp_pcg.restype = ctypes.c_int
    lib.ncomp_apply_unscaled.argtypes = [i64, vp, vp, vp, vp, f64, f64, ctypes.c_int, f64, vp]
    lib.ncomp_apply_unscaled.restype = ctypes.c_int
    lib.ncomp_set_threads.argtypes = [ctypes.c_int]
    lib.ncomp_set_progress.argtypes = [ctypes.c_int]
    lib.ncomp_max_threads.restype = ctypes.c_int
    return lib


def set_threads(n: int) -> None:
    """Host threads of the following calls."""
    load().ncomp_set_threads(int(n))


def set_progress(every: int) -> None:
    """Print the iteration count and residual to stderr every `every` PCG iterations (0: never)."""
    load().ncomp_set_progress(int(every))


def max_threads() -> int:
    return int(load().ncomp_max_threads())


def _csr(rowptr, colind, values):
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(colind, dtype=np.int32)
    v = np.ascontiguousarray(values, dtype=np.float64)
    if int(np.asarray(rowptr)[-1]) >= 2 ** 31:
        raise ValueError("nnz must be below 2^31")
    return rp, ci, v


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class OmpResult:
    x_hat: np.ndarray
    iters: int
    converged: bool
    breakdown: bool
    relres: float
    relres_true: float
    relres_true_hat: float
    n_spmv: int
    n_dot: int


def nc_pcg(rowptr, colind, values, b_hat, lambda_min, lambda_max, k, s=1.001, tol=1e-8, maxit=100000,
           flexible=False, lib=None) -> OmpResult:
    """PCG with the degree-k NC preconditioner on the Jacobi-scaled system (as ``nc.nc_pcg``)."""
    rp, ci, v = _csr(rowptr, colind, values)
    n = len(rp) - 1
    b = np.ascontiguousarray(b_hat, dtype=np.float64)
    x = np.zeros(n)
    st = _Stats()
    rc = (lib or load()).ncomp_pcg(n, _p(rp), _p(ci), _p(v), _p(b), float(lambda_min), float(lambda_max), int(k),
                                   float(s), float(tol), int(maxit), int(bool(flexible)), _p(x), ctypes.byref(st))
    if rc != 0:
        raise ValueError("operator diagonal has a non-positive entry")
    return OmpResult(x, st.iters, bool(st.converged), bool(st.breakdown), st.relres, st.relres_true,
                     st.relres_true_hat, st.n_spmv, st.n_dot)


def nc_apply_unscaled(rowptr, colind, values, r_hat, lambda_min, lambda_max, k, s=1.001, lib=None) -> np.ndarray:
    """D^-1/2 p_k(A) D^-1/2 r_hat (as ``nc.nc_apply_unscaled``)."""
    rp, ci, v = _csr(rowptr, colind, values)
    n = len(rp) - 1
    r = np.ascontiguousarray(r_hat, dtype=np.float64)
    z = np.empty(n)
    rc = (lib or load()).ncomp_apply_unscaled(n, _p(rp), _p(ci), _p(v), _p(r), float(lambda_min),
                                              float(lambda_max), int(k), float(s), _p(z))
    if rc != 0:
        raise ValueError("operator diagonal has a non-positive entry")
    return z

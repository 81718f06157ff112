"""ctypes declarations of include/pcheb.h and argument-marshalling wrappers."""

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libpcheb.so"

STATUS = {
    0: "OK",
    1: "INVALID",
    2: "NOT_SPD",
    3: "OOM",
    4: "HIP",
    5: "NOT_CONVERGED",
    6: "BREAKDOWN",
    7: "BUDGET",
    8: "NOT_FOUND",
    9: "PENDING",
}

OP_KIND = {"csr": 0, "sell": 1, "stencil7": 2, "stencil27h": 3}
PREC = {"f64": 0, "f32": 1, "bf16": 2}
FORM = {"chebyshev": 0, "newton": 1}

PCG_FLEXIBLE = 0x1
PCG_X0_GIVEN = 0x2
PCG_TIME_KERNELS = 0x4
PCG_NO_GRAPH = 0x8
PCG_REFRESH = 0x10


class PchebError(RuntimeError):
    """A pcheb call returned a status other than OK (or an expected one)."""

    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class COperator(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("rowptr", ctypes.c_void_p),
        ("colind", ctypes.c_void_p),
        ("values", ctypes.c_void_p),
        ("nnz", ctypes.c_int64),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("cell_coeff", ctypes.c_void_p),
        ("sell_C", ctypes.c_int32),
        ("sell_sigma", ctypes.c_int32),
    ]


class CParams(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32),
        ("lambda_min", ctypes.c_double),
        ("lambda_max", ctypes.c_double),
        ("theta_scale", ctypes.c_double),
        ("prec", ctypes.c_int32),
        ("fuse_steps", ctypes.c_int32),
        ("form", ctypes.c_int32),
        ("block_size", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class CStats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("pad0", ctypes.c_int32),
        ("relres", ctypes.c_double),
        ("relres_true", ctypes.c_double),
        ("relres_true_hat", ctypes.c_double),
        ("n_spmv", ctypes.c_int64),
        ("n_dot", ctypes.c_int64),
        ("seconds", ctypes.c_double),
        ("step_ms", ctypes.c_double),
        ("step_launches", ctypes.c_int64),
    ]


class CServeRequest(ctypes.Structure):
    _fields_ = [
        ("op", COperator),
        ("k", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("lambda_min", ctypes.c_double),
        ("lambda_max", ctypes.c_double),
        ("theta_scale", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("maxit", ctypes.c_int32),
        ("fuse_steps", ctypes.c_int32),
        ("b", ctypes.c_void_p),
        ("x", ctypes.c_void_p),
        ("op_key", ctypes.c_uint64),
    ]


class CServeStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "submitted", "admitted", "completed", "rejected", "cancelled", "queued", "active", "groups",
        "groups_created", "groups_evicted", "bytes_in_use", "bytes_high_water", "budget", "launches")] + [
        ("batch_hist", ctypes.c_int64 * 8)]


_lib = None

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_allocator_refs = None  # the installed callbacks, kept alive while the library may call them


def library_path() -> str:
    return os.path.join(_PKG, _LIB_NAME)


def load_library():
    """Load libpcheb.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2008_01440_amd.build.build()")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
    lib.pcheb_setup.argtypes = [ctypes.POINTER(COperator), ctypes.POINTER(CParams), vp, ctypes.POINTER(vp)]
    lib.pcheb_apply.argtypes = [vp, vp, vp, i32, i64, vp]
    lib.pcheb_matvec.argtypes = [vp, vp, vp, i32, i64, vp]
    lib.pcg_solve.argtypes = [vp, vp, vp, i32, i64, f64, i32, u32, ctypes.POINTER(CStats), vp]
    lib.pcheb_destroy.argtypes = [vp]
    lib.pcheb_group_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]
    lib.pcheb_group_apply.argtypes = [vp, vp, vp, i64, vp]
    lib.pcg_solve_group.argtypes = [vp, vp, vp, i64, f64, i32, u32, ctypes.POINTER(CStats), vp]
    lib.pcheb_group_destroy.argtypes = [vp]
    lib.pcheb_last_error.argtypes = []
    lib.pcheb_last_error.restype = ctypes.c_char_p
    lib.pcheb_footprint_bytes.argtypes = [ctypes.POINTER(COperator), ctypes.POINTER(CParams), i32]
    lib.pcheb_footprint_bytes.restype = ctypes.c_size_t
    lib.pcheb_estimate_bounds.argtypes = [ctypes.POINTER(COperator), vp, i32, ctypes.POINTER(f64),
                                          ctypes.POINTER(f64), vp]
    lib.pcheb_estimate_bounds_noalloc.argtypes = [ctypes.POINTER(COperator), vp, i32, ctypes.POINTER(f64),
                                                  ctypes.POINTER(f64), vp]
    lib.pcheb_estimate_bounds_block.argtypes = [ctypes.POINTER(COperator), i32, vp, i32, ctypes.POINTER(f64),
                                                ctypes.POINTER(f64), vp]
    lib.pcheb_estimate_bounds_pdacg.argtypes = [ctypes.POINTER(COperator), vp, i32, f64, i32, ctypes.POINTER(f64),
                                                ctypes.POINTER(f64), ctypes.POINTER(i32), ctypes.POINTER(f64), vp]
    lib.pcheb_fill_uniform.argtypes = [vp, i64, ctypes.c_uint64, f64, f64, vp]
    lib.pcheb_set_allocator.argtypes = [ALLOC_FN, FREE_FN, vp]
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.pserve_create.argtypes = [ctypes.c_size_t, i32, ctypes.POINTER(vp)]
    lib.pserve_submit.argtypes = [vp, ctypes.POINTER(CServeRequest), u64p]
    lib.pserve_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(CStats)]
    lib.pserve_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(CStats)]
    lib.pserve_cancel.argtypes = [vp, ctypes.c_uint64]
    lib.pserve_get_stats.argtypes = [vp, ctypes.POINTER(CServeStats)]
    lib.pserve_destroy.argtypes = [vp]
    for name in ("pcheb_setup", "pcheb_apply", "pcheb_matvec", "pcg_solve", "pcheb_destroy",
                 "pcheb_group_create", "pcheb_group_apply", "pcg_solve_group", "pcheb_group_destroy",
                 "pcheb_set_allocator", "pcheb_estimate_bounds", "pcheb_estimate_bounds_noalloc", "pcheb_estimate_bounds_block", "pcheb_estimate_bounds_pdacg", "pcheb_fill_uniform", "pserve_create", "pserve_submit", "pserve_poll", "pserve_wait",
                 "pserve_cancel", "pserve_get_stats", "pserve_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def pcheb_last_error() -> str:
    return load_library().pcheb_last_error().decode()


def _check(status, allowed=(0,)):
    if status not in allowed:
        raise PchebError(status, pcheb_last_error())
    return status


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t, dtype_name):
    """Device pointer of a CUDA tensor with the expected dtype: contiguous, or 2-D with
    unit-stride rows (one vector per row, leading dimension = row stride)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device (CUDA/HIP) tensor")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise ValueError(f"expected dtype {dtype_name}, got {t.dtype}")
    if not (t.is_contiguous() or (t.dim() == 2 and t.stride(1) == 1)):
        raise ValueError("expected a contiguous tensor or rows with unit stride")
    return ctypes.c_void_p(t.data_ptr())


def _rhs_layout(t, n):
    """(nrhs, leading dimension) of a vector (n,) or a block of vectors (nrhs, >= n)."""
    if t.dim() == 1:
        return 1, n
    if t.shape[1] != n:
        raise ValueError(f"expected rows of length {n}, got {t.shape[1]}")
    return t.shape[0], t.stride(0)


class Operator:
    """The unscaled SPD operator A_hat; keeps the tensors it borrows alive."""

    def __init__(self, c: COperator, keep=()):
        self.c = c
        self._keep = tuple(keep)

    @property
    def n(self) -> int:
        return int(self.c.n)

    @staticmethod
    def stencil7(nx: int, ny: int = None, nz: int = None) -> "Operator":
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        c = COperator(kind=OP_KIND["stencil7"], n=nx * ny * nz, nx=nx, ny=ny, nz=nz)
        return Operator(c)

    @staticmethod
    def stencil27h(kappa) -> "Operator":
        """kappa: float64 device tensor of shape (nz, ny, nx) (x fastest)."""
        nz, ny, nx = kappa.shape
        c = COperator(kind=OP_KIND["stencil27h"], n=nx * ny * nz, nx=nx, ny=ny, nz=nz,
                      cell_coeff=_dptr(kappa, "float64"))
        return Operator(c, (kappa,))

    @staticmethod
    def csr(rowptr, colind, values, sell: bool = False, sigma: int = 1) -> "Operator":
        """CSR device tensors (int32, int32, float64); sell=True streams it as SELL-C-sigma."""
        n = rowptr.numel() - 1
        c = COperator(kind=OP_KIND["sell" if sell else "csr"], n=n, rowptr=_dptr(rowptr, "int32"),
                      colind=_dptr(colind, "int32"), values=_dptr(values, "float64"), nnz=values.numel(),
                      sell_C=64 if sell else 0, sell_sigma=sigma)
        return Operator(c, (rowptr, colind, values))


class Handle:
    """An owned pcheb_handle (release with pcheb_destroy or as a context manager)."""

    def __init__(self, ptr, op: Operator, params: CParams):
        self.ptr = ptr
        self.op = op
        self.params = params

    @property
    def n(self):
        return self.op.n

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        pcheb_destroy(self)


def _params(k, lambda_min, lambda_max, theta_scale, prec, fuse_steps, form="chebyshev", block_size=1):
    return CParams(k=k, lambda_min=lambda_min, lambda_max=lambda_max, theta_scale=theta_scale,
                   prec=PREC[prec] if isinstance(prec, str) else int(prec), fuse_steps=fuse_steps,
                   form=FORM[form] if isinstance(form, str) else int(form), block_size=int(block_size))


def pcheb_setup(op: Operator, k: int, lambda_min: float, lambda_max: float, theta_scale: float = 1.001,
                prec: str = "f64", fuse_steps: int = 1, stream=None, form: str = "chebyshev",
                block_size: int = 1) -> Handle:
    """form: "chebyshev" (the recurrence of Alg. 2) or "newton" (the recursion of Alg. 1,
    k = 2^nlev - 1).  block_size 3: the second-level preconditioner on the node-block Jacobi
    factor (CSR/SELL); the bounds then refer to W^T A W."""
    lib = load_library()
    p = _params(k, lambda_min, lambda_max, theta_scale, prec, fuse_steps, form, block_size)
    out = ctypes.c_void_p()
    _check(lib.pcheb_setup(ctypes.byref(op.c), ctypes.byref(p), _stream(stream), ctypes.byref(out)))
    return Handle(out, op, p)


def _same_layout(a, b, n):
    la, lb = _rhs_layout(a, n), _rhs_layout(b, n)
    if la != lb:
        raise ValueError("input and output blocks must have the same shape and row stride")
    return la


def pcheb_apply(h: Handle, r, z, stream=None):
    nrhs, ld = _same_layout(r, z, h.n)
    _check(load_library().pcheb_apply(h.ptr, _dptr(r, "float64"), _dptr(z, "float64"), nrhs, ld, _stream(stream)))


def pcheb_matvec(h: Handle, x, y, stream=None):
    nrhs, ld = _same_layout(x, y, h.n)
    _check(load_library().pcheb_matvec(h.ptr, _dptr(x, "float64"), _dptr(y, "float64"), nrhs, ld,
                                        _stream(stream)))


def pcg_solve(h: Handle, b, x, tol: float = 1e-8, maxit: int = 100000, flexible: bool = False,
              x0_given: bool = False, time_kernels: bool = False, graph: bool = True, refresh: bool = False,
              stream=None, check: bool = True) -> dict:
    """Returns the statistics as a dict (status name under 'status').  With check=True,
    BREAKDOWN and errors raise; NOT_CONVERGED is reported in the dict."""
    flags = ((PCG_FLEXIBLE if flexible else 0) | (PCG_X0_GIVEN if x0_given else 0)
             | (PCG_TIME_KERNELS if time_kernels else 0) | (0 if graph else PCG_NO_GRAPH)
             | (PCG_REFRESH if refresh else 0))
    st = CStats()
    nrhs, ld = _same_layout(b, x, h.n)
    status = load_library().pcg_solve(h.ptr, _dptr(b, "float64"), _dptr(x, "float64"), nrhs, ld, tol, maxit,
                                      flags, ctypes.byref(st), _stream(stream))
    if check:
        _check(status, allowed=(0, 5))
    out = {name: getattr(st, name) for name, _ in CStats._fields_ if name != "pad0"}
    out["status"] = STATUS.get(status, str(status))
    return out


def pcheb_destroy(h: Handle):
    if h.ptr:
        _check(load_library().pcheb_destroy(h.ptr))
        h.ptr = None


class Group:
    """An owned pcheb_group over borrowed handles (release with pcheb_group_destroy or as a
    context manager; the handles must outlive it)."""

    def __init__(self, ptr, handles):
        self.ptr = ptr
        self.handles = tuple(handles)

    @property
    def n(self):
        return self.handles[0].n

    def __len__(self):
        return len(self.handles)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        pcheb_group_destroy(self)


def pcheb_group_create(handles) -> Group:
    handles = list(handles)
    arr = (ctypes.c_void_p * len(handles))(*[h.ptr for h in handles])
    out = ctypes.c_void_p()
    _check(load_library().pcheb_group_create(arr, len(handles), ctypes.byref(out)))
    return Group(out, handles)


def _group_layout(g: Group, a, b):
    """Leading dimension of the (count, >= n) blocks a and b, one row per problem."""
    for t in (a, b):
        if t.dim() != 2 or t.shape[0] != len(g):
            raise ValueError(f"expected a block of {len(g)} rows, one per problem")
    count, ld = _same_layout(a, b, g.n)
    return ld


def pcheb_group_apply(g: Group, r, z, stream=None):
    ld = _group_layout(g, r, z)
    _check(load_library().pcheb_group_apply(g.ptr, _dptr(r, "float64"), _dptr(z, "float64"), ld, _stream(stream)))


def pcg_solve_group(g: Group, b, x, tol: float = 1e-8, maxit: int = 100000, flexible: bool = False,
                    x0_given: bool = False, graph: bool = True, stream=None, check: bool = True) -> list:
    """Per-problem statistics as dicts.  With check=True, BREAKDOWN and errors raise;
    NOT_CONVERGED is reported in the dicts."""
    flags = (PCG_FLEXIBLE if flexible else 0) | (PCG_X0_GIVEN if x0_given else 0) | (0 if graph else PCG_NO_GRAPH)
    ld = _group_layout(g, b, x)
    sts = (CStats * len(g))()
    status = load_library().pcg_solve_group(g.ptr, _dptr(b, "float64"), _dptr(x, "float64"), ld, tol, maxit, flags,
                                            sts, _stream(stream))
    if check:
        _check(status, allowed=(0, 5))
    out = []
    for st in sts:
        d = {name: getattr(st, name) for name, _ in CStats._fields_ if name != "pad0"}
        d["status"] = STATUS.get(int(st.status), str(int(st.status)))
        out.append(d)
    return out


def pcheb_group_destroy(g: Group):
    if g.ptr:
        _check(load_library().pcheb_group_destroy(g.ptr))
        g.ptr = None


def pcheb_footprint_bytes(op: Operator, k: int, lambda_min: float = 0.1, lambda_max: float = 2.0,
                          theta_scale: float = 1.001, prec: str = "f64", nrhs: int = 1, fuse_steps: int = 1,
                          form: str = "chebyshev", block_size: int = 1) -> int:
    p = _params(k, lambda_min, lambda_max, theta_scale, prec, fuse_steps, form, block_size)
    return int(load_library().pcheb_footprint_bytes(ctypes.byref(op.c), ctypes.byref(p), nrhs))


def pcheb_estimate_bounds(op: Operator, v0, nsteps: int = 30, stream=None, block_size: int = 1):
    """Lanczos extreme Ritz values of D^-1/2 A_hat D^-1/2 (block_size 1) or of the second-level
    operator W^T A W on the node-block Jacobi factor (block_size 3)."""
    lo, hi = ctypes.c_double(), ctypes.c_double()
    if block_size == 1:
        _check(load_library().pcheb_estimate_bounds(ctypes.byref(op.c), _dptr(v0, "float64"), nsteps,
                                                    ctypes.byref(lo), ctypes.byref(hi), _stream(stream)))
    else:
        _check(load_library().pcheb_estimate_bounds_block(ctypes.byref(op.c), int(block_size), _dptr(v0, "float64"),
                                                          nsteps, ctypes.byref(lo), ctypes.byref(hi), _stream(stream)))
    return lo.value, hi.value


def pcheb_estimate_bounds_noalloc(op: Operator, v0, nsteps: int = 30, stream=None):
    """pcheb_estimate_bounds without device allocation: the workspace is the library's fixed
    per-device scratch array (INVALID when the operator needs more than it holds)."""
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(load_library().pcheb_estimate_bounds_noalloc(ctypes.byref(op.c), _dptr(v0, "float64"), nsteps,
                                                        ctypes.byref(lo), ctypes.byref(hi), _stream(stream)))
    return lo.value, hi.value


def pcheb_estimate_bounds_pdacg(op: Operator, v0, power_iters: int = 30, dacg_tol: float = 1e-2,
                                dacg_maxit: int = 100000, stream=None) -> dict:
    """The paper's bound estimates (Sec. 5.1): lambda_max from `power_iters` power-method steps,
    lambda_min from DACG without preconditioning, stopped at relative eigen-residual `dacg_tol`.
    Returns {"lambda_min", "lambda_max", "dacg_steps", "dacg_relres"}."""
    lo, hi, rr = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    steps = ctypes.c_int32()
    _check(load_library().pcheb_estimate_bounds_pdacg(ctypes.byref(op.c), _dptr(v0, "float64"), int(power_iters),
                                                      float(dacg_tol), int(dacg_maxit), ctypes.byref(lo),
                                                      ctypes.byref(hi), ctypes.byref(steps), ctypes.byref(rr),
                                                      _stream(stream)))
    return {"lambda_min": lo.value, "lambda_max": hi.value, "dacg_steps": steps.value, "dacg_relres": rr.value}


def pcheb_fill_uniform(v, seed: int, lo: float = 0.0, hi: float = 1.0, stream=None):
    """v[i] = lo + (hi - lo) * U_i from the SplitMix64 stream of `seed` (float64 device vector)."""
    _check(load_library().pcheb_fill_uniform(_dptr(v, "float64"), v.numel(), seed & 0xFFFFFFFFFFFFFFFF, lo, hi,
                                             _stream(stream)))


def pcheb_set_allocator(allocator=None):
    """Install `allocator` (an object with alloc(nbytes) -> int device pointer, 0 on failure,
    and free(ptr, nbytes)) as the source of all the library's device memory; None restores
    hipMalloc / hipFree.  Callbacks of an earlier allocator stay alive: blocks it handed out
    are returned to it."""
    global _allocator_refs
    lib = load_library()
    if allocator is None:
        _check(lib.pcheb_set_allocator(ALLOC_FN(), FREE_FN(), None))
        return

    def _alloc(nbytes, _ctx):
        try:
            return int(allocator.alloc(int(nbytes))) or None
        except Exception:  # noqa: BLE001 - reported to the library as a failed allocation
            return None

    def _free(ptr, nbytes, _ctx):
        allocator.free(int(ptr), int(nbytes))

    refs = (ALLOC_FN(_alloc), FREE_FN(_free), allocator)
    _check(lib.pcheb_set_allocator(refs[0], refs[1], None))
    _allocator_refs = (refs, _allocator_refs)


class TorchCachingAllocator:
    """Device memory for the library from PyTorch's caching allocator (torch.cuda.caching_allocator_alloc
    on the current device and stream), with counts of the blocks handed out and returned."""

    def __init__(self):
        self.live = {}
        self.n_alloc = 0
        self.n_free = 0
        self.bytes_alloc = 0

    def alloc(self, nbytes):
        import torch
        ptr = torch.cuda.caching_allocator_alloc(nbytes, device=torch.cuda.current_device())
        self.live[ptr] = nbytes
        self.n_alloc += 1
        self.bytes_alloc += nbytes
        return ptr

    def free(self, ptr, nbytes):
        import torch
        if self.live.pop(ptr, None) is None:
            raise RuntimeError(f"free of a block this allocator did not hand out: {ptr:#x}")
        self.n_free += 1
        torch.cuda.caching_allocator_delete(ptr)


def _stats_dict(st: CStats, status) -> dict:
    out = {name: getattr(st, name) for name, _ in CStats._fields_ if name != "pad0"}
    out["status"] = STATUS.get(status, str(status))
    return out


class Server:
    """A pserve_handle: continuous-batching solve server (see pserve_* in include/pcheb.h).

    Requests borrow their operator tensors and the b / x vectors until they finish;
    the server keeps references to them until then."""

    def __init__(self, hbm_budget: int, max_nrhs: int = 16):
        out = ctypes.c_void_p()
        _check(load_library().pserve_create(int(hbm_budget), int(max_nrhs), ctypes.byref(out)))
        self.ptr = out
        self._keep = {}

    def submit(self, op: Operator, b, x, k: int, tol: float = 1e-8, maxit: int = 100000, prec: str = "f64",
               lambda_min: float = 0.0, lambda_max: float = 0.0, theta_scale: float = 1.001, fuse_steps: int = 1,
               op_key: int = 0) -> int:
        """Queue a solve; lambda_max <= 0 asks the server to estimate the bounds.  Returns the id."""
        if b.shape != (op.n,) or x.shape != (op.n,):
            raise ValueError(f"b and x must be vectors of length {op.n}")
        req = CServeRequest(op=op.c, k=k, prec=PREC[prec] if isinstance(prec, str) else int(prec),
                            lambda_min=lambda_min, lambda_max=lambda_max, theta_scale=theta_scale, tol=tol,
                            maxit=maxit, fuse_steps=fuse_steps, b=_dptr(b, "float64"), x=_dptr(x, "float64"),
                            op_key=op_key)
        import torch
        torch.cuda.current_stream().synchronize()  # b and x are used on the server's own streams
        rid = ctypes.c_uint64()
        _check(load_library().pserve_submit(self.ptr, ctypes.byref(req), ctypes.byref(rid)))
        self._keep[rid.value] = (op, b, x)
        return rid.value

    def poll(self, rid: int):
        """None while running, else the statistics dict (the id is then released)."""
        done = ctypes.c_int32()
        st = CStats()
        _check(load_library().pserve_poll(self.ptr, rid, ctypes.byref(done), ctypes.byref(st)))
        if not done.value:
            return None
        self._keep.pop(rid, None)
        out = _stats_dict(st, st.status)
        if st.status != 0:
            out["error"] = pcheb_last_error()
        return out

    def wait(self, rid: int, check: bool = False) -> dict:
        """Block until the request finishes; the dict's 'status' is its final status."""
        st = CStats()
        status = load_library().pserve_wait(self.ptr, rid, ctypes.byref(st))
        self._keep.pop(rid, None)
        if check:
            _check(status, allowed=(0, 5))
        return _stats_dict(st, status)

    def cancel(self, rid: int):
        _check(load_library().pserve_cancel(self.ptr, rid))

    def stats(self) -> dict:
        st = CServeStats()
        _check(load_library().pserve_get_stats(self.ptr, ctypes.byref(st)))
        out = {name: getattr(st, name) for name, _ in CServeStats._fields_ if name != "batch_hist"}
        out["batch_hist"] = list(st.batch_hist)
        return out

    def close(self):
        if self.ptr:
            _check(load_library().pserve_destroy(self.ptr))
            self.ptr = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

"""The C-ABI library on the host: it loads, exports every declared entry point,
its structs have the layout the C compiler gives them, and argument checks that
run before any device work return the documented statuses (no GPU needed)."""

import ctypes
import os
import re
import shutil
import subprocess

import pytest

import paper_2008_01440_amd as pc
from paper_2008_01440_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcheb.h")

pytestmark = pytest.mark.skipif(not os.path.exists(_abi.library_path()), reason="libpcheb.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?!typedef\b)(?:const\s+)?[a-z_0-9]+\s*\**\s*([a-z_0-9]+)\s*\(", text,
                                 flags=re.M)))


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ("pcheb_setup", "pcheb_apply", "pcg_solve", "pcheb_matvec", "pcheb_destroy", "pcheb_last_error",
                 "pcheb_footprint_bytes", "pcheb_set_allocator", "pcheb_estimate_bounds",
                 "pcheb_estimate_bounds_noalloc", "pcheb_estimate_bounds_pdacg",
                 "pcheb_estimate_bounds_block", "pcheb_group_create", "pcheb_group_apply", "pcg_solve_group",
                 "pcheb_group_destroy", "pserve_create",
                 "pserve_submit", "pserve_poll",
                 "pserve_wait", "pserve_cancel", "pserve_get_stats", "pserve_destroy"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.library_path()], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    lib = pc.load_library()
    for f in declared_functions():
        assert hasattr(lib, f)


STRUCTS = (("pcheb_operator", _abi.COperator), ("pcheb_params", _abi.CParams), ("pcg_stats", _abi.CStats),
           ("pserve_request", _abi.CServeRequest), ("pserve_stats", _abi.CServeStats))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "pcheb.h"\n'
        "#define O(T, f) printf(#T \".\" #f \" %zu\\n\", offsetof(T, f))\n"
        "int main(void) {\n"
        + "".join(f' printf("{c} %zu\\n", sizeof({c}));\n' for c, _ in STRUCTS)
        + "".join(f" O({c}, {f});\n" for c, cls in STRUCTS for f, _ in cls._fields_)
        + " return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True)
    lines = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True,
                                                                text=True).stdout.splitlines())
    for cname, cls in STRUCTS:
        assert int(lines[cname]) == ctypes.sizeof(cls)
        for f, _ in cls._fields_:
            assert int(lines[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)


def _setup_status(op, k=5, lmin=0.1, lmax=1.9, s=1.0, prec=0, form=0, block_size=0):
    lib = pc.load_library()
    p = _abi.CParams(k=k, lambda_min=lmin, lambda_max=lmax, theta_scale=s, prec=prec, fuse_steps=1, form=form,
                     block_size=block_size)
    out = ctypes.c_void_p()
    return lib.pcheb_setup(ctypes.byref(op.c), ctypes.byref(p), None, ctypes.byref(out))


@pytest.mark.parametrize("kw,what", [
    (dict(k=-1), "degree"), (dict(k=1001), "degree"), (dict(lmin=0.0), "lambda"), (dict(lmin=2.0), "lambda"),
    (dict(s=0.99), "theta_scale"), (dict(prec=7), "precision"), (dict(form=2), "form"),
    (dict(k=5, form=1), "Newton"), (dict(k=6, form=1), "Newton"), (dict(k=7, form=1, prec=2), "Newton"),
    (dict(block_size=2), "block_size"), (dict(block_size=3), "block_size"), (dict(block_size=-1), "block_size"),
    (dict(k=33, prec=2), "bfloat16"), (dict(k=100, prec=2), "bfloat16"),
])
def test_setup_rejects_bad_parameters(kw, what):
    assert _setup_status(pc.Operator.stencil7(4), **kw) == 1
    assert what.split("_")[0] in pc.pcheb_last_error()


def test_setup_rejects_bad_operators():
    op = pc.Operator.stencil7(4)
    op.c.n = 65
    assert _setup_status(op) == 1 and "nx*ny*nz" in pc.pcheb_last_error()
    csr = _abi.Operator(_abi.COperator(kind=0, n=10))
    assert _setup_status(csr) == 1 and "CSR" in pc.pcheb_last_error()
    sell = _abi.Operator(_abi.COperator(kind=1, n=10, rowptr=8, colind=8, values=8, nnz=10, sell_C=32,
                                        sell_sigma=1))
    assert _setup_status(sell) == 1 and "64" in pc.pcheb_last_error()
    h27 = _abi.Operator(_abi.COperator(kind=3, n=8, nx=2, ny=2, nz=2))
    assert _setup_status(h27) == 1 and "cell_coeff" in pc.pcheb_last_error()
    bad = _abi.Operator(_abi.COperator(kind=9, n=8, nx=2, ny=2, nz=2))
    assert _setup_status(bad) == 1


def test_null_arguments():
    lib = pc.load_library()
    assert lib.pcheb_setup(None, None, None, None) == 1
    assert lib.pcheb_apply(None, None, None, 1, 1, None) == 1
    assert lib.pcg_solve(None, None, None, 1, 1, 1e-8, 10, 0, None, None) == 1
    assert lib.pcheb_destroy(None) == 0
    lo, hi = ctypes.c_double(), ctypes.c_double()
    assert lib.pcheb_estimate_bounds(None, None, 30, ctypes.byref(lo), ctypes.byref(hi), None) == 1
    assert lib.pcheb_estimate_bounds_pdacg(None, None, 30, 1e-2, 100, ctypes.byref(lo), ctypes.byref(hi), None, None,
                                           None) == 1
    assert lib.pcheb_estimate_bounds_block(None, 3, None, 30, ctypes.byref(lo), ctypes.byref(hi), None) == 1


def test_pdacg_argument_checks():
    """Argument errors are reported before any device work (the operator is never touched)."""
    lib = pc.load_library()
    lo, hi = ctypes.c_double(), ctypes.c_double()
    op = pc.Operator.stencil7(4)
    args = lambda it, tol, mx, a=ctypes.byref(lo), b=ctypes.byref(hi): lib.pcheb_estimate_bounds_pdacg(
        ctypes.byref(op.c), None, it, tol, mx, a, b, None, None, None)
    assert args(0, 1e-2, 10) == 1 and "power_iters" in pc.pcheb_last_error()
    assert args(5, -1.0, 10) == 1 and "dacg_tol" in pc.pcheb_last_error()
    assert args(5, float("nan"), 10) == 1 and "dacg_tol" in pc.pcheb_last_error()
    assert args(5, 1e-2, -1) == 1 and "dacg_maxit" in pc.pcheb_last_error()
    assert args(5, 1e-2, 10, None) == 1 and "null" in pc.pcheb_last_error()
    assert args(5, 1e-2, 10) == 1 and "null" in pc.pcheb_last_error()  # v0 is NULL


def test_server_argument_checks():
    lib = pc.load_library()
    out = ctypes.c_void_p()
    assert lib.pserve_create(1 << 30, 0, ctypes.byref(out)) == 1 and "max_nrhs" in pc.pcheb_last_error()
    assert lib.pserve_create(1 << 30, 65, ctypes.byref(out)) == 1
    assert lib.pserve_create(0, 4, ctypes.byref(out)) == 1 and "budget" in pc.pcheb_last_error()
    assert lib.pserve_create(1 << 30, 4, None) == 1
    rid = ctypes.c_uint64()
    assert lib.pserve_submit(None, None, ctypes.byref(rid)) == 1 and "server" in pc.pcheb_last_error()
    assert lib.pserve_poll(None, 1, None, None) == 1
    assert lib.pserve_wait(None, 1, None) == 1
    assert lib.pserve_cancel(None, 1) == 1
    assert lib.pserve_get_stats(None, None) == 1
    assert lib.pserve_destroy(None) == 0
    assert lib.pcheb_fill_uniform(None, -1, 0, 0.0, 1.0, None) == 1
    assert lib.pcheb_fill_uniform(None, 5, 0, 0.0, 1.0, None) == 1
    assert lib.pcheb_fill_uniform(8, 5, 0, 1.0, 0.0, None) == 1 and "lo <= hi" in pc.pcheb_last_error()


def test_footprint_scales_with_precision_and_rhs():
    op = pc.Operator.stencil7(64)
    f64 = pc.pcheb_footprint_bytes(op, 20, prec="f64")
    f32 = pc.pcheb_footprint_bytes(op, 20, prec="f32")
    bf = pc.pcheb_footprint_bytes(op, 20, prec="bf16")
    assert f64 > f32 > bf > 64 ** 3 * 40
    assert pc.pcheb_footprint_bytes(op, 20, prec="f32", nrhs=4) > 3 * f32 - 1e6


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "_PKG", str(tmp_path))
    with pytest.raises(RuntimeError, match="missing"):
        _abi.load_library()


def test_block_size_needs_csr_with_node_rows():
    """The node-block first level is for CSR/SELL operators whose size is a multiple of 3."""
    csr = _abi.Operator(_abi.COperator(kind=0, n=10, rowptr=8, colind=8, values=8, nnz=10))
    assert _setup_status(csr, block_size=3) == 1 and "multiple of 3" in pc.pcheb_last_error()
    lib = pc.load_library()
    lo, hi = ctypes.c_double(), ctypes.c_double()
    assert lib.pcheb_estimate_bounds_block(ctypes.byref(pc.Operator.stencil7(3).c), 3, None, 30, ctypes.byref(lo),
                                           ctypes.byref(hi), None) == 1
    assert lib.pcheb_estimate_bounds_block(ctypes.byref(csr.c), 2, None, 30, ctypes.byref(lo),
                                           ctypes.byref(hi), None) == 1 and "block_size" in pc.pcheb_last_error()


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N with N > 1 exits with status 2 and a JSON message, before touching a GPU."""
    import json
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_set_allocator_needs_both_functions():
    lib = pc.load_library()
    alloc = _abi.ALLOC_FN(lambda nbytes, ctx: None)
    free = _abi.FREE_FN(lambda ptr, nbytes, ctx: None)
    assert lib.pcheb_set_allocator(alloc, _abi.FREE_FN(), None) == 1 and "both" in pc.pcheb_last_error()
    assert lib.pcheb_set_allocator(_abi.ALLOC_FN(), free, None) == 1
    assert lib.pcheb_set_allocator(_abi.ALLOC_FN(), _abi.FREE_FN(), None) == 0  # hipMalloc / hipFree again
    pc.pcheb_set_allocator(None)


def test_noalloc_estimator_argument_checks():
    """The allocation-free estimator refuses bad arguments and operators whose workspace exceeds its
    fixed scratch before any device work: 80^3 7-point with 30 steps needs
    8 (31 * 512000 + 2 * 512000 + 93) + 524288 bytes > 128 MiB."""
    lib = pc.load_library()
    lo, hi = ctypes.c_double(), ctypes.c_double()
    call = lambda op, steps, v0=None: lib.pcheb_estimate_bounds_noalloc(
        ctypes.byref(op.c) if op else None, v0, steps, ctypes.byref(lo), ctypes.byref(hi), None)
    assert call(None, 30) == 1 and "null" in pc.pcheb_last_error()
    assert call(pc.Operator.stencil7(4), 0) == 1 and "nsteps" in pc.pcheb_last_error()
    assert call(pc.Operator.stencil7(4), 30, v0=8) == 1 and "aligned" in pc.pcheb_last_error()
    assert call(pc.Operator.stencil7(80), 30) == 1 and "workspace" in pc.pcheb_last_error()
    assert call(pc.Operator.stencil7(79), 1001) == 1 and "nsteps" in pc.pcheb_last_error()


def test_group_argument_checks():
    """Group calls refuse null groups, null or repeated handles and bad counts before any device work
    (a handle pointer is never dereferenced when the list itself is invalid)."""
    lib = pc.load_library()
    out = ctypes.c_void_p()
    handles = (ctypes.c_void_p * 2)(None, None)
    assert lib.pcheb_group_create(None, 1, ctypes.byref(out)) == 1 and "null" in pc.pcheb_last_error()
    assert lib.pcheb_group_create(handles, 0, ctypes.byref(out)) == 1 and "count" in pc.pcheb_last_error()
    assert lib.pcheb_group_create(handles, 1025, ctypes.byref(out)) == 1 and "count" in pc.pcheb_last_error()
    assert lib.pcheb_group_create(handles, 2, ctypes.byref(out)) == 1 and "null handle" in pc.pcheb_last_error()
    assert lib.pcheb_group_create(handles, 1, None) == 1
    assert out.value is None
    assert lib.pcheb_group_apply(None, None, None, 8, None) == 1 and "null group" in pc.pcheb_last_error()
    assert lib.pcg_solve_group(None, None, None, 8, 1e-8, 10, 0, None, None) == 1
    assert lib.pcheb_group_destroy(None) == 0

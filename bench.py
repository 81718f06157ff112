"""Benchmark: NC-preconditioned PCG solves/s on one MI355X.

Workload (one "step" = one complete pcg_solve): 3-D 7-point Poisson on a 256^3
grid (16,777,216 unknowns), Dirichlet boundaries, right-hand side b = A x*
with x* i.i.d. U[-1, 1] (SplitMix64, seed 0), eigenvalue bounds from 30
Lanczos steps on the GPU with lambda_max widened by 1.01, theta scale
s = 1.001, tol 1e-8, x0 = 0.  The headline is the matrix-free operator with
the degree-50 Chebyshev recurrence in float64 (the precision of the paper and
of the configuration), four steps per pass over memory, inside a float64
flexible PCG, timed on the library's default path (HIP-graph replay).  In the
same run it times plain float64 PCG (k = 0, the Jacobi-scaled "diagonal
preconditioner" baseline of the paper), the mixed-precision variants (float32
and bfloat16 recurrences inside the float64 PCG) and the CSR operator; reports
the dominant kernel (the fused pass of four middle Chebyshev steps) against
the HBM roofline with HIP events from separate kernel-timed solves; runs a
short serving leg (200 requests of the mixed 7-/27-point trace at 50 req/s);
and solves the same problem once with the FP64 CPU oracle (the C/OpenMP one,
on all host threads and on one), which gives both the CPU baseline and the
iteration and solution differences of every GPU variant against the oracle.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--k 50] [--prec f64] [--fuse 4] [--sweep]
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PCG solves/s + P_k(A) HBM GB/s vs FP64 plain PCG; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
BF16_MAX_K = 32  # the library refuses bfloat16 recurrences of higher degree
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cheb_step_stencil7_256_traffic.md")
KERNEL_SOURCES = ["common.hpp", "launch.hpp", "fused_stencil.hpp", "fused_launch.hpp"]  # the fused pass and its launch


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2008_01440_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(prec, steps_per_pass):
    """HBM bytes per middle-step launch from the committed rocprofv3 counter summary,
    or None when it is missing or the kernel sources changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and line.startswith("- "):
            key, _, v = line[2:].partition(":")
            vals[key.strip()] = v.strip()
    if vals.get("source_hash") != kernel_source_hash():
        return None
    v = vals.get(f"traffic_bytes_per_launch_{prec}_s{steps_per_pass}")
    return float(v) if v else None


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if xs else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256, help="grid points per axis")
    ap.add_argument("--k", type=int, default=50, help="polynomial degree of the flagship solve")
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16"],
                    help="precision of the headline's recurrence (the others run as variants)")
    ap.add_argument("--fuse", type=int, default=4, help="Chebyshev steps per pass of the matrix-free operator")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 1 GiB device copy (reference dispatch for DRAM byte counters)")
    ap.add_argument("--sweep-fuse", default="1", help="steps per pass tried by the sweep (stencil7 only)")
    ap.add_argument("--sweep", action="store_true", help="sweep degrees, precisions and operators")
    ap.add_argument("--sweep-kinds", default="stencil7,csr,sell", help="operators of the sweep")
    ap.add_argument("--sweep-degrees", default="0,5,10,20,30,50,100", help="degrees of the sweep")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-oracle", default="omp", choices=["omp", "numpy"],
                    help="oracle of the CPU baseline and the parity check: C/OpenMP (all host threads and one) "
                         "or numpy/scipy (one thread)")
    ap.add_argument("--no-variants", action="store_true", help="time the flagship only (no variants, no batching leg)")
    ap.add_argument("--no-serve", action="store_true", help="skip the short serving leg")
    ap.add_argument("--no-batching", action="store_true",
                    help="skip the short batching leg (four right-hand sides of a 64^3 elasticity operator in one "
                         "solve; 16 27-point operators of 32^3 and 64^3 in one grouped solve)")
    ap.add_argument("--bench-serve-requests", type=int, default=200,
                    help="requests of the serving leg of the default run (50 req/s)")
    ap.add_argument("--serve", action="store_true",
                    help="run the serving scenario instead: Poisson arrivals of mixed 7-point / 27-point solves")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-rates", default="50", help="arrival rates (req/s) to run; 'inf' submits all at once")
    ap.add_argument("--serve-nrhs", type=int, default=4, help="concurrent solves per resident operator")
    ap.add_argument("--serve-budget-gib", type=float, default=128.0)
    ap.add_argument("--serve-k", type=int, default=30)
    ap.add_argument("--serve-prec", default="f32", choices=["f64", "f32", "bf16"])
    ap.add_argument("--serve-fuse", type=int, default=4, help="steps per pass of the 7-point requests")
    ap.add_argument("--configs", default="",
                    help="comma-separated subset of c1,c2,c3,c4: per-configuration measurements, one JSON line each")
    ap.add_argument("--paper-scale", default="",
                    help="comma-separated nx of lap3d(nx) solves at the paper's sizes (e.g. 512,1024)")
    ap.add_argument("--paper-bounds", default="exact", choices=["exact", "pdacg"],
                    help="bounds of the --paper-scale solves: closed form, or the paper's power method + DACG")
    ap.add_argument("--nrhs-study", action="store_true",
                    help="C4 elasticity (SELL and CSR, F32, k=20): four right-hand sides in one batched solve "
                         "(matrix read once per launch) against the four solved one at a time")
    ap.add_argument("--cpu-baseline-configs", default="",
                    help="comma-separated c3,c4: the CPU baseline at full size, one FP64 oracle solve (k = 20) on "
                         "the host threads, beside GPU F64 and F32 solves of the same problem")
    ap.add_argument("--group-study", action="store_true",
                    help="work lists: 16 same-shape problems with different operators solved one at a time "
                         "against one grouped solve (27-point harmonic 32^3/64^3/96^3, elasticity 24^3)")
    ap.add_argument("--bounds", action="store_true",
                    help="compare bound estimators (Lanczos, power method + DACG, exact) on the flagship problem")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1 (sharding over several GPUs "
                                   "is a design, not implemented)", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import paper_2008_01440_amd as pc
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pc.load_library()
    if args.serve:
        for rate in args.serve_rates.split(","):
            run_serve(args, float(rate), torch, pc, W, dev)
        return
    if args.paper_scale:
        for nx in (int(v) for v in args.paper_scale.split(",")):
            run_paper_scale(nx, torch, pc, W, dev, args.paper_bounds)
        return
    if args.bounds:
        run_bounds(args, torch, pc, W, dev)
        return
    if args.nrhs_study:
        run_nrhs_study(torch, pc, W, dev)
        return
    if args.group_study:
        run_group_study(torch, pc, W, dev)
        return
    if args.cpu_baseline_configs:
        cpu_baseline_configs([c for c in args.cpu_baseline_configs.split(",") if c], torch, pc, W, dev)
        return
    configs = [c for c in args.configs.split(",") if c]
    for c in configs:
        if c != "c2":
            {"c1": run_c1, "c3": run_c3, "c4": run_c4}[c](torch, pc, W, dev)
    if configs and "c2" not in configs:
        return
    n1 = args.n
    n = n1 ** 3

    t = time.perf_counter()
    rp, ci, v = W.stencil7_csr(n1)
    xstar = W.uniform(0, n, -1.0, 1.0)
    b = W.rhs_from_solution(rp, ci, v, xstar)
    log(f"inputs: {n1}^3 grid, n={n}, nnz={int(rp[-1])} built in {time.perf_counter() - t:.1f}s")
    bt = torch.from_numpy(b).to(dev)
    xs_t = torch.from_numpy(xstar).to(dev)
    op_st = pc.Operator.stencil7(n1)

    v0 = torch.empty(n, dtype=torch.float64, device=dev)
    pc.pcheb_fill_uniform(v0, 7, 0.5, 1.5)  # SplitMix64 U[0.5, 1.5), seed 7, generated on the device
    torch.cuda.synchronize()
    t = time.perf_counter()
    lo, hi_ritz = pc.pcheb_estimate_bounds(op_st, v0, 30)
    torch.cuda.synchronize()
    lanczos_ms = 1e3 * (time.perf_counter() - t)
    hi = 1.01 * hi_ritz
    del v0
    exact_lo, exact_hi = W.stencil7_bounds(n1)
    log(f"bounds: Lanczos(30) [{lo:.6g}, {hi_ritz:.6g}] x1.01 -> {hi:.6g}  (exact [{exact_lo:.6g}, {exact_hi:.6g}]) "
        f"in {lanczos_ms:.0f} ms")

    csr_dev = None

    def operator(kind):
        nonlocal csr_dev
        if kind == "stencil7":
            return op_st
        if csr_dev is None:
            csr_dev = tuple(torch.from_numpy(a).to(dev) for a in (rp, ci, v))
        return pc.Operator.csr(*csr_dev, sell=(kind == "sell"), sigma=1)

    def run(kind, k, prec, steps, warmup, flexible=True, fuse=1, kernel_solves=0, keep_x=False):
        """`steps` timed solves on the default path (HIP-graph replay of iteration pairs), then
        `kernel_solves` more with HIP events around the middle Chebyshev steps of every
        application (events turn graph replay off, so they are timed apart)."""
        t0 = time.perf_counter()
        h = pc.pcheb_setup(operator(kind), k, lo, hi, 1.001, prec, fuse_steps=fuse)
        torch.cuda.synchronize()
        setup_ms = 1e3 * (time.perf_counter() - t0)
        x = torch.zeros(n, dtype=torch.float64, device=dev)
        for _ in range(warmup):
            pc.pcg_solve(h, bt, x, tol=1e-8, maxit=20000, flexible=flexible)
        torch.cuda.synchronize()
        lat, stats = [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            st = pc.pcg_solve(h, bt, x, tol=1e-8, maxit=20000, flexible=flexible)
            torch.cuda.synchronize()
            lat.append(1e3 * (time.perf_counter() - ts))
            stats.append(st)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        err = float(torch.linalg.vector_norm(x - xs_t) / torch.linalg.vector_norm(xs_t))
        step_ms, step_n = 0.0, 0
        if kernel_solves and k >= 3:
            xk = torch.zeros_like(x)
            for _ in range(kernel_solves):
                sk = pc.pcg_solve(h, bt, xk, tol=1e-8, maxit=20000, flexible=flexible, time_kernels=True)
                step_ms += sk["step_ms"]
                step_n += sk["step_launches"]
            torch.cuda.synchronize()
            del xk
        pc.pcheb_destroy(h)
        st = stats[-1]
        res = dict(kind=kind, k=k, prec=prec, fuse=fuse, steps=steps, solves_per_s=steps / total,
                   ms_per_solve=1e3 * total / steps, p50_ms=percentile(lat, 50), p99_ms=percentile(lat, 99),
                   iters=st["iters"], status=st["status"], relres=st["relres"], relres_true=st["relres_true"],
                   err_vs_xstar=err, n_spmv=st["n_spmv"], n_dot=st["n_dot"], setup_ms=setup_ms,
                   step_avg_us=(1e3 * step_ms / step_n) if step_n else None, step_launches=step_n)
        if keep_x:
            res["x"] = x.cpu().numpy()
        del x
        log(f"  {kind:8s} k={k:3d} {prec:4s} S={fuse}: {res['solves_per_s']:8.3f} solves/s  {res['ms_per_solve']:8.2f} ms  "
            f"iters={st['iters']:5d} relres_true={st['relres_true']:.2e} err={err:.2e}"
            + (f"  step {res['step_avg_us']:.1f} us" if step_n else ""))
        return res

    if "c2" in configs:
        rows = []
        for k in (0, 5, 20, 50, 100):
            x64 = None  # the matrix-free FP64 solution at this degree (the first row of each k)
            for kind, prec, fuse in (("stencil7", "f64", 4), ("stencil7", "f32", 4), ("stencil7", "bf16", 4),
                                     ("csr", "f64", 1), ("csr", "f32", 1), ("sell", "f64", 1), ("sell", "f32", 1)):
                if (k == 0 and prec != "f64") or (prec == "bf16" and k > BF16_MAX_K):
                    continue
                r = run(kind, k, prec, 2, 1, flexible=prec != "f64", kernel_solves=1 if k >= 3 else 0,
                        fuse=fuse if k >= 3 else 1, keep_x=True)
                xr = r.pop("x")
                if x64 is None:
                    x64 = xr
                r["rel_diff_vs_f64_solution"] = float(np.linalg.norm(xr - x64) / np.linalg.norm(x64))
                e = {"f64": 8, "f32": 4, "bf16": 2}[prec]
                if r["step_avg_us"]:
                    # per step: the operator's algorithmic bytes (values and column indices of the
                    # nonzeros, row pointers or chunk headers) plus 4 vectors (read y, s, y_{j-2}; write y_j)
                    meta = 4 * (n + 1) if kind == "csr" else 12 * (n // 64 + 1)
                    step_bytes = 4 * e * n if kind == "stencil7" else (e + 4) * int(rp[-1]) + meta + 4 * e * n
                    r["step_alg_gbs"] = round(step_bytes / (r["step_avg_us"] * 1e-6) / 1e9, 1)
                rows.append(r)
        print(json.dumps({"config": "c2", "workload": f"3-D 7-point Poisson {n1}^3, Lanczos(30) bounds x1.01, "
                          "b = A x*, tol 1e-8; matrix-free, CSR and SELL-C-sigma (C = 64, sigma = 1)",
                          "rows": rows}), flush=True)
        return

    if args.sweep:
        rows = []
        for kind in args.sweep_kinds.split(","):
            for prec in ("f64", "f32", "bf16"):
                for k in (int(d) for d in args.sweep_degrees.split(",")):
                    if (k == 0 and prec != "f64") or (prec == "bf16" and k > BF16_MAX_K):
                        continue
                    for fuse in (int(f) for f in args.sweep_fuse.split(",")):
                        if fuse > 1 and (kind != "stencil7" or k < 3):
                            continue
                        rows.append(run(kind, k, prec, 2, 1, kernel_solves=1 if k >= 3 else 0, fuse=fuse))
        print(json.dumps({"sweep": rows}))
        return

    # The headline: NC-PCG in the configuration's precision (float64 by default) on the
    # matrix-free operator, timed on the default path; the kernel times of the roofline
    # come from separate solves with HIP events around the middle Chebyshev steps.
    log("flagship:")
    flag = run("stencil7", args.k, args.prec, args.steps, args.warmup, fuse=args.fuse, kernel_solves=2, keep_x=True)
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 1073741824 bytes read, 1073741824 bytes written")
        del src, dst
    variants = {}
    if not args.no_variants:
        log("variants:")
        variants["fp64_plain_pcg"] = run("stencil7", 0, "f64", args.steps, 1, keep_x=True)
        for prec in ("f64", "f32", "bf16"):
            if prec != args.prec and (prec != "bf16" or args.k <= BF16_MAX_K):
                name = ("fp64" if prec == "f64" else f"mixed_{prec}") + "_nc"
                variants[name] = run("stencil7", args.k, prec, args.steps, 1, fuse=args.fuse, kernel_solves=2,
                                     keep_x=True)
        for prec in ("f64", "f32"):
            variants[f"csr_{prec}_nc"] = run("csr", args.k, prec, 2, 1, kernel_solves=1, keep_x=True)

    ceiling = hbm_triad_ceiling(torch, dev)

    def roofline_of(r):
        """Roofline of a stencil run's dominant kernel (the fused pass of S middle steps, or the
        single middle step): a middle step reads y_{j-1}, y_{j-2} and s and writes y_j (the
        7-point operator has no stored matrix), 4 e n bytes; a pass of S steps reads the same
        three vectors and writes two, 5 e n bytes."""
        prec = r["prec"]
        e = {"f64": 8, "f32": 4, "bf16": 2}[prec]
        S = min(r["fuse"], 4) if r["fuse"] > 1 else 1  # the library's clamp
        if S > 1 and (r["k"] - 2) % S != 0:
            log(f"note: {r['k'] - 2} middle steps are not a multiple of {S}; the timed launches mix pass kinds")
        alg_bytes = (5 if S > 1 else 4) * e * n
        avg_s = r["step_avg_us"] * 1e-6 * S
        achieved = alg_bytes / avg_s / 1e9
        if S > 1:
            name = ("KFusedPass64" if prec == "f64" else "KFusedPass") + f"<S={S},{prec}>"
            name += f" ({S} middle steps per launch)"
        else:
            name = f"KStencil7<SCALED,EpiChebStep<{prec}>> (middle step)"
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(prec, S), "kernel": name,
                "alg_bytes_per_launch": alg_bytes, "avg_launch_us": round(avg_s * 1e6, 2),
                "launches_timed": r["step_launches"] // S,
                "effective_step_gbs": round(4 * e * n / (r["step_avg_us"] * 1e-6) / 1e9, 1),
                "measured_triad_ceiling_gbs": round(ceiling, 1),
                "frac_of_triad_ceiling": round(achieved / ceiling, 4)}

    roofline = roofline_of(flag)

    batching = None
    if not (args.no_batching or args.no_variants):  # --no-variants: the flagship alone
        log("batching: several right-hand sides of one operator, several operators of one shape")
        keep = ("workload", "format", "n", "k", "prec", "nrhs", "problems", "single_solves_s", "batched_solve_s",
                "group_solve_s", "speedup", "bitwise_equal")
        batching = {
            "multi_rhs": [{kk: r[kk] for kk in keep if kk in r}
                          for r in run_nrhs_study(torch, pc, W, dev, N=64, formats=("sell256",), emit=False)],
            "work_list": [{kk: r[kk] for kk in keep if kk in r}
                          for r in run_group_study(torch, pc, W, dev, sizes=(32, 64), elasticity=None, emit=False)],
        }

    serving = None
    if not args.no_serve:
        log("serving:")
        serving = run_serve(args, 50.0, torch, pc, W, dev, nreq=args.bench_serve_requests, emit=False)

    cpu, parity = None, None
    if not args.no_cpu:
        cpu, ref_x, ref_iters = cpu_baseline(rp, ci, v, b, lo, hi, args.k, args.cpu_oracle)
        parity = {"oracle_iters": ref_iters, "bar": "iterations within +-2, relative solution difference <= 1e-6"}
        for name, r in [("headline", flag)] + list(variants.items()):
            if "x" not in r or r["k"] != args.k:
                continue
            d = float(np.linalg.norm(r["x"] - ref_x) / np.linalg.norm(ref_x))
            parity[name] = {"prec": r["prec"], "kind": r["kind"], "iters": r["iters"],
                            "iters_delta": r["iters"] - ref_iters, "rel_diff_vs_oracle": d,
                            "meets_bar": bool(abs(r["iters"] - ref_iters) <= 2 and d <= 1e-6)}
            r["rel_diff_vs_oracle"] = d
        if "fp64_plain_pcg" in variants:
            r = variants["fp64_plain_pcg"]
            r["rel_diff_vs_oracle"] = float(np.linalg.norm(r["x"] - ref_x) / np.linalg.norm(ref_x))

    prec_name = {"f64": "float64", "f32": "float32", "bf16": "bfloat16 storage with float32 arithmetic"}[args.prec]
    out = {
        "metric": METRIC,
        "value": round(flag["solves_per_s"], 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(flag["ms_per_solve"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "dtype_detail": f"P_k(A) recurrence in {prec_name}; outer PCG, dots and residual in f64",
        "data": "synthetic",
        "config": {"workload": f"3-D 7-point Poisson {n1}^3 ({n} unknowns), Dirichlet, b = A x*, x* ~ U[-1,1] "
                               f"seed 0; matrix-free operator; NC degree k={args.k}, theta scale 1.001; bounds "
                               f"Lanczos(30) with lambda_max x1.01; flexible PCG, tol 1e-8, x0 = 0",
                   "n": n, "k": args.k, "precision": args.prec, "operator": "stencil7 (matrix-free)",
                   "steps_per_pass": min(args.fuse, 4) if args.fuse > 1 else 1,
                   "lambda_min": lo, "lambda_max": hi},
        "latency_ms": {"p50": round(flag["p50_ms"], 3), "p99": round(flag["p99_ms"], 3)},
        "iters": flag["iters"],
        "relres_true": flag["relres_true"],
        "err_vs_xstar": flag["err_vs_xstar"],
        "rel_diff_vs_oracle": flag.get("rel_diff_vs_oracle"),
        "setup_ms": round(flag["setup_ms"], 2),
        "lanczos_ms": round(lanczos_ms, 2),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
    }
    if variants:
        keys = ("kind", "k", "prec", "solves_per_s", "ms_per_solve", "p50_ms", "p99_ms", "iters", "relres_true",
                "err_vs_xstar", "rel_diff_vs_oracle", "step_avg_us")
        out["variants"] = {name: {kk: r.get(kk) for kk in keys} for name, r in variants.items()}
        base = variants["fp64_plain_pcg"]["solves_per_s"]
        out["speedup_vs_fp64_plain_pcg"] = round(flag["solves_per_s"] / base, 3)
        out["speedup_vs_fp64_plain_pcg_by_variant"] = {
            name: round(r["solves_per_s"] / base, 3) for name, r in variants.items() if name != "fp64_plain_pcg"}
        for name, r in variants.items():
            if r["kind"] == "stencil7" and r["k"] >= 3 and r["step_avg_us"]:
                out.setdefault("roofline_by_variant", {})[name] = roofline_of(r)
    if batching:
        out["batching"] = batching
    if serving:
        out["serving"] = serving
    print(json.dumps(out))


def _timed_solves(torch, pc, h, b, reps, flexible, time_kernels=False, warmup=1):
    x = torch.zeros_like(b)
    for _ in range(warmup):
        pc.pcg_solve(h, b, x, tol=1e-8, maxit=50000, flexible=flexible, time_kernels=time_kernels)
    torch.cuda.synchronize()
    lat, st = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        st = pc.pcg_solve(h, b, x, tol=1e-8, maxit=50000, flexible=flexible, time_kernels=time_kernels)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    return st, x, lat


def run_c1(torch, pc, W, dev):
    """32^3 7-point Poisson, CSR FP64, k = 10, exact closed-form bounds, tol 1e-8: GPU solve
    latency, and the FP64 oracle's CPU seconds for the same solve on 1 and on all host cores."""
    import oracle
    from threadpoolctl import threadpool_limits

    N, k = 32, 10
    rp, ci, v = W.stencil7_csr(N)
    n = N ** 3
    xs = W.uniform(0, n, -1.0, 1.0)
    b = W.rhs_from_solution(rp, ci, v, xs)
    lo, hi = W.stencil7_bounds(N)
    d = [torch.from_numpy(a).to(dev) for a in (rp, ci, v)]
    bt = torch.from_numpy(b).to(dev)
    with pc.pcheb_setup(pc.Operator.csr(*d), k, lo, hi, 1.001, "f64") as h:
        st, x, lat = _timed_solves(torch, pc, h, bt, 50, False, warmup=3)
    err = float(np.linalg.norm(x.cpu().numpy() - xs) / np.linalg.norm(xs))
    cpu = {}
    cores = os.cpu_count() or 1
    for label, lim in (("1", 1), ("all", cores)):
        with threadpool_limits(limits=lim):
            t0 = time.perf_counter()
            ref = oracle.nc_pcg(rp, ci, v, b, lo, hi, k, s=1.001, tol=1e-8)
            cpu[label] = time.perf_counter() - t0
    print(json.dumps({"config": "c1", "workload": "3-D 7-point Poisson 32^3, CSR FP64, k=10, closed-form bounds, "
                      "b = A x*, tol 1e-8", "gpu_p50_ms": round(1e3 * percentile(lat, 50), 3),
                      "gpu_p99_ms": round(1e3 * percentile(lat, 99), 3), "gpu_solves_per_s": round(len(lat) / sum(lat), 1),
                      "gpu_iters": st["iters"], "oracle_iters": ref.iters, "err_vs_xstar": err,
                      "relres_true": st["relres_true"], "oracle_cpu_s_1core": round(cpu["1"], 4),
                      f"oracle_cpu_s_{cores}threads": round(cpu["all"], 4), "host_cores": cores}), flush=True)


def run_c3(torch, pc, W, dev):
    """192^3 27-point harmonic diffusion, lognormal(0, 2) cells: k in {10, 20, 40, 80} with the
    recurrence in F64, F32 and BF16 (F32 arithmetic), FP64 flexible PCG; errors of the mixed
    solutions against the F64 one."""
    N = 192
    n = N ** 3
    kappa = torch.from_numpy(W.harmonic27_kappa(N, N, N, seed=1)).to(dev)
    op = pc.Operator.stencil27h(kappa)
    xs = torch.empty(n, dtype=torch.float64, device=dev)
    pc.pcheb_fill_uniform(xs, 0, -1.0, 1.0)
    b = torch.empty_like(xs)
    v0 = torch.empty_like(xs)
    pc.pcheb_fill_uniform(v0, 7, 0.5, 1.5)
    lo, hi = pc.pcheb_estimate_bounds(op, v0, 30)
    hi *= 1.01
    # the operator's condition number: DACG's lambda_min (an upper estimate, Temple-tight at its
    # tolerance) and 300 power steps for lambda_max, the paper's estimators (Sec. 5.1)
    t0 = time.perf_counter()
    est = pc.pcheb_estimate_bounds_pdacg(op, v0, 300, 1e-3, 200000)
    est_s = time.perf_counter() - t0
    log(f"c3: Lanczos(30) [{lo:.6g}, {hi / 1.01:.6g}]; power(300) lambda_max {est['lambda_max']:.6g}, DACG(1e-3) "
        f"lambda_min {est['lambda_min']:.6g} in {est['dacg_steps']} steps ({est_s:.2f} s): "
        f"kappa ~ {est['lambda_max'] / est['lambda_min']:.4g}")
    del v0
    rows = []
    with pc.pcheb_setup(op, 0, lo, hi) as h0:
        pc.pcheb_matvec(h0, xs, b)
        st, x, lat = _timed_solves(torch, pc, h0, b, 1, False)
        rows.append({"k": 0, "prec": "f64", "iters": st["iters"], "solves_per_s": round(1 / lat[0], 3),
                     "relres_true": st["relres_true"]})
    for k in (10, 20, 40, 80):
        x64 = None
        for prec in ("f64", "f32", "bf16") if k <= BF16_MAX_K else ("f64", "f32"):
            with pc.pcheb_setup(op, k, lo, hi, 1.001, prec) as h:
                st, x, lat = _timed_solves(torch, pc, h, b, 2, prec != "f64", time_kernels=True)
            e = {"f64": 8, "f32": 4, "bf16": 2}[prec]
            step_bytes = 4 * e * n + 8 * n  # iterates + operator data (kappa, or 1/(2 kappa) and D^-1 in float)
            row = {"k": k, "prec": prec, "iters": st["iters"], "solves_per_s": round(2 / sum(lat), 3),
                   "relres_true": st["relres_true"], "step_us": round(st["step_ms"] * 1e3 / max(1, st["step_launches"]), 2),
                   "err_vs_xstar": float(torch.linalg.vector_norm(x - xs) / torch.linalg.vector_norm(xs))}
            row["step_alg_gbs"] = round(step_bytes / (row["step_us"] * 1e-6) / 1e9, 1) if row["step_us"] else None
            if prec == "f64":
                x64 = x.clone()
            else:
                row["rel_diff_vs_f64_solution"] = float(torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64))
            rows.append(row)
            log(f"  c3 k={k} {prec}: {row}")
    print(json.dumps({"config": "c3", "workload": "27-point harmonic diffusion 192^3, lognormal(0,2) cells seed 1, "
                      "Lanczos(30) bounds x1.01, b = A x*, tol 1e-8", "lambda_min": lo, "lambda_max": hi,
                      "kappa_estimate_lanczos": hi / lo, "dacg_lambda_min": est["lambda_min"],
                      "dacg_steps": est["dacg_steps"], "dacg_relres": est["dacg_relres"],
                      "power300_lambda_max": est["lambda_max"],
                      "kappa_dacg": est["lambda_max"] / est["lambda_min"], "rows": rows}), flush=True)


def run_c4(torch, pc, W, dev):
    """Q1 elasticity 128^3 x 3 (502M nonzeros): F32 recurrence with k in {20, 60} stored as CSR and
    as SELL-C-sigma (C = 64, sigma = 256), FP64 flexible PCG; FP64 plain PCG (k = 0) beside.  Also the
    second-level preconditioner on the 3x3 node-block Jacobi factor (block_size 3, SELL, bounds of
    W^T A W by Lanczos(30) x1.01): block Jacobi PCG (k = 0) and k = 20."""
    N = 128
    rp, ci, v = W.elasticity_q1_csr(N, seed=2)
    n = len(rp) - 1
    nnz = int(rp[-1])
    xs_h = W.uniform(0, n, -1.0, 1.0)
    b = torch.from_numpy(W.rhs_from_solution(rp, ci, v, xs_h)).to(dev)
    xs = torch.from_numpy(xs_h).to(dev)
    d = [torch.from_numpy(a).to(dev) for a in (rp, ci, v)]
    del rp, ci, v, xs_h
    v0 = torch.empty(n, dtype=torch.float64, device=dev)
    pc.pcheb_fill_uniform(v0, 7, 0.5, 1.5)
    lo, hi = pc.pcheb_estimate_bounds(pc.Operator.csr(*d), v0, 30)
    hi *= 1.01
    lo3, hi3 = pc.pcheb_estimate_bounds(pc.Operator.csr(*d), v0, 30, block_size=3)
    hi3 *= 1.01
    del v0
    rows = []
    op = pc.Operator.csr(*d, sell=True, sigma=256)
    for k, prec in ((0, "f64"), (20, "f32")):
        with pc.pcheb_setup(op, k, lo3, hi3, 1.001, prec, block_size=3) as h:
            st, x, lat = _timed_solves(torch, pc, h, b, 1, prec != "f64", time_kernels=k >= 3)
        row = {"format": "sell256", "block_size": 3, "k": k, "prec": prec, "iters": st["iters"],
               "solve_s": round(lat[0], 3), "relres_true": st["relres_true"],
               "err_vs_xstar": float(torch.linalg.vector_norm(x - xs) / torch.linalg.vector_norm(xs))}
        rows.append(row)
        log(f"  c4 {row}")
    for fmt in ("sell256", "csr"):
        op = pc.Operator.csr(*d, sell=fmt != "csr", sigma=256)
        cases = [(0, "f64"), (20, "f32"), (60, "f32")] if fmt == "sell256" else [(20, "f32"), (60, "f32")]
        for k, prec in cases:
            with pc.pcheb_setup(op, k, lo, hi, 1.001, prec) as h:
                st, x, lat = _timed_solves(torch, pc, h, b, 1, prec != "f64", time_kernels=k >= 3)
            row = {"format": fmt, "k": k, "prec": prec, "iters": st["iters"], "solve_s": round(lat[0], 3),
                   "relres_true": st["relres_true"],
                   "err_vs_xstar": float(torch.linalg.vector_norm(x - xs) / torch.linalg.vector_norm(xs))}
            if k >= 3 and st["step_launches"]:
                row["step_us"] = round(st["step_ms"] * 1e3 / st["step_launches"], 1)
                step_bytes = 8 * nnz + 4 * (n + 1) + 16 * n
                row["step_alg_gbs"] = round(step_bytes / (row["step_us"] * 1e-6) / 1e9, 1)
            rows.append(row)
            log(f"  c4 {row}")
    print(json.dumps({"config": "c4", "workload": "Q1 elasticity 128^3 free nodes x 3, E = 1 +- 10% seed 2, nu 0.3, "
                      "Lanczos(30) bounds x1.01, b = A x*, tol 1e-8", "n": n, "nnz": nnz, "lambda_min": lo,
                      "lambda_max": hi, "block3_lambda_min": lo3, "block3_lambda_max": hi3, "rows": rows}),
          flush=True)


def run_nrhs_study(torch, pc, W, dev, nrhs=4, k=20, N=128, formats=("sell256", "csr"), emit=True):
    """Q1 elasticity N^3 x 3 (C4 at N = 128), F32 recurrence of degree k, flexible FP64 PCG, tol
    1e-8: nrhs right-hand sides b_j = A x*_j (x*_j ~ U[-1, 1], seeds 0..nrhs-1) solved in one batched
    call, whose CSR / SELL launches read the matrix once for every four of them, against the same
    right-hand sides solved one at a time.  Each batched solution must equal its single solve
    bit for bit.  One JSON line per operator format (emit), and the rows returned."""
    rows = []
    t0 = time.perf_counter()
    rp, ci, v = W.elasticity_q1_csr(N, seed=2)
    n = len(rp) - 1
    bs = [W.rhs_from_solution(rp, ci, v, W.uniform(j, n, -1.0, 1.0)) for j in range(nrhs)]
    log(f"nrhs study: {n} unknowns, {int(rp[-1])} nonzeros, {nrhs} right-hand sides built in "
        f"{time.perf_counter() - t0:.1f}s")
    d = [torch.from_numpy(a).to(dev) for a in (rp, ci, v)]
    del rp, ci, v
    ld = n + (n % 2)
    B = torch.zeros((nrhs, ld), dtype=torch.float64, device=dev)
    for j, b in enumerate(bs):
        B[j, :n] = torch.from_numpy(b).to(dev)
    del bs
    v0 = torch.empty(n, dtype=torch.float64, device=dev)
    pc.pcheb_fill_uniform(v0, 7, 0.5, 1.5)
    lo, hi = pc.pcheb_estimate_bounds(pc.Operator.csr(*d), v0, 30)
    hi *= 1.01
    del v0
    for fmt in formats:
        op = pc.Operator.csr(*d, sell=fmt != "csr", sigma=256)
        with pc.pcheb_setup(op, k, lo, hi, 1.001, "f32") as h:
            X = torch.zeros((nrhs, ld), dtype=torch.float64, device=dev)
            pc.pcg_solve(h, B[:, :n], X[:, :n], flexible=True)  # warm-up (workspace, graph capture)
            singles, t_single = [], 0.0
            for j in range(nrhs):
                x = torch.zeros(n, dtype=torch.float64, device=dev)
                pc.pcg_solve(h, B[j, :n].contiguous(), x, flexible=True)  # warm-up of the one-slot graph
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st = pc.pcg_solve(h, B[j, :n].contiguous(), x, flexible=True)
                torch.cuda.synchronize()
                t_single += time.perf_counter() - t1
                singles.append((st, x))
            X.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            stb = pc.pcg_solve(h, B[:, :n], X[:, :n], flexible=True)
            torch.cuda.synchronize()
            t_batch = time.perf_counter() - t1
        same = sum(int(torch.equal(X[j, :n], x)) for j, (_, x) in enumerate(singles))
        row = {"mode": "nrhs_study", "workload": f"Q1 elasticity {N}^3 free nodes x 3, seed 2", "format": fmt,
               "n": n, "k": k, "prec": "f32", "nrhs": nrhs,
               "iters": [s["iters"] for s, _ in singles], "batched_iters": stb["iters"],
               "single_solves_s": round(t_single, 4), "batched_solve_s": round(t_batch, 4),
               "speedup": round(t_single / t_batch, 3), "bitwise_equal": f"{same}/{nrhs}"}
        if emit:
            print(json.dumps(row), flush=True)
        rows.append(row)
        log(f"  {fmt}: {nrhs} single solves {t_single:.3f}s, batched {t_batch:.3f}s, {same}/{nrhs} bitwise equal")
    del d
    torch.cuda.empty_cache()
    return rows


def run_group_study(torch, pc, W, dev, count=16, sizes=(32, 64, 96), elasticity=24, emit=True):
    """Work lists: `count` problems of one shape with different operators, solved one after
    another (each on its own handle, graph replay) against one grouped solve (pcheb_group_*),
    whose launches cover every problem's tiles.  Problems: 27-point harmonic operators with
    lognormal(0, 2) coefficient fields (seeds 1..count) on N^3 grids, N in {32, 64, 96}, and Q1
    elasticity on 24^3 elements with Young's modulus fields (seeds 1..count), SELL-C-sigma; bounds
    from 30 Lanczos steps each (x1.01); F32 recurrence of degree k, flexible FP64 PCG, tol 1e-8,
    b = A x*, x* ~ U[-1, 1].  Every grouped solution must equal its single solve bit for bit.
    One JSON line per workload."""
    def cases():
        for N in sizes:
            ops = []
            for sd in range(1, count + 1):
                kappa = W.harmonic27_kappa(N, N, N, seed=sd)
                ops.append(pc.Operator.stencil27h(torch.from_numpy(kappa).to(dev)))
            yield f"27-point harmonic {N}^3, {count} coefficient fields", ops, 30
        if not elasticity:
            return
        ops = []
        for sd in range(1, count + 1):
            rp, ci, v = W.elasticity_q1_csr(elasticity, seed=sd)
            d = [torch.from_numpy(a).to(dev) for a in (rp, ci, v)]
            ops.append(pc.Operator.csr(*d, sell=True, sigma=256))
        yield f"Q1 elasticity {elasticity}^3 elements x 3 (SELL), {count} modulus fields", ops, 20

    rows = []
    for name, ops, k in cases():
        n = ops[0].n
        ld = n + (n % 2)
        B = torch.zeros((count, ld), dtype=torch.float64, device=dev)
        hs = []
        for i, op in enumerate(ops):
            v0 = torch.empty(n, dtype=torch.float64, device=dev)
            pc.pcheb_fill_uniform(v0, 7, 0.5, 1.5)
            lo, hi = pc.pcheb_estimate_bounds(op, v0, 30)
            hs.append(pc.pcheb_setup(op, k, lo, 1.01 * hi, 1.001, "f32"))
            pc.pcheb_matvec(hs[-1], torch.from_numpy(W.uniform(i, n, -1.0, 1.0)).to(dev), B[i, :n])  # b = A x*
        try:
            singles, t_single = [], 0.0
            for i, h in enumerate(hs):
                x = torch.zeros(n, dtype=torch.float64, device=dev)
                pc.pcg_solve(h, B[i, :n].contiguous(), x, flexible=True)  # warm-up (graph capture)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st = pc.pcg_solve(h, B[i, :n].contiguous(), x, flexible=True)
                torch.cuda.synchronize()
                t_single += time.perf_counter() - t1
                singles.append((st, x))
            with pc.pcheb_group_create(hs) as g:
                X = torch.zeros_like(B)
                pc.pcg_solve_group(g, B[:, :n], X[:, :n], flexible=True)  # warm-up (graph capture)
                X.zero_()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                sts = pc.pcg_solve_group(g, B[:, :n], X[:, :n], flexible=True)
                torch.cuda.synchronize()
                t_group = time.perf_counter() - t1
        finally:
            for h in hs:
                pc.pcheb_destroy(h)
        same = sum(int(torch.equal(X[i, :n], x)) for i, (_, x) in enumerate(singles))
        iters = [s["iters"] for s, _ in singles]
        row = {"mode": "group_study", "workload": name, "n": n, "k": k, "prec": "f32", "problems": count,
               "iters_min": min(iters), "iters_max": max(iters),
               "group_iters_match": all(sts[i]["iters"] == iters[i] for i in range(count)),
               "single_solves_s": round(t_single, 4), "group_solve_s": round(t_group, 4),
               "speedup": round(t_single / t_group, 3), "bitwise_equal": f"{same}/{count}",
               "group_solves_per_s": round(count / t_group, 2)}
        if emit:
            print(json.dumps(row), flush=True)
        rows.append(row)
        log(f"  {name}: {count} single solves {t_single:.3f}s, one group {t_group:.3f}s "
            f"({t_single / t_group:.2f}x), iterations {min(iters)}-{max(iters)}, {same}/{count} bitwise equal")
        del ops, B, X
        torch.cuda.empty_cache()
    return rows


def cpu_baseline_configs(which, torch, pc, W, dev, k=20):
    """The CPU baseline of C3 and C4 at full size, with parity: C3 (192^3 27-point harmonic, lognormal(0, 2) seed 1, matrix-free on the GPU) and C4 (Q1
    elasticity 128^3 x 3, seed 2, SELL-C-sigma on the GPU) at full size against the FP64 C/OpenMP
    oracle: b = A x* (x* ~ U[-1, 1], seed 0) and the bounds (30 Lanczos steps of the oracle on the
    scaled operator from a U[0.5, 1.5) start, seed 7; lambda_max x1.01) are formed on the host and
    passed to both sides; one oracle solve (degree k, s = 1.001, flexible, tol 1e-8) on all host
    threads, then GPU solves with the F64 and F32 recurrences.  One JSON line per configuration
    with iterations, oracle seconds and the GPU solutions' relative differences."""
    import oracle
    from oracle import omp

    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    omp.set_threads(threads)
    omp.set_progress(1)
    for cfg in which:
        t0 = time.perf_counter()
        if cfg == "c3":
            N = 192
            kappa = W.harmonic27_kappa(N, N, N, seed=1)
            rp, ci, v = W.harmonic27_csr(kappa)
            op = pc.Operator.stencil27h(torch.from_numpy(kappa).to(dev))
            name = "27-point harmonic diffusion 192^3, lognormal(0,2) cells seed 1 (GPU: matrix-free)"
        elif cfg == "c4":
            rp, ci, v = W.elasticity_q1_csr(128, seed=2)
            d = [torch.from_numpy(a).to(dev) for a in (rp, ci, v)]
            op = pc.Operator.csr(*d, sell=True, sigma=256)
            name = "Q1 elasticity 128^3 free nodes x 3, seed 2 (GPU: SELL-C-sigma, C = 64, sigma = 256)"
        else:
            raise SystemExit(f"--cpu-baseline-configs takes c3 and c4, not {cfg}")
        n = len(rp) - 1
        b = W.rhs_from_solution(rp, ci, v, W.uniform(0, n, -1.0, 1.0))
        log(f"cpu baseline {cfg}: {n} unknowns, {int(rp[-1])} nonzeros built in {time.perf_counter() - t0:.1f}s")
        a, _ = oracle.jacobi_scale(oracle.csr(rp, ci, v))
        steps = [0]

        def mv(x):
            steps[0] += 1
            if steps[0] % 5 == 0:
                log(f"  oracle Lanczos step {steps[0]}")
            return a @ x

        lo, hi = oracle.lanczos_extremes(mv, W.uniform(7, n, 0.5, 1.5), 30)
        hi *= 1.01
        del a
        log(f"  bounds [{lo:.6g}, {hi:.6g}]; oracle solve on {threads} thread(s)")
        t0 = time.perf_counter()
        ref = omp.nc_pcg(rp, ci, v, b, lo, hi, k, s=1.001, tol=1e-8, flexible=True)
        secs = time.perf_counter() - t0
        log(f"  oracle: {ref.iters} iterations in {secs:.1f}s, true relres {ref.relres_true:.2e}")
        bt = torch.from_numpy(b).to(dev)
        row = {"mode": "cpu_baseline_full_size", "config": cfg, "workload": name, "n": n, "nnz": int(rp[-1]), "k": k,
               "lambda_min": lo, "lambda_max": hi, "oracle_iters": ref.iters, "oracle_seconds": round(secs, 2),
               "oracle_threads": threads, "oracle_relres_true": ref.relres_true}
        xr = torch.from_numpy(ref.x_hat).to(dev)
        for prec in ("f64", "f32"):
            with pc.pcheb_setup(op, k, lo, hi, 1.001, prec) as h:
                x = torch.zeros(n, dtype=torch.float64, device=dev)
                st = pc.pcg_solve(h, bt, x, tol=1e-8, flexible=True)
            diff = float(torch.linalg.vector_norm(x - xr) / torch.linalg.vector_norm(xr))
            row[f"gpu_{prec}"] = {"iters": st["iters"], "iters_delta": st["iters"] - ref.iters,
                                  "rel_diff_vs_oracle": diff, "relres_true": st["relres_true"],
                                  "meets_bar": abs(st["iters"] - ref.iters) <= 2 and diff <= 1e-6}
            log(f"  GPU {prec}: {st['iters']} iterations, {diff:.2e} from the oracle's solution")
        print(json.dumps(row), flush=True)
        del rp, ci, v, b, bt, xr, op
        torch.cuda.empty_cache()
    omp.set_progress(0)


PD_POWER_STEPS = 300  # power steps for lambda_max (30 land 2.6% low on 256^3, 300 within 0.3%)
PD_DACG_TOL = 1e-2   # DACG tolerance of Sec. 5.1


def paper_estimate(pc, torch, op, n, dev):
    """The paper's bound estimates (Sec. 5.1) from a SplitMix64 U[0.5, 1.5) start vector (seed 7)."""
    v0 = torch.empty(n, dtype=torch.float64, device=dev)
    pc.pcheb_fill_uniform(v0, 7, 0.5, 1.5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = pc.pcheb_estimate_bounds_pdacg(op, v0, PD_POWER_STEPS, PD_DACG_TOL, 1000000)
    r["seconds"] = time.perf_counter() - t0
    del v0
    torch.cuda.empty_cache()
    return r


def run_paper_scale(nx, torch, pc, W, dev, bounds="exact"):
    """lap3d(nx): the 7-point Poisson problem of the paper's large runs, (nx - 1)^3 unknowns,
    matrix-free, s = 1.001, tol 1e-8, x0 = 0, degrees k = 2^nlev - 1 for nlev in {5, 2, 0}.
    Bounds: closed form (a Lanczos basis does not fit at 1023^3), or the paper's estimators
    (300 power steps, DACG to 1e-2; lambda_max widened by 1.01).  Right-hand sides: b = A_hat 1
    (x* = ones) and b ~ U[0, 1] (SplitMix64 seed 0), both formed on the device.  One solve per
    case (the first includes the capture of its iteration graph); prints a JSON line per case."""
    N = nx - 1
    n = N ** 3
    op = pc.Operator.stencil7(N)
    lo, hi = W.stencil7_bounds(N)
    est = None
    if bounds == "pdacg":
        est = paper_estimate(pc, torch, op, n, dev)
        log(f"lap3d({nx}): power({PD_POWER_STEPS}) + DACG({PD_DACG_TOL}) bounds [{est['lambda_min']:.6g}, "
            f"{est['lambda_max']:.6g}] (exact [{lo:.6g}, {hi:.6g}]), {est['dacg_steps']} DACG steps, "
            f"{est['seconds']:.2f} s")
        lo, hi = est["lambda_min"], 1.01 * est["lambda_max"]
    b = torch.empty(n, dtype=torch.float64, device=dev)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    cases = [(5, "f32", 4, True), (5, "f64", 4, False), (2, "f32", 1, True), (0, "f64", 1, False)]
    for rhs in ("ones", "uniform01"):
        if rhs == "ones":
            x.fill_(1.0)
            with pc.pcheb_setup(op, 0, lo, hi) as h0:
                pc.pcheb_matvec(h0, x, b)
        else:
            pc.pcheb_fill_uniform(b, 0, 0.0, 1.0)
        torch.cuda.synchronize()
        for nlev, prec, fuse, flexible in cases:
            k = 2 ** nlev - 1
            t0 = time.perf_counter()
            h = pc.pcheb_setup(op, k, lo, hi, 1.001, prec, fuse_steps=fuse)
            torch.cuda.synchronize()
            setup_s = time.perf_counter() - t0
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = pc.pcg_solve(h, b, x, tol=1e-8, maxit=20000, flexible=flexible, check=False)
            torch.cuda.synchronize()
            solve_s = time.perf_counter() - t0
            pc.pcheb_destroy(h)
            print(json.dumps({"mode": "paper_scale", "problem": f"lap3d({nx})", "n": n, "rhs": rhs, "nlev": nlev,
                              "bounds": bounds, "lambda_min": lo, "lambda_max": hi,
                              "estimate_s": round(est["seconds"], 3) if est else None,
                              "dacg_steps": est["dacg_steps"] if est else None,
                              "k": k, "prec": prec, "steps_per_pass": fuse, "flexible": flexible,
                              "iters": st["iters"], "status": st["status"], "solve_s": round(solve_s, 3),
                              "setup_s": round(setup_s, 3), "relres_true": st["relres_true"],
                              "n_spmv": st["n_spmv"], "n_dot": st["n_dot"]}), flush=True)
    del b, x
    torch.cuda.empty_cache()


def run_bounds(args, torch, pc, W, dev):
    """Bound estimators on the flagship problem (n^3 7-point Poisson, k, F32, four steps per pass):
    Lanczos(30); the paper's power method (30, 300, 1000 steps) for lambda_max and DACG (1e-2)
    for lambda_min; DACG with Lanczos' lambda_max; the closed-form spectrum.  Estimated upper
    bounds are widened by 1.01, and the paper's 30-step estimate is also used as is (s = 1.001
    only).  For each: the estimate, its time, and the flexible NC-PCG solve with those bounds
    (b = A x*, tol 1e-8, at most 5000 iterations)."""
    n1 = args.n
    n = n1 ** 3
    op = pc.Operator.stencil7(n1)
    rp, ci, v = W.stencil7_csr(n1)
    xstar = W.uniform(0, n, -1.0, 1.0)
    bt = torch.from_numpy(W.rhs_from_solution(rp, ci, v, xstar)).to(dev)
    del rp, ci, v
    exact_lo, exact_hi = W.stencil7_bounds(n1)
    v0 = torch.empty(n, dtype=torch.float64, device=dev)
    pc.pcheb_fill_uniform(v0, 7, 0.5, 1.5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    l_lo, l_hi = pc.pcheb_estimate_bounds(op, v0, 30)
    lanczos_s = time.perf_counter() - t0
    power = {}
    for steps in (30, 300, 1000):
        t0 = time.perf_counter()
        power[steps] = (pc.pcheb_estimate_bounds_pdacg(op, v0, steps, 1.0, 0)["lambda_max"], time.perf_counter() - t0)
    del v0
    est = paper_estimate(pc, torch, op, n, dev)  # PD_POWER_STEPS power steps + DACG
    d_lo, d_s = est["lambda_min"], est["seconds"] - power[PD_POWER_STEPS][1]
    log(f"DACG({PD_DACG_TOL}): lambda_min {d_lo:.6g} in {est['dacg_steps']} steps, {d_s:.3f}s; power: "
        + ", ".join(f"{k} steps {v[0]:.6g} ({v[1]:.3f}s)" for k, v in power.items()))
    rows = []
    cases = [("lanczos30_x1.01", l_lo, 1.01 * l_hi, lanczos_s),
             ("power30_dacg_as_printed", d_lo, power[30][0], power[30][1] + d_s)]
    cases += [(f"power{k}_dacg_x1.01", d_lo, 1.01 * power[k][0], power[k][1] + d_s) for k in (30, 300, 1000)]
    cases += [("dacg_lanczos30_x1.01", d_lo, 1.01 * l_hi, lanczos_s + d_s), ("exact", exact_lo, exact_hi, 0.0)]
    for name, lo, hi, secs in cases:
        h = pc.pcheb_setup(op, args.k, lo, hi, 1.001, args.prec, fuse_steps=args.fuse)
        x = torch.zeros(n, dtype=torch.float64, device=dev)
        pc.pcg_solve(h, bt, x, tol=1e-8, maxit=5000, flexible=True, check=False)  # warm-up (graph capture)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = pc.pcg_solve(h, bt, x, tol=1e-8, maxit=5000, flexible=True, check=False)
        torch.cuda.synchronize()
        solve_s = time.perf_counter() - t0
        pc.pcheb_destroy(h)
        rows.append({"bounds": name, "lambda_min": lo, "lambda_max": hi, "estimate_s": round(secs, 4),
                     "iters": st["iters"], "status": st["status"], "solve_s": round(solve_s, 4),
                     "relres_true": st["relres_true"]})
        log(f"  {name:24s} [{lo:.6g}, {hi:.6g}] est {secs:.3f}s  iters {st['iters']}  {st['status']}  "
            f"solve {solve_s:.3f}s")
    print(json.dumps({"mode": "bounds", "workload": f"3-D 7-point Poisson {n1}^3, k={args.k}, {args.prec}, "
                      f"S={args.fuse}, b = A x*, tol 1e-8", "exact": [exact_lo, exact_hi],
                      "dacg_steps": est["dacg_steps"], "dacg_relres": est["dacg_relres"], "dacg_s": round(d_s, 4),
                      "power": {str(k): {"lambda_max": v[0], "seconds": round(v[1], 4)} for k, v in power.items()},
                      "rows": rows}), flush=True)


def run_serve(args, rate, torch, pc, W, dev, nreq=None, emit=True):
    """Serving scenario: requests arrive as a Poisson process (seeded trace), each a
    solve on a cubic grid with N uniform in [32, 160], half 7-point Laplacian (closed-form
    bounds), half 27-point harmonic lognormal (bounds estimated by the server, counted in
    latency); k = 30, float32 polynomial, float64 flexible PCG, tol 1e-8.  Operators with
    equal (stencil, N) share resident data.  Latency runs from the scheduled arrival to
    the host seeing the request done (solution in its device buffer).  A sample of the
    served solutions is re-solved alone and compared bit for bit."""
    tr = W.serving_trace(args.serve_requests if nreq is None else nreq, rate, seed=3)
    nreq = len(tr["t"])
    t0 = time.perf_counter()
    ops, bounds = {}, {}
    for kind, N, cs in sorted(set(zip(tr["kind"].tolist(), tr["N"].tolist(), tr["coeff_seed"].tolist()))):
        if W.KINDS[kind] == "stencil7":
            ops[(kind, N)] = pc.Operator.stencil7(N)
            bounds[(kind, N)] = W.stencil7_bounds(N)
        else:
            kappa = torch.from_numpy(W.harmonic27_kappa(N, N, N, seed=cs)).to(dev)
            ops[(kind, N)] = pc.Operator.stencil27h(kappa)
            bounds[(kind, N)] = (0.0, 0.0)  # estimated by the server
    torch.cuda.synchronize()
    log(f"serve: {len(ops)} operators staged in {time.perf_counter() - t0:.1f}s; {nreq} requests at {rate} req/s")

    check = {}  # request index -> (b, x) kept for the invariance check
    want_check = set()
    for kind in (0, 1):
        idx = np.nonzero(tr["kind"] == kind)[0]
        want_check.update(idx[:: max(1, len(idx) // 3)][:3].tolist())
    srv = pc.Server(int(args.serve_budget_gib * (1 << 30)), args.serve_nrhs)
    outstanding = {}  # id -> (request index, b, x)
    lat, iters, status = [], [], {}
    failures = []
    rejected = 0
    start = time.perf_counter()
    i = 0
    while i < nreq or outstanding:
        now = time.perf_counter() - start
        while i < nreq and tr["t"][i] <= now:
            kind, N = int(tr["kind"][i]), int(tr["N"][i])
            n = N ** 3
            b = torch.empty(n, dtype=torch.float64, device=dev)
            pc.pcheb_fill_uniform(b, int(tr["rhs_seed"][i]), -1.0, 1.0)
            x = torch.empty(n, dtype=torch.float64, device=dev)
            lo, hi = bounds[(kind, N)]
            try:
                rid = srv.submit(ops[(kind, N)], b, x, args.serve_k, tol=1e-8, prec=args.serve_prec,
                                 lambda_min=lo, lambda_max=hi, fuse_steps=args.serve_fuse if kind == 0 else 1)
                outstanding[rid] = (i, b, x)
            except pc.PchebError as e:
                if e.name != "BUDGET":
                    raise
                rejected += 1
            i += 1
        for rid in list(outstanding):
            st = srv.poll(rid)
            if st is None:
                continue
            j, b, x = outstanding.pop(rid)
            lat.append(time.perf_counter() - start - tr["t"][j])
            iters.append(st["iters"])
            status[st["status"]] = status.get(st["status"], 0) + 1
            if st["status"] != "OK" and len(failures) < 12:
                failures.append({"request": int(j), "op": W.KINDS[int(tr["kind"][j])], "N": int(tr["N"][j]),
                                 "status": st["status"], "iters": st["iters"], "relres": st["relres"],
                                 "error": st.get("error", "")})
            if j in want_check:
                check[j] = (b, x, st)
        if i < nreq and not outstanding:
            time.sleep(max(0.0, min(0.002, tr["t"][i] - (time.perf_counter() - start))))
        else:
            time.sleep(0.0002)
    wall = time.perf_counter() - start
    sv = srv.stats()
    srv.close()

    # invariance: the sampled requests re-solved alone (same bounds) give the same bits
    same = 0
    for j, (b, x, st) in sorted(check.items()):
        kind, N = int(tr["kind"][j]), int(tr["N"][j])
        op = ops[(kind, N)]
        lo, hi = bounds[(kind, N)]
        if hi <= 0:
            v0 = torch.empty(N ** 3, dtype=torch.float64, device=dev)
            pc.pcheb_fill_uniform(v0, 7, 0.5, 1.5)
            lo, hi = pc.pcheb_estimate_bounds(op, v0, 30)
            hi *= 1.01
        with pc.pcheb_setup(op, args.serve_k, lo, hi, 1.001, args.serve_prec,
                            fuse_steps=args.serve_fuse if kind == 0 else 1) as h:
            x1 = torch.empty_like(x)
            st1 = pc.pcg_solve(h, b, x1, tol=1e-8, flexible=True)
        same += int(torch.equal(x, x1) and st1["iters"] == st["iters"])
    done = len(lat)
    out = {
        "mode": "serve", "requests": nreq, "rate_req_per_s": rate, "completed": done, "rejected": rejected,
        "status": status, "wall_s": round(wall, 3), "throughput_solves_per_s": round(done / wall, 3),
        "p50_latency_ms": round(1e3 * percentile(lat, 50), 3) if lat else None,
        "p99_latency_ms": round(1e3 * percentile(lat, 99), 3) if lat else None,
        "max_latency_ms": round(1e3 * max(lat), 3) if lat else None,
        "mean_iters": round(float(np.mean(iters)), 2) if iters else None,
        "k": args.serve_k, "prec": args.serve_prec, "max_nrhs": args.serve_nrhs,
        "budget_gib": args.serve_budget_gib, "hbm_high_water_gib": round(sv["bytes_high_water"] / (1 << 30), 3),
        "groups_created": sv["groups_created"], "groups_evicted": sv["groups_evicted"],
        "launches": sv["launches"], "batch_hist": sv["batch_hist"],
        "invariance": f"{same}/{len(check)} bitwise equal to solo solves",
        "failures": failures,
        "data": "synthetic", "n_gpus": 1,
    }
    if emit:
        print(json.dumps(out), flush=True)
    log(f"serve: {done}/{nreq} done at {rate} req/s, p50 {out['p50_latency_ms']} ms, p99 {out['p99_latency_ms']} ms, "
        f"{out['throughput_solves_per_s']} solves/s, invariance {out['invariance']}")
    return out


def hbm_triad_ceiling(torch, dev, nbytes=1 << 30, reps=20):
    """Achievable HBM bandwidth: c = a + 0.5 b on three 1 GiB float64 vectors (12x the
    256 MB last-level cache), timed with events; 3 GiB moved per pass."""
    m = nbytes // 8
    a = torch.ones(m, dtype=torch.float64, device=dev)
    b = torch.ones(m, dtype=torch.float64, device=dev)
    c = torch.empty(m, dtype=torch.float64, device=dev)
    for _ in range(3):
        torch.add(a, b, alpha=0.5, out=c)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.add(a, b, alpha=0.5, out=c)
    e1.record()
    torch.cuda.synchronize()
    gbs = 3 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b, c
    torch.cuda.empty_cache()
    log(f"triad ceiling: {gbs:.0f} GB/s")
    return gbs


def cpu_baseline(rp, ci, v, b, lo, hi, k, which="omp"):
    """The FP64 oracle solving the headline's problem once, completely (the same operator as a CSR
    matrix, right-hand side, bounds, degree, s = 1.001, flexible beta, tol 1e-8).  By default the
    C/OpenMP oracle (oracle/nc_omp.c), on all the host threads this process may use and on one;
    with which="numpy" the numpy/scipy oracle on one thread (its CSR product is single-threaded).
    Returns (the cpu_baseline object, the oracle's solution from the first run, its iterations)."""
    if which == "numpy":
        import oracle
        from threadpoolctl import threadpool_limits

        t_last = [time.perf_counter()]

        def progress(it, relres):
            now = time.perf_counter()
            log(f"  oracle iteration {it}: relres {relres:.3e} ({now - t_last[0]:.1f}s)")
            t_last[0] = now

        log("cpu oracle (numpy): one full FP64 solve of the same problem, 1 thread")
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            res = oracle.nc_pcg(rp, ci, v, b, lo, hi, k, s=1.001, tol=1e-8, flexible=True, progress=progress)
            dt = time.perf_counter() - t0
        log(f"cpu oracle: {res.iters} iterations ({res.n_spmv} operator products) in {dt:.1f}s")
        cpu = {"value": round(1.0 / dt, 6), "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": f"one complete solve, not extrapolated: FP64 numpy/scipy oracle on 1 thread (scipy's CSR "
                         f"product is single-threaded), same {len(rp) - 1}-unknown problem, k={k}, same bounds, "
                         f"flexible PCG to tol 1e-8: {res.iters} iterations, {res.n_spmv} operator products, "
                         f"{dt:.2f} s",
               "seconds": round(dt, 3), "iters": res.iters, "n_spmv": res.n_spmv, "relres_true": res.relres_true}
        return cpu, res.x_hat, res.iters
    from oracle import omp

    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    runs = []
    for t in dict.fromkeys((threads, 1)):
        omp.set_threads(t)
        log(f"cpu oracle (C/OpenMP): one full FP64 solve of the same problem on {t} thread(s)")
        t0 = time.perf_counter()
        res = omp.nc_pcg(rp, ci, v, b, lo, hi, k, s=1.001, tol=1e-8, flexible=True)
        dt = time.perf_counter() - t0
        log(f"cpu oracle: {t} thread(s): {res.iters} iterations ({res.n_spmv} operator products) in {dt:.1f}s, "
            f"true relres {res.relres_true:.2e}")
        runs.append((t, res, dt))
    t, res, dt = runs[0]
    cpu = {"value": round(1.0 / dt, 6), "unit": "solves/s", "cores": t, "kind": "oracle",
           "sample": f"one complete solve, not extrapolated: the FP64 C/OpenMP oracle (plain CSR PCG, rows split "
                     f"over {t} host threads) on the same {len(rp) - 1}-unknown problem, k={k}, same bounds, flexible "
                     f"PCG to tol 1e-8: {res.iters} iterations, {res.n_spmv} operator products, {dt:.2f} s",
           "seconds": round(dt, 3), "iters": res.iters, "n_spmv": res.n_spmv, "relres_true": res.relres_true,
           "by_threads": {str(tt): {"seconds": round(d, 3), "solves_per_s": round(1.0 / d, 6), "iters": r.iters}
                          for tt, r, d in runs}}
    return cpu, res.x_hat, res.iters


if __name__ == "__main__":
    main()

"""Benchmark of the IFMM hot path on one MI355X.

One step = ifmm_build (host octree, lists, colouring) + ifmm_factor (device
operators, colour-by-colour elimination, top LU) + ifmm_solve of 8
right-hand sides, all inputs resident before the timed region (the solve
takes device pointers).  Workload: N = 1,048,576 points on the ellipsoid with
semi-axes (1, 0.7, 0.3) plus 5 % uniform jitter, Laplace kernel, eps = 1e-6,
sigma = 3, leaves of at most 64 points, Chebyshev 4^3 operators.

Two forms run on the same GPU: "mixed" (FP32 matrix-core Schur and basis
products, sketched recompression sized by the trained rank network) gives
`value`; "fp64" (every step FP64, full eigen-decompositions) is reported
beside it.  For each form, FGMRES(50) on the Chebyshev 5^3 FMM operator with
the form's factorisation as right preconditioner gives the iteration count
at the same tolerance (1e-8).

Prints one JSON line (see the keys below).  `roofline` covers the kernel
class with the largest device time in the timed steps, timed with HIP events
on its own launch stream inside the library; `cpu_baseline` times the CPU
oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IFMM factor s + solve ms/RHS at eps=1e-6, N=1M; mixed vs FP64 on same GPU"
FP64_VECTOR_PEAK = 78.6e12      # 256 CUs x 2.4 GHz x 128 FP64 flop/clk
HBM_PEAK = 8.0e12               # bytes/s
FP32_MFMA_PEAK = 157.3e12      # dense FP32 matrix-core peak
BOUND = {"k_fwd": "hbm", "k_bwd": "hbm", "k_gather": "hbm"}
MFMA_F32 = {"k_schur"}          # runs on FP32 matrix cores in the mixed form


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(N, seed=5):
    import synth
    axes = (1.0, 0.7, 0.3)
    pts = synth.ellipsoid_points(N, seed, axes=axes, jitter=0.05)
    dg = synth.laplace_self_term(N, synth.ellipsoid_area(axes))
    return pts, dg


def cpu_baseline(eps, sigma, nrhs, N_full, budget_s=25.0):
    """The oracle, untuned, on a bounded sample: the same workload at a
    reduced N, scaled linearly in N (the IFMM is O(N))."""
    import numpy as np
    import synth
    from oracle.ifmm import IFMM as Oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    N = 4096
    pts, dg = workload(N)
    b = synth.uniform_rhs(N, nrhs, 201)
    t0 = time.perf_counter()
    F = Oracle(pts, eps=eps, sigma=sigma, diag=dg, leaf_max=64).factor()
    tf = time.perf_counter() - t0
    t0 = time.perf_counter()
    F.solve(b)
    ts = time.perf_counter() - t0
    scale = N_full / N
    return {"value": tf * scale, "unit": "s (factor, extrapolated)", "cores": int(cores), "kind": "oracle",
            "sample": f"oracle factor {tf:.2f} s + solve of {nrhs} RHS {ts:.2f} s on the same workload at "
                      f"N={N}, scaled linearly to N={N_full}; solve {1e3 * ts * scale / nrhs:.1f} ms/RHS"}


def run_form(name, pts, dg, args, bt, xt, F, f_dev):
    """One form of the path: `steps` timed steps (build + factor + solve of the
    RHS block), then FGMRES(50) to 1e-8 on the FMM operator with this form's
    factorisation as the right preconditioner (untimed against the metric)."""
    import numpy as np
    import torch
    from paper_1905_10602_amd import IFMM
    from paper_1905_10602_amd.ifmm import _check, _ptr, load_library
    N = pts.shape[0]
    mixed = name != "fp64"
    os.environ["IFMM_SKETCH"] = "1" if mixed else "0"
    theta = None
    if mixed:
        from paper_1905_10602_amd.rank_model import load
        theta, _ = load()

    def step():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = IFMM(pts, args.eps, args.sigma, diag=dg, leaf_max=64, precision="mixed" if mixed else "fp64")
        if theta is not None:
            h.set_rank_model(theta)
        t1 = time.perf_counter()
        h.factor()
        t2 = time.perf_counter()
        _check(load_library().ifmm_solve(h._h, _ptr(bt), _ptr(xt), args.nrhs, N, 1))
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        return h, {"build_s": t1 - t0, "factor_s": t2 - t1, "solve_s": t3 - t2, "step_s": t3 - t0}

    for w in range(args.warmup):
        h, t = step()
        log(f"{name} warmup {w}: {json.dumps(t)}")
        h.close()
    times = []
    h = None
    for k in range(args.steps):
        if h is not None:
            h.close()
        torch.cuda.synchronize()
        h, t = step()
        torch.cuda.synchronize()
        times.append(t)
        log(f"{name} step {k}: {json.dumps(t)}")
    stats = h.stats()
    x_first = xt[0].cpu().numpy().copy()
    # accuracy of the IFMM solve on the FMM operator, and preconditioned FGMRES
    res = None
    gm = {}
    if F is not None:
        y = F.matvec(xt[0].contiguous())
        res = float(torch.linalg.norm(y - bt[0]) / torch.linalg.norm(bt[0]))
        t0 = time.perf_counter()
        xg, its, rr = F.gmres(f_dev, precond=h, tol=1e-8, restart=50, maxit=200, allow_noconv=True)
        torch.cuda.synchronize()
        gm = {"gmres_iters": its, "gmres_relres": rr, "gmres_s": time.perf_counter() - t0}
        t0 = time.perf_counter()
        xg0, its0, rr0 = F.gmres(f_dev, precond=None, tol=1e-8, restart=50, maxit=400, allow_noconv=True)
        torch.cuda.synchronize()
        gm.update({"gmres_unpreconditioned_iters": its0, "gmres_unpreconditioned_s": time.perf_counter() - t0})
        del xg, xg0
    h.close()
    med = lambda key: statistics.median(t[key] for t in times)
    out = {"factor_s": med("factor_s"), "solve_ms_per_rhs": med("solve_s") * 1e3 / args.nrhs,
           "build_s": med("build_s"), "step_s": med("step_s"), "solve_residual_on_fmm": res, **gm,
           "sketches": stats.get("sketches"), "sketches_rejected": stats.get("sketches_rejected"),
           "rank_predictions": stats.get("rank_predictions"), "t_sync": stats.get("t_sync"), "t_h2d": stats.get("t_h2d"),
           "depth": stats.get("depth"), "top_n": stats.get("top_n"), "device_GB": stats.get("device_bytes", 0) / 1e9,
           "factor_store_GB": stats.get("store_bytes", 0) / 1e9,
           "levels": [{k2: L[k2] for k2 in ("level", "nodes", "colours", "rank_sum", "rank_max", "n_max", "t_elim")}
                      for L in stats.get("levels", [])],
           "kernels_ms": {n: round(k["ms"], 3) for n, k in stats.get("kernels", {}).items()},
           "kernels_rate": {n: {"TFLOP/s": round(k["flops"] / k["ms"] / 1e9, 2) if k["flops"] else None,
                                "GB/s": round(k["bytes"] / k["ms"] / 1e6, 1) if k["bytes"] else None}
                            for n, k in stats.get("kernels", {}).items() if k["ms"] > 0},
           "host_ms": {n: round(v, 1) for n, v in stats.get("host_ms", {}).items()}}
    return out, stats, x_first


def measured_traffic(kernel, form):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    record (FETCH_SIZE / WRITE_SIZE scaled by the copy calibration), or None
    when there is none or the kernel sources changed since it was taken."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_1905_10602_amd", "csrc")
    h = hashlib.sha256()
    for f in ("dense.hpp", "kernels.hpp"):
        with open(os.path.join(src, f), "rb") as fh:
            h.update(fh.read())
    digest = h.hexdigest()[:16]
    for path in glob.glob(os.path.join(ROOT, "profiles", f"{kernel}_hbm_traffic_*.json")):
        with open(path) as fh:
            rec = json.load(fh)
        if rec.get("form") == form and rec.get("kernel_sources_sha256_16") == digest:
            return rec["traffic_bytes_per_launch"]
    return None


def roofline_of(stats, mixed):
    """Roofline of the single kernel with the largest device time (profiler
    classes named "group:..." span several kernels and are skipped)."""
    ks = {n: k for n, k in stats.get("kernels", {}).items() if not n.startswith("group:")}
    if not ks:
        return None
    name, k = max(ks.items(), key=lambda kv: kv[1]["ms"])
    avg_s = k["ms"] / 1e3 / max(k["launches"], 1)
    common = {"kernel": name, "traffic": measured_traffic(name, "mixed" if mixed else "fp64"),
              "launches": k["launches"], "avg_launch_ms": avg_s * 1e3,
              "algorithmic_per_launch": (k["bytes"] if BOUND.get(name) == "hbm" else k["flops"]) / max(k["launches"], 1),
              "algorithmic_bytes_per_launch": k["bytes"] / max(k["launches"], 1)}
    if BOUND.get(name) == "hbm":
        ach = k["bytes"] / max(k["launches"], 1) / avg_s
        return {"bound": "hbm", "achieved": ach / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": ach / HBM_PEAK, **common}
    ach = k["flops"] / max(k["launches"], 1) / avg_s
    if mixed and name in MFMA_F32:
        return {"bound": "mfma", "achieved": ach / 1e12, "peak": FP32_MFMA_PEAK / 1e12, "unit": "TFLOP/s",
                "frac": ach / FP32_MFMA_PEAK, **common}
    return {"bound": "alu", "achieved": ach / 1e12, "peak": FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": ach / FP64_VECTOR_PEAK, **common}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--sigma", type=int, default=3)
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--form", choices=("both", "mixed", "fp64"), default="both")
    ap.add_argument("--no-gmres", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: one GPU only (--gpus 1); sharding a factorisation across GPUs is not implemented",
              file=sys.stderr)
        sys.exit(2)
    os.environ["IFMM_PROF"] = "1"
    os.environ.setdefault("IFMM_LOG", "1")
    import numpy as np
    import torch
    import synth
    from paper_1905_10602_amd import FMM
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    N = args.n
    log(f"workload: ellipsoid N={N}")
    pts, dg = workload(N)
    b = synth.uniform_rhs(N, args.nrhs, 201)
    bt = torch.from_numpy(np.ascontiguousarray(b.T)).cuda()  # (nrhs, N) row-major = (N, nrhs) col-major
    xt = torch.empty_like(bt)
    F, f_dev = None, None
    if not args.no_gmres:
        F = FMM(pts, dg, cheb_order=5, leaf_max=256)  # FMM depth for ~30 points per leaf (not the IFMM's)
        f_dev = bt[0].contiguous()
        log(f"FMM matvec operator built: {json.dumps(F.stats())}")
    forms = {"both": ["mixed", "fp64"], "mixed": ["mixed"], "fp64": ["fp64"]}[args.form]
    res, stats0, xs = {}, None, {}
    for fm in forms:
        log(f"form {fm}")
        out, st, x0 = run_form(fm, pts, dg, args, bt, xt, F, f_dev)
        res[fm] = out
        xs[fm] = x0
        if stats0 is None:
            stats0 = st
    lead = forms[0]
    R = res[lead]
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        cpu = cpu_baseline(args.eps, args.sigma, args.nrhs, N)
    out = {
        "metric": METRIC, "value": R["factor_s"], "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": R["step_s"] * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32mfma" if lead == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": f"ellipsoid (1,0.7,0.3) + 5% jitter, N={N}, Laplace 1/(4 pi r), eps={args.eps}, "
                               f"sigma={args.sigma}, leaf<=64, Chebyshev 4^3, {args.nrhs} RHS; value = "
                               f"{'mixed-precision learned-rank' if lead == 'mixed' else 'plain FP64'} form",
                   "parallelism": "single GPU"},
        "factor_s": R["factor_s"], "solve_ms_per_rhs": R["solve_ms_per_rhs"],
        "forms": res,
        "roofline": roofline_of(stats0, lead == "mixed"), "cpu_baseline": cpu,
    }
    if "mixed" in res and "fp64" in res:
        out["factor_speedup_mixed_vs_fp64"] = res["fp64"]["factor_s"] / res["mixed"]["factor_s"]
        xm, x6 = xs["mixed"], xs["fp64"]
        out["mixed_vs_fp64_solution_rel_diff"] = float(np.linalg.norm(xm - x6) / np.linalg.norm(x6))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

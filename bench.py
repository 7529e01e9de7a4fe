"""Benchmark of the IFMM hot path on one MI355X.

One step = ifmm_build (host octree, lists, colouring) + ifmm_factor (device
operators, colour-by-colour elimination, top LU) + ifmm_solve of 8
right-hand sides, all inputs resident before the timed region (the solve
takes device pointers).  Workload: N = 1,048,576 points on the ellipsoid with
semi-axes (1, 0.7, 0.3) plus 5 % uniform jitter, Laplace kernel, eps = 1e-6,
sigma = 3, Chebyshev 4^3 operators; the IFMM's depth (bottom level) is the
one the library's cost model picks among the depth with leaves of at most 64
points (7 here) and the two coarser ones (Sec. 5.2 tunes it the same way).

Forms on the same GPU:
  mixed      FP32 matrix-core Schur and basis products, sketched recompression
             sized by the trained rank network: gives `value`;
  fp64       every step FP64, full eigen-decompositions;
  heuristic  the mixed form without the network (sketch width from the node's
             current rank): the ablation of the learned part.
The comparison forms take up to three timed steps each (no warm-up of their
own: the lead form's run has loaded the kernels), factor time the median.
For each form: e_res = ||A~ x - b|| / ||b|| with A~ applied through the
Chebyshev 4^3 FMM on the IFMM's own tree (exactly the matrix the IFMM
factorises), and FGMRES(50) on the Chebyshev 5^3 FMM operator with the form's
factorisation as right preconditioner (iterations at tolerance 1e-8).

The whole run keeps to a wall-clock budget (--budget-s, counted from the
start of the process): warm-up is at most one step, the timed mixed steps are
as many of --steps as fit, the comparison forms up to three steps each, and the
GMRES and CPU legs are skipped, with a note, when they no longer fit.  `steps` reports
the count actually timed.  The JSON line is always printed.

`roofline` covers the single kernel with the largest device time in the lead
form, timed with HIP events on its own launch stream inside the library;
`roofline_more` adds the Schur update and the solve.  `cpu_baseline` times
the CPU oracle on two bounded samples of the same workload and extrapolates
linearly in N.

`python bench.py --copy-calibration` only copies 3 x 256 MiB on the device:
the reference kernel whose FETCH_SIZE / WRITE_SIZE counters scale the same
counters of the library's kernels to bytes.
"""
from __future__ import annotations

import time

T_START = time.time()

import argparse  # noqa: E402
import json  # noqa: E402
import os  # noqa: E402
import statistics  # noqa: E402
import sys  # noqa: E402
import traceback  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IFMM factor s + solve ms/RHS at eps=1e-6, N=1M; mixed vs FP64 on same GPU"
FP64_VECTOR_PEAK = 78.6e12      # 256 CUs x 2.4 GHz x 128 FP64 flop/clk
FP64_MFMA_PEAK = 78.6e12        # dense FP64 matrix-core peak
HBM_PEAK = 8.0e12               # bytes/s
FP32_MFMA_PEAK = 157.3e12      # dense FP32 matrix-core peak
BOUND = {"k_solve_fwd_w": "hbm", "k_solve_fwd_upd": "hbm", "k_solve_bwd": "hbm", "k_gather": "hbm",
         "solve": "hbm"}
# k_schur: the Schur update's FP64 products (FP64 matrix cores) and, in the
# mixed form without IFMM_SCHUR_SPLIT, also its far products (FP32 matrix
# cores; the peak is then blended by the flops share); k_schur_far: the
# mixed form's far products alone (FP32 matrix cores)
MFMA_F32 = {"k_schur", "k_schur_far"}
MFMA_F64 = {"k_schur"}


def log(msg):
    print(f"[bench {time.time() - T_START:6.1f}s] {msg}", file=sys.stderr, flush=True)


CMP_STEPS = 3  # timed steps of each comparison form (fp64, heuristic), when they fit


def left(args):
    return args.budget_s - (time.time() - T_START)


def workload(N, seed=5):
    import synth
    axes = (1.0, 0.7, 0.3)
    pts = synth.ellipsoid_points(N, seed, axes=axes, jitter=0.05)
    dg = synth.laplace_self_term(N, synth.ellipsoid_area(axes))
    return pts, dg


def host_info():
    info = {"nproc": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    info["ram_GB"] = round(int(line.split()[1]) / 1e6, 1)
                    break
    except OSError:
        pass
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    return info


def cpu_baseline(eps, sigma, nrhs, N_full, args):
    """The oracle, untuned, on bounded samples of the same workload: N = 4096
    and, when the budget allows, N = 8192; the factor time is extrapolated to
    N_full along the straight line through the two points (the IFMM is O(N);
    with one point, proportionally)."""
    import synth
    from oracle.ifmm import IFMM as Oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    pts_all = {}
    runs = []
    for N in (4096, 8192):
        if runs:
            need = runs[-1]["factor_s"] * 2.6 + runs[-1]["solve_s"] * 2.6 + 10
            if left(args) < need:
                log(f"cpu baseline: N={N} skipped (needs ~{need:.0f} s, {left(args):.0f} s left)")
                break
        pts_all[N] = workload(N)
        pts, dg = pts_all[N]
        b = synth.uniform_rhs(N, nrhs, 201)
        t0 = time.perf_counter()
        F = Oracle(pts, eps=eps, sigma=sigma, diag=dg, leaf_max=64).factor()
        tf = time.perf_counter() - t0
        t0 = time.perf_counter()
        F.solve(b)
        ts = time.perf_counter() - t0
        runs.append({"N": N, "factor_s": tf, "solve_s": ts})
        log(f"cpu baseline N={N}: factor {tf:.2f} s, solve {ts:.2f} s")
    if len(runs) >= 2:
        a, b2 = runs[0], runs[1]
        slope = (b2["factor_s"] - a["factor_s"]) / (b2["N"] - a["N"])
        slope_s = (b2["solve_s"] - a["solve_s"]) / (b2["N"] - a["N"])
        val = b2["factor_s"] + slope * (N_full - b2["N"])
        sol = b2["solve_s"] + slope_s * (N_full - b2["N"])
        how = (f"straight line through the two samples: {slope * 1e3:.3f} ms of factor time per point, "
               f"extrapolated from N={b2['N']} to N={N_full}")
    else:
        a = runs[0]
        val = a["factor_s"] * N_full / a["N"]
        sol = a["solve_s"] * N_full / a["N"]
        how = f"one sample, scaled proportionally from N={a['N']} to N={N_full}"
    return {"value": val, "unit": "s (factor, extrapolated)", "cores": int(cores), "kind": "oracle",
            "sample": "oracle (FP64 numpy/scipy, untuned) factor + solve of the same workload (ellipsoid + jitter, "
                      f"eps={eps}, sigma={sigma}, {nrhs} RHS) at " +
                      ", ".join(f"N={r['N']}: factor {r['factor_s']:.2f} s, solve {r['solve_s']:.2f} s" for r in runs) +
                      f"; {how}; solve extrapolated {1e3 * sol / nrhs:.0f} ms/RHS",
            "samples": runs, "host": host_info()}


def run_form(name, pts, dg, args, bt, xt, F5, F4, f_dev, max_steps, warmup):
    """One form of the path: `warmup` untimed and up to `max_steps` timed steps
    (build + factor + solve of the RHS block, the step count cut by the
    budget), then e_res on A~ and FGMRES(50) to 1e-8 on the order-5 FMM
    operator with this form's factorisation as the right preconditioner
    (untimed against the metric)."""
    import torch
    from paper_1905_10602_amd import IFMM
    from paper_1905_10602_amd.ifmm import _check, _ptr, load_library
    N = pts.shape[0]
    mixed = name != "fp64"
    os.environ["IFMM_SKETCH"] = "1" if mixed else "0"
    theta = None
    if name == "mixed":
        from paper_1905_10602_amd.rank_model import load
        theta, _ = load()

    def step():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = IFMM(pts, args.eps, args.sigma, diag=dg, leaf_max=64, precision="mixed" if mixed else "fp64",
                 bottom_level=args.bottom_level, colouring=args.colouring,
                 tune_cache=args.tune_path if mixed and args.tune_path else None)
        if theta is not None:
            h.set_rank_model(theta)
        t1 = time.perf_counter()
        h.factor()
        t2 = time.perf_counter()
        _check(load_library().ifmm_solve(h._h, _ptr(bt), _ptr(xt), args.nrhs, N, 1))
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        return h, {"build_s": t1 - t0, "factor_s": t2 - t1, "solve_s": t3 - t2, "step_s": t3 - t0}

    for w in range(warmup):
        h, t = step()
        log(f"{name} warmup {w}: {json.dumps(t)}")
        h.close()
    times = []
    h = None
    reserve = args.reserve_s
    while len(times) < max_steps:
        if times and left(args) < times[-1]["step_s"] * 1.15 + reserve:
            log(f"{name}: stopping after {len(times)} timed steps ({left(args):.0f} s left, "
                f"{reserve:.0f} s reserved for the other legs)")
            break
        if h is not None:
            h.close()
        torch.cuda.synchronize()
        h, t = step()
        torch.cuda.synchronize()
        times.append(t)
        log(f"{name} step {len(times) - 1}: {json.dumps(t)}")
    stats = h.stats()
    x_first = xt[0].cpu().numpy().copy()
    gm = {}
    # e_res on the matrix the IFMM factorises (A~ through its exact FMM form,
    # on a tree of the IFMM's depth: with a coarser bottom level the leaves
    # hold more points and A~ has more exact near-field blocks)
    F4_own = None
    if F4 is not None and stats.get("depth") != F4.stats().get("depth"):
        from paper_1905_10602_amd import FMM
        leaf = max(L["n_max"] for L in stats["levels"] if L["level"] == stats["depth"])
        F4_own = F4 = FMM(pts, dg, cheb_order=4, leaf_max=int(leaf))
        gm["e_res_tree_depth"] = F4.stats().get("depth")
    if F4 is not None:
        ys = [F4.matvec(xt[k].contiguous()) for k in range(args.nrhs)]
        gm["e_res"] = max(float(torch.linalg.norm(ys[k] - bt[k]) / torch.linalg.norm(bt[k])) for k in range(args.nrhs))
        gm["e_res_over_eps"] = gm["e_res"] / args.eps
        gm["backward_error"] = max(float(torch.linalg.norm(ys[k] - bt[k]) /
                                         (args.anorm * torch.linalg.norm(xt[k]) + torch.linalg.norm(bt[k])))
                                   for k in range(args.nrhs))
        gm["backward_error_over_eps"] = gm["backward_error"] / args.eps
    # one untimed single-RHS solve: captures its graph (and, with the
    # autotuner, times the wave counts for one right-hand side) before GMRES
    # and the latency below use that path
    x1 = torch.empty_like(bt[0])
    _check(load_library().ifmm_solve(h._h, _ptr(bt[0]), _ptr(x1), 1, N, 1))
    torch.cuda.synchronize()
    if F5 is not None:
        y = F5.matvec(xt[0].contiguous())
        gm["solve_residual_on_cheb5_fmm"] = float(torch.linalg.norm(y - bt[0]) / torch.linalg.norm(bt[0]))
        if left(args) > args.reserve_gmres_s:
            t0 = time.perf_counter()
            xg, its, rr = F5.gmres(f_dev, precond=h, tol=1e-8, restart=50, maxit=100, allow_noconv=True)
            torch.cuda.synchronize()
            gm.update({"gmres_iters": its, "gmres_relres": rr, "gmres_s": time.perf_counter() - t0})
            del xg
        else:
            gm["gmres_skipped"] = f"budget ({left(args):.0f} s left)"
    # single-RHS latency of the solve (graph-captured)
    t0 = time.perf_counter()
    for _ in range(3):
        _check(load_library().ifmm_solve(h._h, _ptr(bt[0]), _ptr(x1), 1, N, 1))
    torch.cuda.synchronize()
    gm["solve_1rhs_ms"] = (time.perf_counter() - t0) * 1e3 / 3
    # per-kernel timing of the solve steps: three eager (uncaptured) solves of
    # the RHS block, each launch between hipEvents on the solve's stream
    os.environ["IFMM_GRAPH"] = "0"
    xe = torch.empty_like(bt)
    for _ in range(3):
        _check(load_library().ifmm_solve(h._h, _ptr(bt), _ptr(xe), args.nrhs, N, 1))
    torch.cuda.synchronize()
    os.environ["IFMM_GRAPH"] = "1"
    gm["eager_solve_equals_graph"] = bool(torch.equal(xe, xt))
    stats = h.stats()
    h.close()
    if F4_own is not None:
        F4_own.close()
    med = lambda key: statistics.median(t[key] for t in times)
    out = {"steps_timed": len(times), "factor_s": med("factor_s"), "solve_ms_per_rhs": med("solve_s") * 1e3 / args.nrhs,
           "build_s": med("build_s"), "step_s": med("step_s"), "step_s_all": [round(t["step_s"], 3) for t in times],
           **gm,
           "sketches": stats.get("sketches"), "sketches_rejected": stats.get("sketches_rejected"),
           "full_decompositions": stats.get("full_decompositions"),
           "rank_predictions": stats.get("rank_predictions"), "t_sync": stats.get("t_sync"), "t_h2d": stats.get("t_h2d"),
           "depth": stats.get("depth"), "top_n": stats.get("top_n"), "device_GB": stats.get("device_bytes", 0) / 1e9,
           "peak_device_GB": stats.get("peak_device_bytes", 0) / 1e9,
           "factor_store_GB": stats.get("store_bytes", 0) / 1e9,
           "levels": [{k2: L.get(k2) for k2 in ("level", "nodes", "colours", "rank_sum", "rank_max", "n_max", "t_elim",
                                                 "rank_hist")}
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


def price(name, k, mixed, f32_flops=None):
    """Roofline entry of one kernel class from its in-library hipEvent record.
    f32_flops: the part of the kernel's flops on FP32 matrix cores (mixed form);
    the peak is then the time-weighted blend of the FP32 and FP64 peaks."""
    la = max(k["launches"], 1)
    avg_s = k["ms"] / 1e3 / la
    common = {"kernel": name, "traffic": measured_traffic(name, "mixed" if mixed else "fp64"),
              "launches": k["launches"], "avg_launch_ms": avg_s * 1e3,
              "algorithmic_per_launch": (k["bytes"] if BOUND.get(name) == "hbm" else k["flops"]) / la,
              "algorithmic_bytes_per_launch": k["bytes"] / la}
    if avg_s <= 0:
        return None
    if BOUND.get(name) == "hbm":
        ach = k["bytes"] / la / avg_s
        return {"bound": "hbm", "achieved": ach / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": ach / HBM_PEAK, **common}
    ach = k["flops"] / la / avg_s
    if mixed and name in MFMA_F32:
        peak = FP32_MFMA_PEAK
        if f32_flops is not None and k["flops"] > 0:
            f = min(max(f32_flops / k["flops"], 0.0), 1.0)  # flops share on FP32 matrix cores
            peak = 1.0 / (f / FP32_MFMA_PEAK + (1.0 - f) / FP64_MFMA_PEAK)
            common["fp32_share_of_flops"] = f
        return {"bound": "mfma", "achieved": ach / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": ach / peak, **common}
    if not mixed and name in MFMA_F64:
        return {"bound": "mfma", "achieved": ach / 1e12, "peak": FP64_MFMA_PEAK / 1e12, "unit": "TFLOP/s",
                "frac": ach / FP64_MFMA_PEAK, **common}
    return {"bound": "alu", "achieved": ach / 1e12, "peak": FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": ach / FP64_VECTOR_PEAK, **common}


def roofline_of(stats, mixed):
    """Roofline of the single kernel with the largest device time (profiler
    classes named "group:..." span several kernels and are skipped)."""
    ks = {n: k for n, k in stats.get("kernels", {}).items() if not n.startswith("group:")}
    if not ks:
        return None
    name, k = max(ks.items(), key=lambda kv: kv[1]["ms"])
    return price(name, k, mixed, _f32_flops(stats, name))


def _f32_flops(stats, name):
    """Flops of `name` on FP32 matrix cores: all of k_schur_far; for k_schur
    the far products' share unless they ran as their own kernel."""
    ks = stats.get("kernels", {})
    if name == "k_schur_far":
        return ks[name]["flops"]
    if name == "k_schur":
        return 0.0 if "k_schur_far" in ks else stats.get("aux", {}).get("schur_far_flops")
    return None


def roofline_more(stats, mixed):
    """The Schur update and the solve (per-colour substitution kernels and the
    whole captured solve) beside the dominant kernel."""
    ks = stats.get("kernels", {})
    out = {}
    for n in ("k_schur", "k_schur_far", "k_eig_values", "k_solve_fwd_w", "k_solve_fwd_upd", "k_solve_bwd"):
        if n in ks:
            out[n] = price(n, ks[n], mixed, _f32_flops(stats, n))
    # the three solve steps together: algorithmic bytes over their summed time
    parts = [ks[n] for n in ("k_solve_fwd_w", "k_solve_fwd_upd", "k_solve_bwd") if n in ks]
    if parts:
        tot = {"ms": sum(p["ms"] for p in parts), "launches": 1, "flops": 0.0, "bytes": sum(p["bytes"] for p in parts)}
        out["solve"] = price("solve", tot, mixed)
    return out


def bem_comparison(args):
    """The FMBEM workload (Laplace single layer on the unit sphere, icosphere of
    327,680 panels, f = 1/|x - (0,0,0.5)|): FGMRES(50) to 1e-8 with the
    Chebyshev 5^3 FMM product and no preconditioner, BD at the leaf level and
    one level coarser (Sec. 4.3), and the IFMM (eps = 1e-3, sigma = 3) in FP64
    and in the mixed form.  One JSON line: iterations, set-up and solve times,
    density error against the closed form."""
    import numpy as np
    import torch
    import synth
    from paper_1905_10602_amd import BD, FMM, IFMM
    v, f = synth.icosphere(7)
    a_ = v[f[:, 0]]
    b_ = v[f[:, 1]]
    c_ = v[f[:, 2]]
    cen = (a_ + b_ + c_) / 3.0
    area = 0.5 * np.linalg.norm(np.cross(b_ - a_, c_ - a_), axis=1)
    st = np.sqrt(area / np.pi) / 2.0
    x0 = np.array([0.0, 0.0, 0.5])
    rhs = 1.0 / np.linalg.norm(cen - x0, axis=1)
    exact = (1.0 - x0 @ x0) / np.linalg.norm(cen - x0, axis=1) ** 3
    N = cen.shape[0]
    log(f"BEM: {N} panels")
    F = FMM(cen, st, weights=area, cheb_order=5, leaf_max=64)
    bt = torch.from_numpy(rhs).cuda()
    res = {"panels": N, "fmm_depth": F.stats()["depth"]}

    def run(name, pre, setup_s):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, it, rr = F.gmres(bt, precond=pre, tol=1e-8, restart=50, maxit=2000, allow_noconv=True)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        xs = x.cpu().numpy()
        res[name] = {"iterations": it, "relres": rr, "setup_s": setup_s, "gmres_s": ts, "total_s": setup_s + ts,
                     "density_error": float(np.linalg.norm(xs - exact) / np.linalg.norm(exact))}
        log(f"BEM {name}: {json.dumps(res[name])}")

    run("none", None, 0.0)
    for coarser in (0, 1):
        t0 = time.perf_counter()
        lvl = F.stats()["depth"] - coarser
        bd = BD(cen, st, weights=area, level=lvl, leaf_max=64)
        torch.cuda.synchronize()
        run(f"BD_level{lvl}", bd, time.perf_counter() - t0)
        bd.close()
    for prec in ("fp64", "mixed"):
        t0 = time.perf_counter()
        h = IFMM(cen, 1e-3, 3, diag=st, weights=area, leaf_max=64, precision=prec, bottom_level=args.bottom_level)
        h.factor()
        torch.cuda.synchronize()
        run(f"IFMM_eps1e-3_{prec}", h, time.perf_counter() - t0)
        res[f"IFMM_eps1e-3_{prec}"]["depth"] = h.depth()
        h.close()
    print(json.dumps({"bem_comparison": res}), flush=True)


def batch_leg(args):
    """The many-geometry workload: 64 independent geometries (seeds 4000..4063,
    spheres, ellipsoids with random semi-axes and cube surfaces, N uniform in
    [2048, 32768]), eps = 1e-4, sigma = 3, mixed form, 4 right-hand sides each:
    ifmm_factor_batch / ifmm_solve_batch (8 host threads, one stream each)
    against the same factorisations and solves one after the other; the
    solutions must agree bit for bit."""
    import numpy as np
    import torch
    import synth
    from paper_1905_10602_amd import IFMM, factor_batch, solve_batch
    geoms = synth.batch_geometries(64, 4000)
    dgs = [synth.laplace_self_term(p.shape[0]) for _, p in geoms]
    rhs = [synth.uniform_rhs(p.shape[0], 4, 4100 + g) for g, (_, p) in enumerate(geoms)]

    def handles():
        return [IFMM(p, 1e-4, 3, diag=dg, leaf_max=64, precision="mixed", bottom_level=args.bottom_level)
                for (_, p), dg in zip(geoms, dgs)]
    out = {"geometries": len(geoms), "points_total": int(sum(p.shape[0] for _, p in geoms)), "rhs_each": 4,
           "eps": 1e-4}
    hs = handles()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    factor_batch(hs, threads=8)
    t1 = time.perf_counter()
    xb = solve_batch(hs, rhs, threads=8)
    t2 = time.perf_counter()
    out.update({"batch_factor_s": t1 - t0, "batch_solve_s": t2 - t1})
    for h in hs:
        h.close()
    if left(args) < 3.0 * (t2 - t0) + 20:
        out["sequential"] = f"skipped ({left(args):.0f} s left)"
        return out
    hs = handles()
    t0 = time.perf_counter()
    for h in hs:
        h.factor()
    t1 = time.perf_counter()
    xs = [h.solve(b) for h, b in zip(hs, rhs)]
    t2 = time.perf_counter()
    out.update({"sequential_factor_s": t1 - t0, "sequential_solve_s": t2 - t1,
                "bitwise_equal": bool(all(np.array_equal(a, b) for a, b in zip(xb, xs)))})
    for h in hs:
        h.close()
    return out


def copy_calibration():
    """Reference copy for the HBM traffic counters: three copies of 256 MiB of FP64."""
    import torch
    n = 32 * 1024 * 1024
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    x.fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("copied 3 x 256 MiB", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--sigma", type=int, default=3)
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--form", choices=("all", "both", "mixed", "fp64", "heuristic"), default="all")
    ap.add_argument("--budget-s", type=float, default=450.0,
                    help="wall-clock budget of the whole run, counted from the start of the process")
    ap.add_argument("--reserve-s", type=float, default=-1.0,
                    help="seconds kept free for the legs after the timed mixed steps (default: estimated)")
    ap.add_argument("--reserve-gmres-s", type=float, default=20.0)
    ap.add_argument("--bottom-level", type=int, default=-1,
                    help="IFMM depth: -1 = chosen by the cost model among the depth of leaves of <= 64 points and "
                         "the two coarser ones (default), 0 = leaves of <= 64 points, >= 2 = forced")
    ap.add_argument("--colouring", choices=("stride", "lookback"), default="stride")
    ap.add_argument("--no-tune", action="store_true",
                    help="built-in tile and wave choices (default: the autotuner, tuned in the mixed form's warm-up "
                         "step and reused by the heuristic form; the FP64 form keeps the built-in choices)")
    ap.add_argument("--no-gmres", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-geometry batch leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--bem", action="store_true", help="only the FMBEM preconditioner comparison (327,680 panels)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: one GPU only (--gpus 1); sharding a factorisation across GPUs is not implemented",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.bem:
        bem_comparison(args)
        return
    os.environ["IFMM_PROF"] = "1"
    os.environ.setdefault("IFMM_LOG", "1")
    import numpy as np
    import torch
    import synth
    from paper_1905_10602_amd import FMM
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    N = args.n
    log(f"workload: ellipsoid N={N}; budget {args.budget_s:.0f} s")
    args.tune_path = None
    if not args.no_tune:  # a fresh autotuner cache per run
        import tempfile
        fd, args.tune_path = tempfile.mkstemp(prefix="ifmm_tune_", suffix=".txt")
        os.close(fd)
        os.unlink(args.tune_path)
    pts, dg = workload(N)
    b = synth.uniform_rhs(N, args.nrhs, 201)
    bt = torch.from_numpy(np.ascontiguousarray(b.T)).cuda()  # (nrhs, N) row-major = (N, nrhs) col-major
    xt = torch.empty_like(bt)
    F5, F4, f_dev = None, None, None
    notes = []
    if not args.no_gmres:
        F5 = FMM(pts, dg, cheb_order=5, leaf_max=256)  # FMM depth for ~30 points per leaf (not the IFMM's)
        f_dev = bt[0].contiguous()
        log(f"FMM (order 5) built: {json.dumps(F5.stats())}")
    F4 = FMM(pts, dg, cheb_order=4, leaf_max=64)  # the IFMM's own tree and operators: exactly A~
    # ||A~||_2 from power iteration (A~ is symmetric for unit weights): the
    # scale of the normwise backward error ||A~ x - b|| / (||A~|| ||x|| + ||b||)
    v = torch.from_numpy(synth.uniform_rhs(N, 1, 77)[:, 0].copy()).cuda()
    v /= torch.linalg.norm(v)
    anorm = 0.0
    for _ in range(30):
        w = F4.matvec(v)
        anorm = float(torch.linalg.norm(w))
        v = w / anorm
    args.anorm = anorm
    log(f"FMM (order 4, the IFMM's tree) built; ||A~||_2 ~ {anorm:.4e}")
    forms = {"all": ["mixed", "fp64", "heuristic"], "both": ["mixed", "fp64"], "mixed": ["mixed"], "fp64": ["fp64"],
             "heuristic": ["heuristic"]}[args.form]
    res, stats0, xs = {}, None, {}
    lead = forms[0]
    est_step = None
    for fm in forms:
        if fm != lead:
            # a comparison form: one step, when it fits
            need = (est_step or 60.0) * (2.0 if fm == "fp64" else 1.2) + 15
            if left(args) < need:
                notes.append(f"form {fm} skipped: needs ~{need:.0f} s, {left(args):.0f} s left")
                log(notes[-1])
                continue
        log(f"form {fm}")
        try:
            if fm == lead:
                out, st, x0 = run_form(fm, pts, dg, argparse.Namespace(**{**vars(args), "reserve_s": _reserve(args, forms)}),
                                       bt, xt, F5, F4, f_dev, max(args.steps, 1), min(args.warmup, 1))
                est_step = out["step_s"]
            else:
                # up to CMP_STEPS steps, keeping time for the legs still to come
                rest = forms[forms.index(fm) + 1:]
                keep = sum((est_step or 60.0) * (2.0 if r == "fp64" else 1.2) + 15 for r in rest)
                keep += (0.0 if args.no_batch else 90.0) + (0.0 if args.no_cpu_baseline else 80.0)
                out, st, x0 = run_form(fm, pts, dg, argparse.Namespace(**{**vars(args), "reserve_s": keep}),
                                       bt, xt, F5, F4, f_dev, CMP_STEPS, 0)
        except Exception as e:  # keep the line: report the failure of this form
            traceback.print_exc()
            notes.append(f"form {fm} failed: {e}")
            if fm == lead:
                break
            continue
        res[fm] = out
        xs[fm] = x0
        if stats0 is None:
            stats0 = st
    batch = None
    if not args.no_batch and left(args) > 120:
        log("many-geometry batch (64 geometries)")
        try:
            batch = batch_leg(args)
            log(f"batch: {json.dumps(batch)}")
        except Exception as e:
            traceback.print_exc()
            notes.append(f"batch leg failed: {e}")
    elif not args.no_batch:
        notes.append(f"batch leg skipped: {left(args):.0f} s left")
    cpu = None
    if not args.no_cpu_baseline and left(args) > 30:
        log("cpu baseline (oracle on bounded samples)")
        try:
            cpu = cpu_baseline(args.eps, args.sigma, args.nrhs, N, args)
        except Exception as e:
            traceback.print_exc()
            notes.append(f"cpu baseline failed: {e}")
    elif not args.no_cpu_baseline:
        notes.append(f"cpu baseline skipped: {left(args):.0f} s left")
    R = res.get(lead, {})
    out = {
        "metric": METRIC, "value": R.get("factor_s"), "unit": "s", "n_gpus": 1, "steps": R.get("steps_timed", 0),
        "warmup": min(args.warmup, 1), "ms_per_step": R["step_s"] * 1e3 if R else None, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32mfma" if lead != "fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": f"ellipsoid (1,0.7,0.3) + 5% jitter, N={N}, Laplace 1/(4 pi r), eps={args.eps}, "
                               f"sigma={args.sigma}, depth {R.get('depth')} (bottom level "
                               f"{'by the cost model' if args.bottom_level == -1 else args.bottom_level}; leaves of <= 64 "
                               f"points at depth 7), Chebyshev 4^3, {args.nrhs} RHS; value = factor s of the "
                               f"{'mixed-precision learned-rank' if lead == 'mixed' else lead} form",
                   "parallelism": "single GPU", "bottom_level": args.bottom_level, "colouring": args.colouring,
                   "autotuner": "off" if args.no_tune else "mixed and heuristic forms (tuned in the warm-up step)"},
        "factor_s": R.get("factor_s"), "solve_ms_per_rhs": R.get("solve_ms_per_rhs"),
        "steps_requested": args.steps, "warmup_requested": args.warmup,
        "forms": res,
        "roofline": roofline_of(stats0, lead != "fp64") if stats0 else None,
        "roofline_more": roofline_more(stats0, lead != "fp64") if stats0 else None,
        "cpu_baseline": cpu, "batch_64_geometries": batch, "notes": notes, "wall_s": time.time() - T_START,
    }
    if "mixed" in res and "fp64" in res:
        out["factor_speedup_mixed_vs_fp64"] = res["fp64"]["factor_s"] / res["mixed"]["factor_s"]
        xm, x6 = xs["mixed"], xs["fp64"]
        out["mixed_vs_fp64_solution_rel_diff"] = float(np.linalg.norm(xm - x6) / np.linalg.norm(x6))
    if "mixed" in res and "heuristic" in res:
        out["learned_rank_ablation"] = {
            k: {"mixed": res["mixed"].get(k), "heuristic": res["heuristic"].get(k)}
            for k in ("factor_s", "sketches", "sketches_rejected", "full_decompositions")}
    if args.tune_path and os.path.exists(args.tune_path):
        with open(args.tune_path) as fh:
            out["autotuner_choices"] = [ln.strip() for ln in fh if ln.strip() and not ln.startswith("#")]
        os.unlink(args.tune_path)
    print(json.dumps(out), flush=True)


def _reserve(args, forms):
    """Seconds to keep free after the lead form's timed steps: the comparison
    forms (CMP_STEPS steps each), GMRES, the batch leg and the CPU sample.
    Estimated before the first step from the workload size."""
    if args.reserve_s >= 0:
        return args.reserve_s
    scale = args.n / float(1 << 20)
    est = 0.0
    if "fp64" in forms:
        est += 20.0 * CMP_STEPS * scale + 10
    if "heuristic" in forms:
        est += 18.0 * CMP_STEPS * scale + 10
    if not args.no_gmres:
        est += 5.0 * len(forms)
    if not args.no_cpu_baseline:
        est += 80.0
    if not args.no_batch:
        est += 45.0
    return est


if __name__ == "__main__":
    main()

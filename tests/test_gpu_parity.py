"""Parity of the HIP factorisation and solve with the CPU oracle.

All device work goes through the C ABI (paper_1905_10602_amd.ifmm).  Expected
values come from the oracle (oracle/) run on the same seeded inputs.
Tolerances:
  * eps -> 0: both reproduce the dense LU solve of the represented matrix,
    so they must agree with it to 1e-10 (relative forward error);
  * eps = 1e-6: the two implementations take the same truncation decisions
    except within a narrow band around the threshold (Gram eigenvalues on the
    GPU vs an SVD in the oracle), so the solutions agree within 10 eps
    relative, and the GPU solution has a normwise backward error <= 10 eps.
"""
import numpy as np
import pytest

import synth
from oracle.ifmm import IFMM as Oracle, dense_tilde

pytestmark = pytest.mark.gpu


def _case(shape, N, seed):
    kw = {"jitter": 0.05} if shape == "ellipsoid" else {}
    pts = synth.geometry_points(shape, N, seed, **kw)
    area = {"sphere": 4 * np.pi, "ellipsoid": 2.6, "cube": 24.0}[shape]
    return pts, synth.laplace_self_term(N, area)


def _gpu(pts, eps, sigma, dg, leaf, **kw):
    from paper_1905_10602_amd import IFMM
    return IFMM(pts, eps, sigma, diag=dg, leaf_max=leaf, **kw).factor()


@pytest.mark.parametrize("shape,N,leaf,sigma", [("sphere", 500, 8, 3), ("cube", 600, 12, 6)])
def test_exact_limit_matches_dense_lu(shape, N, leaf, sigma):
    print(f"case exact {shape} N={N} leaf={leaf} sigma={sigma}", flush=True)
    pts, dg = _case(shape, N, 21)
    b = synth.uniform_rhs(N, 2, 101)
    At = dense_tilde(pts, None, dg, leaf_max=leaf)
    xd = np.linalg.solve(At, b)
    h = _gpu(pts, 1e-14, sigma, dg, leaf)
    assert h.depth() >= 3
    x = h.solve(b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10


@pytest.mark.parametrize("shape,N,leaf,sigma,eps", [
    ("sphere", 4096, 64, 6, 1e-6),      # the N = 4096 sphere workload
    ("sphere", 1500, 24, 3, 1e-4),      # strong compression, depth 3
    ("ellipsoid", 3000, 32, 3, 1e-6),
    ("cube", 2000, 20, 6, 1e-5),
])
def test_matches_oracle(shape, N, leaf, sigma, eps):
    print(f"case oracle {shape} N={N} leaf={leaf} sigma={sigma} eps={eps}", flush=True)
    pts, dg = _case(shape, N, 1)
    b = synth.uniform_rhs(N, 3, 101)
    ref = Oracle(pts, eps=eps, sigma=sigma, diag=dg, leaf_max=leaf).factor()
    xo = ref.solve(b)
    h = _gpu(pts, eps, sigma, dg, leaf)
    x = h.solve(b)
    rel = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    assert rel <= 10 * eps, rel
    # Ranks agree except near the truncation threshold: the GPU takes
    # eigenvalues of W^T W, which carry an absolute error ~u lam_1, i.e. ~1e-4
    # relative at the threshold eps^2 lam_1, where the oracle's SVD of W is
    # more accurate; a decision in that band can differ by one.
    for lvl in range(2, ref.depth + 1):
        ro = ref.state[lvl]["r"]
        rg = h.ranks(lvl)
        assert np.mean(ro != rg) <= 0.10
        assert np.abs(ro - rg).max() <= 2


def test_weighted_columns_and_diag_vector():
    N = 1200
    pts = synth.sphere_points(N, 4)
    rng = np.random.default_rng(4)
    w = rng.uniform(0.5, 2.0, N) * (4 * np.pi / N)
    dg = w * synth.laplace_self_term(N) * (N / (4 * np.pi))
    b = synth.uniform_rhs(N, 1, 7)[:, 0]
    eps = 1e-6
    ref = Oracle(pts, eps=eps, sigma=3, diag=dg, weights=w, leaf_max=20).factor()
    h = _gpu(pts, eps, 3, dg, 20, weights=w)
    x, xo = h.solve(b), ref.solve(b)
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 10 * eps


def test_multi_rhs_device_pointers_and_determinism():
    import torch
    N = 2500
    pts, dg = _case("sphere", N, 3)
    h = _gpu(pts, 1e-6, 3, dg, 32)
    b = synth.uniform_rhs(N, 4, 11)
    x = h.solve(b)
    for k in range(4):
        xk = h.solve(b[:, k])
        assert np.allclose(xk, x[:, k], rtol=0, atol=1e-12 * np.abs(x).max())
    bt = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    xt = h.solve(bt).cpu().numpy()
    assert np.array_equal(xt, x)
    # refactorisation and a second handle give bitwise-identical results
    x2 = h.factor().solve(b)
    assert np.array_equal(x2, x)
    x3 = _gpu(pts, 1e-6, 3, dg, 32).solve(b)
    assert np.array_equal(x3, x)


def test_backward_error_at_eps():
    N = 3000
    pts, dg = _case("sphere", N, 8)
    b = synth.uniform_rhs(N, 1, 5)[:, 0]
    At = dense_tilde(pts, None, dg, leaf_max=40)
    for eps in (1e-3, 1e-6):
        x = _gpu(pts, eps, 3, dg, 40).solve(b)
        r = np.linalg.norm(At @ x - b)
        assert r / (np.linalg.norm(At, 2) * np.linalg.norm(x) + np.linalg.norm(b)) <= 10 * eps


def test_m2l_capacity_growth_path(monkeypatch):
    # without headroom every rank increase reallocates the node's M2L blocks
    monkeypatch.setenv("IFMM_IL_TIGHT", "1")
    N, eps = 3000, 1e-6
    pts, dg = _case("ellipsoid", N, 2)
    b = synth.uniform_rhs(N, 2, 3)
    h = _gpu(pts, eps, 3, dg, 32)
    assert h.stats()["grown"] > 0
    x = h.solve(b)
    xo = Oracle(pts, eps=eps, sigma=3, diag=dg, leaf_max=32).factor().solve(b)
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 10 * eps


@pytest.mark.parametrize("big_d", [1, 40, 100])
def test_blocked_pivot_path_exact_limit(monkeypatch, big_d):
    # every pivot of order >= big_d takes the blocked multi-workgroup LU of the
    # augmented matrix; orders of 1..~400 cover partial panels and ragged tails
    monkeypatch.setenv("IFMM_BIG_D", str(big_d))
    print(f"case blocked exact big_d={big_d}", flush=True)
    pts, dg = _case("sphere", 900, 21)
    b = synth.uniform_rhs(900, 2, 101)
    At = dense_tilde(pts, None, dg, leaf_max=16)
    xd = np.linalg.solve(At, b)
    x = _gpu(pts, 1e-14, 3, dg, 16).solve(b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10


def test_blocked_pivot_path_matches_oracle(monkeypatch):
    monkeypatch.setenv("IFMM_BIG_D", "64")
    N, eps = 3000, 1e-6
    pts, dg = _case("ellipsoid", N, 2)
    b = synth.uniform_rhs(N, 2, 3)
    x = _gpu(pts, eps, 3, dg, 32).solve(b)
    xo = Oracle(pts, eps=eps, sigma=3, diag=dg, leaf_max=32).factor().solve(b)
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 10 * eps


@pytest.mark.parametrize("shape,N,leaf,sigma,eps", [("sphere", 4096, 64, 6, 1e-6), ("ellipsoid", 3000, 32, 3, 1e-6),
                                                    ("sphere", 1500, 24, 3, 1e-4)])
def test_mixed_precision_error_vs_oracle(shape, N, leaf, sigma, eps):
    # FP32 matrix cores for the Schur and basis-change products: the solution
    # stays within 10 eps of the FP64 oracle (the FP32 rounding of an operand,
    # 6e-8 relative, is 0.06 eps at eps = 1e-6, well inside the truncation)
    print(f"case mixed {shape} N={N} eps={eps}", flush=True)
    pts, dg = _case(shape, N, 1)
    b = synth.uniform_rhs(N, 2, 101)
    xo = Oracle(pts, eps=eps, sigma=sigma, diag=dg, leaf_max=leaf).factor().solve(b)
    h = _gpu(pts, eps, sigma, dg, leaf, precision="mixed")
    x = h.solve(b)
    rel = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    x64 = _gpu(pts, eps, sigma, dg, leaf).solve(b)
    rel64 = np.linalg.norm(x64 - xo) / np.linalg.norm(xo)
    print(f"mixed error vs oracle {rel:.3e} (fp64 {rel64:.3e})", flush=True)
    assert rel <= 10 * eps
    assert not np.array_equal(x, x64)  # the FP32 path really ran


def test_top_tau_and_forced_depth_match_oracle():
    # tau = 4: levels 3 and 2 are eliminated one node per step (Sec. 4.2's
    # matrix-parallel top); the oracle with the same tau, and a forced
    # coarser depth, both within 10 eps
    N, eps = 3000, 1e-6
    print(f"case top tau=4 and depth 3, ellipsoid N={N}", flush=True)
    pts, dg = _case("ellipsoid", N, 9)
    b = synth.uniform_rhs(N, 2, 61)
    xo = Oracle(pts, eps=eps, sigma=3, diag=dg, leaf_max=16, tau=4).factor().solve(b)
    x = _gpu(pts, eps, 3, dg, 16, top_tau=4).solve(b)
    rel = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    print(f"tau=4 vs oracle {rel:.3e}", flush=True)
    assert rel <= 10 * eps
    xo3 = Oracle(pts, eps=eps, sigma=3, diag=dg, leaf_max=16, depth=3).factor().solve(b)
    h3 = _gpu(pts, eps, 3, dg, 16, bottom_level=3)
    assert h3.depth() == 3
    rel3 = np.linalg.norm(h3.solve(b) - xo3) / np.linalg.norm(xo3)
    print(f"depth 3 vs oracle {rel3:.3e}", flush=True)
    assert rel3 <= 10 * eps


def test_fp64_matrix_core_schur_matches_oracle(monkeypatch):
    # IFMM_F64_MFMA=1: FP64 Schur products on the FP64 matrix cores
    # (v_mfma_f64_16x16x4f64); same 10 eps bar against the oracle as the FMA
    # tile.  The tile itself is checked against numpy in the kernel tests.
    N, eps = 3000, 1e-6
    print(f"case FP64 matrix-core Schur sphere N={N}", flush=True)
    pts, dg = _case("sphere", N, 8)
    b = synth.uniform_rhs(N, 2, 41)
    xo = Oracle(pts, eps=eps, sigma=3, diag=dg, leaf_max=40).factor().solve(b)
    monkeypatch.setenv("IFMM_F64_MFMA", "1")
    xm = _gpu(pts, eps, 3, dg, 40).solve(b)
    monkeypatch.setenv("IFMM_F64_MFMA", "0")
    xf = _gpu(pts, eps, 3, dg, 40).solve(b)
    rel = np.linalg.norm(xm - xo) / np.linalg.norm(xo)
    print(f"matrix-core Schur vs oracle {rel:.3e}; bitwise equal to the FMA tile: {np.array_equal(xm, xf)}",
          flush=True)
    assert rel <= 10 * eps
    assert np.linalg.norm(xm - xf) <= 10 * eps * np.linalg.norm(xf)


def test_schur_near_far_kernels_match_one_kernel(monkeypatch):
    # IFMM_SCHUR_SPLIT=1: the mixed form's near (FP64) and far (FP32) Schur
    # products as two kernels on two streams; every product is the same
    # arithmetic as in the single kernel, so the solutions agree bit for bit
    N, eps = 6000, 1e-6
    print(f"case Schur near / far kernels ellipsoid N={N}", flush=True)
    pts, dg = _case("ellipsoid", N, 13)
    b = synth.uniform_rhs(N, 2, 81)
    out = {}
    for v in ("1", "0"):
        monkeypatch.setenv("IFMM_SCHUR_SPLIT", v)
        h = _gpu(pts, eps, 3, dg, 32, precision="mixed")
        out[v] = h.solve(b)
    assert np.array_equal(out["1"], out["0"])


def test_split_backward_tiles_match_unsplit(monkeypatch):
    # colours with few backward row tiles split each tile's inner dimension
    # over several workgroups and add the partial sums in order; against one
    # task per tile (IFMM_SOLVE_SPLIT=0) only the summation order differs
    N, eps = 20000, 1e-6
    print(f"case split backward tiles sphere N={N}", flush=True)
    pts, dg = _case("sphere", N, 12)
    b = synth.uniform_rhs(N, 8, 71)
    out = {}
    for v in ("1", "0"):
        monkeypatch.setenv("IFMM_SOLVE_SPLIT", v)
        h = _gpu(pts, eps, 3, dg, 64)
        st = h.stats()
        out[v] = (h.solve(b), h.solve(b[:, :1]), [lv["rank_sum"] for lv in st["levels"]],
                  sum(lv["solve_split_tiles"] for lv in st["levels"]))
    (x1, y1, r1, s1), (x0, y0, r0, s0) = out["1"], out["0"]
    print(f"split tiles: {s1} (split) / {s0} (unsplit)", flush=True)
    assert s1 > 0 and s0 == 0
    assert r1 == r0
    rel = np.linalg.norm(x1 - x0) / np.linalg.norm(x0)
    rel1 = np.linalg.norm(y1 - y0) / np.linalg.norm(y0)
    print(f"split vs unsplit: {rel:.2e} (8 RHS), {rel1:.2e} (1 RHS)", flush=True)
    assert rel <= 1e-12 and rel1 <= 1e-12


def test_mixed_solve_reads_fp32_blocks(monkeypatch):
    # mixed form with IFMM_SOLVE32=1: the solve reads FP32 copies of the
    # stored L and G blocks (FP64 vectors and pivot inverses).  Against the
    # same factorisation with FP64 blocks (the default) the store shrinks, the
    # ranks are the same, the solutions differ only by the FP32 rounding of the
    # blocks, and the normwise backward error on A~ stays <= 10 eps
    N, eps = 3000, 1e-6
    print(f"case mixed FP32 solve blocks sphere N={N}", flush=True)
    pts, dg = _case("sphere", N, 8)
    b = synth.uniform_rhs(N, 2, 31)
    out = {}
    for v in ("1", "0"):
        monkeypatch.setenv("IFMM_SOLVE32", v)
        h = _gpu(pts, eps, 3, dg, 40, precision="mixed")
        st = h.stats()
        out[v] = (h.solve(b), st["store_bytes"], [lv["rank_sum"] for lv in st["levels"]])
    (x32, s32, r32), (x64, s64, r64) = out["1"], out["0"]
    rel = np.linalg.norm(x32 - x64) / np.linalg.norm(x64)
    print(f"FP32 vs FP64 solve blocks: rel diff {rel:.3e}, store {s32} vs {s64} bytes", flush=True)
    assert r32 == r64
    assert s32 < 0.75 * s64
    assert not np.array_equal(x32, x64)
    assert rel <= 10 * eps
    At = dense_tilde(pts, None, dg, leaf_max=40)
    for c in range(2):
        r = np.linalg.norm(At @ x32[:, c] - b[:, c])
        assert r / (np.linalg.norm(At, 2) * np.linalg.norm(x32[:, c]) + np.linalg.norm(b[:, c])) <= 10 * eps


def test_phase_b_wave_form_matches_workgroup_form(monkeypatch):
    # mixed form: where every rank of a level is <= 32 the basis change of the
    # M2L blocks runs one block per wave; with leaves of <= 32 points that is
    # the case on the leaf level.  Against the one-workgroup-per-node form the
    # solution differs only by FP32 rounding and the ranks chosen on every
    # level stay the same (a block updated from stale data would shift them)
    N, eps = 3000, 1e-6
    print(f"case phase-B wave form ellipsoid N={N}", flush=True)
    pts, dg = _case("ellipsoid", N, 7)
    b = synth.uniform_rhs(N, 2, 17)
    out = {}
    for w in ("1", "0"):
        monkeypatch.setenv("IFMM_PB_WAVE", w)
        h = _gpu(pts, eps, 3, dg, 32, precision="mixed")
        out[w] = (h.solve(b), [lv["rank_sum"] for lv in h.stats()["levels"]])
    (x1, r1), (x0, r0) = out["1"], out["0"]
    rel = np.linalg.norm(x1 - x0) / np.linalg.norm(x0)
    print(f"wave vs workgroup: rel diff {rel:.3e}, rank sums {r1} vs {r0}", flush=True)
    assert not np.array_equal(x1, x0)  # the wave form really ran
    assert rel <= 20 * eps
    for a, c in zip(r1, r0):
        assert abs(a - c) <= 0.01 * c + 2


@pytest.mark.parametrize("shape,N,leaf,sigma,eps", [("sphere", 4096, 64, 6, 1e-6), ("ellipsoid", 3000, 32, 3, 1e-6)])
def test_sketched_recompression(monkeypatch, shape, N, leaf, sigma, eps):
    # Gram matrices of order >= 64 first try the randomised range finder with
    # the node's current rank plus oversampling; accepted sketches must give the
    # same solution quality as the full eigen-decomposition (IFMM_SKETCH=0)
    monkeypatch.setenv("IFMM_SKETCH_MIN", "64")
    print(f"case sketch {shape} N={N}", flush=True)
    pts, dg = _case(shape, N, 1)
    b = synth.uniform_rhs(N, 2, 101)
    xo = Oracle(pts, eps=eps, sigma=sigma, diag=dg, leaf_max=leaf).factor().solve(b)
    h = _gpu(pts, eps, sigma, dg, leaf)
    st = h.stats()
    print(f"sketches {st['sketches']} rejected {st['sketches_rejected']} narrow {st['sketches_narrow']}", flush=True)
    assert st["sketches"] > st["sketches_rejected"]
    x = h.solve(b)
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 10 * eps
    monkeypatch.setenv("IFMM_SKETCH", "0")
    h0 = _gpu(pts, eps, sigma, dg, leaf)
    assert h0.stats()["sketches"] == 0
    x0 = h0.solve(b)
    assert np.linalg.norm(x0 - xo) / np.linalg.norm(xo) <= 10 * eps


def test_batched_geometries_match_individual_runs():
    # many independent geometries factorised and solved concurrently (one
    # stream and host thread each): bitwise the results of separate runs
    from paper_1905_10602_amd import factor_batch, solve_batch
    geoms = synth.batch_geometries(6, 4000, nmin=1500, nmax=4000)
    eps = 1e-4
    hs, refs, rhs = [], [], []
    for g, (shape, pts) in enumerate(geoms):
        dg = synth.laplace_self_term(pts.shape[0], 4 * np.pi)
        hs.append(_gpu_unfactored(pts, eps, 3, dg, 32))
        refs.append(_gpu(pts, eps, 3, dg, 32))
        rhs.append(synth.uniform_rhs(pts.shape[0], 4, 300 + g))
    factor_batch(hs, threads=4)
    xs = solve_batch(hs, rhs, threads=4)
    for h, r, b, x in zip(hs, refs, rhs, xs):
        assert np.array_equal(x, r.solve(b))
        assert np.array_equal(h.solve(b), x)
    # one of them against the oracle
    shape, pts = geoms[0]
    dg = synth.laplace_self_term(pts.shape[0], 4 * np.pi)
    xo = Oracle(pts, eps=eps, sigma=3, diag=dg, leaf_max=32).factor().solve(rhs[0])
    assert np.linalg.norm(xs[0] - xo) / np.linalg.norm(xo) <= 10 * eps


def _gpu_unfactored(pts, eps, sigma, dg, leaf, **kw):
    from paper_1905_10602_amd import IFMM
    return IFMM(pts, eps, sigma, diag=dg, leaf_max=leaf, **kw)


def test_graph_captured_solve_replays(monkeypatch):
    # the solve is captured into a HIP graph and replayed while the vectors
    # repeat; every replay, with eager work and synchronisations in between,
    # must equal the eager (uncaptured) solve bitwise
    import torch
    N = 3000
    pts, dg = _case("ellipsoid", N, 4)
    b = synth.uniform_rhs(N, 3, 9)
    bt = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    monkeypatch.setenv("IFMM_GRAPH", "0")
    he = _gpu(pts, 1e-6, 3, dg, 32)
    ref = he.solve(bt).cpu().numpy()
    monkeypatch.setenv("IFMM_GRAPH", "1")
    hg = _gpu(pts, 1e-6, 3, dg, 32)
    from paper_1905_10602_amd.ifmm import _check, _ptr, load_library
    Bc = bt.t().contiguous()
    X = torch.empty_like(Bc)
    for rep in range(4):
        _check(load_library().ifmm_solve(hg._h, _ptr(Bc), _ptr(X), 3, N, 1))
        assert np.array_equal(X.t().cpu().numpy(), ref), rep
        junk = torch.randn(1000, 1000, device="cuda", dtype=torch.float64) @ torch.randn(1000, 1000, device="cuda",
                                                                                          dtype=torch.float64)
        torch.cuda.synchronize()
        del junk
    # a different right-hand-side count recaptures; host vectors use the staging buffer
    x1 = hg.solve(b[:, 0])
    assert np.array_equal(x1, he.solve(b[:, 0]))
    assert np.array_equal(hg.solve(b), ref)


def _cfg2(sigma):
    """The N = 65,536 sphere workload with the oracle's stored solutions
    (tests/golden/make_cfg2.py, oracle only)."""
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    ref = np.load(os.path.join(here, f"cfg2_sphere65536_sigma{sigma}.npz"))
    N = 65536
    pts = synth.sphere_points(N, 2)
    dg = synth.laplace_self_term(N)
    b = np.asfortranarray(np.concatenate([synth.uniform_rhs(N, 1, s) for s in range(201, 209)], axis=1))
    return pts, dg, b, ref


@pytest.mark.parametrize("sigma", [3, 6])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sphere_65536_eight_rhs_vs_oracle_fixture(sigma, precision):
    # FP64 and mixed GPU solves of 8 right-hand sides against the oracle's
    # stored solutions at eps = 1e-6.  At this size A~ has condition numbers
    # ~1e5 (i.i.d. points come arbitrarily close), so two factorisations that
    # are each eps-accurate (rank decisions of the GPU's Gram eigenvalues and
    # the oracle's SVD differ inside the truncation band) can differ by
    # ~eps cond(A~) in the solution.  The bar is therefore the normwise
    # backward error on A~ (applied exactly through the Chebyshev 4^3 FMM on
    # the IFMM's own tree): <= 10 eps for the GPU, and its residual no larger
    # than the oracle's times 2; the difference of the two solutions is
    # reported, and the ranks per level agree except inside the band (R9).
    import torch
    from paper_1905_10602_amd import FMM
    print(f"case cfg2 sphere N=65536 sigma={sigma} {precision}", flush=True)
    pts, dg, b, ref = _cfg2(sigma)
    eps = float(ref["eps"])
    h = _gpu(pts, eps, sigma, dg, 64, precision=precision)
    assert h.depth() == int(ref["depth"])
    bt = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    xg = h.solve(bt)
    xo = torch.from_numpy(np.ascontiguousarray(ref["x"])).cuda()
    F = FMM(pts, dg, cheb_order=4, leaf_max=64)
    v = torch.ones(pts.shape[0], dtype=torch.float64, device="cuda")
    for _ in range(30):
        w = F.matvec(v / torch.linalg.norm(v))
        v = w
    anorm = float(torch.linalg.norm(v))
    for c in range(b.shape[1]):
        bc = bt[:, c].contiguous()
        rg = float(torch.linalg.norm(F.matvec(xg[:, c].contiguous()) - bc))
        ro = float(torch.linalg.norm(F.matvec(xo[:, c].contiguous()) - bc))
        nb = float(torch.linalg.norm(bc))
        bwg = rg / (anorm * float(torch.linalg.norm(xg[:, c])) + nb)
        bwo = ro / (anorm * float(torch.linalg.norm(xo[:, c])) + nb)
        fwd = float(torch.linalg.norm(xg[:, c] - xo[:, c]) / torch.linalg.norm(xo[:, c]))
        print(f"  column {c}: backward error GPU {bwg:.2e} oracle {bwo:.2e}; residual GPU {rg / nb:.2e} "
              f"oracle {ro / nb:.2e}; GPU vs oracle {fwd:.2e}", flush=True)
        assert bwg <= 10 * eps
        assert rg <= 2.0 * ro + 10 * eps * nb
    for lvl in range(2, int(ref["depth"]) + 1):
        ro_ = ref[f"ranks_level{lvl}"].astype(int)
        rg_ = h.ranks(lvl).astype(int)
        print(f"  level {lvl}: rank sum GPU {rg_.sum()} oracle {ro_.sum()}; ranks differ at "
              f"{np.mean(ro_ != rg_):.3f} of the nodes, by at most {np.abs(ro_ - rg_).max()}", flush=True)
        # decisions inside the truncation band change what later levels see,
        # so individual ranks drift upwards in the tree; the totals agree
        assert abs(rg_.sum() - ro_.sum()) <= 0.05 * ro_.sum() + 2, lvl


def test_autotuner_cache_written_then_reused(tmp_path):
    # options.tune_cache: the first factorisation with an empty cache times the
    # two Schur tiles on alternating colours of every level, the first solve
    # times every solve step at 1, 4 and 8 waves per workgroup; both write
    # their choices.  Handles built later with the same cache reuse them
    # without timing and give bitwise-identical results; all stay within the
    # 10 eps bar against the oracle.
    N, eps = 3000, 1e-6
    print(f"case autotuner cache sphere N={N}", flush=True)
    pts, dg = _case("sphere", N, 8)
    b = synth.uniform_rhs(N, 8, 51)
    xo = Oracle(pts, eps=eps, sigma=3, diag=dg, leaf_max=40).factor().solve(b)
    cache = tmp_path / "tune.txt"
    for precision in ("fp64", "mixed"):
        x1 = _gpu(pts, eps, 3, dg, 40, precision=precision, tune_cache=str(cache)).solve(b)
        text = cache.read_text()
        depth = _gpu(pts, eps, 3, dg, 40).stats()["depth"]
        for l in range(2, depth + 1):
            assert f"schur {precision} d{depth} l{l} = " in text
            assert f"solve_bwd {precision} d{depth} l{l} k8 = " in text
        assert f"solve {precision} d{depth} k8 = 1" in text
        x2 = _gpu(pts, eps, 3, dg, 40, precision=precision, tune_cache=str(cache)).solve(b)
        assert cache.read_text() == text  # nothing left to tune
        x3 = _gpu(pts, eps, 3, dg, 40, precision=precision, tune_cache=str(cache)).solve(b)
        assert np.array_equal(x2, x3)
        for x in (x1, x2):
            rel = np.linalg.norm(x - xo) / np.linalg.norm(xo)
            print(f"{precision} tuned vs oracle {rel:.3e}", flush=True)
            assert rel <= 10 * eps

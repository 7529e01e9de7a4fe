"""Unit tests of individual device routines against numpy (through an
internal, undeclared test symbol of the library)."""
import ctypes as C
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _syev(mats, k, jacobi):
    lib = C.CDLL(os.path.join(ROOT, "paper_1905_10602_amd", "libifmm.so"))
    f = lib.ifmm_internal_syev
    f.restype = C.c_int
    f.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int]
    cnt, n = len(mats), mats[0].shape[0]
    A = np.ascontiguousarray(np.stack([np.asfortranarray(m).ravel(order="F") for m in mats]))
    lam = np.zeros((cnt, n))
    V = np.zeros((cnt, k * n))
    rc = f(A.ctypes.data, cnt, n, k, lam.ctypes.data, V.ctypes.data, int(jacobi))
    assert rc == 0
    return lam, [V[c].reshape((n, k), order="F") for c in range(cnt)]


def _mats(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for kind in range(4):
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        if kind == 0:
            lam = np.logspace(0, -16, n)
        elif kind == 1:   # degenerate top eigenvalues
            lam = np.logspace(0, -12, n)
            lam[1:4] = lam[0]
        elif kind == 2:   # rank deficient Gram
            Z = rng.standard_normal((n, max(1, n // 3)))
            out.append(Z @ Z.T)
            continue
        else:
            lam = rng.uniform(0, 1, n)
        out.append((Q * lam) @ Q.T)
    return [0.5 * (m + m.T) for m in out]


@pytest.mark.parametrize("n,jacobi,k", [(n, j, 24) for n in (1, 2, 3, 7, 40, 131, 300) for j in (0, 1)] +
                         [(513, 0, 24), (1024, 0, 24), (1190, 0, 300), (2048, 0, 64)])
def test_syev_matches_numpy(n, jacobi, k):
    # orders up to the largest the solver takes (2048); the factorisation of
    # the N = 1M ellipsoid decomposes Gram matrices up to order ~1190
    print(f"case syev n={n} jacobi={jacobi} k={k}", flush=True)
    mats = _mats(n, n)
    k = max(1, min(n, k))
    lam, V = _syev(mats, k, jacobi)
    for G, l, X in zip(mats, lam, V):
        ref = np.linalg.eigvalsh(G)[::-1]
        s = max(abs(ref[0]), 1e-300)
        assert np.abs(l - ref).max() <= 1e-13 * s * max(1, n / 10)
        lk = l[:k]
        # eigen-residual and orthonormality of the k leading vectors
        assert np.linalg.norm(G @ X - X * lk) <= 1e-12 * s * max(1, n / 10)
        assert np.linalg.norm(X.T @ X - np.eye(k)) <= 1e-10


def test_syev_on_ifmm_gram_matrices():
    # the Gram matrices W^T W of the recompressions of a strongly compressing
    # case (sphere, N = 1500, leaf 24, eps = 1e-4), taken from the oracle
    import synth
    import oracle.ifmm as OI
    grams = []
    orig = OI._right_svd

    def spy(W):
        grams.append(W.T @ W)
        return orig(W)

    OI._right_svd = spy
    try:
        N = 1500
        pts = synth.sphere_points(N, 1)
        OI.IFMM(pts, eps=1e-4, sigma=3, diag=synth.laplace_self_term(N), leaf_max=24).factor()
    finally:
        OI._right_svd = orig
    by_n = {}
    for G in grams:
        by_n.setdefault(G.shape[0], []).append(0.5 * (G + G.T))
    worst = 0.0
    for n, mats in sorted(by_n.items()):
        ks = []
        for G in mats:
            lam = np.linalg.eigvalsh(G)[::-1]
            ks.append(int(np.sum(lam > 1e-8 * lam[0])) if lam[0] > 0 else 0)
        k = max(max(ks), 1)
        lam, V = _syev(mats, k, 0)
        for G, l, X, kk in zip(mats, lam, V, ks):
            if kk == 0:
                continue
            w, Q = np.linalg.eigh(G)
            Q = Q[:, ::-1][:, :kk]
            Xk = X[:, :kk]
            err = np.linalg.norm(Xk @ Xk.T - Q @ Q.T)
            worst = max(worst, err)
            assert err < 1e-6, (n, kk, err)


@pytest.mark.parametrize("m,n,k,tA,tB", [(64, 64, 64, 0, 0), (130, 70, 33, 0, 0), (5, 200, 300, 1, 0),
                                         (77, 9, 1, 0, 1), (100, 100, 0, 1, 1), (20, 30, 7, 0, 0),
                                         (32, 32, 32, 1, 1), (9, 3, 32, 1, 0), (100, 90, 129, 0, 1),
                                         (70, 130, 96, 1, 0), (64, 64, 95, 0, 0)])
@pytest.mark.parametrize("f32", [0, 1, 2, 3])
def test_workgroup_gemm_fp64_and_fp32_matrix_cores(m, n, k, tA, tB, f32):
    # f32: 0 FP64 FMA tile, 1 / 2 FP32 matrix-core tiles, 3 FP64 matrix-core tile
    # (untransposed operands; transposed cases take the FMA tile)
    lib = C.CDLL(os.path.join(ROOT, "paper_1905_10602_amd", "libifmm.so"))
    f = lib.ifmm_internal_gemm
    f.restype = C.c_int
    f.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_double,
                  C.c_void_p, C.c_int]
    rng = np.random.default_rng(m + n + k)
    A = rng.standard_normal((k, m) if tA else (m, k))
    B = rng.standard_normal((n, k) if tB else (k, n))
    Cm = rng.standard_normal((m, n))
    Af, Bf, Cf = np.asfortranarray(A), np.asfortranarray(B), np.asfortranarray(Cm.copy())
    assert f(m, n, k, -1.5, Af.ctypes.data, tA, Bf.ctypes.data, tB, 0.5, Cf.ctypes.data, f32) == 0
    opA = A.T if tA else A
    opB = B.T if tB else B
    ref = -1.5 * opA @ opB + 0.5 * Cm
    small = m <= 32 and n <= 32 and k <= 32  # one-pass FP64 product for tiny tiles, whatever the flag
    if f32 in (1, 2) and not small:
        # operands rounded to FP32 and FP32 accumulation: |error| <= c k u32 |A||B|
        bound = 1.5 * (k + 2) * 2.0 ** -23 * (np.abs(opA) @ np.abs(opB)) + 1e-300
        assert np.all(np.abs(Cf - ref) <= bound)
        if k > 1:
            assert not np.allclose(Cf, ref, rtol=0, atol=1e-12)  # really FP32
    else:
        assert np.allclose(Cf, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def _blocked_solve(D, B):
    lib = C.CDLL(os.path.join(ROOT, "paper_1905_10602_amd", "libifmm.so"))
    f = lib.ifmm_internal_blocked_solve
    f.restype = C.c_int
    f.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
    cnt, d, W = len(D), D[0].shape[0], B[0].shape[1]
    Dd = np.ascontiguousarray(np.stack([m.ravel(order="F") for m in D]))
    Bd = np.ascontiguousarray(np.stack([m.ravel(order="F") for m in B]))
    X = np.zeros_like(Bd)
    info = np.zeros(cnt, dtype=np.int32)
    assert f(Dd.ctypes.data, cnt, d, Bd.ctypes.data, W, X.ctypes.data, info.ctypes.data) == 0
    return [X[c].reshape((d, W), order="F") for c in range(cnt)], info


@pytest.mark.parametrize("d,W", [(63, 40), (64, 64), (65, 129), (700, 300), (1500, 700), (1537, 257)])
def test_blocked_pivot_solve_matches_numpy(d, W):
    # the multi-workgroup LU of the augmented system that large pivots take,
    # up to orders beyond the largest of the N = 1M ellipsoid (~1,480): a
    # dense matrix and a saddle-point matrix [[P, B^T], [B, 0]] like the
    # pivots of the extended system (its zero block needs the row pivoting)
    print(f"case blocked solve d={d} W={W}", flush=True)
    rng = np.random.default_rng(d + W)
    dense = rng.standard_normal((d, d)) + 4.0 * np.sqrt(d) * np.eye(d)
    r = d // 3
    n = d - r
    P = rng.standard_normal((n, n))
    P = P @ P.T / n + np.eye(n)
    Bm = rng.standard_normal((r, n))
    saddle = np.zeros((d, d))
    saddle[:n, :n] = P
    saddle[:n, n:] = Bm.T
    saddle[n:, :n] = Bm
    Ds = [np.asfortranarray(dense), np.asfortranarray(saddle)]
    Bs = [np.asfortranarray(rng.standard_normal((d, W))) for _ in Ds]
    Xs, info = _blocked_solve(Ds, Bs)
    assert np.all(info == 0)
    for D, B, X in zip(Ds, Bs, Xs):
        ref = np.linalg.solve(D, B)
        res = np.linalg.norm(D @ X - B) / (np.linalg.norm(D) * np.linalg.norm(X))
        assert res <= 1e-14 * d, res
        assert np.linalg.norm(X - ref) / np.linalg.norm(ref) <= 1e-13 * np.linalg.cond(D)

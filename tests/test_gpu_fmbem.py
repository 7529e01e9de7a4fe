"""Parity of the HIP FMM product and FGMRES driver with the CPU oracle.

* fmm_matvec computes A~ x, the Chebyshev-FMM representation of A: it must
  equal the oracle's FMM (oracle/fmm.py, itself pinned to the block-wise A~)
  up to rounding, 1e-12 relative;
* at sizes the oracle cannot reach, sampled rows are compared with the direct
  sum A x (interpolation error of the order-5 FMM, < 1e-4 relative);
* fmm_gmres follows the same FGMRES(m) recurrence as oracle/krylov.py: with
  the same operator (rounding apart) the iteration counts agree within one
  and the solutions within the tolerance times a small factor;
* the BEM solution converges to the closed-form density of a point source.
"""
import numpy as np
import pytest

import synth
from oracle import bem
from oracle.fmm import FMM as OracleFMM
from oracle.ifmm import IFMM as OracleIFMM
from oracle.krylov import fgmres

pytestmark = pytest.mark.gpu


def _panels(subdiv):
    V, T = synth.icosphere(subdiv)
    c, a = bem.panels(V, T)
    return c, a, bem.self_terms(a)


@pytest.mark.parametrize("shape,N,leaf,nc", [("sphere", 3000, 32, 5), ("ellipsoid", 2500, 16, 4),
                                             ("cube", 1800, 24, 5), ("sphere", 40, 64, 5)])
def test_fmm_matvec_matches_oracle(shape, N, leaf, nc):
    from paper_1905_10602_amd import FMM
    print(f"case fmm {shape} N={N} leaf={leaf} nc={nc}", flush=True)
    kw = {"jitter": 0.05} if shape == "ellipsoid" else {}
    pts = synth.geometry_points(shape, N, 7, **kw)
    rng = np.random.default_rng(8)
    w = rng.uniform(0.5, 1.5, N)
    dg = rng.uniform(1.0, 2.0, N)
    x = synth.uniform_rhs(N, 1, 9)[:, 0]
    yo = OracleFMM(pts, w, dg, leaf_max=leaf, cheb_order=nc).matvec(x)
    F = FMM(pts, dg, weights=w, cheb_order=nc, leaf_max=leaf)
    y = F.matvec(x)
    assert np.linalg.norm(y - yo) <= 1e-12 * np.linalg.norm(yo)
    st = F.stats()
    assert st["N"] == N and st["K"] == nc ** 3 and st["matvecs"] == 1


def test_fmm_matvec_device_pointers_and_repeat():
    import torch
    from paper_1905_10602_amd import FMM
    N = 5000
    pts = synth.sphere_points(N, 3)
    F = FMM(pts, synth.laplace_self_term(N), cheb_order=5, leaf_max=32)
    x = synth.uniform_rhs(N, 1, 4)[:, 0]
    y = F.matvec(x)
    yt = F.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.array_equal(y, yt)
    assert np.array_equal(F.matvec(x), y)


def test_fmm_matvec_sampled_rows_at_bem_size():
    # the icosphere of subdivision 6 (81,920 panels): sampled rows against the direct sum
    from paper_1905_10602_amd import FMM
    c, a, st = _panels(6)
    N = c.shape[0]
    x = synth.uniform_rhs(N, 1, 12)[:, 0]
    y = FMM(c, st, weights=a, cheb_order=5, leaf_max=64).matvec(x)
    rows = np.random.default_rng(1).choice(N, 64, replace=False)
    for i in rows:
        d = np.linalg.norm(c - c[i], axis=1)
        d[i] = 1.0
        ai = a / (4 * np.pi * d)
        ai[i] = st[i]
        ref = ai @ x
        assert abs(y[i] - ref) <= 1e-4 * np.abs(ai) @ np.abs(x)


def test_gmres_matches_oracle_fgmres():
    from paper_1905_10602_amd import FMM, IFMM
    c, a, st = _panels(4)  # 5120 panels
    f = bem.point_source(c)
    leaf = 32
    # no preconditioner: the same operator up to rounding
    of = OracleFMM(c, a, st, leaf_max=leaf, cheb_order=5)
    xo, ito, rro = fgmres(of.matvec, f, tol=1e-8, restart=30, maxit=300)
    F = FMM(c, st, weights=a, cheb_order=5, leaf_max=leaf)
    x, it, rr = F.gmres(f, tol=1e-8, restart=30, maxit=300)
    assert rr <= 1e-8 and abs(it - ito) <= 1
    assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)
    # true residual of the returned iterate (fresh product)
    assert np.linalg.norm(F.matvec(x) - f) <= 2e-8 * np.linalg.norm(f)
    # IFMM preconditioner (Alg. 5) on both sides
    eps = 1e-3
    P = IFMM(c, eps, 3, diag=st, weights=a, leaf_max=leaf).factor()
    po = OracleIFMM(c, eps=eps, sigma=3, diag=st, weights=a, leaf_max=leaf).factor()
    xo2, ito2, _ = fgmres(of.matvec, f, precond=po.solve, tol=1e-8, restart=30, maxit=300)
    x2, it2, rr2 = F.gmres(f, precond=P, tol=1e-8, restart=30, maxit=300)
    assert rr2 <= 1e-8 and abs(it2 - ito2) <= 1
    assert it2 < it
    assert np.linalg.norm(x2 - xo2) <= 1e-6 * np.linalg.norm(xo2)


def test_fmbem_converges_to_closed_form_density():
    from paper_1905_10602_amd import IFMM, fmbem_gmres
    c, a, st = _panels(5)  # 20480 panels
    f = bem.point_source(c)
    P = IFMM(c, 1e-3, 3, diag=st, weights=a, leaf_max=64).factor()
    sol, it, rr = fmbem_gmres(c, a, st, f, precond=P, tol=1e-8, restart=50, maxit=200)
    assert rr <= 1e-8 and it <= 30
    ex = bem.exact_density(c)
    assert np.linalg.norm(sol - ex) / np.linalg.norm(ex) < 0.01


def test_gmres_errors():
    from paper_1905_10602_amd import FMM, IFMM, IfmmError
    c, a, st = _panels(3)
    F = FMM(c, st, weights=a)
    f = bem.point_source(c)
    with pytest.raises(IfmmError) as e:
        F.gmres(f, restart=0)
    assert e.value.status == "IFMM_EINVAL"
    P = IFMM(c, 1e-3, 3, diag=st, weights=a)
    with pytest.raises(IfmmError) as e:
        F.gmres(f, precond=P)  # not factored
    assert e.value.status == "IFMM_ESTATE"
    # too few iterations: ENOCONV, iterate and counters still returned
    x, it, rr = F.gmres(f, tol=1e-14, restart=5, maxit=3, allow_noconv=True)
    assert it == 3 and rr > 1e-14 and np.all(np.isfinite(x))
    with pytest.raises(IfmmError) as e:
        F.gmres(f, tol=1e-14, restart=5, maxit=3)
    assert e.value.status == "IFMM_ENOCONV"
    # a zero right-hand side returns x = 0 at once
    x, it, rr = F.gmres(np.zeros_like(f))
    assert it == 0 and not np.any(x)

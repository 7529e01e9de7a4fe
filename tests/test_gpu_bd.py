"""The block-diagonal preconditioner BD (bd_build / bd_apply / fmm_gmres_bd)
against the CPU oracle (oracle/bd.py): the application agrees to roundoff
(the blocks are dense LU solves on both sides), and FGMRES with BD takes the
oracle's iteration count (+-1) at the same tolerance."""
import numpy as np
import pytest

import synth
from oracle.bd import BD as OracleBD
from oracle.bem import panels, point_source, self_terms

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("sub,leaf,coarser", [(4, 16, 0), (4, 16, 1), (5, 64, 1)])
def test_bd_apply_matches_oracle(sub, leaf, coarser):
    from paper_1905_10602_amd import BD
    from oracle.tree import Tree
    v, f = synth.icosphere(sub)
    c, a = panels(v, f)
    st = self_terms(a)
    level = Tree(c, leaf_max=leaf, sigma=3).depth - coarser
    print(f"case bd icosphere {sub} N={c.shape[0]} level={level}", flush=True)
    ref = OracleBD(c, st, weights=a, level=level, leaf_max=leaf)
    bd = BD(c, st, weights=a, level=level, leaf_max=leaf)
    assert bd.stats()["level"] == level
    r = np.random.default_rng(sub).standard_normal(c.shape[0])
    z, zo = bd.apply(r), ref.apply(r)
    assert np.linalg.norm(z - zo) / np.linalg.norm(zo) <= 1e-11


def test_fmbem_gmres_with_bd_matches_oracle():
    import torch
    from paper_1905_10602_amd import BD, FMM
    from oracle.bem import dense_matrix
    from oracle.krylov import fgmres
    v, f = synth.icosphere(4)
    c, a = panels(v, f)
    st = self_terms(a)
    b = point_source(c)
    F = FMM(c, st, weights=a, cheb_order=5, leaf_max=16)
    out = {}
    for level in (0, 3):
        bd = BD(c, st, weights=a, level=level, leaf_max=16)
        x, it, rr = F.gmres(torch.from_numpy(b).cuda(), precond=bd, tol=1e-8, restart=50)
        out[level] = it
        A = dense_matrix(c, a)  # the FMM product is A to ~1e-6 at order 5; iterations agree within one
        ref = OracleBD(c, st, weights=a, level=bd.stats()["level"], leaf_max=16)
        _, ito, _ = fgmres(lambda y: A @ y, b, precond=ref.apply, tol=1e-8, restart=50)
        print(f"BD level {bd.stats()['level']}: GPU {it} iterations (relres {rr:.1e}), oracle {ito}", flush=True)
        assert rr <= 1e-8 and abs(it - ito) <= 1

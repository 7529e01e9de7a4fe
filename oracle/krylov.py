"""Oracle: restarted, right-preconditioned flexible GMRES.

Test infrastructure only (see the package header).

Alg. 4 of the paper solves the BEM system with GMRES(m) from x = 0, stopping
when the relative residual ||A x - b|| / ||b|| falls below tol (Sec. 5.1);
the preconditioner of Alg. 5 returns v ~ A^-1 r.  Written here from Saad's
textbook statement of FGMRES(m) (right preconditioning, the preconditioned
directions z_j kept, so the preconditioner may vary between calls):

  r = b - A x;  beta = ||r||;  v_1 = r / beta;  g = beta e_1
  for j = 1..m:
      z_j = M v_j;  w = A z_j
      h_{:, j} = V^T w;  w -= V h_{:, j}       classical Gram-Schmidt ...
      c = V^T w;  w -= V c;  h_{:, j} += c      ... applied twice (CGS2)
      h_{j+1, j} = ||w||;  v_{j+1} = w / h_{j+1, j}
      Givens rotations reduce column j of H to upper triangular form and
      rotate g; |g_{j+1}| is the residual norm of the least-squares iterate
      stop when |g_{j+1}| <= tol ||b||
  x += Z y with R y = g (back substitution); restart from the new residual.

Returns the iterate, the number of inner iterations and the final relative
residual estimate |g_{j+1}| / ||b||.
"""
from __future__ import annotations

import numpy as np


def givens(a: float, b: float):
    """(c, s) with [c s; -s c] [a; b] = [r; 0], r = hypot(a, b) >= 0."""
    if b == 0.0:
        return (1.0, 0.0) if a >= 0.0 else (-1.0, 0.0)
    r = np.hypot(a, b)
    return a / r, b / r


def fgmres(matvec, b, precond=None, tol=1e-8, restart=50, maxit=1000, x0=None):
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    M = (lambda v: v) if precond is None else precond
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), 0, 0.0
    its = 0
    relres = np.linalg.norm(b - matvec(x)) / bnorm
    while its < maxit:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        relres = beta / bnorm
        if relres <= tol:
            break
        m = min(restart, maxit - its)
        V = np.zeros((n, m + 1))
        Z = np.zeros((n, m))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        k = 0
        for j in range(m):
            Z[:, j] = M(V[:, j])
            w = matvec(Z[:, j])
            h = V[:, :j + 1].T @ w
            w = w - V[:, :j + 1] @ h
            c = V[:, :j + 1].T @ w
            w = w - V[:, :j + 1] @ c
            H[:j + 1, j] = h + c
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            its += 1
            relres = abs(g[j + 1]) / bnorm
            if relres <= tol or H[j, j] == 0.0:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:, :k] @ y
        if relres <= tol:
            break
    return x, its, relres

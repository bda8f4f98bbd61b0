"""Oracle: restarted (flexible) GMRES with right preconditioning, FP64.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only tests, the smoke check and the CPU-baseline leg of
the benchmark do.

The paper's accelerator is restarted GMRES with a relative-residual stopping
test on the row-scaled system (section 5); its remark on right
preconditioning (section 3.3, C B^{-1} has the same spectrum) is the form used
here.  Steps, in textbook order (Saad's GMRES/FGMRES with modified
Gram-Schmidt and Givens rotations):

  r = b - C x;  beta = ||r||;  v_1 = r / beta;  g = beta e_1
  for j = 1 .. restart:
      z_j = B^{-1} v_j                      (kept for FGMRES)
      w = C z_j
      for i = 1 .. j:  h_ij = <w, v_i>;  w = w - h_ij v_i     (MGS)
        or, with ortho = "cgs2", classical Gram-Schmidt applied twice:
        h = V_j^T w; w = w - V_j h; c = V_j^T w; w = w - V_j c; h += c
      h_{j+1,j} = ||w||;  v_{j+1} = w / h_{j+1,j}
      apply rotations 1..j-1 to column j; new rotation from (h_jj, h_{j+1,j})
      with t = hypot(a, b), c = a/t, s = b/t (b = 0: c = 1, s = 0);
      g_{j+1} = -s g_j, g_j = c g_j
      stop the cycle when |g_{j+1}| <= tol ||b|| or h_{j+1,j} == 0
  y = R^{-1} g (back substitution);  x += Z y (FGMRES) or x += B^{-1} V y
  converged iff the true residual ||b - C x|| / ||b|| <= tol, else restart.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    converged: bool
    true_relres: float
    est_history: list = field(default_factory=list)
    true_history: list = field(default_factory=list)


def givens(a: float, b: float):
    if b == 0.0:
        return 1.0, 0.0
    t = float(np.hypot(a, b))
    return a / t, b / t


def gmres(matvec, precond, b, x0=None, restart=30, tol=1e-8, maxit=1000, flexible=True, ortho="mgs"):
    if ortho not in ("mgs", "cgs2"):
        raise ValueError(ortho)
    b = np.asarray(b, dtype=np.float64)
    N = b.size
    x = np.zeros(N) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return GmresResult(np.zeros(N), 0, True, 0.0)
    its = 0
    est_hist, true_hist = [], []
    r = b - matvec(x)
    relres = float(np.linalg.norm(r)) / bnorm
    true_hist.append(relres)
    if relres <= tol:
        return GmresResult(x, 0, True, relres, est_hist, true_hist)
    while its < maxit:
        beta = float(np.linalg.norm(r))
        V = np.zeros((restart + 1, N))
        Z = np.zeros((restart, N)) if flexible else None
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        jdone = 0
        for j in range(restart):
            z = precond(V[j])
            if flexible:
                Z[j] = z
            w = matvec(z)
            if ortho == "mgs":
                for i in range(j + 1):
                    H[i, j] = float(np.dot(w, V[i]))
                    w = w - H[i, j] * V[i]
            else:
                Vj = V[:j + 1]
                h = Vj @ w
                w = w - Vj.T @ h
                c = Vj @ w
                w = w - Vj.T @ c
                H[:j + 1, j] = h + c
            H[j + 1, j] = float(np.linalg.norm(w))
            breakdown = H[j + 1, j] == 0.0
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            jdone = j + 1
            est_hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or its >= maxit or breakdown:
                break
        y = np.zeros(jdone)
        for i in range(jdone - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:jdone], y[i + 1:jdone])) / H[i, i]
        if flexible:
            x = x + Z[:jdone].T @ y
        else:
            x = x + precond(V[:jdone].T @ y)
        r = b - matvec(x)
        relres = float(np.linalg.norm(r)) / bnorm
        true_hist.append(relres)
        if relres <= tol:
            return GmresResult(x, its, True, relres, est_hist, true_hist)
    return GmresResult(x, its, False, relres, est_hist, true_hist)


def solve_system(pre, b_unscaled, restart=30, tol=1e-8, maxit=1000, flexible=True, x0=None, ortho="mgs"):
    """Solve the row-scaled system C~ x = R b with B from `pre` (right)."""
    bt = pre.R * b_unscaled
    return gmres(lambda v: pre.C @ v, pre.apply, bt, x0=x0, restart=restart, tol=tol,
                 maxit=maxit, flexible=flexible, ortho=ortho)


def exact_solve(rowptr, colidx, vals, b):
    """Sparse direct solve of the unscaled system (SuperLU)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    N = len(rowptr) - 1
    C = sp.csc_matrix(sp.csr_matrix((vals, colidx, rowptr), shape=(N, N)))
    return spl.splu(C).solve(np.asarray(b, dtype=np.float64))

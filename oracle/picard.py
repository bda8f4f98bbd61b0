"""Oracle: the Picard (Oseen) outer iteration for the steady Navier-Stokes
equations.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only tests, the smoke check and the CPU-baseline leg of
the benchmark do.

Section 1 obtains the block 2x2 system C x = b as one Picard linearisation
of the steady Navier-Stokes equations: the convecting velocity is frozen at
the previous iterate, which gives an Oseen problem.  The outer loop, plainly:

    x_0 = 0 (the first system is the Stokes problem: no wind)
    for q = 0, 1, ...:
        assemble C_q = C(w(x_q)), b_q = b(w(x_q)), w(x) the velocity part of x
        r_q = |R_q (b_q - C_q x_q)| / |R_q b_q|   (the discrete Navier-Stokes
              residual of the row-scaled system, R_q the row scaling of C_q, so
              that r_q is the residual the Krylov solver reports for x_q)
        stop if r_q <= tol
        x_{q+1} = the preconditioned (F)GMRES solution of C_q x = b_q,
                  started from x_q

The partition is built once, from C_0 (the sparsity pattern does not depend
on the wind), and reused for every step; the preconditioner is set up anew
for every C_q.  The paper runs no outer loop of its own (its systems are
single Oseen steps), so the stopping rule above is a reading.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from oracle.krylov import solve_system
from oracle.partition import build_partition
from oracle.precond import MSCN, Preconditioner, row_scale
from workloads.mac_oseen import FaceWind, make_oseen_mac


def assemble(n, nu, x, stretch=None, seed=0, forcing=None):
    """C(w(x)), b(w(x)) of the Oseen system linearised at x."""
    return make_oseen_mac(n, nu, wind=FaceWind.from_solution(x, n), stretch=stretch, seed=seed,
                          forcing=forcing)


def scaled_residual(rp, ci, v, b, x):
    """|R (b - C x)| / |R b| with R the row scaling of C (section 5)."""
    R, _ = row_scale(rp, ci, v)
    C = sp.csr_matrix((v, ci, rp), shape=(len(b), len(b)))
    return float(np.linalg.norm(R * (b - C @ x)) / np.linalg.norm(R * b))


def ns_residual(n, nu, x, stretch=None, seed=0, forcing=None):
    """The discrete steady Navier-Stokes residual of x (row-scaled)."""
    rp, ci, v, b, meta = assemble(n, nu, x, stretch, seed, forcing)
    return scaled_residual(rp, ci, v, b, x)


@dataclass
class PicardResult:
    x: np.ndarray
    converged: bool
    residuals: list = field(default_factory=list)   # r_q, q = 0..steps
    lin_iters: list = field(default_factory=list)   # linear iterations of each solve


def picard(n, nu, stretch=None, seed=0, m=4, sz=64, mode=MSCN, overlap=0, tol=1e-6, maxit=40,
           restart=50, lin_tol=1e-10, lin_maxit=5000, forcing=None):
    N = 3 * n * n - 2 * n - 1
    x = np.zeros(N)
    part = None
    out = PicardResult(x, False)
    for q in range(maxit + 1):
        rp, ci, v, b, meta = assemble(n, nu, x, stretch, seed, forcing)
        r = scaled_residual(rp, ci, v, b, x)
        out.residuals.append(r)
        if r <= tol:
            out.converged = True
            break
        if q == maxit:
            break
        if part is None:
            part = build_partition(N, rp, ci, v, m, sz)
        pre = Preconditioner(N, rp, ci, v, part, mode, overlap=overlap)
        res = solve_system(pre, b, restart=restart, tol=lin_tol, maxit=lin_maxit, flexible=True, x0=x)
        out.lin_iters.append(res.iters)
        x = res.x
    out.x = x
    return out

"""Pins of the oracle's restarted (F)GMRES (section 5 accelerator; right
preconditioning per the section 3.3 remark)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from oracle.krylov import exact_solve, givens, gmres, solve_system
from oracle.partition import build_partition
from oracle.precond import MSCN, Preconditioner
from workloads.mac_oseen import make_oseen_mac


def _pre(n=16, nu=0.1, m=4, sz=32, seed=1001, st=None):
    rp, ci, v, b, meta = make_oseen_mac(n, nu, stretch=st, seed=seed)
    P = build_partition(meta["N"], rp, ci, v, m, sz)
    return rp, ci, v, b, meta, Preconditioner(meta["N"], rp, ci, v, P, MSCN)


def test_givens():
    for a, b in [(3.0, 4.0), (-1.0, 2.0), (1e-300, 1e-300), (5.0, 0.0), (0.0, -2.0)]:
        c, s = givens(a, b)
        assert abs(c * c + s * s - 1) < 1e-15
        assert abs(-s * a + c * b) <= 1e-15 * max(abs(a), abs(b))
    assert givens(2.0, 0.0) == (1.0, 0.0)


@pytest.mark.parametrize("ortho", ["mgs", "cgs2"])
@pytest.mark.parametrize("flexible", [True, False])
@pytest.mark.parametrize("j", [1, 3, 7])
def test_first_iterates_minimise_over_explicit_krylov_basis(flexible, j, ortho):
    """After j steps from x0 = 0, x_j = B^{-1} K y with K spanning
    {r0, (C B^-1) r0, ...} and y the least-squares minimiser (either
    orthogonalisation: both span the same Krylov space)."""
    rp, ci, v, b, meta, pre = _pre()
    bt = pre.R * b
    res = gmres(lambda x: pre.C @ x, pre.apply, bt, restart=j, maxit=j, tol=1e-30,
                flexible=flexible, ortho=ortho)
    assert res.iters == j
    N = meta["N"]
    K = np.zeros((N, j))
    q = bt.copy()
    for i in range(j):
        K[:, i] = q
        q = pre.C @ pre.apply(q)
    Q, _ = np.linalg.qr(K)
    AQ = np.column_stack([pre.C @ pre.apply(Q[:, i]) for i in range(j)])
    y, *_ = np.linalg.lstsq(AQ, bt, rcond=None)
    x = pre.apply(Q @ y)
    assert np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x)


def test_cgs2_and_mgs_agree_and_keep_the_basis_orthonormal():
    """Classical Gram-Schmidt applied twice gives the same iterates as MGS (to
    rounding) and an orthonormal basis to working precision."""
    rp, ci, v, b, meta, pre = _pre(24, 0.02, st=1.05)
    bt = pre.R * b
    runs = {o: gmres(lambda x: pre.C @ x, pre.apply, bt, restart=40, maxit=120, tol=1e-30, ortho=o)
            for o in ("mgs", "cgs2")}
    a, c = runs["mgs"], runs["cgs2"]
    assert a.iters == c.iters == 120
    assert np.linalg.norm(a.x - c.x) <= 1e-9 * np.linalg.norm(a.x)
    np.testing.assert_allclose(c.est_history, a.est_history, rtol=1e-7)
    # the basis itself: rebuild one cycle's V with the same CGS2 steps
    N = meta["N"]
    V = np.zeros((41, N))
    V[0] = bt / np.linalg.norm(bt)
    for j in range(40):
        w = pre.C @ pre.apply(V[j])
        Vj = V[:j + 1]
        h = Vj @ w
        w = w - Vj.T @ h
        cc = Vj @ w
        w = w - Vj.T @ cc
        V[j + 1] = w / np.linalg.norm(w)
    assert np.abs(V @ V.T - np.eye(41)).max() <= 1e-13


def test_finite_termination():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((25, 25)) + 6 * np.eye(25)
    bb = rng.standard_normal(25)
    res = gmres(lambda x: A @ x, lambda x: x, bb, restart=25, maxit=25, tol=1e-12)
    assert res.converged and res.iters <= 25
    assert np.linalg.norm(res.x - np.linalg.solve(A, bb)) < 1e-9


def test_solution_matches_sparse_direct():
    rp, ci, v, b, meta, pre = _pre()
    res = solve_system(pre, b, restart=30, tol=1e-10, maxit=500, flexible=False)
    assert res.converged and res.true_relres <= 1e-10
    xe = exact_solve(rp, ci, v, b)
    C = sp.csc_matrix(sp.csr_matrix((v, ci, rp)))
    kappa = np.linalg.cond(C.toarray())
    assert np.linalg.norm(res.x - xe) <= 10 * kappa * 1e-10 * np.linalg.norm(xe)


def test_restart_and_true_residual_history():
    rp, ci, v, b, meta, pre = _pre(24, 0.02, 4, 16, st=1.05)
    res = solve_system(pre, b, restart=5, tol=1e-8, maxit=2000, flexible=True)
    assert res.converged
    C = pre.C
    bt = pre.R * b
    assert abs(np.linalg.norm(bt - C @ res.x) / np.linalg.norm(bt) - res.true_relres) < 1e-14
    assert len(res.true_history) >= 2 and res.true_history[-1] <= 1e-8
    assert res.iters == len(res.est_history)


def test_zero_rhs():
    res = gmres(lambda x: x, lambda x: x, np.zeros(5))
    assert res.converged and res.iters == 0 and not res.x.any()


def test_maxit_reports_not_converged():
    rp, ci, v, b, meta, pre = _pre()
    res = solve_system(pre, b, restart=30, tol=1e-14, maxit=3)
    assert not res.converged and res.iters == 3

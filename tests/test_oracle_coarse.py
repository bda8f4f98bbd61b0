"""Pins of the oracle's coarse-grid correction of the interface solve (the
coarse grid correction that section 6 proposes; the reading is stated in
oracle/coarse.py): the coarse space is built by the stated graph rules
(a path graph worked by hand in tests/golden/coarse_path_pieces.txt), its
pieces satisfy their invariants, its columns are orthonormal, the two-level
interface solve reproduces the coarse space exactly (M S Z = Z), a coarse
space spanning the whole separator gives the exact Schur complement inverse
and so B = C (Banachiewicz, the lemma of section 3.3), and Theorem 2's
spectrum statement carries over with Shat^{-1} replaced by M."""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle.coarse import CoarseCorrection, coarse_matrix, coarse_space, near_graph, velocity_classes
from oracle.krylov import gmres
from oracle.partition import Partition, build_partition
from oracle.precond import MSCN, Preconditioner
from workloads.mac_oseen import make_oseen_mac, unknown_positions

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _system(n=16, nu=0.1, st=None, m=4, sz=64, seed=1001):
    rp, ci, v, b, meta = make_oseen_mac(n, nu, stretch=st, seed=seed)
    P = build_partition(meta["N"], rp, ci, v, m, sz)
    return rp, ci, v, b, meta, P


def _golden_path():
    pieces, cols = [], []
    with open(os.path.join(GOLDEN, "coarse_path_pieces.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = line.split()
            if w[0] == "piece":
                pieces.append([int(x) for x in w[3:]])
            else:
                den = float(w[5].split("sqrt(")[1].rstrip("):"))
                cols.append((int(w[3]), w[4], np.array([float(x) for x in w[6:]]) / np.sqrt(den)))
    return pieces, cols


def test_path_graph_pieces_match_hand_worked_example():
    n = 10
    rows, colsx = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                rows.append(i)
                colsx.append(j)
    A = sp.csr_matrix((np.ones(len(rows)), (rows, colsx)), shape=(n, n))
    A.sort_indices()
    part = Partition(N=n, m=0, sz=n, perm=np.arange(n), part=np.full(n, -1), int_offsets=np.array([0]),
                     sep_size=n, agg_offsets=np.array([0, n]), drange_offsets=np.array([0, 0]),
                     drange_nodes=np.zeros(0, np.int64), pair=np.full(n, -1), is_pressure=np.zeros(n, bool))
    offs, pos, zcols = coarse_space(n, A.indptr, A.indices, part, piece=4)
    pieces, gcols = _golden_path()
    assert [list(pos[offs[c]:offs[c + 1]]) for c in range(len(offs) - 1)] == pieces
    assert len(zcols) == len(gcols)
    for (c, v), (gc, kind, gv) in zip(zcols, gcols):
        assert c == gc
        np.testing.assert_allclose(v, gv, rtol=0, atol=1e-15)


def test_velocity_classes_are_the_velocity_components():
    rp, ci, v, b, meta = make_oseen_mac(12, 0.01, stretch=1.05, seed=3)
    N = meta["N"]
    from oracle.partition import pressure_like
    isp = pressure_like(N, np.asarray(rp), np.asarray(ci), np.asarray(v))
    cls = velocity_classes(N, rp, ci, isp)
    _, _, kind = unknown_positions(meta)
    assert np.all(cls[kind == 2] == -1)
    assert np.all(cls[kind == 0] == 0) and np.all(cls[kind == 1] == 1)


@pytest.mark.parametrize("n,st,m,P", [(16, None, 4, 32), (24, 1.05, 6, 16), (20, None, 5, 7)])
def test_pieces_invariants(n, st, m, P):
    rp, ci, v, b, meta, part = _system(n, 0.01, st, m, 32)
    N = meta["N"]
    offs, pos, zcols = coarse_space(N, rp, ci, part, piece=P)
    sep = part.perm[part.n_int:]
    vel = np.nonzero(~part.is_pressure[sep])[0]
    # disjoint, covering every non-pressure separator position, at most P each
    assert sorted(pos.tolist()) == vel.tolist()
    sizes = np.diff(offs)
    assert sizes.max() <= P and sizes.min() >= 1
    H2 = near_graph(N, rp, ci)
    cls = velocity_classes(N, rp, ci, part.is_pressure)
    for c in range(len(offs) - 1):
        mem = sep[pos[offs[c]:offs[c + 1]]]
        assert len(set(cls[mem].tolist())) == 1
        sub = H2[mem][:, mem]
        ncomp = sp.csgraph.connected_components(sub, directed=False)[0]
        assert ncomp == 1
    Z = coarse_matrix(offs, pos, zcols, part.sep_size).toarray()
    np.testing.assert_allclose(Z.T @ Z, np.eye(Z.shape[1]), atol=1e-13)


def _dense_S(pre):
    D, E, F, G, _ = pre.dense_blocks()
    return G - F @ np.linalg.solve(D, E)


def test_two_level_solve_reproduces_the_coarse_space():
    rp, ci, v, b, meta, part = _system(16, 0.05, 1.05, 4, 24)
    pre = Preconditioner(meta["N"], rp, ci, v, part, MSCN, coarse=8)
    S = _dense_S(pre)
    Z = pre.coarse.Z.toarray()
    assert Z.shape[1] > 4
    MSZ = np.column_stack([pre.schur_solve(S @ Z[:, c]) for c in range(Z.shape[1])])
    np.testing.assert_allclose(MSZ, Z, atol=1e-9 * np.abs(Z).max())


def test_full_coarse_space_gives_exact_schur_inverse():
    """Z = I on the separator: M = S^{-1}, so B = C (Banachiewicz)."""
    rp, ci, v, b, meta, part = _system(12, 0.1, None, 3, 16)
    pre = Preconditioner(meta["N"], rp, ci, v, part, MSCN)
    pre.coarse = CoarseCorrection(pre, sp.identity(part.sep_size, format="csc"))
    rng = np.random.default_rng(5)
    x = rng.standard_normal(meta["N"])
    y = pre.apply(pre.C @ x)
    assert np.linalg.norm(y - x) <= 1e-9 * np.linalg.norm(x)
    res = gmres(lambda u: pre.C @ u, pre.apply, pre.R * b, restart=10, tol=1e-8, maxit=10)
    assert res.converged and res.iters == 1


def test_theorem2_spectrum_with_the_coarse_correction():
    """B^{-1} C has |D| unit eigenvalues; the rest are those of M S."""
    rp, ci, v, b, meta, part = _system(10, 0.1, None, 3, 16)
    pre = Preconditioner(meta["N"], rp, ci, v, part, MSCN, coarse=6)
    N, ni, ns = meta["N"], part.n_int, part.sep_size
    C = pre.C.toarray()
    BinvC = np.column_stack([pre.apply(C[:, c]) for c in range(N)])
    ev = np.linalg.eigvals(BinvC)
    S = _dense_S(pre)
    evs = np.linalg.eigvals(np.column_stack([pre.schur_solve(S[:, c]) for c in range(ns)]))
    ones = np.abs(ev - 1.0) < 1e-7
    assert ones.sum() >= ni
    rest = np.sort_complex(np.concatenate([ev[~ones], np.ones(ones.sum() - ni)]))
    np.testing.assert_allclose(np.sort_complex(evs), rest, atol=1e-6 * max(1.0, np.abs(evs).max()))


def test_coarse_correction_cuts_iterations():
    rp, ci, v, b, meta, part = _system(32, 0.01, None, 8, 64, seed=7)
    its = {}
    for P in (0, 32):
        pre = Preconditioner(meta["N"], rp, ci, v, part, MSCN, coarse=P)
        r = gmres(lambda u: pre.C @ u, pre.apply, pre.R * b, restart=50, tol=1e-8, maxit=2000, ortho="cgs2")
        assert r.converged
        its[P] = r.iters
    assert its[32] < 0.6 * its[0]

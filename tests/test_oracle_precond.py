"""Pins of the oracle preconditioner against what the paper and the
mathematics fix: the block-LU definition of B (MSCN definition, section 3.3),
Banachiewicz's block inverse (the lemma of section 3.3), Theorem 2's spectrum,
the LUM special case (section 5 remark that MSCN equals LUM when the coupling
blocks vanish) and the worked example of section 3.2."""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle.partition import Partition, build_partition
from oracle.precond import EXACT_BJ, LUM, MSCN, MSCN_LITERAL, MSCNR, BandILU, BandLU, Preconditioner, row_scale
from workloads.mac_oseen import make_oseen_mac

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _system(n=16, nu=0.1, st=None, m=4, sz=64, seed=1001):
    rp, ci, v, b, meta = make_oseen_mac(n, nu, stretch=st, seed=seed)
    P = build_partition(meta["N"], rp, ci, v, m, sz)
    return rp, ci, v, b, meta, P


def test_row_scaling_unit_max():
    rp, ci, v, b, meta = make_oseen_mac(10, 0.01, stretch=1.05, seed=1)
    R, sv = row_scale(rp, ci, v)
    for i in range(meta["N"]):
        assert abs(np.abs(sv[rp[i]:rp[i + 1]]).max() - 1.0) < 1e-15


def test_band_lu_matches_dense_solve():
    rp, ci, v, b, meta, P = _system(12, 0.01, 1.05, 3, 16)
    pre = Preconditioner(meta["N"], rp, ci, v, P, MSCN)
    Cp = pre.C[P.perm][:, P.perm].toarray()
    rng = np.random.default_rng(0)
    for (a, bb, lu) in pre.blocks:
        y = rng.standard_normal(bb - a)
        x = lu.solve(y)
        ref = np.linalg.solve(Cp[a:bb, a:bb], y)
        assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("mode,overlap,tau", [(MSCN, 0, 0.0), (LUM, 0, 0.0), (MSCNR, 0, 0.0), (MSCN, 23, 0.0),
                                              (MSCNR, 5, 0.0), (LUM, 23, 0.0), (MSCN, 0, 1e-2)])
def test_apply_equals_dense_block_factorisation(mode, overlap, tau):
    """x = B^{-1} y with B = [D 0; F S][D^-1 0; 0 S^-1][D E; 0 S] built densely
    (with tau > 0, D is the product of the incomplete factors)."""
    rp, ci, v, b, meta, P = _system(16, 0.1, None, 4, 24)
    pre = Preconditioner(meta["N"], rp, ci, v, P, mode, overlap=overlap, ilu_tol=tau)
    D, E, F, G, Sh = pre.dense_blocks()
    if tau > 0:
        D = D.copy()
        for (a, bb, f) in pre.blocks:
            D[a:bb, a:bb] = (f.L @ f.U)[np.argsort(f.perm)]
    ni, ns = D.shape[0], Sh.shape[0]
    L = np.block([[D, np.zeros((ni, ns))], [F, Sh]])
    M = sla.block_diag(np.linalg.inv(D), np.linalg.inv(Sh))
    U = np.block([[D, E], [np.zeros((ns, ni)), Sh]])
    B = L @ M @ U
    rng = np.random.default_rng(1)
    y = rng.standard_normal(meta["N"])
    x = pre.apply_permuted(y)
    ref = np.linalg.solve(B, y)
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)
    # B reproduces C~ everywhere except in the separator block, where it holds
    # G - F D^-1 E + Shat... i.e. B(2,2) = F D^-1 E + Shat
    if tau > 0:
        return
    assert np.allclose(B[:ni, :], np.block([[D, E]]), atol=1e-12)
    assert np.allclose(B[ni:, :ni], F, atol=1e-12)
    assert np.allclose(B[ni:, ni:], F @ np.linalg.solve(D, E) + Sh, atol=1e-10)


def test_exact_schur_gives_B_equal_C():
    """Banachiewicz: with Shat = S the factorised B equals C~, so
    apply(C~ x) = x and GMRES converges in one step."""
    rp, ci, v, b, meta, P = _system(16, 0.1, None, 4, 10 ** 6)
    assert P.k == 1
    pre = Preconditioner(meta["N"], rp, ci, v, P, EXACT_BJ)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(meta["N"])
    assert np.linalg.norm(pre.apply(pre.C @ x) - x) <= 1e-12 * np.linalg.norm(x)
    from oracle.krylov import solve_system
    res = solve_system(pre, b, restart=10, tol=1e-10)
    assert res.iters == 1 and res.converged


def test_theorem2_spectrum():
    """B^{-1} C~ has |D| eigenvalues equal to one; the remaining ones are the
    eigenvalues of Shat^{-1} S (Theorem 2)."""
    rp, ci, v, b, meta, P = _system(16, 0.1, None, 4, 32)
    pre = Preconditioner(meta["N"], rp, ci, v, P, MSCN)
    D, E, F, G, Sh = pre.dense_blocks()
    Cp = pre.C[P.perm][:, P.perm].toarray()
    N = meta["N"]
    BinvC = np.column_stack([pre.apply_permuted(Cp[:, j]) for j in range(N)])
    ev = np.linalg.eigvals(BinvC)
    ni = D.shape[0]
    S = G - F @ np.linalg.solve(D, E)
    evS = np.linalg.eigvals(np.linalg.solve(Sh, S))
    near1 = np.abs(ev - 1.0) < 1e-8
    assert near1.sum() >= ni
    # the structure (expLeftPre): [[I, *], [0, Shat^-1 S]]
    assert np.allclose(BinvC[:ni, :ni], np.eye(ni), atol=1e-9)
    assert np.abs(BinvC[ni:, :ni]).max() < 1e-9
    # remaining eigenvalues match those of Shat^{-1} S (as multisets)
    rest = np.sort_complex(np.linalg.eigvals(BinvC[ni:, ni:]))
    assert np.allclose(rest, np.sort_complex(evS), atol=1e-7)


def test_lum_equals_mscn_when_coupling_vanishes():
    """S_i = G_i - F_i D^-1 E_i reduces to G_i when E_i = F_i = 0."""
    rp, ci, v, b, meta, P = _system(16, 0.1, None, 4, 24)
    C = sp.csr_matrix((v, ci, rp)).tolil()
    sep = set(P.separator().tolist())
    dn = set(P.drange_nodes.tolist())
    coo = sp.csr_matrix((v, ci, rp)).tocoo()
    for r, c in zip(coo.row, coo.col):
        if (r in sep and c in dn) or (r in dn and c in sep):
            C[r, c] = 0.0
    C = C.tocsr()
    C.sort_indices()
    p1 = Preconditioner(meta["N"], C.indptr, C.indices, C.data, P, MSCN)
    p2 = Preconditioner(meta["N"], C.indptr, C.indices, C.data, P, LUM)
    for a, bb in zip(p1.S_blocks, p2.S_blocks):
        assert np.array_equal(a, bb)


def test_mscnr_keeps_mscn_row_sums():
    """The rowsum variant (section 3.1 step 2; Algorithm 1): S_i 1 equals the
    full mini Schur complement's S_i 1, the off-diagonal entries are G_i's,
    and the lumped correction is not trivially zero on this workload."""
    rp, ci, v, b, meta, P = _system(16, 0.05, 1.05, 4, 24)
    full = Preconditioner(meta["N"], rp, ci, v, P, MSCN)
    lum = Preconditioner(meta["N"], rp, ci, v, P, LUM)
    rs = Preconditioner(meta["N"], rp, ci, v, P, MSCNR)
    moved = 0.0
    for Sf, G, Sr in zip(full.S_blocks, lum.S_blocks, rs.S_blocks):
        one = np.ones(Sf.shape[0])
        scale = np.abs(Sf).sum(axis=1) + 1e-300
        assert np.all(np.abs(Sr @ one - Sf @ one) <= 1e-12 * scale)
        off = ~np.eye(Sf.shape[0], dtype=bool)
        assert np.array_equal(Sr[off], G[off])
        moved = max(moved, float(np.abs(np.diag(Sr) - np.diag(G)).max(initial=0.0)))
    assert moved > 1e-3


def test_mscnr_equals_lum_when_coupling_vanishes():
    """With E_i = F_i = 0 the lumped correction vanishes: S_i = G_i."""
    rp, ci, v, b, meta, P = _system(16, 0.1, None, 4, 24)
    C = sp.csr_matrix((v, ci, rp)).tolil()
    sep = set(P.separator().tolist())
    dn = set(P.drange_nodes.tolist())
    coo = sp.csr_matrix((v, ci, rp)).tocoo()
    for r, c in zip(coo.row, coo.col):
        if (r in sep and c in dn) or (r in dn and c in sep):
            C[r, c] = 0.0
    C = C.tocsr()
    C.sort_indices()
    p1 = Preconditioner(meta["N"], C.indptr, C.indices, C.data, P, MSCNR)
    p2 = Preconditioner(meta["N"], C.indptr, C.indices, C.data, P, LUM)
    for a, bb in zip(p1.S_blocks, p2.S_blocks):
        assert np.array_equal(a, bb)


def _ext_sets(P, i, w):
    sep = P.perm[P.n_int:]
    a, b = P.agg_offsets[i], P.agg_offsets[i + 1]
    dr = P.drange(i) if w == 0 else np.concatenate([P.drange(i), P.drange(i + 1)])
    return sep[a:b + w], dr


def _interior_block(j=0, st=1.05, nu=0.05):
    rp, ci, v, b, meta, P = _system(16, nu, st, 4, 24)
    pre = Preconditioner(meta["N"], rp, ci, v, P, MSCN)
    Cp = pre.C[P.perm][:, P.perm].tocsr()
    a, bb = P.int_offsets[j], P.int_offsets[j + 1]
    return Cp[a:bb, a:bb]


def test_band_ilu_without_dropping_is_the_band_lu():
    A = _interior_block()
    y = np.random.default_rng(0).standard_normal(A.shape[0])
    ref = BandLU(A).solve(y)
    assert np.linalg.norm(BandILU(A, 0.0).solve(y) - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("tau", [1e-4, 1e-2])
def test_band_ilu_error_lives_on_the_dropped_positions(tau):
    """P A = L U + R: R vanishes wherever L or U keeps an entry and stays
    below tau ||A(:, k)|| where an entry was dropped (the defining property
    of a threshold incomplete factorisation)."""
    A = _interior_block()
    f = BandILU(A, tau)
    Ad = A.toarray()
    R = Ad[f.perm] - f.L @ f.U
    kept = (np.tril(f.L, -1) != 0) | (f.U != 0)
    scale = np.abs(Ad).max()
    assert np.abs(R[kept]).max() <= 1e-13 * scale
    cn = np.sqrt((Ad * Ad).sum(axis=0))
    assert np.all(np.abs(R) <= tau * cn[None, :] * (1 + 1e-12) + 1e-13 * scale)
    assert np.abs(R).max() > 0     # something was dropped


def _zero_pivot_block():
    """Interior 0 of a 16 x 16 cavity stretched 1.3 (nu = 1/100, m = 8): with
    tau = 1e-2 the dropped fill leaves column 79 without a nonzero candidate."""
    rp, ci, v, b, meta, P = _system(16, 0.01, 1.3, 8, 64)
    R, sv = row_scale(rp, ci, v)
    C = sp.csr_matrix((sv, ci, rp), shape=(meta["N"], meta["N"]))
    Cp = C[P.perm][:, P.perm]
    return Cp[:P.int_offsets[1], :P.int_offsets[1]].tocsr()


def test_band_ilu_zero_pivot_compensation():
    """Reading R24: a column whose every pivot candidate is zero after the
    drops takes tau ||A(:, j)|| as its pivot.  P A = L U + R still holds with
    R on the dropped positions (below tau ||A(:, k)||), and at a compensated
    pivot R_jj = -tau ||A(:, j)|| exactly; the exact LU refuses the block as
    singular only where it is (here it is not)."""
    A = _zero_pivot_block()
    tau = 1e-2
    f = BandILU(A, tau)
    assert f.compensated == [79]
    Ad = A.toarray()
    cn = np.sqrt((Ad * Ad).sum(axis=0))
    R = Ad[f.perm] - f.L @ f.U
    scale = np.abs(Ad).max()
    for j in f.compensated:
        assert f.U[j, j] == tau * cn[j]
        assert abs(R[j, j] + tau * cn[j]) <= 1e-13 * scale
        R[j, j] = 0.0
    kept = (np.tril(f.L, -1) != 0) | (f.U != 0)
    assert np.abs(R[kept]).max() <= 1e-13 * scale
    assert np.all(np.abs(R) <= tau * cn[None, :] * (1 + 1e-12) + 1e-13 * scale)
    # the exact factorisation of the same block exists, and a smaller tau
    # leaves no column without a candidate
    BandLU(A)
    assert BandILU(A, 1e-4).compensated == []


def test_band_ilu_drops_more_with_larger_tau():
    A = _interior_block()
    nz = [BandILU(A, tau).nnz() for tau in (0.0, 1e-4, 1e-2, 1e-1)]
    assert nz[0] > nz[1] >= nz[2] >= nz[3] and nz[0] > nz[2]


def test_overlap_widths():
    """w_i = min(w, s_i - 1, s_{i+1}) for i < k and w_k = 0 (Algorithm 1:
    w_i below the aggregate's own size; the extension stays in aggregate i+1)."""
    rp, ci, v, b, meta, P = _system(16, 0.1, None, 4, 24)
    s = np.diff(P.agg_offsets)
    assert s[-1] < s[0]      # a short remainder aggregate at the end
    for w in (1, 7, 23, 100):
        pre = Preconditioner(meta["N"], rp, ci, v, P, LUM, overlap=w)
        want = [min(w, s[i] - 1, s[i + 1]) for i in range(P.k - 1)] + [0]
        assert pre.widths.tolist() == want


def test_overlapped_block_is_local_schur_complement():
    """Each extended block is the Schur complement of its local system
    [D_e E_e; F_e G_e]: its inverse is the trailing block of the local
    inverse (block-inverse identity, independent of how S_i^e is formed)."""
    rp, ci, v, b, meta, P = _system(16, 0.05, 1.05, 4, 24)
    pre = Preconditioner(meta["N"], rp, ci, v, P, MSCN, overlap=23)
    C = pre.C
    checked = 0
    for i, Se in enumerate(pre.S_blocks):
        nodes, dr = _ext_sets(P, i, int(pre.widths[i]))
        assert Se.shape == (len(nodes), len(nodes))
        if len(dr) == 0:
            continue
        idx = np.concatenate([dr, nodes])
        loc = C[idx][:, idx].toarray()
        tail = np.linalg.inv(loc)[len(dr):, len(dr):]
        ref = np.linalg.inv(Se)
        assert np.abs(tail - ref).max() <= 1e-9 * np.abs(ref).max()
        checked += pre.widths[i] > 0
    assert checked >= 2


def test_olum_shat_is_g_on_the_column_pattern():
    """With S_i^e = G_i^e the column-wise assembly gives Shat(r, c) = G(r, c)
    for c in aggregate i and r in aggregate i or in the first w_i rows of
    aggregate i+1, and zero everywhere else (block lower bidiagonal)."""
    rp, ci, v, b, meta, P = _system(16, 0.1, None, 4, 24)
    pre = Preconditioner(meta["N"], rp, ci, v, P, LUM, overlap=23)
    D, E, F, G, Sh = pre.dense_blocks()
    mask = np.zeros_like(G, dtype=bool)
    off = P.agg_offsets
    for i in range(P.k):
        mask[off[i]:off[i + 1] + pre.widths[i], off[i]:off[i + 1]] = True
    assert np.array_equal(Sh[mask], G[mask])
    assert not Sh[~mask].any()
    assert np.abs(G[~mask & np.tril(np.ones_like(mask), -1).astype(bool)]).max() > 0  # G is cut


def test_overlap_lowers_iterations():
    """The overlap Remark of section 3.1 (and the tables of section 5): the
    overlapped method needs fewer iterations than the non-overlapped one."""
    from oracle.krylov import solve_system
    rp, ci, v, b, meta, P = _system(48, 0.005, 1.05, 6, 40, seed=1002)
    its = {}
    for w in (0, 39):
        pre = Preconditioner(meta["N"], rp, ci, v, P, MSCN, overlap=w)
        r = solve_system(pre, b, restart=50, tol=1e-8, maxit=2000, flexible=True)
        assert r.converged
        its[w] = r.iters
    assert its[39] < 0.95 * its[0], its


def test_single_subdomain_is_exact():
    rp, ci, v, b, meta = make_oseen_mac(8, 0.1, seed=3)
    P = build_partition(meta["N"], rp, ci, v, 1, 8)
    pre = Preconditioner(meta["N"], rp, ci, v, P, MSCN)
    x = np.random.default_rng(0).standard_normal(meta["N"])
    assert np.linalg.norm(pre.apply(pre.C @ x) - x) <= 1e-12 * np.linalg.norm(x)


def _read_fig1():
    d = {}
    with open(os.path.join(GOLDEN, "fig1_aggregates.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *rest = line.split()
            d[k] = rest
    return d


def test_fig1_block_extraction():
    """Section 3.2 worked example: uneven consecutive aggregates of a 16-node
    G, the 4th local matrix is C([10,11,26,27],[10,11,26,27])."""
    g = _read_fig1()
    nD, nG = int(g["n_D"][0]), int(g["n_G"][0])
    aggs = [[int(t) for t in a.split(",")] for a in g["aggregates"]]
    k4 = int(g["check_aggregate"][0]) - 1
    want = [int(t) - 1 for t in g["local_matrix_global_indices"]]
    N = nD + nG
    rng = np.random.default_rng(5)
    C = rng.standard_normal((N, N)) + 8 * N * np.eye(N)
    Cs = sp.csr_matrix(C)
    offs = np.concatenate([[0], np.cumsum([len(a) for a in aggs])])
    assert offs[-1] == nG and [a[0] for a in aggs] == [o + 1 for o in offs[:-1]]
    P = Partition(N=N, m=1, sz=0, perm=np.arange(N), part=np.r_[np.zeros(nD, int), -np.ones(nG, int)],
                  int_offsets=np.array([0, nD]), sep_size=nG, agg_offsets=offs,
                  drange_offsets=offs.copy(), drange_nodes=np.arange(nG), pair=-np.ones(nG, int))
    pre = Preconditioner(N, Cs.indptr, Cs.indices, Cs.data, P, MSCN_LITERAL, row_scaling=False)
    idx = [int(t) for t in P.drange(k4)] + [int(t) for t in P.aggregate(k4)]
    assert idx == want
    Cl = C[np.ix_(want, want)]
    Dl, El, Fl, Gl = Cl[:2, :2], Cl[:2, 2:], Cl[2:, :2], Cl[2:, 2:]
    assert np.allclose(pre.S_blocks[k4], Gl - Fl @ np.linalg.solve(Dl, El), rtol=0, atol=1e-13)


def test_singular_interior_detected_without_closure():
    """A pressure-only diagonal block (zero rows) must be reported singular."""
    A = sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 0.0]]))
    BandLU(A)  # nonsingular with pivoting
    with pytest.raises(Exception):
        BandLU(sp.csr_matrix(np.array([[0.0, 0.0], [0.0, 1.0]])))


def test_fill_factor_hand_count():
    """A tridiagonal matrix of 9 nodes (diagonal 4, neighbours -1), two
    subdomains: the bisection puts node 4 in the separator and nodes 0-3,
    5-8 in the interiors.  Each 4 x 4 tridiagonal interior factors without
    pivoting (diagonally dominant) into 3 multipliers and 4 + 3 entries of U;
    the 1 x 1 interface block is one entry; E and F hold C(3,4), C(5,4) and
    C(4,3), C(4,5).  So the preconditioner holds 10 + 10 + 1 + 2 + 2 = 25
    nonzeros, and C holds 3 * 9 - 2 = 25: fill factor 1."""
    n = 9
    rows, cols, vals = [], [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                rows.append(i)
                cols.append(j)
                vals.append(4.0 if i == j else -1.0)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    A.sort_indices()
    P = build_partition(n, A.indptr, A.indices, A.data, 2, 8)
    assert list(P.perm[P.n_int:]) == [4]
    pre = Preconditioner(n, A.indptr, A.indices, A.data, P, MSCN)
    assert pre.fill_factor() == 1.0

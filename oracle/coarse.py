"""Oracle: a coarse-grid correction of the interface solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only tests, the smoke check and the CPU-baseline leg of
the benchmark do.

Section 6 names a coarse grid correction as the way to improve the method's
convergence further, without specifying it.  The reading built here keeps the
method purely algebraic and leaves Algorithm 2 untouched except for its
interface step:

Coarse space Z (|Sigma| x nc, orthonormal columns), from the matrix graph and
the partition only:
  * H is the symmetrised pattern of C without self-loops; pressure-like nodes
    (zero or absent diagonal) are left out of the coarse space;
  * velocity classes: the connected components of H restricted to the
    non-pressure nodes (for the MAC Oseen matrices, one class per velocity
    component, as the convection-diffusion block does not couple them);
  * two separator nodes are *near* when they belong to the same class and are
    adjacent in H or share a neighbour in H (distance at most two);
  * pieces: walking the separator in order, every node not yet in a piece
    starts one, which grows breadth first through near nodes not yet in a
    piece (neighbours in ascending position) until it holds P nodes or
    cannot grow;
  * every piece K contributes the normalised constant 1_K / sqrt(|K|) and,
    when |K| >= 3, a normalised linear coordinate along it: breadth-first
    levels (in the near graph restricted to K) from the node last reached
    from K's first node (ties: smaller position), minus their mean, divided
    by their 2-norm.  A piece whose levels are all equal contributes the
    constant only.

Two-level interface solve (a deflation of the preconditioned Schur operator):
with the exact interface Schur complement S = G - F D^{-1} E (section 3.1),
  E_c = Z^T S Z,   x2 = Z y + Shat^{-1} (t - S Z y),   y = E_c^{-1} Z^T t.
S Z is formed once, column by column, from its definition (every column of
E Z is solved by the interior factors, as Algorithm 2 solves with D).  The
block factorisation of the MSCN definition then holds with Shat^{-1} replaced
by M = Q + Shat^{-1}(I - S Q), Q = Z E_c^{-1} Z^T, so Theorem 2 still gives
|D| unit eigenvalues and the rest are those of M S; M S Z = Z, so the coarse
space itself is reproduced exactly.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def near_graph(N, rowptr, colidx) -> sp.csr_matrix:
    """Distance <= 2 adjacency of H (the symmetrised pattern without loops)."""
    A = sp.csr_matrix((np.ones(len(colidx)), np.asarray(colidx), np.asarray(rowptr)), shape=(N, N))
    H = ((A + A.T) != 0).astype(np.int64).tocsr()
    H.setdiag(0)
    H.eliminate_zeros()
    H2 = ((H @ H + H) != 0).astype(np.int8).tocsr()
    H2.setdiag(0)
    H2.eliminate_zeros()
    H2.sort_indices()
    return H2


def _levels(adj, start):
    """Breadth-first levels over a small adjacency list (dict of sorted lists)."""
    lev = {start: 0}
    frontier = [start]
    while frontier:
        nxt = []
        for a in frontier:
            for b in adj[a]:
                if b not in lev:
                    lev[b] = lev[a] + 1
                    nxt.append(b)
        frontier = nxt
    return lev


def velocity_classes(N, rowptr, colidx, is_p):
    """Class of every non-pressure node (-1 for pressure-like nodes): the
    connected components of H restricted to the non-pressure nodes, numbered
    in order of their smallest node."""
    import scipy.sparse.csgraph as csg
    A = sp.csr_matrix((np.ones(len(colidx)), np.asarray(colidx), np.asarray(rowptr)), shape=(N, N))
    H = ((A + A.T) != 0).tocsr()
    v = np.nonzero(~is_p)[0]
    ncomp, lab = csg.connected_components(H[v][:, v], directed=False)
    first = np.full(ncomp, N)
    np.minimum.at(first, lab, v)
    rank = np.empty(ncomp, dtype=np.int64)
    rank[np.argsort(first, kind="stable")] = np.arange(ncomp)
    cls = np.full(N, -1, dtype=np.int64)
    cls[v] = rank[lab]
    return cls


def coarse_space(N, rowptr, colidx, part, piece=32):
    """Returns (offsets, positions, zcols): piece c holds separator positions
    positions[offsets[c]:offsets[c+1]] (in the order they joined the piece);
    zcols is a list of (piece, values) pairs in column order, values aligned
    with the piece's positions."""
    if piece < 1:
        raise ValueError("piece size must be >= 1")
    H2 = near_graph(N, rowptr, colidx)
    sep = part.perm[part.n_int:]
    cls = velocity_classes(N, rowptr, colidx, part.is_pressure)
    ns = len(sep)
    where = np.full(N, -1, dtype=np.int64)
    where[sep] = np.arange(ns)
    adj = {}
    for p in range(ns):
        g = int(sep[p])
        if cls[g] < 0:
            continue
        nb = H2.indices[H2.indptr[g]:H2.indptr[g + 1]]
        nb = nb[(where[nb] >= 0) & (cls[nb] == cls[g])]
        adj[p] = sorted(int(where[x]) for x in nb)
    owner = np.full(ns, -1, dtype=np.int64)
    offs, pos_all, zcols = [0], [], []
    for p in range(ns):
        if p not in adj or owner[p] >= 0:
            continue
        c = len(offs) - 1
        members = [p]
        owner[p] = c
        frontier = [p]
        while frontier and len(members) < piece:
            nxt = []
            for a in frontier:
                for b in adj[a]:
                    if owner[b] < 0 and len(members) < piece:
                        owner[b] = c
                        members.append(b)
                        nxt.append(b)
            frontier = nxt
        pos_all.extend(members)
        offs.append(len(pos_all))
        s = len(members)
        zcols.append((c, np.full(s, 1.0 / np.sqrt(s))))
        if s >= 3:
            inner = {q: [b for b in adj[q] if owner[b] == c] for q in members}
            lev0 = _levels(inner, members[0])
            far = max(lev0.values())
            r = min(q for q in members if lev0[q] == far)
            lev = _levels(inner, r)
            t = np.array([lev[q] for q in members], dtype=np.float64)
            t -= t.mean()
            nt = float(np.linalg.norm(t))
            if nt > 0.0:
                zcols.append((c, t / nt))
    return np.array(offs, dtype=np.int64), np.array(pos_all, dtype=np.int64), zcols


def coarse_matrix(comp_offsets, comp_pos, zcols, ns) -> sp.csc_matrix:
    """Z as a sparse |Sigma| x nc matrix."""
    rows, cols, vals = [], [], []
    for j, (c, v) in enumerate(zcols):
        p = comp_pos[comp_offsets[c]:comp_offsets[c + 1]]
        rows.append(p)
        cols.append(np.full(len(p), j))
        vals.append(v)
    if not zcols:
        return sp.csc_matrix((ns, 0))
    return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(ns, len(zcols)))


class CoarseCorrection:
    """S Z, E_c = Z^T S Z and its LU, from a Preconditioner's blocks and a
    coarse space Z (|Sigma| x nc, sparse or dense)."""

    def __init__(self, pre, Z):
        Z = sp.csc_matrix(Z)
        self.Z = Z
        nc = Z.shape[1]
        self.nc = nc
        # S Z = G Z - F D^{-1} (E Z), D^{-1} one interior block at a time
        EZ = (pre.E @ Z).tocsc()
        SZ = (pre.G @ Z).toarray()
        for (a, b, lu) in pre.blocks:
            blk = EZ[a:b].tocsc()
            cols = np.nonzero(np.diff(blk.indptr))[0]
            if len(cols) == 0:
                continue
            W = lu.solve(blk[:, cols].toarray())
            SZ[:, cols] -= pre.F[:, a:b] @ W
        self.SZ = SZ
        self.Ec = (Z.T @ SZ) if nc else np.zeros((0, 0))
        if nc:
            self.Ec_lu = sla.lu_factor(self.Ec)
            d = np.abs(np.diag(self.Ec_lu[0]))
            if d.min() <= 1e-13 * max(np.abs(self.Ec).max(), 1e-300):
                raise RuntimeError("coarse matrix is singular")

    @classmethod
    def from_pieces(cls, pre, N, rowptr, colidx, piece):
        offs, pos, zcols = coarse_space(N, rowptr, colidx, pre.part, piece)
        cc = cls(pre, coarse_matrix(offs, pos, zcols, pre.part.sep_size))
        cc.offsets, cc.positions, cc.zcols = offs, pos, zcols
        return cc

    def solve(self, t, shat_solve):
        """x2 = Z y + Shat^{-1}(t - S Z y), y = E_c^{-1} Z^T t."""
        if self.nc == 0:
            return shat_solve(t)
        y = sla.lu_solve(self.Ec_lu, self.Z.T @ t)
        return self.Z @ y + shat_solve(t - self.SZ @ y)

"""Oracle: the algebraic non-overlapping domain-decomposition preconditioner.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only tests, the smoke check and the CPU-baseline leg of
the benchmark do.

Plain FP64, no blocking or fusion beyond what the paper states:

* row scaling (section 5): every row of C (and of b) is divided by the
  largest absolute value in that row;
* blocks of P^T C P = [D E; F G] (section 3.3), D = blkDiag(A_11..A_mm)
  (Algorithm 2);
* interior factors: each A_jj by a LAPACK band LU with partial pivoting
  (the section 4 remark that D_ii is factorised exactly, [L,U] = lu(D_ii)),
  or by the threshold ILU of BandILU (section 5's inexact solver);
* mini Schur complements (section 3.1 steps 2-4; Algorithm 1):
    MSCN      S_i = G_i - F_i D_{r_i}^{-1} E_i with the D-range of the
              partition (interior velocity neighbours of the aggregate);
    MSCN_LIT  the same with Algorithm 1's literal index-range pairing;
    LUM       S_i = G_i (Definition of the LUM method);
    MSCNR     the rowsum variant (section 3.1 step 2; Algorithm 1): with
              MSCN's D-range, S_i = G_i - diag(F_i D_{r_i}^{-1} E_i 1), 1 the
              all-ones vector; the printed expression subtracts a vector
              from a matrix, read here as lumping each row's sum of the
              correction onto the diagonal;
    EXACT_BJ  S_i = S(agg_i, agg_i), the diagonal blocks of the exact
              Schur complement S = G - F D^{-1} E (a test reference and the
              learned extension's target, not one of the paper's methods);
  then Shat = blkDiag(S_i), each block LU-factorised with partial pivoting;
* overlapped aggregates (the overlap Remark of section 3.1; Algorithm 1's
  overlapped branch; OMSCN / OMSCNR / OLUM): aggregate i is extended by
  the first w_i separator positions of aggregate i+1, with
  w_i = min(w, s_i - 1, s_{i+1}) (Algorithm 1 requires w_i < s_i; the
  second bound keeps the extension inside aggregate i+1) and w_k = 0.  The
  extended block S_i^e is formed by the mode's formula on the extended node
  set, with the D-range of aggregate i followed by that of aggregate i+1.
  Assembly (section 3.1 step 4, read column-wise): the columns of S_i^e that
  belong to aggregate i's own nodes, all of their rows, are written into
  those columns of Shat, which is then block lower bidiagonal; it is
  factorised as one sparse matrix;
* apply (Algorithm 2, with E and F placed as the block factorisation of the
  MSCN definition requires):
    z1 = D^{-1} y1;  x2 = Shat^{-1} (y2 - F z1);  x1 = z1 - D^{-1} (E x2).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.linalg import lapack

MSCN, MSCN_LITERAL, LUM, EXACT_BJ, LEARNED, MSCNR = 0, 1, 2, 3, 4, 5


class SingularBlock(RuntimeError):
    pass


def row_scale(rowptr, colidx, vals):
    """R_ii = 1 / max_j |C_ij| (section 5); returns (R, scaled values)."""
    rowptr = np.asarray(rowptr)
    N = len(rowptr) - 1
    if np.any(np.diff(rowptr) == 0):
        raise ValueError("row scaling needs every row to hold an entry")
    R = 1.0 / np.maximum.reduceat(np.abs(vals), rowptr[:-1])
    rows = np.repeat(np.arange(N), np.diff(rowptr))
    return R, vals * R[rows]


class BandLU:
    """LAPACK band LU with partial pivoting of one interior block."""

    def __init__(self, A: sp.spmatrix):
        A = sp.coo_matrix(A)
        n = A.shape[0]
        self.n = n
        if n == 0:
            return
        kl = int(max(0, (A.row - A.col).max()))
        ku = int(max(0, (A.col - A.row).max()))
        ab = np.zeros((2 * kl + ku + 1, n))
        ab[kl + ku + A.row - A.col, A.col] = A.data
        lub, piv, info = lapack.dgbtrf(ab, kl, ku)
        if info > 0:
            raise SingularBlock(f"zero pivot at column {info - 1}")
        self.kl, self.ku, self.lub, self.piv = kl, ku, lub, piv
        d = np.abs(lub[kl + ku, :])
        self.pivot_ratio = float(d.min() / max(np.abs(A.data).max(), 1e-300))

    def solve(self, y):
        if self.n == 0:
            return np.zeros_like(y)
        x, info = lapack.dgbtrs(self.lub, self.kl, self.ku, y, self.piv)
        assert info == 0
        return x


class BandILU:
    """Incomplete LU with threshold tau of one interior block (the inexact
    interior solver of the experiments in section 5; Algorithm 2 allows an
    inexact solve).  Reading: right-looking elimination with partial
    pivoting inside the band, as the exact factorisation, where at step j
      * a multiplier is dropped (not stored, its row not updated) when
        |a_ij| < tau ||A(:, j)||_2, a_ij the entry before division by the
        pivot (equivalently |l_ij u_jj| < tau ||A(:, j)||_2);
      * an entry of the pivot row is dropped when |u_jk| < tau ||A(:, k)||_2;
      * the pivot itself is never dropped;
    with ||A(:, k)|| the column norms of the block before elimination.
    Partial pivoting picks the first row whose magnitude is within a
    relative PIVOT_TIE of the column's largest (the paper does not say how
    equal candidates are ordered; on the uniform grids exact and 1-ulp ties
    are common, and this rule makes the choice independent of rounding).
    Dense getrf-style storage (later swaps move earlier multipliers), so
    P A = L U + R with R supported on the dropped positions.  tau = 0 gives
    the exact band LU."""

    PIVOT_TIE = 1e-12

    def __init__(self, A: sp.spmatrix, tau: float):
        A = sp.csr_matrix(A)
        n = A.shape[0]
        self.n = n
        self.tau = float(tau)
        self.compensated = []
        if n == 0:
            return
        coo = A.tocoo()
        kl = int(max(0, (coo.row - coo.col).max()))
        ku = int(max(0, (coo.col - coo.row).max()))
        W = A.toarray()
        cn = np.sqrt((W * W).sum(axis=0))
        perm = np.arange(n)
        for j in range(n):
            hi = min(n, j + kl + 1)            # rows that can hold column j
            mag = np.abs(W[j:hi, j])
            p = j + int(np.argmax(mag >= (1.0 - self.PIVOT_TIE) * mag.max()))
            if W[p, j] == 0.0:
                # every candidate of column j is zero (the dropped fill took
                # what would have been the pivot): with dropping, the pivot
                # becomes tau ||A(:, j)||, a diagonal compensation of the
                # size of the largest entry dropped in that column (reading
                # of the incomplete factorisation); the exact LU refuses
                if tau > 0.0 and cn[j] > 0.0:
                    p = j
                    W[j, j] = tau * cn[j]
                    self.compensated.append(j)
                else:
                    raise SingularBlock(f"zero pivot at column {j}")
            if p != j:
                W[[j, p], :] = W[[p, j], :]
                perm[[j, p]] = perm[[p, j]]
            cr = min(n, j + kl + ku + 1)       # columns of U row j (fill stays in the band)
            u = W[j, j + 1:cr].copy()
            drop_u = np.abs(u) < tau * cn[j + 1:cr]
            u[drop_u] = 0.0
            W[j, j + 1:cr] = u
            a = W[j + 1:hi, j].copy()
            drop_l = np.abs(a) < tau * cn[j]
            l = a / W[j, j]
            l[drop_l] = 0.0
            W[j + 1:hi, j] = l
            W[j + 1:hi, j + 1:cr] -= np.outer(l, u)
        self.kl, self.ku = kl, ku
        self.perm = perm
        self.L = np.tril(W, -1) + np.eye(n)
        self.U = np.triu(W)

    def nnz(self):
        """Stored entries of L (below the unit diagonal) and U."""
        if self.n == 0:
            return 0
        return int(np.count_nonzero(np.tril(self.L, -1)) + np.count_nonzero(self.U))

    def solve(self, y):
        if self.n == 0:
            return np.zeros_like(y)
        z = sla.solve_triangular(self.L, np.asarray(y)[self.perm], lower=True, unit_diagonal=True)
        return sla.solve_triangular(self.U, z, lower=False)


class Preconditioner:
    """B of the MSCN definition (section 3.3) built by Algorithm 1."""

    def __init__(self, N, rowptr, colidx, vals, part, mode=MSCN, row_scaling=True,
                 learned_S=None, overlap=0, ilu_tol=0.0, coarse=0):
        if overlap < 0:
            raise ValueError("overlap must be >= 0")
        if overlap > 0 and mode not in (MSCN, MSCNR, LUM):
            raise ValueError("overlapped aggregates are defined for MSCN, MSCNR and LUM")
        self.N = N
        self.part = part
        vals = np.asarray(vals, dtype=np.float64)
        if row_scaling:
            self.R, sv = row_scale(rowptr, colidx, vals)
        else:
            self.R, sv = np.ones(N), vals
        self.C = sp.csr_matrix((sv, colidx, rowptr), shape=(N, N))
        Cp = self.C[part.perm][:, part.perm].tocsr()
        ni = part.n_int
        self.ni = ni
        self.E = Cp[:ni, ni:].tocsr()      # interiors x separator
        self.F = Cp[ni:, :ni].tocsr()      # separator x interiors
        self.G = Cp[ni:, ni:].tocsr()
        self.blocks = []
        for j in range(part.m):
            a, b = part.int_offsets[j], part.int_offsets[j + 1]
            blk = BandILU(Cp[a:b, a:b], ilu_tol) if ilu_tol > 0 else BandLU(Cp[a:b, a:b])
            self.blocks.append((a, b, blk))
        self.mode = mode
        self.overlap = overlap
        k = part.k
        s = np.diff(part.agg_offsets)
        self.widths = np.zeros(k, dtype=np.int64)
        if overlap > 0:
            for i in range(k - 1):
                self.widths[i] = min(overlap, s[i] - 1, s[i + 1])
        self.S_blocks = self._schur_blocks(mode, learned_S)
        self.S_lu = []
        self.coarse = None
        if overlap > 0:
            self._assemble_overlapped()
        else:
            self._factor_blocks()
        if coarse:
            from .coarse import CoarseCorrection
            self.coarse = CoarseCorrection.from_pieces(self, N, rowptr, colidx, int(coarse))

    def _factor_blocks(self):
        for i, S in enumerate(self.S_blocks):
            if S.shape[0] == 0:
                self.S_lu.append(None)
                continue
            lu, piv = sla.lu_factor(S, check_finite=True)
            d = np.abs(np.diag(lu))
            if d.min() <= 1e-13 * max(np.abs(S).max(), 1e-300):
                raise SingularBlock(f"interface block {i} is singular")
            self.S_lu.append((lu, piv))

    def _assemble_overlapped(self):
        """Shat from the extended blocks, column-wise (section 3.1 step 4).
        Its diagonal blocks are the leading s_i x s_i parts of the S_i^e;
        each must be nonsingular (Shat is block lower triangular)."""
        off = self.part.agg_offsets
        ns = self.part.sep_size
        rows, cols, vals = [], [], []
        for i, Se in enumerate(self.S_blocks):
            a, b = off[i], off[i + 1]
            A = Se[:b - a, :b - a]
            if A.size:
                lu, piv = sla.lu_factor(A)
                if np.abs(np.diag(lu)).min() <= 1e-13 * max(np.abs(A).max(), 1e-300):
                    raise SingularBlock(f"interface block {i} is singular")
            rr, cc = np.meshgrid(np.arange(Se.shape[0]), np.arange(b - a), indexing="ij")
            rows.append((a + rr).ravel())
            cols.append((a + cc).ravel())
            vals.append(Se[:, :b - a].ravel())
        r = np.concatenate(rows) if rows else np.zeros(0, np.int64)
        c = np.concatenate(cols) if cols else np.zeros(0, np.int64)
        v = np.concatenate(vals) if vals else np.zeros(0)
        self.Shat = sp.csc_matrix((v, (r, c)), shape=(ns, ns))
        self.Shat_lu = spla.splu(self.Shat) if ns else None

    # ---- Algorithm 1 ----
    def _schur_blocks(self, mode, learned_S):
        part = self.part
        C = self.C
        pos = np.empty(self.N, dtype=np.int64)
        pos[part.perm] = np.arange(self.N)
        sep = part.perm[part.n_int:]
        out = []
        for i in range(part.k):
            agg = part.aggregate(i)
            w = int(self.widths[i])
            if w > 0:
                agg = sep[part.agg_offsets[i]:part.agg_offsets[i + 1] + w]
            Gi = C[agg][:, agg].toarray()
            if mode == LUM:
                out.append(Gi)
            elif mode in (MSCN, MSCN_LITERAL):
                if mode == MSCN_LITERAL:
                    # Algorithm 1's pairing: the same local positions of D
                    if part.n_int < part.sep_size:
                        raise ValueError("literal D-range pairing needs |D| >= |Sigma|")
                    dr = part.perm[part.agg_offsets[i]:part.agg_offsets[i + 1]]
                else:
                    dr = part.drange(i)
                    if w > 0:
                        dr = np.concatenate([dr, part.drange(i + 1)])
                if len(dr) == 0:
                    out.append(Gi)
                    continue
                Di = C[dr][:, dr].toarray()
                Ei = C[dr][:, agg].toarray()
                Fi = C[agg][:, dr].toarray()
                lu, piv = sla.lu_factor(Di)
                if np.abs(np.diag(lu)).min() <= 1e-13 * np.abs(Di).max():
                    raise SingularBlock(f"D-range block {i} is singular")
                out.append(Gi - Fi @ sla.lu_solve((lu, piv), Ei))
            elif mode == MSCNR:
                dr = part.drange(i)
                if w > 0:
                    dr = np.concatenate([dr, part.drange(i + 1)])
                if len(dr) == 0:
                    out.append(Gi)
                    continue
                Di = C[dr][:, dr].toarray()
                Ei = C[dr][:, agg].toarray()
                Fi = C[agg][:, dr].toarray()
                lu, piv = sla.lu_factor(Di)
                if np.abs(np.diag(lu)).min() <= 1e-13 * np.abs(Di).max():
                    raise SingularBlock(f"D-range block {i} is singular")
                e = Ei @ np.ones(len(agg))                  # E_i 1
                c = Fi @ sla.lu_solve((lu, piv), e)         # F_i D_{r_i}^{-1} E_i 1
                out.append(Gi - np.diag(c))
            elif mode == EXACT_BJ:
                cols = pos[agg] - self.ni
                S = Gi.copy()
                for (a, b, lu) in self.blocks:
                    Ej = self.E[a:b][:, cols].toarray()
                    if not Ej.any():
                        continue
                    Fj = self.F[cols][:, a:b].toarray()
                    S -= Fj @ lu.solve(Ej)
                out.append(S)
            elif mode == LEARNED:
                out.append(np.asarray(learned_S[i], dtype=np.float64))
            else:
                raise ValueError(mode)
        return out

    # ---- Algorithm 2 ----
    def interior_solve(self, y1):
        z = np.empty_like(y1)
        for (a, b, lu) in self.blocks:
            z[a:b] = lu.solve(y1[a:b])
        return z

    def schur_solve(self, t):
        if self.coarse is not None:
            return self.coarse.solve(t, self.shat_solve)
        return self.shat_solve(t)

    def shat_solve(self, t):
        if self.overlap > 0:
            return self.Shat_lu.solve(t) if len(t) else np.zeros_like(t)
        x = np.empty_like(t)
        off = self.part.agg_offsets
        for i, f in enumerate(self.S_lu):
            a, b = off[i], off[i + 1]
            if f is not None:
                x[a:b] = sla.lu_solve(f, t[a:b])
        return x

    def apply_permuted(self, yp):
        """x = B^{-1} y for vectors in the permuted order P^T."""
        ni = self.ni
        y1, y2 = yp[:ni], yp[ni:]
        z1 = self.interior_solve(y1)
        x2 = self.schur_solve(y2 - self.F @ z1)
        x1 = z1 - self.interior_solve(self.E @ x2)
        return np.concatenate([x1, x2])

    def apply(self, y):
        """x = B^{-1} y in the original numbering (y, x of the scaled system)."""
        perm = self.part.perm
        x = np.empty_like(y)
        x[perm] = self.apply_permuted(y[perm])
        return x

    # ---- dense forms for small checks ----
    def dense_blocks(self):
        Cp = self.C[self.part.perm][:, self.part.perm].toarray()
        ni = self.ni
        D, E, F, G = Cp[:ni, :ni], Cp[:ni, ni:], Cp[ni:, :ni], Cp[ni:, ni:]
        if self.overlap > 0:
            Shat = self.Shat.toarray()
        else:
            Shat = sla.block_diag(*self.S_blocks) if self.S_blocks else np.zeros((0, 0))
        return D, E, F, G, Shat

    def fill_factor(self):
        """Fill factor of section 5: the nonzeros of the preconditioner over
        nnz(C).  Counted: the nonzero entries of every interior factor (the
        multipliers of L and all of U, as LAPACK's band storage holds them),
        the stored entries of Shat (dense s_i x s_i blocks, with overlapped
        aggregates also their lower blocks) and the entries of E and F that
        Algorithm 2 applies."""
        nz = 0
        for (a, b, lu) in self.blocks:
            if lu.n:
                nz += np.count_nonzero(lu.lub) if isinstance(lu, BandLU) else lu.nnz()
        if self.overlap > 0:
            nz += self.Shat.nnz
        else:
            nz += sum(S.size for S in self.S_blocks)
        nz += self.E.nnz + self.F.nnz
        return nz / self.C.nnz

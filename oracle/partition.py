"""Oracle: substructuring of C into interiors and an interface (separator).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only tests, the smoke check and the CPU-baseline leg of
the benchmark do.

The paper obtains P^T C P = [D E; F G] from a graph partitioner (section 1,
substructuring paragraph; section 3.3, matrix view): removing the separator
disconnects the graph so that the (1,1) block D is block-diagonal, one block
A_jj per subdomain (Algorithm 2 notation).  It names METIS without fixing an
algorithm, so this module states one deterministic partitioner precisely:

 (i)   pressure-like set Pi = rows whose diagonal is absent or exactly 0.0;
 (ii)  H = symmetrised pattern of C without self-loops;
 (iii) recursive level-set bisection RB(V, mV): components of H[V] in order
       of their smallest index, each rooted at a pseudo-peripheral node
       (start at the component's smallest index, BFS, move to the last-level
       node of least degree in H[V] (ties: smaller index) while the
       eccentricity grows), their BFS level sets concatenated; with
       mA = ceil(mV/2), the separator level t is the first with
       cum(levels <= t) * mV >= |V| * mA.  A velocity-only separator is
       enforced by moving every pressure node q of level t (ascending) to the
       A side and pulling its B-side neighbours into the separator.  Parts
       are numbered depth first, A before B;
 (iv)  closure: for every subdomain and every pressure component K of its
       interior (pressure nodes joined through shared interior velocity
       nodes, ordered by smallest index) whose constant vector is in the null
       space of the interior block (sum over q in K of C(v, q) == 0.0 for all
       adjacent interior velocity rows v), one pair (q in K, separator
       velocity neighbour f) is chosen: ranked by |C(q,f)| / max|C(q,:)|,
       then |C(f,q)| / max|C(f,:)| (larger first), then smaller q, then
       smaller f, the best pair whose f is still unclaimed; q moves to the
       separator, paired with f.  If every f is claimed the best pair is used
       and a shared-pair warning is returned.  (A weakly coupled pair would
       leave the interface block nearly singular on stretched grids);
 (v)   orderings: each interior by reverse Cuthill-McKee on H[int_j] per
       component (components by smallest index; CM children by (degree in
       H[int_j], index); each component's CM list reversed); the separator by
       ascending index of its non-closure nodes, each followed by the closure
       nodes paired with it (ascending);
 (vi)  aggregates of consecutive separator positions (section 3.1 step 1,
       consecutive-numbering aggregation; Algorithm 1 breakpoints r_i):
       r_1 = 0, r_{i+1} = min(r_i + sz, |Sigma|), moved forward while it
       would separate a closure node from the node it is paired with;
 (vii) D-ranges: walking the separator in order, each aggregate collects the
       not-yet-collected interior velocity neighbours (ascending) of its
       nodes (section 3.1 step 2b allows a D-range "slightly larger" than
       the aggregate; the worked example of section 3.2 takes the D-nodes
       that have direct edges to the aggregate).

Everything is integer work except the exact-zero test in (iv).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

WARN_SHARED_PAIR = 1


@dataclass
class Partition:
    N: int
    m: int
    sz: int
    perm: np.ndarray            # new position -> original index
    part: np.ndarray            # original index -> subdomain id, -1 = separator
    int_offsets: np.ndarray     # m+1 offsets into perm for the interiors
    sep_size: int
    agg_offsets: np.ndarray     # k+1 offsets into the separator order
    drange_offsets: np.ndarray  # k+1
    drange_nodes: np.ndarray    # original indices
    pair: np.ndarray            # per separator position: original index of f or -1
    status: int = 0
    is_pressure: np.ndarray = field(default=None, repr=False)

    @property
    def k(self) -> int:
        return len(self.agg_offsets) - 1

    @property
    def n_int(self) -> int:
        return int(self.int_offsets[-1])

    def interior(self, j: int) -> np.ndarray:
        return self.perm[self.int_offsets[j]:self.int_offsets[j + 1]]

    def separator(self) -> np.ndarray:
        return self.perm[self.n_int:]

    def aggregate(self, i: int) -> np.ndarray:
        s = self.separator()
        return s[self.agg_offsets[i]:self.agg_offsets[i + 1]]

    def drange(self, i: int) -> np.ndarray:
        return self.drange_nodes[self.drange_offsets[i]:self.drange_offsets[i + 1]]


# --------------------------------------------------------------------------
# graph helpers
# --------------------------------------------------------------------------

def pressure_like(N, rowptr, colidx, vals) -> np.ndarray:
    """Rows whose diagonal entry is absent or exactly zero."""
    rows = np.repeat(np.arange(N), np.diff(rowptr))
    d = np.zeros(N)
    has = np.zeros(N, dtype=bool)
    on = rows == colidx
    d[rows[on]] = vals[on]
    has[rows[on]] = True
    return (~has) | (d == 0.0)


def sym_pattern(N, rowptr, colidx) -> sp.csr_matrix:
    A = sp.csr_matrix((np.ones(len(colidx)), colidx, rowptr), shape=(N, N))
    H = ((A + A.T) != 0).astype(np.int8).tocsr()
    H.setdiag(0)
    H.eliminate_zeros()
    H.sort_indices()
    return H


def _bfs_levels(indptr, indices, root):
    """BFS distance of every node from root (-1 when unreachable)."""
    n = len(indptr) - 1
    level = np.full(n, -1, dtype=np.int64)
    level[root] = 0
    frontier = np.array([root], dtype=np.int64)
    d = 0
    while frontier.size:
        starts = indptr[frontier]
        lens = indptr[frontier + 1] - starts
        tot = int(lens.sum())
        if tot == 0:
            break
        base = np.repeat(starts - np.concatenate(([0], np.cumsum(lens)[:-1])), lens)
        nb = indices[base + np.arange(tot)]
        nb = np.unique(nb[level[nb] == -1])
        d += 1
        level[nb] = d
        frontier = nb
    return level


def _pseudo_peripheral(indptr, indices, deg, start):
    """Root of a component: move to the least-degree (then smallest index)
    last-level node while the eccentricity grows."""
    r = start
    lev = _bfs_levels(indptr, indices, r)
    ecc = int(lev.max())
    while True:
        last = np.nonzero(lev == ecc)[0]
        order = np.lexsort((last, deg[last]))
        c = int(last[order[0]])
        lev_c = _bfs_levels(indptr, indices, c)
        ecc_c = int(lev_c.max())
        if ecc_c > ecc:
            r, lev, ecc = c, lev_c, ecc_c
        else:
            return r, lev


def _components_by_min(Hs: sp.csr_matrix):
    ncomp, lab = csg.connected_components(Hs, directed=False)
    first = np.full(ncomp, np.iinfo(np.int64).max)
    np.minimum.at(first, lab, np.arange(len(lab)))
    return lab, np.argsort(first, kind="stable"), first


# --------------------------------------------------------------------------
# (iii) recursive bisection
# --------------------------------------------------------------------------

def _bisect(H, is_p, V, mV):
    mA = (mV + 1) // 2
    Hs = H[V][:, V].tocsr()
    Hs.sort_indices()
    indptr, indices = Hs.indptr.astype(np.int64), Hs.indices.astype(np.int64)
    deg = np.diff(indptr)
    lab, comp_order, first = _components_by_min(Hs)
    level_sets = []
    for c in comp_order:
        root, lev = _pseudo_peripheral(indptr, indices, deg, int(first[c]))
        for d in range(int(lev.max()) + 1):
            level_sets.append(np.nonzero(lev == d)[0])
    sizes = np.array([len(s) for s in level_sets], dtype=np.int64)
    cum = np.cumsum(sizes)
    t = int(np.nonzero(cum * mV >= len(V) * mA)[0][0])
    side = np.empty(len(V), dtype=np.int8)   # 0 = A, 1 = S, 2 = B
    for d, s in enumerate(level_sets):
        side[s] = 0 if d < t else (1 if d == t else 2)
    # velocity-only separator
    s_press = np.sort(level_sets[t][is_p[V[level_sets[t]]]])
    for q in s_press:
        side[q] = 0
        nb = indices[indptr[q]:indptr[q + 1]]
        nb = nb[side[nb] == 2]
        side[nb] = 1
    return V[side == 0], V[side == 1], V[side == 2], mA, mV - mA


def _recursive_bisection(H, is_p, N, m):
    part = np.full(N, -1, dtype=np.int64)
    parts = []

    def rb(V, mV):
        if mV == 1:
            part[V] = len(parts)
            parts.append(V)
            return
        if len(V) == 0:
            for _ in range(mV):
                parts.append(V)
            return
        A, S, B, mA, mB = _bisect(H, is_p, V, mV)
        rb(A, mA)
        rb(B, mB)

    rb(np.arange(N, dtype=np.int64), m)
    return part


# --------------------------------------------------------------------------
# (iv) closure of interior pressure components
# --------------------------------------------------------------------------

def _coef(rowptr, colidx, vals, r, c):
    """|C(r, c)| (0.0 when the entry is absent)."""
    for e in range(rowptr[r], rowptr[r + 1]):
        if colidx[e] == c:
            return abs(float(vals[e]))
    return 0.0


def _closure(N, rowptr, colidx, vals, H, is_p, part, m):
    status = 0
    rowmax = np.zeros(N)
    nonempty = np.diff(rowptr) > 0
    if nonempty.any():
        rowmax[nonempty] = np.maximum.reduceat(np.abs(vals), rowptr[:-1][nonempty])
    rel = lambda r, c: _coef(rowptr, colidx, vals, r, c) / rowmax[r] if rowmax[r] > 0 else 0.0
    in_sep = part < 0
    pair_of = {}          # moved q -> f
    claimed = np.zeros(N, dtype=bool)
    Hi, Hp = H.indices, H.indptr
    for j in range(m):
        nodes = np.nonzero(part == j)[0]
        pn = nodes[is_p[nodes]]
        if pn.size == 0:
            continue
        # bipartite pressure/velocity graph inside the interior
        sub = H[nodes][:, nodes].tocoo()
        keep = is_p[nodes[sub.row]] != is_p[nodes[sub.col]]
        Bg = sp.csr_matrix((np.ones(int(keep.sum())), (sub.row[keep], sub.col[keep])),
                           shape=(len(nodes), len(nodes)))
        ncomp, lab = csg.connected_components(Bg, directed=False)
        comps = {}
        for q_local, q in zip(np.nonzero(is_p[nodes])[0], pn):
            comps.setdefault(lab[q_local], []).append(int(q))
        for K in sorted(comps.values(), key=lambda K: min(K)):
            K = sorted(K)
            Kset = set(K)
            vels = np.nonzero((lab == lab[np.searchsorted(nodes, K[0])]) & ~is_p[nodes])[0]
            closed = True
            for vloc in vels:
                v = nodes[vloc]
                s = 0.0
                for e in range(rowptr[v], rowptr[v + 1]):
                    if int(colidx[e]) in Kset:
                        s += vals[e]
                if s != 0.0:
                    closed = False
                    break
            if not closed:
                continue
            cand = []
            for q in K:
                nb = Hi[Hp[q]:Hp[q + 1]]
                for f in nb[in_sep[nb] & ~is_p[nb]]:
                    f = int(f)
                    s1 = rel(q, f)
                    s2 = rel(f, q)
                    cand.append((-s1, -s2, q, f))
            if not cand:
                continue
            cand.sort()
            pick = next(((q, f) for _, _, q, f in cand if not claimed[f]), None)
            if pick is None:
                pick = (cand[0][2], cand[0][3])
                status = WARN_SHARED_PAIR
            q, f = pick
            part[q] = -1
            in_sep[q] = True
            claimed[f] = True
            pair_of[q] = f
    return pair_of, status


# --------------------------------------------------------------------------
# (v) orderings
# --------------------------------------------------------------------------

def _rcm(H, nodes):
    if len(nodes) == 0:
        return nodes
    Hs = H[nodes][:, nodes].tocsr()
    Hs.sort_indices()
    indptr, indices = Hs.indptr.astype(np.int64), Hs.indices.astype(np.int64)
    deg = np.diff(indptr)
    lab, comp_order, first = _components_by_min(Hs)
    visited = np.zeros(len(nodes), dtype=bool)
    out = []
    for c in comp_order:
        root, _ = _pseudo_peripheral(indptr, indices, deg, int(first[c]))
        cm = [root]
        visited[root] = True
        head = 0
        while head < len(cm):
            u = cm[head]
            head += 1
            nb = indices[indptr[u]:indptr[u + 1]]
            nb = nb[~visited[nb]]
            if nb.size:
                nb = nb[np.lexsort((nb, deg[nb]))]
                visited[nb] = True
                cm.extend(int(x) for x in nb)
        out.extend(cm[::-1])
    return nodes[np.array(out, dtype=np.int64)]


# --------------------------------------------------------------------------
# driver
# --------------------------------------------------------------------------

def build_partition(N, rowptr, colidx, vals, m, sz) -> Partition:
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    if m < 1 or sz < 1:
        raise ValueError("need m >= 1 and sz >= 1")
    is_p = pressure_like(N, rowptr, colidx, vals)
    H = sym_pattern(N, rowptr, colidx)
    part = _recursive_bisection(H, is_p, N, m)
    pair_of, status = _closure(N, rowptr, colidx, vals, H, is_p, part, m)

    perm, offs = [], [0]
    for j in range(m):
        o = _rcm(H, np.nonzero(part == j)[0])
        perm.append(o)
        offs.append(offs[-1] + len(o))
    sep = np.nonzero(part < 0)[0]
    reps = {}
    for q, f in pair_of.items():
        reps.setdefault(f, []).append(q)
    base = [int(s) for s in sep if int(s) not in pair_of]
    sep_order, pair = [], []
    for s in base:
        sep_order.append(s)
        pair.append(-1)
        for q in sorted(reps.get(s, [])):
            sep_order.append(q)
            pair.append(s)
    # closure nodes whose f is not itself a separator node cannot occur:
    # f is always chosen among separator velocity nodes.
    assert len(sep_order) == len(sep)
    perm.append(np.array(sep_order, dtype=np.int64))
    perm = np.concatenate(perm) if perm else np.zeros(0, np.int64)
    nsep = len(sep_order)
    pair = np.array(pair, dtype=np.int64)

    # (vi) aggregates
    agg = [0]
    r = 0
    while r < nsep:
        e = min(r + sz, nsep)
        while e < nsep and pair[e] >= 0:
            e += 1
        agg.append(e)
        r = e
    agg = np.array(agg, dtype=np.int64)

    # (vii) D-ranges
    n_int = offs[-1]
    assigned = np.zeros(N, dtype=bool)
    interior_vel = (part >= 0) & ~is_p
    Hi, Hp = H.indices, H.indptr
    dn, do = [], [0]
    sep_nodes = perm[n_int:]
    for i in range(len(agg) - 1):
        for g in sep_nodes[agg[i]:agg[i + 1]]:
            nb = Hi[Hp[g]:Hp[g + 1]]
            nb = nb[interior_vel[nb] & ~assigned[nb]]
            assigned[nb] = True
            dn.extend(int(x) for x in nb)
        do.append(len(dn))
    return Partition(N=N, m=m, sz=sz, perm=perm.astype(np.int64), part=part,
                     int_offsets=np.array(offs, dtype=np.int64), sep_size=nsep,
                     agg_offsets=agg, drange_offsets=np.array(do, dtype=np.int64),
                     drange_nodes=np.array(dn, dtype=np.int64), pair=pair,
                     status=status, is_pressure=is_p)

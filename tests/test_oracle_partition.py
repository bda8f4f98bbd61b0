"""Pins of the oracle partition: invariants that the substructuring of the
paper (section 1; section 3.3; Algorithm 2's D = blkDiag(A_jj)) requires."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.partition import build_partition, pressure_like
from workloads.mac_oseen import Wind, make_oseen_mac

CASES = [(6, 0.1, None, 2), (16, 0.1, None, 4), (24, 0.01, 1.05, 5), (32, 0.002, 1.05, 8),
         (20, 0.05, None, 1), (12, 0.02, None, 7)]


def _check_invariants(N, rp, ci, v, P):
    C = sp.csr_matrix((v, ci, rp), shape=(N, N))
    is_p = pressure_like(N, rp, ci, v)
    # permutation
    assert np.array_equal(np.sort(P.perm), np.arange(N))
    # part agrees with the interior ranges
    for j in range(P.m):
        assert np.all(P.part[P.interior(j)] == j)
    assert np.all(P.part[P.separator()] == -1)
    # no coupling between different interiors
    coo = C.tocoo()
    pr, pc = P.part[coo.row], P.part[coo.col]
    bad = (pr >= 0) & (pc >= 0) & (pr != pc)
    assert not bad.any()
    # separator pressure nodes are exactly the closure nodes, each right after its pair
    sep = P.separator()
    assert np.array_equal(is_p[sep], P.pair >= 0)
    for s in range(P.sep_size):
        if P.pair[s] >= 0:
            prev = sep[s - 1]
            assert prev == P.pair[s] or P.pair[s - 1] == P.pair[s]
    # aggregates cover the separator and never split a closure node from its pair
    assert P.agg_offsets[0] == 0 and P.agg_offsets[-1] == P.sep_size
    assert np.all(np.diff(P.agg_offsets) > 0) or P.sep_size == 0
    for a in P.agg_offsets[1:-1]:
        assert P.pair[a] < 0
    # D-ranges: disjoint interior velocity nodes adjacent to their aggregate
    dn = P.drange_nodes
    assert len(np.unique(dn)) == len(dn)
    assert np.all(P.part[dn] >= 0) and not is_p[dn].any()
    H = (abs(C) + abs(C).T).tocsr()
    for i in range(P.k):
        agg = P.aggregate(i)
        nbrs = set(H[agg].indices.tolist())
        assert set(P.drange(i).tolist()) <= nbrs
    # every interior block nonsingular (dense rank)
    Cp = C[P.perm][:, P.perm].toarray()
    for j in range(P.m):
        a, b = P.int_offsets[j], P.int_offsets[j + 1]
        if b > a:
            s = np.linalg.svd(Cp[a:b, a:b], compute_uv=False)
            assert s.min() > 1e-10 * s.max()


@pytest.mark.parametrize("n,nu,st,m", CASES)
def test_partition_invariants(n, nu, st, m):
    rp, ci, v, b, meta = make_oseen_mac(n, nu, stretch=st, seed=7)
    P = build_partition(meta["N"], rp, ci, v, m, 16)
    assert P.status == 0
    _check_invariants(meta["N"], rp, ci, v, P)


def test_partition_random_wind_and_sizes():
    rng = np.random.default_rng(11)
    for _ in range(6):
        n = int(rng.integers(4, 14))
        w = Wind.random_modes(rng)
        rp, ci, v, b, meta = make_oseen_mac(n, float(rng.uniform(0.01, 0.2)), wind=w, seed=1)
        m = int(rng.integers(1, 6))
        P = build_partition(meta["N"], rp, ci, v, m, int(rng.integers(3, 30)))
        _check_invariants(meta["N"], rp, ci, v, P)


def test_pressure_rows_detected():
    rp, ci, v, b, meta = make_oseen_mac(8, 0.1, seed=1)
    is_p = pressure_like(meta["N"], rp, ci, v)
    nv = meta["n_u"] + meta["n_v"]
    assert not is_p[:nv].any() and is_p[nv:].all()


def test_single_subdomain_has_no_separator():
    rp, ci, v, b, meta = make_oseen_mac(8, 0.1, seed=1)
    P = build_partition(meta["N"], rp, ci, v, 1, 8)
    assert P.sep_size == 0 and P.k == 0
    assert np.array_equal(np.sort(P.interior(0)), np.arange(meta["N"]))


def test_deterministic():
    rp, ci, v, b, meta = make_oseen_mac(20, 0.01, stretch=1.05, seed=1)
    P1 = build_partition(meta["N"], rp, ci, v, 6, 20)
    P2 = build_partition(meta["N"], rp, ci, v, 6, 20)
    for a in ("perm", "part", "int_offsets", "agg_offsets", "drange_offsets", "drange_nodes", "pair"):
        assert np.array_equal(getattr(P1, a), getattr(P2, a))

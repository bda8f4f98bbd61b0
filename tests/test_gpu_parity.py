"""GPU parity of libaddns against the FP64 oracle (same seeded inputs).

Tolerances (FP64 paths): every quantity below is a short chain of FP64 dense
kernels applied to row-scaled data (|entries| <= 1).  The GPU replaces the
band triangular recurrences by GEMVs with explicitly inverted diagonal
blocks of the same LU factors, so its rounding error is a small multiple of
eps * cond(A_jj) * nb; for the interior blocks here cond(A_jj) < 1e5, giving
the 1e-9 relative bound on interior solves and applies.  Mini Schur blocks
S_i are O(d) flops of FP64 Gaussian elimination: 1e-11 relative to max|S_i|.
GMRES iterates at equal iteration counts: 1e-10 relative in the 2-norm (the
stated target), and element by element 1e-8 of each interior block's and the
separator's largest entry (an iterate combines applies with cancelling
coefficients, so a block of small entries carries a larger share of their
error).  Interior solves and applies are compared element by element, per
interior block and separator, against the 1e-9 bound.
Mixed storage: FP32 factors carry a relative storage error of 2^-24 ~ 6e-8
per entry, amplified by the same cond factor: 1e-4 on an apply; FP16 interface
inverses (11-bit mantissa, per-block scale) perturb the interface part by
~5e-4 relative: 5e-2 on an apply.  Mixed forms are judged by the FP64 GMRES
true residual reaching tol.
"""
import json
import os

import numpy as np
import pytest

from tests.gpu_systems import blocks_of, blockwise_err, gpu_precond, make_system, oracle_precond, relerr

torch = pytest.importorskip("torch")
from paper_1104_3349_amd import addns  # noqa: E402
from oracle.krylov import gmres  # noqa: E402

pytestmark = pytest.mark.gpu

MEASURED = {}


@pytest.fixture(scope="module", autouse=True)
def _dump_measurements():
    yield
    out = os.environ.get("ADDNS_PARITY_OUT")
    if out:
        with open(out, "w") as f:
            json.dump(MEASURED, f, indent=1, sort_keys=True)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = {
    "cavity16": dict(n=16, nu=0.1, m=4, sz=64, stretch=None, seed=1001),
    "mid": dict(n=48, nu=0.005, m=6, sz=40, stretch=1.05, seed=7),
    "cavity128": dict(n=128, nu=0.01, m=16, sz=64, stretch=None, seed=1002),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    S = make_system(**CASES[request.param])
    return request.param, S


@pytest.mark.parametrize("schur", [addns.SCHUR_MSCN, addns.SCHUR_LUM, addns.SCHUR_MSCNR])
def test_schur_blocks(case, schur):
    name, S = case
    ora = oracle_precond(S, schur)
    part, pc = gpu_precond(S, schur)
    tot = sum(x.size for x in ora.S_blocks)
    got = pc.schur_blocks(tot)
    off = 0
    worst = 0.0
    for blk in ora.S_blocks:
        g = got[off:off + blk.size].reshape(blk.shape)
        off += blk.size
        worst = max(worst, float(np.abs(g - blk).max() / max(np.abs(blk).max(), 1e-300)))
    MEASURED[f"schur_{name}_{schur}"] = worst
    assert worst <= 1e-11


def test_interior_solve(case):
    name, S = case
    ora = oracle_precond(S)
    part, pc = gpu_precond(S)
    rng = np.random.default_rng(5)
    y1 = rng.standard_normal(ora.ni)
    z_ref = ora.interior_solve(y1)
    d_y, d_z = _cuda(y1), torch.zeros(ora.ni, dtype=torch.float64, device="cuda")
    addns.interior_solve(pc, d_y, d_z)
    torch.cuda.synchronize()
    e = blockwise_err(d_z.cpu().numpy(), z_ref, blocks_of(ora.part, "interior"))
    MEASURED[f"interior_{name}"] = e
    assert e <= 1e-9


@pytest.mark.parametrize("schur", [addns.SCHUR_MSCN, addns.SCHUR_LUM, addns.SCHUR_MSCNR])
def test_apply(case, schur):
    name, S = case
    ora = oracle_precond(S, schur)
    part, pc = gpu_precond(S, schur)
    rng = np.random.default_rng(6)
    y = rng.standard_normal(S.N)
    x_ref = ora.apply(y)
    d_y, d_x = _cuda(y), torch.zeros(S.N, dtype=torch.float64, device="cuda")
    addns.apply_precond(pc, d_y, d_x)
    torch.cuda.synchronize()
    x1 = d_x.cpu().numpy()
    e = blockwise_err(x1, x_ref, blocks_of(ora.part))
    MEASURED[f"apply_{name}_{schur}"] = e
    assert e <= 1e-9
    # bitwise reproducible
    d_x2 = torch.zeros_like(d_x)
    addns.apply_precond(pc, d_y, d_x2)
    torch.cuda.synchronize()
    assert np.array_equal(d_x2.cpu().numpy(), x1)


@pytest.mark.parametrize("mult", [2, 3])
def test_block_multiplier_same_operator(case, mult):
    """Larger sweep blocks regroup the same LU factors: the apply agrees with
    the oracle to the FP64 bound for every tile shape."""
    name, S = case
    ora = oracle_precond(S)
    part = addns.build_partition(S.N, S.rp, S.ci, S.v, S.m, S.sz)
    pc = addns.setup_precond(part, S.N, _cuda(S.rp), _cuda(S.ci), _cuda(S.v), block_mult=mult)
    y = np.random.default_rng(9).standard_normal(S.N)
    d_x = torch.zeros(S.N, dtype=torch.float64, device="cuda")
    addns.apply_precond(pc, _cuda(y), d_x)
    torch.cuda.synchronize()
    e = blockwise_err(d_x.cpu().numpy(), ora.apply(y), blocks_of(ora.part))
    MEASURED[f"apply_mult{mult}_{name}"] = e
    assert e <= 1e-9


@pytest.mark.parametrize("iprec,sprec,tol", [(addns.F32, addns.F32, 1e-4),
                                             (addns.F32, addns.F16_SCALED, 5e-2)])
def test_apply_mixed(case, iprec, sprec, tol):
    name, S = case
    ora = oracle_precond(S)
    part, pc = gpu_precond(S, addns.SCHUR_MSCN, iprec, sprec)
    y = np.random.default_rng(8).standard_normal(S.N)
    x_ref = ora.apply(y)
    d_y, d_x = _cuda(y), torch.zeros(S.N, dtype=torch.float64, device="cuda")
    addns.apply_precond(pc, d_y, d_x)
    torch.cuda.synchronize()
    e = relerr(d_x.cpu().numpy(), x_ref)
    MEASURED[f"apply_mixed_{name}_{iprec}_{sprec}"] = e
    assert e <= tol


@pytest.mark.parametrize("flexible,schur,ortho", [(True, addns.SCHUR_MSCN, "cgs2"), (False, addns.SCHUR_MSCN, "cgs2"),
                                                  (True, addns.SCHUR_MSCNR, "cgs2"), (True, addns.SCHUR_MSCN, "mgs"),
                                                  (False, addns.SCHUR_MSCN, "mgs")])
def test_gmres_equal_iterations(case, flexible, schur, ortho):
    """Iterates after the same number of steps agree to 1e-10 relative, for
    either orthogonalisation (against the oracle's of the same kind)."""
    name, S = case
    ora = oracle_precond(S, schur)
    part, pc = gpu_precond(S, schur)
    k = 12 if name != "cavity128" else 8
    restart = 5
    bt = ora.R * S.b
    ref = gmres(lambda x: ora.C @ x, ora.apply, bt, restart=restart, tol=1e-300, maxit=k,
                flexible=flexible, ortho=ortho)
    d_b, d_x = _cuda(S.b), torch.zeros(S.N, dtype=torch.float64, device="cuda")
    r = addns.gmres_solve(pc, d_b, d_x, restart=restart, maxit=k, tol=1e-300, flexible=flexible,
                          history=True, ortho=ortho)
    assert r["iters"] == k and not r["converged"]
    x = d_x.cpu().numpy()
    e = relerr(x, ref.x)
    eb = blockwise_err(x, ref.x, blocks_of(ora.part))
    MEASURED[f"gmres_equal_its_{name}_{flexible}_{schur}_{ortho}"] = [e, eb]
    assert e <= 1e-10 and eb <= 1e-8
    assert abs(r["true_relres"] - ref.true_relres) <= 1e-8 * max(ref.true_relres, 1e-300) + 1e-14
    np.testing.assert_allclose(r["history"], ref.est_history, rtol=1e-8, atol=0)


def test_gmres_converges_like_oracle():
    S = make_system(**CASES["cavity16"])
    ora = oracle_precond(S)
    part, pc = gpu_precond(S)
    bt = ora.R * S.b
    ref = gmres(lambda x: ora.C @ x, ora.apply, bt, restart=30, tol=1e-8, maxit=500, flexible=False)
    d_b, d_x = _cuda(S.b), torch.zeros(S.N, dtype=torch.float64, device="cuda")
    r = addns.gmres_solve(pc, d_b, d_x, restart=30, maxit=500, tol=1e-8, flexible=False)
    assert r["converged"] and r["true_relres"] <= 1e-8
    assert abs(r["iters"] - ref.iters) <= 1
    MEASURED["cavity16_its"] = [r["iters"], ref.iters]
    x = d_x.cpu().numpy()
    assert relerr(x, ref.x) <= 1e-6  # both at residual 1e-8; cond(C~) ~ 1e3


def test_gmres_deterministic():
    S = make_system(**CASES["mid"])
    part, pc = gpu_precond(S)
    d_b = _cuda(S.b)
    xs = []
    for _ in range(2):
        d_x = torch.zeros(S.N, dtype=torch.float64, device="cuda")
        addns.gmres_solve(pc, d_b, d_x, restart=20, maxit=40, tol=1e-12)
        xs.append(d_x.cpu().numpy())
    assert np.array_equal(xs[0], xs[1])


@pytest.mark.parametrize("iprec,sprec", [(addns.F32, addns.F32), (addns.F32, addns.F16_SCALED)])
def test_mixed_precision_reaches_tolerance(iprec, sprec):
    S = make_system(**CASES["mid"])
    part, pc = gpu_precond(S, addns.SCHUR_MSCN, iprec, sprec)
    d_b, d_x = _cuda(S.b), torch.zeros(S.N, dtype=torch.float64, device="cuda")
    r = addns.gmres_solve(pc, d_b, d_x, restart=50, maxit=3000, tol=1e-8, flexible=True)
    MEASURED[f"mixed_mid_{iprec}_{sprec}"] = [r["iters"], r["true_relres"]]
    assert r["converged"] and r["true_relres"] <= 1e-8


def test_single_subdomain_exact():
    """m = 1: no interface, B = C~, so GMRES converges in one step."""
    S = make_system(n=10, nu=0.05, m=1, sz=8, seed=4)
    part, pc = gpu_precond(S)
    d_b, d_x = _cuda(S.b), torch.zeros(S.N, dtype=torch.float64, device="cuda")
    r = addns.gmres_solve(pc, d_b, d_x, restart=5, maxit=5, tol=1e-10)
    assert r["iters"] == 1 and r["converged"]


def _generic_system(n=20, seed=3):
    """A non-saddle, diagonally dominant nonsymmetric 5-point matrix."""
    import scipy.sparse as sp
    from tests.gpu_systems import System
    rng = np.random.default_rng(seed)
    N = n * n
    I = np.arange(N)
    rows, cols = [I], [I]
    for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        i, j = I % n + di, I // n + dj
        ok = (i >= 0) & (i < n) & (j >= 0) & (j < n)
        rows.append(I[ok])
        cols.append((j * n + i)[ok])
    r, c = np.concatenate(rows), np.concatenate(cols)
    vals = np.where(r == c, 6.0, -1.0) + 0.3 * rng.standard_normal(r.size)
    A = sp.csr_matrix((vals, (r, c)), shape=(N, N))
    A.sort_indices()
    b = rng.standard_normal(N)
    return System(n, N, A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data, b, {}, 4, 10)


@pytest.mark.parametrize("schur", [addns.SCHUR_MSCN, addns.SCHUR_MSCN_LITERAL, addns.SCHUR_LUM,
                                   addns.SCHUR_MSCNR])
def test_generic_matrix(schur):
    """The method is purely algebraic: a matrix without saddle-point
    structure goes through the same path (literal Algorithm-1 pairing is
    well posed here because every diagonal block is dominant)."""
    S = _generic_system()
    ora = oracle_precond(S, schur)
    part, pc = gpu_precond(S, schur)
    y = np.random.default_rng(1).standard_normal(S.N)
    d_x = torch.zeros(S.N, dtype=torch.float64, device="cuda")
    addns.apply_precond(pc, _cuda(y), d_x)
    torch.cuda.synchronize()
    e = relerr(d_x.cpu().numpy(), ora.apply(y))
    MEASURED[f"generic_{schur}"] = e
    assert e <= 1e-9


def test_literal_drange_singular_on_saddle_point():
    """Algorithm 1's literal pairing can put a pressure node without its
    velocity partners into D_{r_i}; oracle and GPU both report it singular."""
    from oracle.precond import SingularBlock
    S = make_system(n=24, nu=0.05, m=4, sz=16, seed=9)
    with pytest.raises(SingularBlock):
        oracle_precond(S, addns.SCHUR_MSCN_LITERAL)
    with pytest.raises(addns.AddnsError) as e:
        gpu_precond(S, addns.SCHUR_MSCN_LITERAL)
    assert e.value.code == addns.ERR_SINGULAR


@pytest.mark.parametrize("n,m,sz", [(2, 2, 1), (3, 2, 4), (4, 3, 2), (6, 5, 7)])
def test_tiny_grids(n, m, sz):
    S = make_system(n=n, nu=0.1, m=m, sz=sz, seed=n)
    ora = oracle_precond(S)
    part, pc = gpu_precond(S)
    y = np.random.default_rng(2).standard_normal(S.N)
    d_x = torch.zeros(S.N, dtype=torch.float64, device="cuda")
    addns.apply_precond(pc, _cuda(y), d_x)
    torch.cuda.synchronize()
    assert relerr(d_x.cpu().numpy(), ora.apply(y)) <= 1e-9


def test_singular_interior_reported():
    """An isolated zero-diagonal node cannot be closed: setup must report
    ADDNS_ERR_SINGULAR and name the block."""
    S = make_system(n=6, nu=0.1, m=2, sz=8, seed=1)
    N = S.N + 1
    rp = np.concatenate([S.rp, [S.rp[-1] + 1]]).astype(np.int32)
    ci = np.concatenate([S.ci, [S.N]]).astype(np.int32)
    v = np.concatenate([S.v, [0.0]])
    part = addns.build_partition(N, rp, ci, v, 2, 8)
    with pytest.raises(addns.AddnsError) as e:
        addns.setup_precond(part, N, _cuda(rp), _cuda(ci), _cuda(v))
    assert e.value.code == addns.ERR_SINGULAR and "interior block" in str(e.value)


def test_setup_argument_errors():
    S = make_system(n=6, nu=0.1, m=2, sz=8, seed=1)
    part = addns.build_partition(S.N, S.rp, S.ci, S.v, 2, 8)
    with pytest.raises(addns.AddnsError) as e:
        addns.setup_precond(part, S.N + 1, _cuda(S.rp), _cuda(S.ci), _cuda(S.v))
    assert e.value.code == addns.ERR_ARG
    for mode in (-1, addns.SCHUR_MSCNR + 1):
        with pytest.raises(addns.AddnsError) as e:
            addns.setup_precond(part, S.N, _cuda(S.rp), _cuda(S.ci), _cuda(S.v), schur=mode)
        assert e.value.code == addns.ERR_ARG and "schur mode" in str(e.value)
    for bad in (-1, 3):
        with pytest.raises(addns.AddnsError) as e:
            addns.setup_precond(part, S.N, _cuda(S.rp), _cuda(S.ci), _cuda(S.v), block_sizing=bad)
        assert e.value.code == addns.ERR_ARG and "block_sizing" in str(e.value)
    part2, pc = gpu_precond(S)
    d = torch.zeros(S.N, dtype=torch.float64, device="cuda")
    with pytest.raises(addns.AddnsError):
        addns.apply_precond(pc, d, d)
    x = torch.zeros_like(d)
    for bad in (dict(restart=0), dict(restart=1025), dict(tol=0.0), dict(maxit=-1), dict(ortho=7)):
        kw = dict(restart=10, maxit=10, tol=1e-8)
        kw.update(bad)
        with pytest.raises(addns.AddnsError) as e:
            addns.gmres_solve(pc, d, x, raise_noconv=True, **kw)
        assert e.value.code == addns.ERR_ARG, bad


# ---------------------------------------------------------------------------
# batched systems (block-diagonal concatenation, lockstep FGMRES)
# ---------------------------------------------------------------------------
BATCH = [dict(n=12, nu=0.05, m=3, sz=16, seed=41), dict(n=20, nu=0.01, m=5, sz=24, seed=42),
         dict(n=8, nu=0.2, m=2, sz=8, seed=43), dict(n=16, nu=0.02, m=4, sz=32, stretch=1.05, seed=44)]


def _batched(**kw):
    import scipy.sparse as sp
    systems = [make_system(**c) for c in BATCH]
    parts = [addns.build_partition(S.N, S.rp, S.ci, S.v, S.m, S.sz) for S in systems]
    cat = addns.partition_concat(parts)
    big = sp.block_diag([sp.csr_matrix((S.v, S.ci, S.rp), shape=(S.N, S.N)) for S in systems]).tocsr()
    big.sort_indices()
    b = np.concatenate([S.b for S in systems])
    offs = np.concatenate([[0], np.cumsum([S.N for S in systems])])
    pc = addns.setup_precond(cat, big.shape[0], _cuda(big.indptr.astype(np.int32)),
                             _cuda(big.indices.astype(np.int32)), _cuda(big.data), **kw)
    return systems, pc, b, offs


@pytest.mark.parametrize("sizing", [1, 2])
def test_batched_apply_is_blockwise(sizing):
    """The concatenated systems (bands 11 to 27 wide) with one block size for
    every interior or each its own, element by element per system."""
    systems, pc, b, offs = _batched(block_sizing=sizing)
    y = np.random.default_rng(3).standard_normal(offs[-1])
    d_x = torch.zeros(offs[-1], dtype=torch.float64, device="cuda")
    addns.apply_precond(pc, _cuda(y), d_x)
    torch.cuda.synchronize()
    x = d_x.cpu().numpy()
    for q, S in enumerate(systems):
        ora = oracle_precond(S)
        ref = ora.apply(y[offs[q]:offs[q + 1]])
        assert blockwise_err(x[offs[q]:offs[q + 1]], ref, blocks_of(ora.part)) <= 1e-9


def test_batched_gmres_equal_iterations():
    systems, pc, b, offs = _batched()
    k, restart = 9, 4
    d_x = torch.zeros(offs[-1], dtype=torch.float64, device="cuda")
    res, code = addns.gmres_solve_batched(pc, offs, _cuda(b), d_x, restart=restart, maxit=k, tol=1e-300,
                                          history=True)
    x = d_x.cpu().numpy()
    for q, S in enumerate(systems):
        ora = oracle_precond(S)
        ref = gmres(lambda z: ora.C @ z, ora.apply, ora.R * S.b, restart=restart, tol=1e-300, maxit=k)
        assert res[q]["iters"] == k
        e = relerr(x[offs[q]:offs[q + 1]], ref.x)
        MEASURED[f"batched_equal_its_{q}"] = e
        assert e <= 1e-10
        np.testing.assert_allclose(res[q]["history"], ref.est_history, rtol=1e-8)


def test_batched_converges_per_system():
    systems, pc, b, offs = _batched()
    d_x = torch.zeros(offs[-1], dtype=torch.float64, device="cuda")
    res, code = addns.gmres_solve_batched(pc, offs, _cuda(b), d_x, restart=20, maxit=2000, tol=1e-8)
    assert code == addns.OK
    for q, S in enumerate(systems):
        part, p1 = gpu_precond(S)
        d1 = torch.zeros(S.N, dtype=torch.float64, device="cuda")
        r1 = addns.gmres_solve(p1, _cuda(S.b), d1, restart=20, maxit=2000, tol=1e-8, flexible=True)
        assert res[q]["converged"] and res[q]["true_relres"] <= 1e-8
        assert abs(res[q]["iters"] - r1["iters"]) <= 1
    MEASURED["batched_its"] = [r["iters"] for r in res]


def test_apply_captured_in_graph_replays_exactly():
    """addns_apply_precond only launches kernels, so it can be captured in a
    graph.  Every replay (with eager work and synchronisations in between)
    must equal the eager apply of the same input bit for bit."""
    S = make_system(**CASES["mid"])
    part, pc = gpu_precond(S, iprec=addns.F32, sprec=addns.F32)
    y = torch.zeros(S.N, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(y)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        addns.apply_precond(pc, y, x)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        addns.apply_precond(pc, y, x)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    for rep in range(4):
        yin = _cuda(rng.standard_normal(S.N))
        y.copy_(yin)
        g.replay()
        torch.cuda.synchronize()
        got = x.cpu().numpy().copy()
        ref = torch.zeros_like(x)
        addns.apply_precond(pc, yin, ref)
        torch.cuda.synchronize()
        assert np.array_equal(got, ref.cpu().numpy()), rep
        x.zero_()  # eager work between replays


def test_bench_workload_fp64_iterations_within_one():
    """The 128 x 128 workload, FP64 factors, FGMRES(50) with modified
    Gram-Schmidt (the Arnoldi form of the contract): the GPU's iteration
    count to 1e-8 is within one of the oracle's."""
    S = make_system(**CASES["cavity128"])
    ora = oracle_precond(S)
    ref = gmres(lambda x: ora.C @ x, ora.apply, ora.R * S.b, restart=50, tol=1e-8, maxit=3000, flexible=True,
                ortho="mgs")
    part, pc = gpu_precond(S)
    d_x = torch.zeros(S.N, dtype=torch.float64, device="cuda")
    r = addns.gmres_solve(pc, _cuda(S.b), d_x, restart=50, maxit=3000, tol=1e-8, flexible=True, ortho="mgs")
    MEASURED["cavity128_fp64_its"] = [r["iters"], ref.iters]
    assert ref.converged and r["converged"] and r["true_relres"] <= 1e-8
    assert abs(r["iters"] - ref.iters) <= 1, (r["iters"], ref.iters)


_FORM_REF = {}


def _bench_apply_reference():
    """The bench workload, a seeded vector and the oracle's apply of it
    (computed once for every forced sweep form)."""
    if not _FORM_REF:
        S = make_system(**CASES["cavity128"])
        ora = oracle_precond(S)
        y = np.random.default_rng(12).standard_normal(S.N)
        _FORM_REF.update(S=S, y=y, ref=ora.apply(y), blocks=blocks_of(ora.part))
    return _FORM_REF


@pytest.mark.parametrize("chunks", [1, 2, 6])
@pytest.mark.parametrize("zero_skip", [1, 2])
@pytest.mark.parametrize("sizing", [1, 2])
def test_every_sweep_form_matches_oracle(chunks, zero_skip, sizing):
    """Each interior-sweep form the setup can choose (chunk count, with and
    without loading only the nonzero rows, one block size for every interior
    or each its own: the bench workload's bands differ, 93 to 130), forced,
    against the oracle."""
    R = _bench_apply_reference()
    S = R["S"]
    part, pc = gpu_precond(S, sweep_chunks=chunks, sweep_zero_skip=zero_skip, block_sizing=sizing)
    assert pc.info()["sweep_chunks"] == chunks
    d_x = torch.zeros(S.N, dtype=torch.float64, device="cuda")
    addns.apply_precond(pc, _cuda(R["y"]), d_x)
    torch.cuda.synchronize()
    e = blockwise_err(d_x.cpu().numpy(), R["ref"], R["blocks"])
    MEASURED[f"sweep_form_{chunks}_{zero_skip}_{sizing}"] = e
    assert e <= 1e-9


def test_wide_band_interiors():
    """Interiors with bands of 188 to 190 (a 128 x 128 cavity in 4
    subdomains): the blocked band LU with four 64-row slots per lane, then
    the sweep; interior solve and apply element by element against the
    oracle."""
    S = make_system(n=128, nu=0.01, m=4, sz=64, seed=1)
    ora = oracle_precond(S)
    part, pc = gpu_precond(S)
    assert pc.info()["kl"] >= 185
    y = np.random.default_rng(31).standard_normal(S.N)
    d_x = torch.zeros(S.N, dtype=torch.float64, device="cuda")
    addns.apply_precond(pc, _cuda(y), d_x)
    y1 = y[:ora.ni].copy()
    d_z = torch.zeros(ora.ni, dtype=torch.float64, device="cuda")
    addns.interior_solve(pc, _cuda(y1), d_z)
    torch.cuda.synchronize()
    assert blockwise_err(d_z.cpu().numpy(), ora.interior_solve(y1), blocks_of(ora.part, "interior")) <= 1e-9
    assert blockwise_err(d_x.cpu().numpy(), ora.apply(y), blocks_of(ora.part)) <= 1e-9


def test_unblocked_band_lu_interiors():
    """A band too wide for the blocked LU's register panel (a 96 x 96 cavity
    as one subdomain, KL = 287 > 248): the unblocked elimination, then the
    block conversions and the sweep; interior solve element by element
    against the oracle."""
    S = make_system(n=96, nu=0.05, m=1, sz=64, seed=5)
    ora = oracle_precond(S)
    part, pc = gpu_precond(S)
    assert pc.info()["kl"] > 248
    y1 = np.random.default_rng(33).standard_normal(ora.ni)
    d_z = torch.zeros(ora.ni, dtype=torch.float64, device="cuda")
    addns.interior_solve(pc, _cuda(y1), d_z)
    torch.cuda.synchronize()
    assert blockwise_err(d_z.cpu().numpy(), ora.interior_solve(y1), blocks_of(ora.part, "interior")) <= 1e-9


def test_per_interior_blocks_gmres_matches_oracle():
    """Per-interior block sizes in the FP64 solve of the bench workload: the
    iteration count within one of the oracle's (MGS), the true residual met."""
    S = make_system(**CASES["cavity128"])
    ora = oracle_precond(S)
    ref = gmres(lambda x: ora.C @ x, ora.apply, ora.R * S.b, restart=50, tol=1e-8, maxit=3000, flexible=True,
                ortho="mgs")
    part, pc = gpu_precond(S, block_sizing=2)
    d_x = torch.zeros(S.N, dtype=torch.float64, device="cuda")
    r = addns.gmres_solve(pc, _cuda(S.b), d_x, restart=50, maxit=3000, tol=1e-8, flexible=True, ortho="mgs")
    assert r["converged"] and r["true_relres"] <= 1e-8
    assert abs(r["iters"] - ref.iters) <= 1, (r["iters"], ref.iters)


def test_two_default_setups_solve_bit_for_bit():
    """The setup's choices (chunk count, block size, zero-slot form) never
    depend on a timing that could change the rounding: two setups of the
    same input with default options give the same iterates bit for bit."""
    S = make_system(**CASES["cavity128"])
    xs, its = [], []
    for _ in range(2):
        part, pc = gpu_precond(S, iprec=addns.F32, sprec=addns.F32, block_mult=0, sweep_chunks=0)
        d_x = torch.zeros(S.N, dtype=torch.float64, device="cuda")
        r = addns.gmres_solve(pc, _cuda(S.b), d_x, restart=50, maxit=200, tol=1e-8, flexible=True)
        xs.append(d_x.cpu().numpy())
        its.append(r["iters"])
    assert its[0] == its[1] and np.array_equal(xs[0], xs[1])


def test_fill_factor_matches_oracle():
    """Section 5's fill factor from the library's counts equals the oracle's
    on the 16 x 16 system (exact FP64 band LU on both sides)."""
    S = make_system(**CASES["cavity16"])
    ora = oracle_precond(S)
    part, pc = gpu_precond(S)
    a, c = pc.fill()
    assert c == len(S.v)
    ff = a / c
    MEASURED["fill_cavity16"] = [ff, ora.fill_factor()]
    assert abs(ff - ora.fill_factor()) <= 1e-3 * ora.fill_factor()

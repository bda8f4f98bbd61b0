"""Full-size checks of the GPU path on the stretched workloads (256² and
512², FP32 interior factors as configured), where an element-by-element
comparison with the FP64 oracle would measure the conditioning of the
interior blocks rather than the code.  Instead, properties that hold at any
size are checked in FP64 on the host, from the oracle's partition and
blocks:

* the interface blocks S_i the GPU built (FP64 setup) equal the oracle's
  MSCN blocks (section 3.1; Algorithm 1) to 1e-11 relative;
* the interior solve z1 = D^{-1} y1 has a small normwise backward error
  |D z1 - y1| / (|D| |z1| + |y1|) (infinity norms): at most 1e-4 with FP32
  factors (storage roundoff 2^-24 = 6e-8, grown by the explicitly inverted
  diagonal blocks of the sweep, nb = 136) and 1e-12 with FP64;
* the apply satisfies the relations of Algorithm 2 (reading R2):
  x2 = Shat^{-1}(y2 - F z1) blockwise, with a per-block backward error at
  most 8 u cond(S_i) + 1e-12 (u the storage roundoff of the inverses,
  FP16 with scale: 2^-11; the inverses are explicit, so the block's
  condition number enters), and D x1 = y1 - E x2 with the interior bound;
* GMRES reports the true residual of the iterate it returns.
"""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")
from oracle.partition import build_partition as oracle_partition  # noqa: E402
from oracle.precond import MSCN, Preconditioner, row_scale  # noqa: E402
from paper_1104_3349_amd import addns  # noqa: E402
from workloads.configs import CAVITY256_STRETCHED, CAVITY512_STRETCHED  # noqa: E402

pytestmark = pytest.mark.gpu

U = {addns.F64: 2.0 ** -53, addns.F32: 2.0 ** -24, addns.F16_SCALED: 2.0 ** -11}
PREC = {0: addns.F64, 1: addns.F32, 2: addns.F16_SCALED}


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module", params=["cavity256s", "cavity512s"])
def full(request):
    cfg = {"cavity256s": CAVITY256_STRETCHED, "cavity512s": CAVITY512_STRETCHED}[request.param]
    rp, ci, v, b, meta = cfg.build()
    N = meta["N"]
    P = oracle_partition(N, rp, ci, v, cfg.m, cfg.sz)
    ora = Preconditioner(N, rp, ci, v, P, MSCN)
    part = addns.build_partition(N, rp, ci, v, cfg.m, cfg.sz)
    iprec, sprec = PREC[cfg.interior_prec], PREC[cfg.schur_prec]
    pc = addns.setup_precond(part, N, _cuda(rp), _cuda(ci), _cuda(v), interior_prec=iprec,
                             schur_prec=sprec, block_mult=1)
    torch.cuda.synchronize()
    return dict(cfg=cfg, N=N, rp=rp, ci=ci, v=v, b=b, P=P, ora=ora, pc=pc, iprec=iprec, sprec=sprec)


def _inf(A):
    return float(abs(A).sum(axis=1).max()) if sp.issparse(A) else float(np.abs(A).sum(axis=1).max())


TOL_INTERIOR = {addns.F32: 1e-4, addns.F64: 1e-12}


def test_schur_blocks_equal_oracle(full):
    ora, pc = full["ora"], full["pc"]
    tot = sum(x.size for x in ora.S_blocks)
    got = full["pc"].schur_blocks(tot)
    off, worst = 0, 0.0
    for blk in ora.S_blocks:
        g = got[off:off + blk.size].reshape(blk.shape)
        off += blk.size
        worst = max(worst, float(np.abs(g - blk).max() / max(np.abs(blk).max(), 1e-300)))
    assert worst <= 1e-11


def test_interior_solve_backward_error(full):
    ora, pc, P = full["ora"], full["pc"], full["P"]
    ni = ora.ni
    Cp = ora.C[P.perm][:, P.perm].tocsr()
    D = Cp[:ni, :ni].tocsr()
    y1 = np.random.default_rng(3).standard_normal(ni)
    d_z = torch.zeros(ni, dtype=torch.float64, device="cuda")
    addns.interior_solve(pc, _cuda(y1), d_z)
    torch.cuda.synchronize()
    z1 = d_z.cpu().numpy()
    eta = np.abs(D @ z1 - y1).max() / (_inf(D) * np.abs(z1).max() + np.abs(y1).max())
    assert eta <= TOL_INTERIOR[full["iprec"]], eta


def test_apply_satisfies_algorithm2(full):
    ora, pc, P = full["ora"], full["pc"], full["P"]
    N, ni = full["N"], ora.ni
    Cp = ora.C[P.perm][:, P.perm].tocsr()
    D, E, F = Cp[:ni, :ni].tocsr(), Cp[:ni, ni:].tocsr(), Cp[ni:, :ni].tocsr()
    y = np.random.default_rng(4).standard_normal(N)
    d_x = torch.zeros(N, dtype=torch.float64, device="cuda")
    addns.apply_precond(pc, _cuda(y), d_x)
    torch.cuda.synchronize()
    x = d_x.cpu().numpy()
    yp, xp = y[P.perm], x[P.perm]
    y1, y2, x1, x2 = yp[:ni], yp[ni:], xp[:ni], xp[ni:]
    # the forward interior solve is the same kernel on the same input
    d_z = torch.zeros(ni, dtype=torch.float64, device="cuda")
    addns.interior_solve(pc, _cuda(y1), d_z)
    torch.cuda.synchronize()
    z1 = d_z.cpu().numpy()
    t = y2 - F @ z1
    # interface, block by block with the oracle's FP64 blocks
    us = U[full["sprec"]]
    off = P.agg_offsets
    worst = 0.0
    for i, S in enumerate(ora.S_blocks):
        a, b = off[i], off[i + 1]
        ti, xi = t[a:b], x2[a:b]
        cond = _inf(S) * _inf(np.linalg.inv(S))
        eta = np.abs(S @ xi - ti).max() / (_inf(S) * np.abs(xi).max() + np.abs(ti).max() + 1e-300)
        worst = max(worst, eta / (8 * us * cond + 1e-12))
    assert worst <= 1.0, worst
    # backward sweep: D x1 = y1 - E x2, with w = z1 - x1 = D^{-1}(E x2)
    r = D @ x1 - (y1 - E @ x2)
    scale = _inf(D) * (np.abs(z1).max() + np.abs(z1 - x1).max()) + np.abs(y1).max() + _inf(E) * np.abs(x2).max()
    eta = np.abs(r).max() / scale
    assert eta <= TOL_INTERIOR[full["iprec"]], eta


def test_gmres_reports_true_residual(full):
    pc, N = full["pc"], full["N"]
    d_b = _cuda(full["b"])
    d_x = torch.zeros(N, dtype=torch.float64, device="cuda")
    r = addns.gmres_solve(pc, d_b, d_x, restart=50, maxit=60, tol=1e-8)
    x = d_x.cpu().numpy()
    R, sv = row_scale(full["rp"], full["ci"], full["v"])
    C = sp.csr_matrix((sv, full["ci"], full["rp"]), shape=(N, N))
    bs = R * full["b"]
    true = np.linalg.norm(bs - C @ x) / np.linalg.norm(bs)
    # 60 iterations stop short of 1e-8 on these stretched workloads (their
    # convergence is reported by the benchmark, not asserted here); what is
    # checked is that the reported residual is the true one of the iterate
    assert r["iters"] == 60 or r["converged"]
    assert abs(true - r["true_relres"]) <= 1e-10 * max(true, 1e-300) + 1e-15


def test_ilu_setup_compensates_instead_of_refusing(full):
    """ILU(1e-4) interiors (the tolerance of section 5) on the stretched
    workloads.  The dropped fill leaves some columns without a nonzero pivot
    candidate; with the compensated pivot of reading R24 the setups no longer
    refuse with a zero pivot.  On the 256 x 256 workload the factors and the
    interior solve are finite in FP64 and FP32, with fewer stored entries than
    the exact factors.  On the 512 x 512 workload (cells 2e-7 high) the
    incomplete factors are numerically useless, and the library says so
    instead of returning garbage: in FP32 storage the inverted diagonal
    blocks overflow and the setup refuses (ADDNS_ERR_SINGULAR); in FP64 the
    interior solve overflows and GMRES reports a non-finite estimate."""
    cfg, N, pc0 = full["cfg"], full["N"], full["pc"]
    part = addns.build_partition(N, full["rp"], full["ci"], full["v"], cfg.m, cfg.sz)
    args = (part, N, _cuda(full["rp"]), _cuda(full["ci"]), _cuda(full["v"]))
    ni = full["ora"].ni
    y1 = _cuda(np.random.default_rng(4).standard_normal(ni))
    big = cfg is CAVITY512_STRETCHED
    for iprec in (addns.F64, addns.F32):
        if big and iprec == addns.F32:
            with pytest.raises(addns.AddnsError) as e:
                addns.setup_precond(*args, interior_prec=iprec, schur_prec=full["sprec"], block_mult=1, ilu_tol=1e-4)
            assert e.value.code == addns.ERR_SINGULAR and "not finite" in str(e.value)
            continue
        pc = addns.setup_precond(*args, interior_prec=iprec, schur_prec=full["sprec"], block_mult=1, ilu_tol=1e-4)
        assert pc.info()["interior_nnz"] < pc0.info()["interior_nnz"]
        d_z = torch.zeros(ni, dtype=torch.float64, device="cuda")
        addns.interior_solve(pc, y1, d_z)
        torch.cuda.synchronize()
        if not big:
            assert bool(torch.isfinite(d_z).all())
        else:
            assert not bool(torch.isfinite(d_z).all())
            d_x = torch.zeros(N, dtype=torch.float64, device="cuda")
            with pytest.raises(addns.AddnsError) as e:
                addns.gmres_solve(pc, _cuda(full["b"]), d_x, restart=50, maxit=20, tol=1e-8)
            assert "non-finite" in str(e.value)


def test_interior_solve_sampled_blocks_match_oracle(full):
    """Element-by-element parity at full size on sampled interiors: the GPU's
    FP64 interior solve against the oracle's LAPACK band solve of the same
    interiors (the first, the last and six seeded others).  Per interior the
    largest entry error, relative to the largest entry, stays below
    kappa_1(A_jj) u (u = 2^-53; kappa_1 estimated from the oracle's LU by
    onenormest), the forward error bound of a backward-stable solve; the
    measured errors are 1e-16 to 1e-10 at kappa_1 up to 8e11, at most 0.03 of
    the bound."""
    import scipy.sparse.linalg as spla
    cfg, N, ora, P = full["cfg"], full["N"], full["ora"], full["P"]
    part = addns.build_partition(N, full["rp"], full["ci"], full["v"], cfg.m, cfg.sz)
    pc = addns.setup_precond(part, N, _cuda(full["rp"]), _cuda(full["ci"]), _cuda(full["v"]),
                             interior_prec=addns.F64, schur_prec=addns.F64)
    ni = ora.ni
    y1 = np.random.default_rng(9).standard_normal(ni)
    d_z = torch.zeros(ni, dtype=torch.float64, device="cuda")
    addns.interior_solve(pc, _cuda(y1), d_z)
    torch.cuda.synchronize()
    z = d_z.cpu().numpy()
    sample = sorted({0, cfg.m - 1, *np.random.default_rng(3).choice(cfg.m, 6, replace=False).tolist()})
    for j in sample:
        a, b, lu = ora.blocks[j]
        ref = lu.solve(y1[a:b])
        err = np.abs(z[a:b] - ref).max() / np.abs(ref).max()
        A = ora.C[P.perm[a:b]][:, P.perm[a:b]].tocsc()
        At = A.T.tocsc()
        inv = spla.LinearOperator(A.shape, matvec=lu.solve, rmatvec=lambda x, At=At: spla.spsolve(At, x))
        kappa = spla.norm(A, 1) * spla.onenormest(inv)
        assert err <= max(1e-12, kappa * 2.0 ** -53), (j, err, kappa)


def test_apply_matches_oracle_blockwise(full):
    """The FP64 apply at full size against the oracle's, element by element
    per interior and for the separator: Algorithm 2 with the same blocks on
    both sides.  The bound follows the interiors' conditioning (kappa_1 up to
    1e6 on the 256 x 256 workload, up to 8e11 on the 512 x 512 one, so
    kappa_1 u reaches 1e-10 and 1e-4): 1e-10 and 1e-6.  Measured: 3e-12 and
    2e-8 (the worst interior), medians about 1e-13."""
    cfg, N, ora, P = full["cfg"], full["N"], full["ora"], full["P"]
    part = addns.build_partition(N, full["rp"], full["ci"], full["v"], cfg.m, cfg.sz)
    pc = addns.setup_precond(part, N, _cuda(full["rp"]), _cuda(full["ci"]), _cuda(full["v"]),
                             interior_prec=addns.F64, schur_prec=addns.F64)
    y = np.random.default_rng(11).standard_normal(N)
    d_x = torch.zeros(N, dtype=torch.float64, device="cuda")
    addns.apply_precond(pc, _cuda(y), d_x)
    torch.cuda.synchronize()
    x, ref = d_x.cpu().numpy(), ora.apply(y)
    blocks = [P.interior(j) for j in range(cfg.m)] + [P.separator()]
    errs = [np.abs(x[i] - ref[i]).max() / np.abs(ref[i]).max() for i in blocks if len(i)]
    tol = 1e-6 if cfg is CAVITY512_STRETCHED else 1e-10
    assert max(errs) <= tol, max(errs)
    assert float(np.median(errs)) <= 1e-11

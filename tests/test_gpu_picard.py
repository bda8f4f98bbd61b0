"""GPU Picard outer loop (section 1) and the refactor entry point it uses,
against the FP64 oracle's Picard loop and against fresh setups."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle.picard import picard as oracle_picard  # noqa: E402
from paper_1104_3349_amd import addns  # noqa: E402
from paper_1104_3349_amd import picard as gpu_picard  # noqa: E402
from tests.gpu_systems import make_system, relerr  # noqa: E402
from workloads.mac_oseen import Wind  # noqa: E402

pytestmark = pytest.mark.gpu


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _apply(pc, y):
    d_x = torch.zeros(len(y), dtype=torch.float64, device="cuda")
    addns.apply_precond(pc, _cuda(y), d_x)
    torch.cuda.synchronize()
    return d_x.cpu().numpy()


@pytest.mark.parametrize("kw", [dict(), dict(interior_prec=addns.F32, schur_prec=addns.F32),
                                dict(overlap=23), dict(schur=addns.SCHUR_MSCNR)])
def test_refactor_equals_fresh_setup(kw):
    """Refactoring with another wind's values gives bit for bit the apply of
    a fresh setup on those values (same partition and sweep shape), and
    refactoring back restores the first apply exactly."""
    S1 = make_system(n=24, nu=0.02, m=4, sz=24, seed=3)
    S2 = make_system(n=24, nu=0.02, m=4, sz=24, seed=3, wind=Wind((0.3, -1.0, 0.5, 2.0), 1.5))
    assert np.array_equal(S1.rp, S2.rp) and np.array_equal(S1.ci, S2.ci)
    part = addns.build_partition(S1.N, S1.rp, S1.ci, S1.v, S1.m, S1.sz)
    d_rp, d_ci = _cuda(S1.rp), _cuda(S1.ci)
    pc = addns.setup_precond(part, S1.N, d_rp, d_ci, _cuda(S1.v), block_mult=1, **kw)
    y = np.random.default_rng(4).standard_normal(S1.N)
    x1 = _apply(pc, y)
    addns.refactor_precond(pc, d_rp, d_ci, _cuda(S2.v))
    fresh = addns.setup_precond(part, S2.N, d_rp, d_ci, _cuda(S2.v), block_mult=1, **kw)
    x2 = _apply(pc, y)
    assert np.array_equal(x2, _apply(fresh, y))
    assert not np.array_equal(x1, x2)
    addns.refactor_precond(pc, d_rp, d_ci, _cuda(S1.v))
    assert np.array_equal(_apply(pc, y), x1)


def test_refactor_keeps_a_captured_apply_valid():
    """Buffers keep their addresses: an apply captured in a graph before the
    refactor replays with the new factors."""
    S1 = make_system(n=24, nu=0.02, m=4, sz=24, seed=3)
    S2 = make_system(n=24, nu=0.02, m=4, sz=24, seed=3, wind=Wind((0.3, -1.0, 0.5, 2.0), 1.5))
    part = addns.build_partition(S1.N, S1.rp, S1.ci, S1.v, S1.m, S1.sz)
    d_rp, d_ci = _cuda(S1.rp), _cuda(S1.ci)
    pc = addns.setup_precond(part, S1.N, d_rp, d_ci, _cuda(S1.v), interior_prec=addns.F32,
                             schur_prec=addns.F32, block_mult=1)
    y = torch.from_numpy(np.random.default_rng(5).standard_normal(S1.N)).cuda()
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
    addns.refactor_precond(pc, d_rp, d_ci, _cuda(S2.v))
    want = _apply(pc, y.cpu().numpy())
    for _ in range(3):
        x.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), want)


def test_failed_refactor_leaves_no_factors_until_the_next_one():
    S = make_system(n=6, nu=0.1, m=2, sz=8, seed=1)
    N = S.N + 1
    rp = np.concatenate([S.rp, [S.rp[-1] + 1]]).astype(np.int32)
    ci = np.concatenate([S.ci, [S.N]]).astype(np.int32)
    good = np.concatenate([S.v, [1.0]])
    bad = np.concatenate([S.v, [0.0]])      # an isolated zero diagonal: singular interior
    part = addns.build_partition(N, rp, ci, good, 2, 8)
    d_rp, d_ci = _cuda(rp), _cuda(ci)
    pc = addns.setup_precond(part, N, d_rp, d_ci, _cuda(good), block_mult=1)
    y = np.random.default_rng(1).standard_normal(N)
    x_good = _apply(pc, y)
    with pytest.raises(addns.AddnsError) as e:
        addns.refactor_precond(pc, d_rp, d_ci, _cuda(bad))
    assert e.value.code == addns.ERR_SINGULAR
    with pytest.raises(addns.AddnsError) as e:
        _apply(pc, y)
    assert e.value.code == addns.ERR_ARG and "refactor" in str(e.value)
    addns.refactor_precond(pc, d_rp, d_ci, _cuda(good))
    assert np.array_equal(_apply(pc, y), x_good)
    with pytest.raises(addns.AddnsError):
        addns.refactor_precond(pc, None, d_ci, _cuda(good))


def test_picard_matches_oracle():
    """FP64 factors: the same number of outer steps, the same residual
    history, the same fixed point (16x16 lid-driven cavity, nu = 1/100)."""
    kw = dict(m=4, sz=24, tol=1e-8, maxit=30, restart=50)
    ora = oracle_picard(16, 0.01, lin_tol=1e-9, forcing=gpu_picard.ZERO_FORCING, **kw)
    gpu = gpu_picard.solve(16, 0.01, interior_prec=addns.F64, schur_prec=addns.F64, lin_tol=1e-9, **kw)
    assert ora.converged and gpu["converged"]
    assert len(gpu["residuals"]) == len(ora.residuals)
    np.testing.assert_allclose(gpu["residuals"], ora.residuals, rtol=1e-5, atol=1e-13)
    assert relerr(gpu["x"], ora.x) <= 1e-8
    assert all(abs(a - b) <= 1 for a, b in zip(gpu["lin_iters"], ora.lin_iters))


@pytest.mark.parametrize("overlap", [0, 31])
def test_picard_mixed_precision_converges(overlap):
    """FP32 factors (and overlapped aggregates) reach the same fixed point in
    the same number of outer steps, within one."""
    kw = dict(m=4, sz=32, tol=1e-8, maxit=40, restart=50)
    ora = oracle_picard(32, 0.01, lin_tol=1e-9, forcing=gpu_picard.ZERO_FORCING, **kw)
    gpu = gpu_picard.solve(32, 0.01, overlap=overlap, lin_tol=1e-9, **kw)
    assert gpu["converged"] and gpu["residuals"][-1] <= 1e-8
    assert abs(len(gpu["residuals"]) - len(ora.residuals)) <= 1
    assert relerr(gpu["x"], ora.x) <= 1e-6

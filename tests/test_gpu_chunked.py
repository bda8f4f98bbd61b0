"""Chunked interior sweep (opts.sweep_chunks): every interior's lower and
upper block recurrences cut into p chunks that are swept side by side from a
zero carry or state and then corrected with their responses to the true
one.  The factors are the same L and U as the single-workgroup sweep's, so
the interior solve D^{-1} y and the apply of Algorithm 2 must agree with it,
and with the oracle, to rounding:

* FP64 factors: the chunked form adds the corrections X_c d_c and Y_c s_c
  to zero-state results instead of carrying them through the steps, a
  reassociation of the same sums; the sweep's own error against the oracle is
  at 1e-9 (cond(D) ~ 1e3..1e5 times 1e-16 per step), and the two forms agree
  to 1e-11 relative;
* FP32 factors: the responses are stored in FP32 like the factors
  (roundoff 6e-8 per entry), so the chunked and single-workgroup results
  differ by a few 1e-7 of the result's norm times the growth of the
  corrections; 2e-5 relative is the bound used (the FP32 sweep itself is
  ~1e-4 from the FP64 oracle on these systems);
* the Krylov iteration count with FP32 factors to 1e-8 is unchanged to one
  iteration.
"""
import numpy as np
import pytest

from tests.gpu_systems import gpu_precond, make_system, oracle_precond, relerr
from workloads.mac_oseen import Wind

torch = pytest.importorskip("torch")
from paper_1104_3349_amd import addns  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = {
    "cavity16": dict(n=16, nu=0.1, m=4, sz=64, stretch=None, seed=1001),
    "mid": dict(n=48, nu=0.005, m=6, sz=40, stretch=1.05, seed=7),
    "cavity128": dict(n=128, nu=0.01, m=16, sz=64, stretch=None, seed=1002),
}


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    return request.param, make_system(**CASES[request.param])


def max_chunks(part, pc):
    """Upper blocks of the shortest non-empty interior: the largest p."""
    offs = part.export().int_offsets
    nbu = pc.info()["nb_upper"]
    sizes = np.diff(offs)
    return int(min(-(-int(n) // nbu) for n in sizes if n > 0))


def _solve(pc, y):
    d_z = torch.zeros(len(y), dtype=torch.float64, device="cuda")
    addns.interior_solve(pc, _cuda(y), d_z)
    torch.cuda.synchronize()
    return d_z.cpu().numpy()


def _apply(pc, y):
    d_x = torch.zeros(len(y), dtype=torch.float64, device="cuda")
    addns.apply_precond(pc, _cuda(y), d_x)
    torch.cuda.synchronize()
    return d_x.cpu().numpy()


def _chunk_counts(pmax):
    return sorted({2, max(2, pmax // 2), pmax} & set(range(2, pmax + 1)))


@pytest.mark.parametrize("iprec,tol", [(addns.F64, 1e-11), (addns.F32, 2e-5)])
def test_chunked_interior_solve_matches_single(case, iprec, tol):
    name, S = case
    part, pc1 = gpu_precond(S, iprec=iprec, sprec=iprec, sweep_chunks=1)
    assert pc1.info()["sweep_chunks"] == 1
    pmax = max_chunks(part, pc1)
    assert pmax >= 2, name
    n_int = part.info()["n_interior"]
    y = np.random.default_rng(5).standard_normal(n_int)
    z1 = _solve(pc1, y)
    for p in _chunk_counts(pmax):
        _, pcp = gpu_precond(S, iprec=iprec, sprec=iprec, part=part, sweep_chunks=p)
        assert pcp.info()["sweep_chunks"] == p
        assert relerr(_solve(pcp, y), z1) <= tol, (name, p)


def test_chunked_apply_matches_oracle(case):
    name, S = case
    ora = oracle_precond(S)
    part, pc1 = gpu_precond(S, sweep_chunks=1)
    pmax = max_chunks(part, pc1)
    y = np.random.default_rng(6).standard_normal(S.N)
    ref = ora.apply(y)
    for p in _chunk_counts(pmax):
        _, pcp = gpu_precond(S, part=part, sweep_chunks=p)
        # both interior solves of the apply (z1 = D^-1 y1 and x1 = z1 - D^-1 E x2)
        assert relerr(_apply(pcp, y), ref) <= 1e-9, (name, p)


def test_chunked_gmres_iterations_unchanged():
    S = make_system(**CASES["cavity128"])
    d_b = _cuda(S.b)
    its = {}
    for p in (1, 4):
        part, pc = gpu_precond(S, iprec=addns.F32, sprec=addns.F32, sweep_chunks=p)
        d_x = torch.zeros(S.N, dtype=torch.float64, device="cuda")
        r = addns.gmres_solve(pc, d_b, d_x, restart=50, maxit=3000, tol=1e-8)
        assert r["converged"] and r["true_relres"] <= 1e-8, p
        its[p] = r["iters"]
    assert abs(its[4] - its[1]) <= 1, its


def test_sweep_chunks_out_of_range():
    S = make_system(**CASES["cavity16"])
    part, pc = gpu_precond(S, sweep_chunks=1)
    pmax = max_chunks(part, pc)
    for bad in (pmax + 1, -1):
        with pytest.raises(addns.AddnsError) as e:
            gpu_precond(S, part=part, sweep_chunks=bad)
        assert e.value.code == addns.ERR_ARG, bad


def test_auto_chunks_reported_and_exact():
    """The default (0) keeps the chunked form only where it times faster;
    either way the apply matches the oracle."""
    S = make_system(**CASES["cavity128"])
    ora = oracle_precond(S)
    part, pc = gpu_precond(S)
    p = pc.info()["sweep_chunks"]
    assert 1 <= p <= max_chunks(part, pc)
    y = np.random.default_rng(8).standard_normal(S.N)
    assert relerr(_apply(pc, y), ora.apply(y)) <= 1e-9


def test_chunked_refactor_equals_fresh_setup():
    """A refactor recomputes the responses with the new factors: bit for bit
    what a fresh setup with the same chunk count gives."""
    S = make_system(**CASES["mid"])
    part, pc = gpu_precond(S, iprec=addns.F32, sprec=addns.F32, sweep_chunks=3)
    v2 = S.v * (1.0 + 0.01 * np.random.default_rng(9).standard_normal(len(S.v)))
    addns.refactor_precond(pc, _cuda(S.rp), _cuda(S.ci), _cuda(v2))
    torch.cuda.synchronize()
    S2 = make_system(**CASES["mid"])
    S2.v = v2
    _, fresh = gpu_precond(S2, iprec=addns.F32, sprec=addns.F32, part=part, sweep_chunks=3)
    y = np.random.default_rng(10).standard_normal(S.N)
    assert pc.info()["sweep_chunks"] == 3
    assert np.array_equal(_apply(pc, y), _apply(fresh, y))


def test_chunked_apply_captured_in_graph_replays_exactly():
    S = make_system(**CASES["mid"])
    part, pc = gpu_precond(S, iprec=addns.F32, sprec=addns.F32, sweep_chunks=2)
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
    rng = np.random.default_rng(12)
    for rep in range(3):
        yin = _cuda(rng.standard_normal(S.N))
        y.copy_(yin)
        g.replay()
        torch.cuda.synchronize()
        got = x.cpu().numpy().copy()
        ref = torch.zeros_like(x)
        addns.apply_precond(pc, yin, ref)
        torch.cuda.synchronize()
        assert np.array_equal(got, ref.cpu().numpy()), rep
        x.zero_()


@pytest.mark.parametrize("p", [2, 3])
def test_chunked_refactor_keeps_a_captured_apply_valid(p):
    """The chunk structure (coupling columns and carry positions) follows the
    factor values, so a refactor with another wind may change it; every chunk
    buffer is sized for the plan's largest structure, so the apply captured
    before the refactor replays with the new factors and structure."""
    S1 = make_system(**CASES["mid"])
    S2 = make_system(**CASES["mid"], wind=Wind((0.3, -1.0, 0.5, 2.0), 1.5))
    _, pc = gpu_precond(S1, iprec=addns.F32, sprec=addns.F32, sweep_chunks=p)
    bytes1 = pc.info()["chunk_bytes"]
    y = _cuda(np.random.default_rng(13).standard_normal(S1.N))
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
    addns.refactor_precond(pc, _cuda(S1.rp), _cuda(S1.ci), _cuda(S2.v))
    torch.cuda.synchronize()
    assert pc.info()["sweep_chunks"] == p
    # the new wind couples other positions: the structure did change
    assert pc.info()["chunk_bytes"] != bytes1
    want = _apply(pc, y.cpu().numpy())
    for rep in range(3):
        x.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), want), rep

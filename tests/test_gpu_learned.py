"""GPU parity of the exact block-Jacobi interface blocks and of the learned
interface correction (an extension beyond the paper) against the oracle.

Tolerances:
* EXACT_BJ blocks S_i = S(agg_i, agg_i) of S = G - F D^{-1} E (section 1):
  FP64 column solves with the interior factors, then FP64 products; error
  ~ eps * cond(A_jj): 1e-11 relative to max|S_i|, as for the MSCN blocks.
* Features are FP64 arithmetic rounded once to FP32: 2 ulp of FP32.
  Targets S - G are rounded to FP32 from FP64 blocks that carry the 1e-11
  error above: 1e-11 * max|S| + 2 ulp.
* Network outputs in FP32 against the FP64 oracle: 64-term FP32 sums,
  1e-5 relative.  BF16 inference against the oracle's BF16 emulation: the
  inputs of every layer are rounded identically, but a hidden activation can
  land on the other side of a BF16 rounding boundary (FP32 versus FP64
  accumulation), one BF16 ulp = 2^-8: 2e-2 relative to the output norm.
* Gradient: FP32 accumulation over ~1000 samples in a fixed order against
  FP64 backpropagation: 1e-4 relative (the norm-wise bound of the training
  precision contract).
Solves with a learned form are judged only by the FP64 true residual.
"""
import numpy as np
import pytest

from tests.gpu_systems import gpu_precond, make_system, oracle_precond, relerr

torch = pytest.importorskip("torch")
from oracle import mlp  # noqa: E402
from paper_1104_3349_amd import addns  # noqa: E402

pytestmark = pytest.mark.gpu

F32_ULP = 2.0 ** -23


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _system(n=24, nu=0.02, m=4, sz=16, stretch=1.05, seed=11):
    return make_system(n, nu, m, sz=sz, stretch=stretch, seed=seed)


def _blocks_err(got, blocks):
    off, worst = 0, 0.0
    for blk in blocks:
        g = got[off:off + blk.size].reshape(blk.shape)
        off += blk.size
        worst = max(worst, float(np.abs(g - blk).max() / max(np.abs(blk).max(), 1e-300)))
    return worst


@pytest.mark.parametrize("n,m,sz", [(16, 4, 64), (24, 4, 16), (40, 9, 24)])
def test_exact_bj_blocks(n, m, sz):
    S = _system(n=n, m=m, sz=sz)
    ora = oracle_precond(S, addns.SCHUR_EXACT_BJ)
    part, pc = gpu_precond(S, addns.SCHUR_EXACT_BJ)
    tot = sum(x.size for x in ora.S_blocks)
    assert _blocks_err(pc.schur_blocks(tot), ora.S_blocks) <= 1e-11


def test_exact_single_aggregate_converges_in_one_iteration():
    """Banachiewicz: with Shat = S the preconditioner is C~ itself."""
    S = make_system(16, 0.1, 4, sz=10 ** 6, seed=1001)
    part, pc = gpu_precond(S, addns.SCHUR_EXACT_BJ)
    assert part.info()["k"] == 1
    d_b = _cuda(S.b)
    d_x = torch.zeros(S.N, dtype=torch.float64, device="cuda")
    r = addns.gmres_solve(pc, d_b, d_x, restart=10, maxit=10, tol=1e-10, flexible=False)
    assert r["converged"] and r["iters"] == 1


def _gpu_samples(pc):
    n = addns.dtn_samples(pc)
    X = torch.zeros((n, 7), dtype=torch.float32, device="cuda")
    Y = torch.zeros((n, 5), dtype=torch.float32, device="cuda")
    M = torch.zeros((n, 5), dtype=torch.float32, device="cuda")
    assert addns.dtn_samples(pc, X, Y, M) == n
    torch.cuda.synchronize()
    return X, Y, M


@pytest.mark.parametrize("stretch,nu,teacher", [(None, 0.05, addns.SCHUR_MSCN), (1.05, 0.002, addns.SCHUR_MSCN),
                                                (1.05, 0.002, addns.SCHUR_EXACT_BJ)])
def test_samples_match_oracle(stretch, nu, teacher):
    S = _system(n=32, nu=nu, m=4, sz=24, stretch=stretch)
    ora = oracle_precond(S, teacher)
    smp = mlp.samples(ora)
    part, pc = gpu_precond(S, teacher)
    X, Y, M = _gpu_samples(pc)
    X, Y, M = X.cpu().numpy(), Y.cpu().numpy(), M.cpu().numpy()
    assert X.shape[0] == len(smp.rows) > 0
    assert np.array_equal(M, smp.M.astype(np.float32))
    assert np.all(np.abs(X - smp.X) <= 2 * F32_ULP * np.abs(smp.X) + 1e-15)
    smax = max(np.abs(b).max() for b in ora.S_blocks)
    assert np.all(np.abs(Y - smp.Y) <= 1e-11 * smax + 2 * F32_ULP * np.abs(smp.Y))


def _oracle_data(seed=3):
    S = _system(n=40, nu=0.01, m=4, sz=24, stretch=1.05, seed=seed)
    ora = oracle_precond(S, addns.SCHUR_MSCN)
    return S, ora, mlp.samples(ora)


def _random_weights(seed, scale=0.2):
    return (np.random.default_rng(seed).standard_normal(mlp.N_PARAM) * scale).astype(np.float32)


def _forward_scales(w, X, round_bf16):
    """Per-output error scales of the forward pass: the network with every
    weight and input replaced by its absolute value (the scale of a forward
    error bound), and, with BF16 rounding, the effect of moving every rounded
    activation by one BF16 unit (2^-7 of its size) on the output."""
    p = mlp.unpack(w)
    if round_bf16:
        p = {k: mlp.bf16(v) for k, v in p.items()}
        X = mlp.bf16(X)
    A = {k: np.abs(v) for k, v in p.items()}
    h1 = np.maximum(X @ p["W1"].T + p["b1"], 0.0)
    h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0.0)
    s1 = np.abs(X) @ A["W1"].T + A["b1"]
    s2 = s1 @ A["W2"].T + A["b2"]
    scale = s2 @ A["W3"].T + A["b3"]
    flips = (h1 @ A["W2"].T + h2) @ A["W3"].T * 2.0 ** -7 if round_bf16 else 0.0
    return scale, flips


def test_forward_fp32_and_bf16():
    """Matrix-core forward against the oracle's, element by element.  FP32:
    three layers of FP32 accumulation over at most 64 terms stay within
    3e-5 of the absolute-value network.  BF16: the same, plus one BF16 unit
    per hidden activation whose rounding may fall the other way when the FP32
    sum and the FP64 sum straddle a rounding boundary."""
    S, ora, smp = _oracle_data()
    w = _random_weights(1)
    X32 = smp.X.astype(np.float32)
    d_X = _cuda(X32)
    d_P = torch.zeros((len(X32), 5), dtype=torch.float32, device="cuda")
    addns.dtn_forward(w, d_X, d_P, bf16=False)
    torch.cuda.synchronize()
    ref = mlp.forward(w, X32)
    scale, _ = _forward_scales(w, X32.astype(np.float64), False)
    assert np.all(np.abs(d_P.cpu().numpy() - ref) <= 3e-5 * scale)
    addns.dtn_forward(w, d_X, d_P, bf16=True)
    torch.cuda.synchronize()
    ref = mlp.forward(w, X32, round_bf16=True)
    scale, flips = _forward_scales(w, X32.astype(np.float64), True)
    got = d_P.cpu().numpy()
    assert np.all(np.abs(got - ref) <= 3e-5 * scale + flips)
    assert relerr(got, ref) <= 2e-2
    # a ragged count (not a multiple of the 16-sample tile)
    n = 37
    d_P2 = torch.full((n, 5), -7.0, dtype=torch.float32, device="cuda")
    addns.dtn_forward(w, _cuda(X32[:n]), d_P2, bf16=False)
    torch.cuda.synchronize()
    assert np.all(np.abs(d_P2.cpu().numpy() - mlp.forward(w, X32[:n])) <= 3e-5 * scale[:n])


def test_gradient_matches_oracle_backprop():
    S, ora, smp = _oracle_data()
    n = min(len(smp.rows), 1000)
    assert n > 64  # several workgroups
    X, Y, M = (a[:n].astype(np.float32) for a in (smp.X, smp.Y, smp.M))
    # scale targets to O(1) so that the loss is not dominated by rounding
    Y = (Y / max(np.abs(Y).max(), 1e-30)).astype(np.float32)
    w = _random_weights(2)
    g, loss = addns.dtn_grad(w, _cuda(X), _cuda(Y), _cuda(M))
    loss_ref, g_ref = mlp.loss_grad(w, X, Y, M)
    assert abs(loss - loss_ref) <= 1e-5 * abs(loss_ref)
    assert relerr(g, g_ref) <= 1e-4
    # tensor by tensor (a wrong bias or a transposed weight would not hide in
    # the norm of the larger tensors)
    got, ref = mlp.unpack(g), mlp.unpack(g_ref)
    for name in got:
        assert relerr(got[name], ref[name]) <= 1e-4, name
    # ragged tail: a count that is not a multiple of the workgroup size
    g2, loss2 = addns.dtn_grad(w, _cuda(X[:77]), _cuda(Y[:77]), _cuda(M[:77]))
    loss_ref2, g_ref2 = mlp.loss_grad(w, X[:77], Y[:77], M[:77])
    assert relerr(g2, g_ref2) <= 1e-4 and abs(loss2 - loss_ref2) <= 1e-5 * abs(loss_ref2)


def test_training_deterministic_and_descends():
    S = _system(n=32, nu=0.01, m=4, sz=24)
    part, pc = gpu_precond(S, addns.SCHUR_MSCN)
    X, Y, M = _gpu_samples(pc)
    w1, l1 = addns.dtn_train(X, Y, M, epochs=8, batch=64, lr=3e-3, seed=9)
    w2, l2 = addns.dtn_train(X, Y, M, epochs=8, batch=64, lr=3e-3, seed=9)
    assert np.array_equal(w1, w2) and np.array_equal(l1, l2)
    assert np.all(np.isfinite(l1)) and l1[-1] < l1[0]
    # continuing from given weights with zero epochs returns them unchanged
    w3, _ = addns.dtn_train(X, Y, M, epochs=0, batch=64, lr=1e-3, seed=1, init=w1)
    assert np.array_equal(w3, w1)


@pytest.mark.parametrize("bf16", [False, True])
def test_learned_setup_blocks_and_apply(bf16):
    S, ora, smp = _oracle_data(seed=5)
    w = _random_weights(4, 0.05)
    X32 = smp.X.astype(np.float32)
    delta = mlp.forward(w, X32, round_bf16=bf16)
    blocks = mlp.learned_blocks(ora, smp, delta)
    part, pc = gpu_precond(S, addns.SCHUR_LEARNED, learned_model=w, learned_bf16=bf16)
    assert pc.info()["learned_count"] == len(smp.rows)
    got = pc.schur_blocks(sum(b.size for b in blocks))
    dmax = np.abs(delta).max()
    off = 0
    for b in blocks:
        g = got[off:off + b.size].reshape(b.shape)
        off += b.size
        tol = (2e-2 if bf16 else 1e-5) * dmax + 1e-12 * np.abs(b).max()
        assert np.abs(g - b).max() <= tol
    if not bf16:
        from oracle.precond import LEARNED, Preconditioner
        from oracle.partition import build_partition
        P = build_partition(S.N, S.rp, S.ci, S.v, S.m, S.sz)
        ref = Preconditioner(S.N, S.rp, S.ci, S.v, P, LEARNED, learned_S=blocks)
        y = np.random.default_rng(8).standard_normal(S.N)
        d_x = torch.zeros(S.N, dtype=torch.float64, device="cuda")
        addns.apply_precond(pc, _cuda(y), d_x)
        torch.cuda.synchronize()
        assert relerr(d_x.cpu().numpy(), ref.apply(y)) <= 1e-4


def test_judged_solve_accepts_and_falls_back():
    S = make_system(32, 0.01, 4, sz=32, seed=21)
    part = addns.build_partition(S.N, S.rp, S.ci, S.v, S.m, S.sz)
    _, plain = gpu_precond(S, addns.SCHUR_MSCN, part=part)
    d_b = _cuda(S.b)
    d_x = torch.zeros(S.N, dtype=torch.float64, device="cuda")
    ref = addns.gmres_solve(plain, d_b, d_x, restart=30, maxit=2000, tol=1e-8)
    assert ref["converged"]
    x_plain = d_x.cpu().numpy().copy()
    # zero network = LUM blocks: converges, accepted
    zero = np.zeros(mlp.N_PARAM, np.float32)
    _, lz = gpu_precond(S, addns.SCHUR_LEARNED, part=part, learned_model=zero)
    d_x.zero_()
    r = addns.gmres_solve_judged(lz, plain, d_b, d_x, restart=30, maxit=2000, tol=1e-8)
    assert r["accepted"] and r["converged"] and r["true_relres"] <= 1e-8
    # a network that adds 1e3 to every diagonal of Shat: the interface part of
    # the preconditioner is lost, the learned solve misses the tolerance within
    # the plain method's budget, and the judge returns the plain solve
    bad = np.zeros(mlp.N_PARAM, np.float32)
    bad[-3] = 1e3  # b3 of the diagonal slot
    _, lb = gpu_precond(S, addns.SCHUR_LEARNED, part=part, learned_model=bad)
    d_x.zero_()
    r = addns.gmres_solve_judged(lb, plain, d_b, d_x, restart=30, maxit=ref["iters"] + 2, tol=1e-8)
    assert not r["accepted"]
    assert r["converged"] and r["iters"] == ref["iters"]
    assert np.array_equal(d_x.cpu().numpy(), x_plain)


def test_learned_argument_errors():
    S = _system(n=16, m=4, sz=16)
    with pytest.raises(addns.AddnsError) as e:
        gpu_precond(S, addns.SCHUR_LEARNED)  # no model
    assert e.value.code == addns.ERR_ARG
    zero = np.zeros(mlp.N_PARAM, np.float32)
    part, pl = gpu_precond(S, addns.SCHUR_LEARNED, learned_model=zero)
    n = addns.dtn_samples(pl)  # a size query works on any handle
    assert n > 1
    X = torch.zeros((n, 7), dtype=torch.float32, device="cuda")
    with pytest.raises(addns.AddnsError):
        addns.dtn_samples(pl, X, X, X)  # a LEARNED handle has no teacher blocks
    part, pe = gpu_precond(S, addns.SCHUR_MSCN)
    small = torch.zeros((n - 1, 7), dtype=torch.float32, device="cuda")
    with pytest.raises(addns.AddnsError) as e:
        addns.dtn_samples(pe, small, small, small)  # capacity too small
    assert e.value.code == addns.ERR_ARG
    with pytest.raises(addns.AddnsError):
        addns.dtn_samples(pe, X, X, None)  # targets without masks


def test_trained_network_gains_over_the_method_without_it():
    """Train on 300 seeded 64 x 64 systems (MSCN teacher), then solve a
    held-out system: the learned blocks G_i + Delta_i must need fewer
    iterations than the same mode without the network (Delta = 0, i.e. LUM's
    S_i = G_i) and than MSCN itself, and the judge must accept them."""
    from paper_1104_3349_amd import learned
    from workloads.configs import F32, Workload, training_workloads
    X, Y, M = learned.collect_samples(training_workloads(300), 100)
    w, loss = addns.dtn_train(X, Y, M, epochs=20, batch=1024, lr=2e-3, seed=0)
    assert loss[-1] < loss[0]
    wl = Workload("heldout", 64, 1 / 500, None, 4, 64, 50, True, 1e-8, 78, F32, F32)
    S = make_system(wl.n, wl.nu, wl.m, sz=wl.sz, seed=wl.seed)
    part = addns.build_partition(S.N, S.rp, S.ci, S.v, S.m, S.sz)
    d_b = _cuda(S.b)
    d_x = torch.zeros(S.N, dtype=torch.float64, device="cuda")
    its = {}
    for name, kw in (("lum", dict(schur=addns.SCHUR_LUM)), ("mscn", dict(schur=addns.SCHUR_MSCN)),
                     ("zero", dict(schur=addns.SCHUR_LEARNED, learned_model=np.zeros_like(w))),
                     ("learned", dict(schur=addns.SCHUR_LEARNED, learned_model=w))):
        _, pc = gpu_precond(S, part=part, **kw)
        d_x.zero_()
        r = addns.gmres_solve(pc, d_b, d_x, restart=50, maxit=5000, tol=1e-8)
        assert r["converged"], name
        its[name] = r["iters"]
    _, plain = gpu_precond(S, part=part)
    _, lp = gpu_precond(S, addns.SCHUR_LEARNED, part=part, learned_model=w)
    d_x.zero_()
    r = addns.gmres_solve_judged(lp, plain, d_b, d_x, restart=50, maxit=5000, tol=1e-8)
    print("iterations", its)
    assert r["accepted"] and r["iters"] == its["learned"]
    assert its["zero"] == its["lum"]
    assert its["learned"] < its["lum"]
    assert its["learned"] < its["mscn"]

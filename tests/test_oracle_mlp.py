"""Pins of the learned-correction oracle (an extension beyond the paper):
the network against torch's own layers, the backpropagated gradient against
finite differences and torch autograd, BF16 rounding against its definition,
and the samples against a dense exact Schur complement S = G - F D^{-1} E
(section 1) and the symmetry of the diffusion-only operator."""
import numpy as np
import pytest
import torch

from oracle import mlp
from oracle.partition import build_partition
from oracle.precond import EXACT_BJ, LEARNED, LUM, Preconditioner
from workloads.mac_oseen import Wind, make_oseen_mac


def _weights(seed=0, scale=0.3):
    return np.random.default_rng(seed).standard_normal(mlp.N_PARAM) * scale


def _torch_net(w):
    p = mlp.unpack(w)
    net = torch.nn.Sequential(torch.nn.Linear(7, 64), torch.nn.ReLU(), torch.nn.Linear(64, 64),
                              torch.nn.ReLU(), torch.nn.Linear(64, 5)).double()
    with torch.no_grad():
        for lin, (wn, bn) in zip((net[0], net[2], net[4]), (("W1", "b1"), ("W2", "b2"), ("W3", "b3"))):
            lin.weight.copy_(torch.from_numpy(p[wn].copy()))
            lin.bias.copy_(torch.from_numpy(p[bn].copy()))
    return net


def test_param_count():
    assert mlp.N_PARAM == 4997
    w = _weights()
    assert np.array_equal(mlp.pack(mlp.unpack(w)), w)


def test_forward_matches_torch_layers():
    w = _weights(1)
    X = np.random.default_rng(2).standard_normal((40, 7))
    ref = _torch_net(w)(torch.from_numpy(X)).detach().numpy()
    assert np.allclose(mlp.forward(w, X), ref, rtol=1e-13, atol=1e-13)


def test_gradient_matches_autograd_and_differences():
    rng = np.random.default_rng(3)
    w = _weights(4)
    X = rng.standard_normal((33, 7))
    Y = rng.standard_normal((33, 5))
    M = (rng.random((33, 5)) < 0.7).astype(float)
    loss, g = mlp.loss_grad(w, X, Y, M)
    net = _torch_net(w)
    out = net(torch.from_numpy(X))
    tl = ((torch.from_numpy(M) * (out - torch.from_numpy(Y)) ** 2).sum()) / X.shape[0]
    tl.backward()
    tg = mlp.pack({"W1": net[0].weight.grad, "b1": net[0].bias.grad, "W2": net[2].weight.grad,
                   "b2": net[2].bias.grad, "W3": net[4].weight.grad, "b3": net[4].bias.grad})
    assert abs(loss - tl.item()) <= 1e-12 * abs(loss)
    assert np.allclose(g, tg, rtol=1e-10, atol=1e-12)
    # central differences on a spread of coordinates, one in each tensor
    h = 1e-6
    for idx in [0, 300, 450, 600, 2000, 4500, 4700, 4993, 4996]:
        e = np.zeros_like(w)
        e[idx] = h
        fd = (mlp.loss_grad(w + e, X, Y, M)[0] - mlp.loss_grad(w - e, X, Y, M)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(g[idx])), idx


def test_bf16_rounding_definition():
    e = 2.0 ** -8
    vals = np.array([1.0, 1.0 + e, 1.0 + 3 * e, -2.0 - 2 * e, 1.0 + e + 2 ** -20, 0.0])
    want = np.array([1.0, 1.0, 1.0 + 4 * e, -2.0, 1.0 + 2 * e, 0.0])
    assert np.array_equal(mlp.bf16(vals), want)


def _pre(n=16, nu=0.05, wind=None, m=4, sz=16, mode=EXACT_BJ, seed=7, stretch=None):
    rp, ci, v, b, meta = make_oseen_mac(n, nu, wind=wind, stretch=stretch, seed=seed)
    P = build_partition(meta["N"], rp, ci, v, m, sz)
    return Preconditioner(meta["N"], rp, ci, v, P, mode), meta


def test_samples_targets_are_exact_schur_entries():
    pre, meta = _pre(stretch=1.05)
    smp = mlp.samples(pre)
    assert len(smp.rows) > 0
    D, E, F, G, _ = pre.dense_blocks()
    S = G - F @ np.linalg.solve(D, E)           # dense exact Schur complement
    Gs = G
    part = pre.part
    sep = part.perm[part.n_int:]
    pos = {int(g): c for c, g in enumerate(sep)}
    hits = 0
    for t in range(len(smp.rows)):
        c = smp.seps[t]
        assert sep[c] == smp.rows[t]
        assert smp.nb[t, 2] == smp.rows[t] and smp.M[t, 2] == 1.0
        for q in range(5):
            o = smp.nb[t, q]
            if smp.M[t, q] == 0:
                assert smp.Y[t, q] == 0.0
                continue
            d = pos[int(o)]
            assert abs(smp.Y[t, q] - (S[c, d] - Gs[c, d])) <= 1e-12 * max(1.0, abs(S[c, d]))
            hits += 1
    assert hits > len(smp.rows)  # off-diagonal slots inside aggregates too


def test_samples_slots_and_features():
    pre, meta = _pre()
    smp = mlp.samples(pre, with_targets=False)
    C = pre.C.toarray()
    for t in range(len(smp.rows)):
        g = smp.rows[t]
        lo = [o for o in smp.nb[t, :2] if o >= 0]
        hi = [o for o in smp.nb[t, 3:] if o >= 0]
        assert all(o < g for o in lo) and all(o > g for o in hi)
        if smp.nb[t, 0] >= 0:
            assert g - smp.nb[t, 0] > g - smp.nb[t, 1]
        if smp.nb[t, 4] >= 0:
            assert smp.nb[t, 4] - g > smp.nb[t, 3] - g
        for q in range(5):
            o = smp.nb[t, q]
            assert smp.X[t, q] == (C[g, o] if o >= 0 else 0.0)
        assert smp.X[t, 2] == 1.0  # the diagonal dominates its row: scaled to one


def test_skew_features_vanish_without_wind():
    pre, meta = _pre(wind=Wind(scale=0.0))
    smp = mlp.samples(pre, with_targets=False)
    assert np.abs(smp.X[:, 5:]).max() <= 1e-14
    pre2, _ = _pre(wind=Wind(scale=1.0))
    smp2 = mlp.samples(pre2, with_targets=False)
    assert np.abs(smp2.X[:, 5:]).max() > 1e-3


def test_learned_blocks_special_cases():
    pre, meta = _pre()
    smp = mlp.samples(pre)
    lum, _ = _pre(mode=LUM)
    zero = mlp.learned_blocks(pre, smp, np.zeros_like(smp.Y))
    for a, b in zip(zero, lum.S_blocks):
        assert np.array_equal(a, b)
    exact = mlp.learned_blocks(pre, smp, smp.Y)
    for i, (a, s) in enumerate(zip(exact, pre.S_blocks)):
        g = lum.S_blocks[i]
        on = a != g
        assert np.allclose(a[on], s[on], rtol=1e-12, atol=1e-14)
    # the LEARNED oracle mode with a zero correction is the LUM preconditioner
    rp, ci, v, b, meta2 = make_oseen_mac(16, 0.05, seed=7)
    learned = Preconditioner(meta2["N"], rp, ci, v, pre.part, LEARNED, learned_S=zero)
    y = np.random.default_rng(5).standard_normal(meta2["N"])
    assert np.array_equal(learned.apply(y), lum.apply(y))

"""Oracle: the learned interface correction (an extension beyond the paper).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only tests, the smoke check and the CPU-baseline leg of
the benchmark do.

The paper approximates the exact interface Schur complement
S = G - F D^{-1} E (section 1; the algebraic Dirichlet-to-Neumann map) by the
block diagonal Shat of mini Schur complements (section 3.1, Algorithm 1).
The extension learns a correction of G_i instead:  S_i ~ G_i + Delta_i, with
Delta_i on G's own stencil pattern, predicted per separator velocity row by
a small network and trained on the interface blocks of a teacher mode of
oracle.precond (MSCN, whose blocks are exact Schur complements of the local
D-range systems, or EXACT_BJ, the diagonal blocks of the exact S).
Everything here is plain FP64 numpy.

Samples.  One per separator position c (permuted order) whose node g is a
velocity unknown (not pressure-like).  Its velocity neighbours o != g in
row g of C, split into o < g and o > g (original numbering) and each side
sorted by |o - g|, fill five slots
    [second lower, nearest lower, g itself, nearest upper, second upper]
(missing -> empty slot).  Features (7), with C~ = R C the row-scaled matrix:
    x_q = C~(g, o_q)                         q = 0..4 (0 for empty slots)
    k_q = R_g (C(g, o_q) - C(o_q, g)) / 2    (skew, convective part)
    x_5 = k_3 - k_1,  x_6 = k_4 - k_0.
Targets: y_q = S_i(g, o_q) - G_i(g, o_q), S_i the teacher's block, when o_q
is a separator node of the same aggregate i (mask 1), else 0 (mask 0).

Network: 7 -> 64 -> 64 -> 5 with ReLU, parameters packed as
W1[64][7] b1[64] W2[64][64] b2[64] W3[5][64] b3[5] (4997 numbers).
Loss: (1/count) sum_k sum_q mask_kq (p_kq - y_kq)^2.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

N_IN, N_H, N_OUT = 7, 64, 5
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(w):
    """Named views of a flat parameter vector."""
    w = np.asarray(w, dtype=np.float64)
    assert w.shape == (N_PARAM,)
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = w[o:o + n].reshape(shp)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as
    float64.  Inputs are first rounded to float32."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(w, X, round_bf16=False):
    """Network output for features X[count][7] (FP64; optionally with weights,
    inputs and hidden activations rounded to BF16)."""
    p = unpack(w)
    if round_bf16:
        p = {k: bf16(v) for k, v in p.items()}
        X = bf16(X)
    h1 = np.maximum(X @ p["W1"].T + p["b1"], 0.0)
    if round_bf16:
        h1 = bf16(h1)
    h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0.0)
    if round_bf16:
        h2 = bf16(h2)
    return h2 @ p["W3"].T + p["b3"]


def loss_grad(w, X, Y, M):
    """Loss and its gradient with respect to the packed parameters (FP64
    backpropagation through the two ReLU layers)."""
    p = unpack(w)
    X, Y, M = (np.asarray(a, dtype=np.float64) for a in (X, Y, M))
    n = X.shape[0]
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    out = h2 @ p["W3"].T + p["b3"]
    r = M * (out - Y)
    loss = float(np.sum(r * (out - Y))) / n
    d_out = 2.0 * r / n
    g = {"W3": d_out.T @ h2, "b3": d_out.sum(0)}
    d_a2 = (d_out @ p["W3"]) * (a2 > 0.0)
    g["W2"] = d_a2.T @ h1
    g["b2"] = d_a2.sum(0)
    d_a1 = (d_a2 @ p["W2"]) * (a1 > 0.0)
    g["W1"] = d_a1.T @ X
    g["b1"] = d_a1.sum(0)
    return loss, pack(g)


@dataclass
class Samples:
    rows: np.ndarray     # original index g of each sample
    seps: np.ndarray     # separator position c of each sample
    nb: np.ndarray       # [count][5] original neighbour index or -1
    X: np.ndarray        # [count][7]
    Y: np.ndarray        # [count][5] (zeros where no target)
    M: np.ndarray        # [count][5] mask


def samples(pre, with_targets=True):
    """Samples of an oracle Preconditioner; the targets come from its
    S_blocks (the teacher mode it was built with)."""
    part = pre.part
    C = pre.C.tocsr()                # row-scaled C~
    R = pre.R
    is_p = part.is_pressure
    ni = part.n_int
    sep = part.perm[ni:]
    agg_of = np.repeat(np.arange(part.k), np.diff(part.agg_offsets))
    pos_in_sep = np.full(part.N, -1, dtype=np.int64)
    pos_in_sep[sep] = np.arange(len(sep))
    rows, seps, nbs, Xs, Ys, Ms = [], [], [], [], [], []
    for c, g in enumerate(sep):
        if is_p[g]:
            continue
        lo, hi = [], []
        for o in C.indices[C.indptr[g]:C.indptr[g + 1]]:
            if o == g or is_p[o]:
                continue
            (lo if o < g else hi).append(int(o))
        lo.sort(key=lambda o: g - o)
        hi.sort(key=lambda o: o - g)
        slots = [lo[1] if len(lo) > 1 else -1, lo[0] if lo else -1, int(g),
                 hi[0] if hi else -1, hi[1] if len(hi) > 1 else -1]
        f = np.zeros(5)
        k = np.zeros(5)
        for q, o in enumerate(slots):
            if o < 0:
                continue
            f[q] = C[g, o]
            if q != 2:
                # R_g (C(g,o) - C(o,g)) / 2 with C(i,j) = C~(i,j) / R_i
                k[q] = 0.5 * R[g] * (C[g, o] / R[g] - C[o, g] / R[o])
        x = np.concatenate([f, [k[3] - k[1], k[4] - k[0]]])
        y = np.zeros(5)
        m = np.zeros(5)
        if with_targets:
            i = agg_of[c]
            a0 = part.agg_offsets[i]
            S = pre.S_blocks[i]
            Gi = C[part.aggregate(i)][:, part.aggregate(i)].toarray()
            for q, o in enumerate(slots):
                if o < 0 or pos_in_sep[o] < 0 or agg_of[pos_in_sep[o]] != i:
                    continue
                a, b = c - a0, pos_in_sep[o] - a0
                y[q] = S[a, b] - Gi[a, b]
                m[q] = 1.0
        rows.append(int(g))
        seps.append(c)
        nbs.append(slots)
        Xs.append(x)
        Ys.append(y)
        Ms.append(m)
    return Samples(np.array(rows, dtype=np.int64), np.array(seps, dtype=np.int64),
                   np.array(nbs, dtype=np.int64).reshape(-1, 5), np.array(Xs).reshape(-1, 7),
                   np.array(Ys).reshape(-1, 5), np.array(Ms).reshape(-1, 5))


def learned_blocks(pre, smp: Samples, delta):
    """G_i + Delta_i for every aggregate: G's blocks with delta[count][5]
    added on the sample slots that lie in the sample's own aggregate (the
    blocks of the LEARNED mode)."""
    part = pre.part
    C = pre.C.tocsr()
    ni = part.n_int
    sep = part.perm[ni:]
    agg_of = np.repeat(np.arange(part.k), np.diff(part.agg_offsets))
    pos_in_sep = np.full(part.N, -1, dtype=np.int64)
    pos_in_sep[sep] = np.arange(len(sep))
    blocks = []
    for i in range(part.k):
        agg = part.aggregate(i)
        blocks.append(C[agg][:, agg].toarray())
    for t in range(len(smp.rows)):
        c = smp.seps[t]
        i = agg_of[c]
        a0 = part.agg_offsets[i]
        for q, o in enumerate(smp.nb[t]):
            if o < 0 or pos_in_sep[o] < 0 or agg_of[pos_in_sep[o]] != i:
                continue
            blocks[i][c - a0, pos_in_sep[o] - a0] += delta[t, q]
    return blocks

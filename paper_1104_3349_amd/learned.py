"""Driver of the learned interface correction (an extension beyond the paper).

Training data are the interface blocks S_i of a teacher mode (MSCN's mini
Schur complements by default, or EXACT_BJ's diagonal blocks of the exact
S = G - F D^{-1} E) computed by libaddns on the GPU for many seeded small
systems at once (their partitions concatenated, so each chunk is one
setup); the network is trained on the GPU by addns_dtn_train and written
with addns_dtn_save.  Every numerical step runs
in libaddns; this module only generates seeded inputs and moves buffers.

    python -m paper_1104_3349_amd.learned --count 2000 --out dtn.bin
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import addns


def block_diag_device(built, device):
    """Device CSR (int32 / float64) of diag(C_0, C_1, ...) and the row
    offsets of the systems; `built` holds (rowptr, colidx, vals, b, meta)."""
    import torch
    Ns = [bd[4]["N"] for bd in built]
    offs = np.concatenate([[0], np.cumsum(Ns)]).astype(np.int64)
    nnz = np.concatenate([[0], np.cumsum([len(bd[1]) for bd in built])]).astype(np.int64)
    if offs[-1] > np.iinfo(np.int32).max or nnz[-1] > np.iinfo(np.int32).max:
        raise ValueError("block-diagonal system exceeds int32 sizes")
    rp = np.concatenate([built[0][0][:1]] + [bd[0][1:] + nnz[q] for q, bd in enumerate(built)])
    ci = np.concatenate([bd[1] + offs[q] for q, bd in enumerate(built)])
    v = np.concatenate([bd[2] for bd in built])
    b = np.concatenate([bd[3] for bd in built])
    to = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
    return (int(offs[-1]), to(rp, np.int32), to(ci, np.int32), to(v, np.float64), to(b, np.float64),
            offs.astype(np.int32))


def collect_samples(workloads, chunk=100, device="cuda:0", log=None, teacher=addns.SCHUR_MSCN):
    """Features, targets and masks (device float32 tensors) of every
    workload's separator velocity rows, from teacher-mode setups of `chunk`
    systems at a time."""
    import torch
    Xs, Ys, Ms = [], [], []
    for c0 in range(0, len(workloads), chunk):
        wls = workloads[c0:c0 + chunk]
        built = [w.build() for w in wls]
        parts = [addns.build_partition(bd[4]["N"], bd[0], bd[1], bd[2], w.m, w.sz)
                 for w, bd in zip(wls, built)]
        cat = addns.partition_concat(parts)
        N, d_rp, d_ci, d_v, _, _ = block_diag_device(built, device)
        pc = addns.setup_precond(cat, N, d_rp, d_ci, d_v, schur=teacher)
        n = addns.dtn_samples(pc)
        X = torch.empty((n, 7), dtype=torch.float32, device=device)
        Y = torch.empty((n, 5), dtype=torch.float32, device=device)
        M = torch.empty((n, 5), dtype=torch.float32, device=device)
        addns.dtn_samples(pc, X, Y, M)
        torch.cuda.synchronize()
        Xs.append(X)
        Ys.append(Y)
        Ms.append(M)
        del pc
        if log:
            log(f"samples: systems {c0}..{c0 + len(wls) - 1}, {n} rows")
    return torch.cat(Xs), torch.cat(Ys), torch.cat(Ms)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--count", type=int, default=2000, help="training systems (seeds 5000+t)")
    ap.add_argument("--chunk", type=int, default=100, help="systems per teacher setup")
    ap.add_argument("--teacher", choices=("mscn", "exact_bj"), default="mscn")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", required=True, help="weights file to write")
    a = ap.parse_args(argv)
    import torch

    from workloads.configs import training_workloads

    def log(msg):
        print(msg, flush=True)

    t0 = time.perf_counter()
    teacher = addns.SCHUR_MSCN if a.teacher == "mscn" else addns.SCHUR_EXACT_BJ
    X, Y, M = collect_samples(training_workloads(a.count), a.chunk, log=log, teacher=teacher)
    t1 = time.perf_counter()
    # the rows of the last 5% (the last systems' rows) are held out for validation
    nval = max(1, X.shape[0] // 20)
    ntr = X.shape[0] - nval
    w, loss = addns.dtn_train(X[:ntr], Y[:ntr], M[:ntr], epochs=a.epochs, batch=a.batch, lr=a.lr,
                              seed=a.seed)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    _, vloss = addns.dtn_grad(w, X[ntr:], Y[ntr:], M[ntr:])
    zero = np.zeros_like(w)
    _, vzero = addns.dtn_grad(zero, X[ntr:], Y[ntr:], M[ntr:])
    addns.dtn_save(a.out, w)
    print(json.dumps({"samples": int(X.shape[0]), "train": ntr, "val": nval,
                      "data_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2),
                      "loss_first": float(loss[0]) if len(loss) else None,
                      "loss_last": float(loss[-1]) if len(loss) else None,
                      "val_loss": vloss, "val_loss_zero_model": vzero, "out": a.out}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

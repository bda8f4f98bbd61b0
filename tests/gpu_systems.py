"""Shared set-up for GPU parity tests: one seeded system, prepared both by
the oracle (CPU, FP64) and by libaddns (GPU), from the same generator call."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from oracle.partition import build_partition as oracle_partition
from oracle.precond import EXACT_BJ, LUM, MSCN, MSCN_LITERAL, MSCNR, Preconditioner
from paper_1104_3349_amd import addns
from workloads.mac_oseen import Wind, make_oseen_mac

ORACLE_MODE = {addns.SCHUR_MSCN: MSCN, addns.SCHUR_LUM: LUM, addns.SCHUR_MSCN_LITERAL: MSCN_LITERAL,
               addns.SCHUR_EXACT_BJ: EXACT_BJ, addns.SCHUR_MSCNR: MSCNR}


@dataclass
class System:
    n: int
    N: int
    rp: np.ndarray
    ci: np.ndarray
    v: np.ndarray
    b: np.ndarray
    meta: dict
    m: int
    sz: int


def make_system(n, nu, m, sz=64, stretch=None, seed=1, wind=None):
    rp, ci, v, b, meta = make_oseen_mac(n, nu, wind=wind or Wind(), stretch=stretch, seed=seed)
    return System(n, meta["N"], rp, ci, v, b, meta, m, sz)


def oracle_precond(S: System, schur=addns.SCHUR_MSCN, overlap=0, ilu_tol=0.0):
    P = oracle_partition(S.N, S.rp, S.ci, S.v, S.m, S.sz)
    return Preconditioner(S.N, S.rp, S.ci, S.v, P, ORACLE_MODE[schur], overlap=overlap, ilu_tol=ilu_tol)


def gpu_precond(S: System, schur=addns.SCHUR_MSCN, iprec=addns.F64, sprec=addns.F64, part=None,
                **kw):
    import torch
    if part is None:
        part = addns.build_partition(S.N, S.rp, S.ci, S.v, S.m, S.sz)
    d_rp = torch.from_numpy(S.rp).cuda()
    d_ci = torch.from_numpy(S.ci).cuda()
    d_v = torch.from_numpy(S.v).cuda()
    pc = addns.setup_precond(part, S.N, d_rp, d_ci, d_v, schur=schur, interior_prec=iprec,
                             schur_prec=sprec, **kw)
    torch.cuda.synchronize()
    return part, pc


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    d = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (d if d > 0 else 1.0))


def blocks_of(part, numbering="original"):
    """Index sets compared separately: every interior block and the separator.
    numbering: "original" (vectors in C's numbering), "permuted" (P^T order),
    or "interior" (permuted interior part only)."""
    m = len(part.int_offsets) - 1
    if numbering == "original":
        return [part.interior(j) for j in range(m)] + [part.separator()]
    ranges = [np.arange(part.int_offsets[j], part.int_offsets[j + 1]) for j in range(m)]
    if numbering == "interior":
        return ranges
    return ranges + [np.arange(part.n_int, part.N)]


def blockwise_err(got, ref, blocks):
    """Element-by-element error: the largest |got_i - ref_i| of each block,
    relative to that block's largest |ref_i|, maximised over the blocks (an
    error confined to a small block is not diluted by the others)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    worst = 0.0
    for idx in blocks:
        if len(idx) == 0:
            continue
        scale = float(np.abs(ref[idx]).max())
        d = float(np.abs(got[idx] - ref[idx]).max())
        worst = max(worst, d / scale if scale > 0 else d)
    return worst

"""Picard outer iteration on the GPU.

Section 1 obtains the Oseen system as one Picard linearisation of the steady
Navier-Stokes equations; a full steady solve repeats it, freezing the wind
at the previous velocity iterate.  Per outer step q:

  host    the generator assembles the values of C(w(x_q)) and b (input
          generation: the sparsity pattern never changes);
  device  addns_precond_refactor recomputes the preconditioner for the new
          values on the plan of the first step (partition built once);
          addns_gmres_solve with maxit = 0 returns the row-scaled residual
          r_q of x_q; unless r_q <= tol, FGMRES solves C_q x = b_q from x_q.

Every numerical step of the method runs in libaddns; this module moves
buffers and calls the generator.

    python -m paper_1104_3349_amd.picard --n 128 --nu 0.01 --m 16
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import addns

ZERO_FORCING = (lambda x, y: 0.0 * x, lambda x, y: 0.0 * y)


def solve(n, nu, stretch=None, seed=0, m=16, sz=64, schur=addns.SCHUR_MSCN, overlap=0,
          interior_prec=addns.F32, schur_prec=addns.F32, tol=1e-8, maxit=40, restart=50, lin_tol=None,
          lin_maxit=5000, forcing=ZERO_FORCING, device="cuda:0", log=None):
    """Run the outer loop; returns a dict with the final x (host), the
    residual history r_0..r_q, linear iterations per step and timings."""
    import torch

    from workloads.mac_oseen import FaceWind, make_oseen_mac

    lin_tol = tol / 10 if lin_tol is None else lin_tol
    dev = torch.device(device)
    N = 3 * n * n - 2 * n - 1
    x = np.zeros(N)
    d_x = torch.zeros(N, dtype=torch.float64, device=dev)
    part = pc = d_rp = d_ci = None
    out = {"residuals": [], "lin_iters": [], "assemble_s": 0.0, "setup_s": 0.0, "refactor_s": 0.0,
           "solve_s": 0.0, "converged": False}
    for q in range(maxit + 1):
        t0 = time.perf_counter()
        rp, ci, v, b, meta = make_oseen_mac(n, nu, wind=FaceWind.from_solution(x, n), stretch=stretch,
                                            seed=seed, forcing=forcing)
        t1 = time.perf_counter()
        out["assemble_s"] += t1 - t0
        d_v = torch.from_numpy(v).to(dev)
        d_b = torch.from_numpy(b).to(dev)
        if pc is None:
            part = addns.build_partition(N, rp, ci, v, m, sz)
            d_rp = torch.from_numpy(rp).to(dev)
            d_ci = torch.from_numpy(ci).to(dev)
            pc = addns.setup_precond(part, N, d_rp, d_ci, d_v, schur=schur, interior_prec=interior_prec,
                                     schur_prec=schur_prec, overlap=overlap, block_mult=1)
            torch.cuda.synchronize()
            out["setup_s"] += time.perf_counter() - t1
        else:
            addns.refactor_precond(pc, d_rp, d_ci, d_v)
            torch.cuda.synchronize()
            out["refactor_s"] += time.perf_counter() - t1
        t2 = time.perf_counter()
        r = addns.gmres_solve(pc, d_b, d_x, restart=restart, maxit=0, tol=tol, use_x0=True)["true_relres"]
        out["residuals"].append(r)
        if log:
            log(f"picard step {q}: residual {r:.3e}")
        if r <= tol:
            out["converged"] = True
            out["solve_s"] += time.perf_counter() - t2
            break
        if q == maxit:
            out["solve_s"] += time.perf_counter() - t2
            break
        res = addns.gmres_solve(pc, d_b, d_x, restart=restart, maxit=lin_maxit, tol=lin_tol, use_x0=True)
        torch.cuda.synchronize()
        out["solve_s"] += time.perf_counter() - t2
        out["lin_iters"].append(res["iters"])
        x = d_x.cpu().numpy().copy()
    out["x"] = x
    out["steps"] = len(out["lin_iters"])
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--nu", type=float, default=0.01)
    ap.add_argument("--m", type=int, default=16)
    ap.add_argument("--sz", type=int, default=64)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--overlap", type=int, default=0)
    a = ap.parse_args(argv)
    t = time.perf_counter()
    res = solve(a.n, a.nu, m=a.m, sz=a.sz, tol=a.tol, overlap=a.overlap, log=lambda s: print(s, flush=True))
    res.pop("x")
    res["total_s"] = round(time.perf_counter() - t, 3)
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())

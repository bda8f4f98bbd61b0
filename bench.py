"""Benchmark: time to a 1e-8 true relative residual and preconditioner-apply
bandwidth on one MI355X.

One step = setup_precond + gmres_solve (FGMRES(50), tol 1e-8) on the
128 x 128 uniform MAC Oseen cavity (nu = 1/100, 16 subdomains), the largest
workload of the set that the method solves to 1e-8 with FGMRES(50): FP32
interior and interface factors, the coarse-grid correction of the interface
solve (pieces of 32), CGS2 Arnoldi, FP64 outer solver; inputs resident in
HBM.  The partition is built once beforehand and excluded, as in the paper's
timings.  Median of the timed steps after the warm-up ones.  Beside it: the
plain FP64 path (FP64 factors, no coarse correction) with CGS2 and with MGS
under the same protocol, the other forms of the paper, and the 512 x 512
stretched workload's apply bandwidth and interior-solve roofline (HBM
resident) with its FGMRES(50) result.

Prints one JSON line.  --gpus above 1 is not supported (one GPU per box).
"""
from __future__ import annotations

import argparse
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def _events_ms(fn, reps, torch):
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


PEAK = 8.0e12  # MI355X HBM3E bytes/s


def _events_median_ms(fn, reps, torch):
    """Median of `reps` launches of fn, each bracketed by HIP events on the
    current stream (the stream the library launches on)."""
    import numpy as np
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record(s)
        fn()
        e1.record(s)
    torch.cuda.synchronize()
    return float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))


def measured_traffic(workload="cavity128"):
    """Calibrated FETCH_SIZE + WRITE_SIZE bytes per interior-solve launch from
    the committed rocprofv3 summary of `workload`; None once the kernel source
    differs from the one that was profiled."""
    import hashlib
    import re
    prof = os.path.join(ROOT, "profiles", f"interior_solve_{workload}_pmc.md")
    src = os.path.join(ROOT, "paper_1104_3349_amd", "csrc", "kernels_apply.hip")
    try:
        text = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    h = re.search(r"kernel_source_sha256_prefix: (\w+)", text)
    if not m or not h or h.group(1) != sha:
        return None
    return int(m.group(1))


def cpu_baseline(cfg, coarse, ortho, runs=3):
    """The oracle as it stands on the host: full solves (setup + FGMRES to
    tol) of the same workload and method options; median of `runs`."""
    import numpy as np

    from oracle.krylov import gmres
    from oracle.partition import build_partition as oracle_partition
    from oracle.precond import MSCN, Preconditioner

    rp, ci, v, b, meta = cfg.build()
    N = meta["N"]
    P = oracle_partition(N, rp, ci, v, cfg.m, cfg.sz)
    walls, cpus, its = [], [], []
    for _ in range(runs):
        r0 = resource.getrusage(resource.RUSAGE_SELF)
        t0 = time.perf_counter()
        pre = Preconditioner(N, rp, ci, v, P, MSCN, coarse=coarse)
        res = gmres(lambda z: pre.C @ z, pre.apply, pre.R * b, restart=cfg.restart, tol=cfg.tol, maxit=20000,
                    flexible=cfg.flexible, ortho=ortho)
        walls.append(time.perf_counter() - t0)
        r1 = resource.getrusage(resource.RUSAGE_SELF)
        cpus.append((r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime))
        its.append(res.iters)
    k = int(np.argsort(walls)[len(walls) // 2])
    return {"value": round(walls[k], 4), "unit": "s", "cores": max(1, int(round(cpus[k] / walls[k]))),
            "kind": "oracle",
            "sample": f"{runs} full oracle solves (setup + FGMRES({cfg.restart}) to {cfg.tol:g}, coarse pieces "
                      f"{coarse}, {ortho}), median; {its[k]} iterations; host cpus {os.cpu_count()}"}


def bench_batched(args):
    """96 independent Oseen systems (seeded grids 32..128, nu log-uniform in
    [1/500, 1/20], random recirculating winds, 4..16 subdomains): one
    concatenated preconditioner and one lockstep FGMRES(50), against solving
    the same systems one after another with the same library."""
    import numpy as np
    import scipy.sparse as sp
    import torch

    from paper_1104_3349_amd import addns
    from workloads.configs import batched_workloads

    dev = torch.device("cuda:0")
    wls = batched_workloads(96)
    built = [w.build() for w in wls]
    parts = [addns.build_partition(bd[4]["N"], bd[0], bd[1], bd[2], w.m, w.sz) for w, bd in zip(wls, built)]
    cat = addns.partition_concat(parts)
    big = sp.block_diag([sp.csr_matrix((bd[2], bd[1], bd[0]), shape=(bd[4]["N"],) * 2) for bd in built])
    big = big.tocsr()
    big.sort_indices()
    Ns = [bd[4]["N"] for bd in built]
    offs = np.concatenate([[0], np.cumsum(Ns)]).astype(np.int32)
    N = int(offs[-1])
    d_rp = torch.from_numpy(big.indptr.astype(np.int32)).to(dev)
    d_ci = torch.from_numpy(big.indices.astype(np.int32)).to(dev)
    d_v = torch.from_numpy(big.data).to(dev)
    d_b = torch.from_numpy(np.concatenate([bd[3] for bd in built])).to(dev)
    d_x = torch.zeros(N, dtype=torch.float64, device=dev)

    split = []

    def step():
        ts = time.perf_counter()
        pc = addns.setup_precond(cat, N, d_rp, d_ci, d_v, interior_prec=addns.F32, schur_prec=addns.F32,
                                 block_sizing=args.block_sizing, sweep_chunks=args.sweep_chunks,
                                 block_mult=args.block_mult, coarse=args.coarse)
        torch.cuda.synchronize()
        tm = time.perf_counter()
        d_x.zero_()
        res, code = addns.gmres_solve_batched(pc, offs, d_b, d_x, restart=50, maxit=20000, tol=1e-8)
        torch.cuda.synchronize()
        split.append((tm - ts, time.perf_counter() - tm))
        return pc, res

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    split.clear()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pc, res = step()
    torch.cuda.synchronize()
    T = (time.perf_counter() - t0) / max(args.steps, 1)
    its = [r["iters"] for r in res]
    # the same systems one at a time
    t1 = time.perf_counter()
    seq_its = []
    for w, bd, p in zip(wls, built, parts):
        n = bd[4]["N"]
        pcs = addns.setup_precond(p, n, *(torch.from_numpy(a).to(dev) for a in (bd[0], bd[1], bd[2])),
                                  interior_prec=addns.F32, schur_prec=addns.F32, block_mult=args.block_mult,
                                  coarse=args.coarse)
        xs = torch.zeros(n, dtype=torch.float64, device=dev)
        r = addns.gmres_solve(pcs, torch.from_numpy(bd[3]).to(dev), xs, restart=50, maxit=20000, tol=1e-8,
                              ortho="mgs")
        seq_its.append(r["iters"])
    torch.cuda.synchronize()
    T_seq = time.perf_counter() - t1
    info = pc.info()
    print(json.dumps({
        "metric": "time to 1e-8 rel. residual (s), 96 independent systems", "value": round(T, 4),
        "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(T * 1e3, 2), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 outer / f32 factors", "data": "synthetic",
        "config": {"workload": "batched96", "systems": len(wls), "N_total": N,
                   "subdomains_total": int(sum(w.m for w in wls)), "krylov": "FGMRES(50)", "ortho": "mgs",
                   "coarse_piece": args.coarse, "block_mult": info["block_mult"],
                   "sweep_chunks": info["sweep_chunks"]},
        "setup_s": round(float(np.median([x[0] for x in split])), 4),
        "solve_s": round(float(np.median([x[1] for x in split])), 4),
        "converged": int(sum(r["converged"] for r in res)), "iters_max": max(its),
        "iters_median": float(np.median(its)), "sequential_same_library_s": round(T_seq, 3),
        "sequential_iters_max": max(seq_its), "speedup_vs_sequential": round(T_seq / T, 2)}))


def bench_picard(args):
    """Steady Navier-Stokes by the Picard outer loop of section 1 on the
    128 x 128 lid-driven cavity (nu = 1/100, lid only, 16 subdomains): host
    assembly of each Oseen system, refactor on the first step's plan, FGMRES
    from the previous iterate, to a row-scaled residual of 1e-8; FP32 factors
    against FP64 factors, and with overlapped aggregates."""
    import torch

    from paper_1104_3349_amd import addns, picard

    torch.cuda.set_device(0)
    runs = {}
    for name, kw in (("f32", dict()), ("f64", dict(interior_prec=addns.F64, schur_prec=addns.F64)),
                     ("f32_omscn", dict(overlap=63))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = picard.solve(128, 0.01, m=16, sz=64, tol=1e-8, maxit=40, **kw)
        torch.cuda.synchronize()
        r.pop("x")
        r["total_s"] = round(time.perf_counter() - t0, 4)
        for key in ("assemble_s", "setup_s", "refactor_s", "solve_s"):
            r[key] = round(r[key], 4)
        r["final_residual"] = r["residuals"][-1]
        r["residuals"] = [float("%.3e" % x) for x in r["residuals"]]
        runs[name] = r
    main_run = runs["f32"]
    print(json.dumps({
        "metric": "time to 1e-8 rel. residual (s) + precond-apply GB/s; plain FP64 vs mixed/learned",
        "value": main_run["total_s"] if main_run["converged"] else None, "unit": "s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(main_run["total_s"] * 1e3, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 outer / f32 factors", "data": "synthetic",
        "config": {"workload": "picard128", "grid": "128x128 MAC lid-driven cavity", "nu": 0.01,
                   "subdomains": 16, "aggregate_size": 64, "krylov": "FGMRES(50), warm start",
                   "outer": "Picard to row-scaled NS residual 1e-8"},
        "runs": runs}))


# Network arithmetic per sample: 7 -> 64 -> 64 -> 5 multiply-adds, forward;
# the backward pass costs twice the forward (input and weight gradients).
MLP_FWD_FLOP = 2 * (7 * 64 + 64 * 64 + 64 * 5)


def network_timing(addns, torch, X, Y, M, w, reps):
    """Whole-call medians of the network entry points over every training
    row: the BF16 and FP32 forward passes and the full-data gradient (each
    call also uploads the weights and synchronises)."""
    import numpy as np
    n = int(X.shape[0])
    P = torch.empty((n, 5), dtype=torch.float32, device=X.device)
    out = {"rows": n, "fwd_flop_per_row": MLP_FWD_FLOP}
    for name, fn in (("forward_bf16", lambda: addns.dtn_forward(w, X, P, bf16=True)),
                     ("forward_f32", lambda: addns.dtn_forward(w, X, P, bf16=False)),
                     ("gradient_f32", lambda: addns.dtn_grad(w, X, Y, M))):
        fn()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        ms = float(np.median(ts)) * 1e3
        flop = MLP_FWD_FLOP * (3 if name.startswith("gradient") else 1) * n
        out[name] = {"call_ms": round(ms, 4), "rows_per_s": round(n / ms * 1e3),
                     "tflops": round(flop / ms / 1e9, 3)}
    return out


def bench_learned(args):
    """Learned interface correction: samples from 2000 seeded 64 x 64 systems
    (MSCN teacher), GPU training, then the judged FGMRES(50) on the 512 x 512
    stretched cavity (nu = 1/500, 256 subdomains) against plain MSCN, and
    on a held-out 64 x 64 system of the training distribution's kind."""
    import numpy as np
    import torch

    from paper_1104_3349_amd import addns, learned
    from workloads.configs import CAVITY512_STRETCHED, F32, Workload, training_workloads

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    nsys, epochs = (200, 3) if args.mlp_profile else (2000, 30)
    X, Y, M = learned.collect_samples(training_workloads(nsys), 100)
    t1 = time.perf_counter()
    w, loss = addns.dtn_train(X, Y, M, epochs=epochs, batch=1024, lr=2e-3, seed=0)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    net = network_timing(addns, torch, X, Y, M, w, reps=args.reps if args.mlp_profile else 5)
    if args.mlp_profile:
        print(json.dumps({"mlp_profile": True, "rows": int(X.shape[0]), "train_s": round(t2 - t1, 3),
                          "network": net}))
        return
    held = Workload("uniform64_nu0.002_m4_heldout", 64, 1 / 500, None, 4, 64, 50, True, 1e-8, 78, F32, F32)
    out = {}
    for wl, maxit in ((held, 5000), (CAVITY512_STRETCHED, args.learned_maxit)):
        rp, ci, v, b, meta = wl.build()
        N = meta["N"]
        part = addns.build_partition(N, rp, ci, v, wl.m, wl.sz)
        d = [torch.from_numpy(a).to(dev) for a in (rp, ci, v)]
        d_b = torch.from_numpy(b).to(dev)
        d_x = torch.zeros(N, dtype=torch.float64, device=dev)
        res = {}
        plain = None
        for name, kw in (("mscn", dict(schur=addns.SCHUR_MSCN)), ("lum", dict(schur=addns.SCHUR_LUM)),
                         ("mscnr", dict(schur=addns.SCHUR_MSCNR)),
                         ("learned_bf16", dict(schur=addns.SCHUR_LEARNED, learned_model=w,
                                               learned_bf16=True))):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            try:
                pc = addns.setup_precond(part, N, *d, interior_prec=F32, schur_prec=F32, block_mult=1, **kw)
            except addns.AddnsError as e:  # e.g. numerically singular interface blocks
                res[name] = {"setup_error": str(e)}
                continue
            if name == "mscn":
                plain = pc
            d_x.zero_()
            if name == "learned_bf16" and plain is not None:
                r = addns.gmres_solve_judged(pc, plain, d_b, d_x, restart=wl.restart, maxit=maxit, tol=wl.tol)
            else:
                r = addns.gmres_solve(pc, d_b, d_x, restart=wl.restart, maxit=maxit, tol=wl.tol)
            torch.cuda.synchronize()
            res[name] = {"seconds": round(time.perf_counter() - ts, 4), "iters": r["iters"],
                         "converged": r["converged"], "true_relres": r["true_relres"]}
            if "accepted" in r:
                res[name]["accepted"] = r["accepted"]
        out[wl.name] = res
    e = out[CAVITY512_STRETCHED.name]["learned_bf16"]
    if "seconds" not in e:
        e = {"seconds": None}
    print(json.dumps({
        "metric": "time to 1e-8 rel. residual (s) + precond-apply GB/s; plain FP64 vs mixed/learned",
        "value": e["seconds"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": None if e["seconds"] is None else round(e["seconds"] * 1e3, 3),
        "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 outer / f32 factors / bf16 network", "data": "synthetic",
        "config": {"workload": "learned512", "eval": CAVITY512_STRETCHED.name, "train_systems": 2000,
                   "train_rows": int(X.shape[0]), "krylov": "FGMRES(50)", "maxit": args.learned_maxit},
        "data_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2), "network": net,
        "loss_first": float(loss[0]), "loss_last": float(loss[-1]), "results": out}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--coarse", type=int, default=32, help="coarse-correction piece size (0 = none)")
    ap.add_argument("--ortho", default="cgs2", choices=["cgs2", "mgs"])
    ap.add_argument("--no-large", action="store_true", help="skip the 512 x 512 stretched measurements")
    ap.add_argument("--large-maxit", type=int, default=300)
    ap.add_argument("--profile-workload", default="cavity128", choices=["cavity128", "cavity512s"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the MSCNR/LUM/overlapped solves")
    ap.add_argument("--sweep-chunks", type=int, default=0,
                    help="chunks per interior of the interior sweep (0 = the library's choice)")
    ap.add_argument("--kernel-profile", action="store_true",
                    help="only the dominant kernel (interior solve) x reps, plus a 256 MiB device "
                         "copy of known size to calibrate memory counters")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--profile-overlap", type=int, default=0,
                    help="with --kernel-profile: also run reps applies with overlapped aggregates of this "
                         "width (OMSCN), for the share of the chain kernels in the apply")
    ap.add_argument("--block-sizing", type=int, default=0, choices=[0, 1, 2],
                    help="sweep block sizes: 0 = the library's rule, 1 = one for all, 2 = per interior")
    ap.add_argument("--workload", default="cavity128",
                    choices=["cavity128", "batched96", "learned512", "picard128"],
                    help="cavity128: the headline single system; batched96: 96 independent "
                         "systems solved together; learned512: train the interface network and "
                         "judge it on the 512 x 512 stretched cavity (both reported separately)")
    ap.add_argument("--learned-maxit", type=int, default=1000)
    ap.add_argument("--mlp-profile", action="store_true",
                    help="learned512 only: samples from 200 systems, 3 epochs, then the network "
                         "kernels x reps (for a kernel trace or counters)")
    ap.add_argument("--block-mult", type=int, default=None,
                    help="sweep tile multiplier (0 is taken as 1)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the multi-GPU path is a design, not a build "
              "(every box here has one GPU)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1104_3349_amd import addns
    from workloads.configs import CAVITY128 as cfg

    if args.workload == "picard128":
        return bench_picard(args)
    if args.workload == "learned512":
        return bench_learned(args)
    if args.workload == "batched96":
        if args.block_mult is None:
            args.block_mult = 0
        return bench_batched(args)
    if args.block_mult is None:
        args.block_mult = 1

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rp, ci, v, b, meta = cfg.build()
    N = meta["N"]
    part = addns.build_partition(N, rp, ci, v, cfg.m, cfg.sz)
    d_rp, d_ci, d_v = (torch.from_numpy(a).to(dev) for a in (rp, ci, v))
    d_b = torch.from_numpy(b).to(dev)
    d_x = torch.zeros(N, dtype=torch.float64, device=dev)
    maxit = 20000

    def step(iprec, sprec, schur=addns.SCHUR_MSCN, overlap=0, ilu_tol=0.0, coarse=None, ortho=None):
        coarse = args.coarse if coarse is None else coarse
        ortho = args.ortho if ortho is None else ortho
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pc = addns.setup_precond(part, N, d_rp, d_ci, d_v, schur=schur, interior_prec=iprec, schur_prec=sprec,
                                 block_sizing=args.block_sizing,
                                 block_mult=args.block_mult, overlap=overlap, ilu_tol=ilu_tol,
                                 sweep_chunks=args.sweep_chunks, coarse=coarse)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        d_x.zero_()
        r = addns.gmres_solve(pc, d_b, d_x, restart=cfg.restart, maxit=maxit, tol=cfg.tol,
                              flexible=cfg.flexible, ortho=ortho)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return pc, r, (t2 - t0, t1 - t0, t2 - t1)

    def timed(steps, warmup, **kw):
        """Median over `steps` timed steps after `warmup` untimed ones."""
        for _ in range(warmup):
            step(**kw)
        ts, last = [], None
        for _ in range(steps):
            pc, r, t = step(**kw)
            ts.append(t)
            last = (pc, r)
        ts = np.array(ts)
        return last[0], last[1], {"seconds": round(float(np.median(ts[:, 0])), 5),
                                  "setup_s": round(float(np.median(ts[:, 1])), 5),
                                  "solve_s": round(float(np.median(ts[:, 2])), 5),
                                  "iters": last[1]["iters"], "true_relres": last[1]["true_relres"],
                                  "converged": bool(last[1]["converged"])}

    iprec, sprec = addns.F32, addns.F32
    if args.kernel_profile:
        wl = cfg
        if args.profile_workload == "cavity512s":
            from workloads.configs import CAVITY512_STRETCHED as wl
            rp, ci, v, b, meta = wl.build()
            N = meta["N"]
            part = addns.build_partition(N, rp, ci, v, wl.m, wl.sz)
            d_rp, d_ci, d_v = (torch.from_numpy(a).to(dev) for a in (rp, ci, v))
        pc = addns.setup_precond(part, N, d_rp, d_ci, d_v, interior_prec=iprec, schur_prec=sprec,
                                 block_sizing=args.block_sizing,
                                 block_mult=args.block_mult, sweep_chunks=args.sweep_chunks)
        n_int = int(part.info()["n_interior"])
        d_y1 = torch.randn(n_int, dtype=torch.float64, device=dev)
        d_z1 = torch.empty_like(d_y1)
        for _ in range(args.reps):
            addns.interior_solve(pc, d_y1, d_z1)
        if args.profile_overlap > 0:
            # the chain in segments (the default), then as one chain
            d_y = torch.randn(N, dtype=torch.float64, device=dev)
            d_o = torch.empty_like(d_y)
            for seg in (0, 1 << 30):
                po = addns.setup_precond(part, N, d_rp, d_ci, d_v, interior_prec=iprec, schur_prec=sprec,
                                         block_mult=args.block_mult, overlap=args.profile_overlap,
                                         overlap_segment=seg)
                for _ in range(args.reps):
                    addns.apply_precond(po, d_y, d_o)
                del po
        src = torch.ones(256 * 2 ** 20 // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        info = pc.info()
        print(json.dumps({"kernel_profile": True, "workload": wl.name, "reps": args.reps,
                          "copy_bytes": 256 * 2 ** 20,
                          "interior_bytes_method": info["band_words"] * 4 + 20 * n_int,
                          "chunk_bytes": info["chunk_bytes"], "factor_bytes": info["factor_bytes"],
                          "sweep_chunks": info["sweep_chunks"]}))
        return

    def interior_roofline(pc, part, sf, reps=100):
        """HIP-event median of `reps` interior solves on the current stream and
        the method's bytes per solve: band factors L (kl_j) and U (kl_j + ku_j
        + 1) per row of interior j, pivots, the vector in and out.  The chunked sweep's
        response matrices are reported beside them as overhead."""
        info = pc.info()
        n_int = int(part.info()["n_interior"])
        d_y1 = torch.randn(n_int, dtype=torch.float64, device=dev)
        d_z1 = torch.empty_like(d_y1)
        t = _events_median_ms(lambda: addns.interior_solve(pc, d_y1, d_z1), reps, torch)
        b_int = info["band_words"] * sf + 4 * n_int + 16 * n_int
        kern = "k_chunk_lower + k_chunk_upper + k_chunk_fix" if info["sweep_chunks"] > 1 else "k_interior_solve"
        ach = b_int / (t * 1e-3)
        return {"bound": "hbm", "kernel": kern, "achieved": round(ach / 1e9, 2), "peak": PEAK / 1e9,
                "unit": "GB/s", "frac": round(ach / PEAK, 4), "traffic": None, "launch_ms": round(t, 4),
                "bytes_per_launch": int(b_int), "overhead_bytes_per_launch": int(info["chunk_bytes"])}

    def apply_bw(pc, n, reps=100):
        info = pc.info()
        d_y = torch.randn(n, dtype=torch.float64, device=dev)
        d_o = torch.empty_like(d_y)
        t = _events_median_ms(lambda: addns.apply_precond(pc, d_y, d_o), reps, torch)
        # method bytes of one apply: the chunked sweep's response matrices
        # (read twice, once per interior solve) are reported as overhead
        mb = info["bytes_apply"] - 2 * info["chunk_bytes"]
        return {"apply_ms": round(t, 4), "apply_GBps": round(mb / (t * 1e-3) / 1e9, 2),
                "apply_frac_hbm": round(mb / (t * 1e-3) / PEAK, 4),
                "bytes_apply": int(mb), "chunk_overhead_bytes": 2 * int(info["chunk_bytes"])}

    # a first setup on a fresh partition handle: includes the host planning
    # (gather maps, sweep geometry, coarse-space structure) that later setups
    # on the same partition reuse
    part_fresh = addns.build_partition(N, rp, ci, v, cfg.m, cfg.sz)
    torch.cuda.synchronize()
    t_cold = time.perf_counter()
    pc_cold = addns.setup_precond(part_fresh, N, d_rp, d_ci, d_v, interior_prec=iprec, schur_prec=sprec,
                                  block_sizing=args.block_sizing,
                                  block_mult=args.block_mult, sweep_chunks=args.sweep_chunks, coarse=args.coarse)
    torch.cuda.synchronize()
    first_setup_s = time.perf_counter() - t_cold
    del pc_cold
    pc, r, main_t = timed(args.steps, args.warmup, iprec=iprec, sprec=sprec)
    info = pc.info()
    sf = 4 if iprec == addns.F32 else 8
    roof = interior_roofline(pc, part, sf)
    roof["traffic"] = measured_traffic()
    bw = apply_bw(pc, N)
    nnz_pre, nnz_c = pc.fill()

    legs = {}
    if not args.no_plain:
        # the plain path: FP64 factors, the paper's one-level interface solve
        for name, kw in (("plain_f64_cgs2", dict(iprec=addns.F64, sprec=addns.F64, coarse=0, ortho="cgs2")),
                         ("plain_f64_mgs", dict(iprec=addns.F64, sprec=addns.F64, coarse=0, ortho="mgs")),
                         ("mixed_f32_one_level", dict(iprec=addns.F32, sprec=addns.F32, coarse=0)),
                         ("f64_coarse", dict(iprec=addns.F64, sprec=addns.F64)),
                         ("mixed_f32_coarse_mgs", dict(iprec=addns.F32, sprec=addns.F32, ortho="mgs"))):
            _, _, legs[name] = timed(args.plain_steps, 1, **kw)

    forms = None
    if not args.no_forms:
        forms = {}
        for name, kw in (("mscnr", dict(schur=addns.SCHUR_MSCNR, coarse=0)),
                         ("lum", dict(schur=addns.SCHUR_LUM, coarse=0)),
                         ("omscn", dict(overlap=cfg.sz - 1, coarse=0)),
                         ("omscnr", dict(schur=addns.SCHUR_MSCNR, overlap=cfg.sz - 1, coarse=0)),
                         ("mscn_ilu1e-4", dict(ilu_tol=1e-4, coarse=0)),
                         ("mscn_ilu1e-4_coarse", dict(ilu_tol=1e-4))):
            pcf, rf, tf = step(iprec, sprec, **kw)
            forms[name] = {"seconds": round(tf[0], 4), "iters": rf["iters"], "converged": rf["converged"]}
            if "ilu_tol" in kw:
                forms[name]["interior_fill"] = round(pcf.info()["interior_nnz"] / len(v), 2)

    big = None
    if not args.no_large:
        big = bench_large(args, addns, torch, dev)

    plain_s = legs.get("plain_f64_cgs2", {}).get("seconds")
    line = {
        "metric": "time to 1e-8 rel. residual (s) + precond-apply GB/s; plain FP64 vs mixed/learned",
        "value": main_t["seconds"], "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(main_t["seconds"] * 1e3, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 outer / f32 factors", "data": "synthetic",
        "config": {"workload": cfg.name, "N": N, "nnz": int(len(v)), "subdomains": cfg.m,
                   "aggregate_size": cfg.sz, "krylov": f"FGMRES({cfg.restart})", "tol": cfg.tol,
                   "factors": "f32/f32", "ortho": args.ortho, "coarse_piece": args.coarse,
                   "sweep_chunks": info["sweep_chunks"], "block_mult": info["block_mult"]},
        "setup_s": main_t["setup_s"], "solve_s": main_t["solve_s"],
        "first_setup_s": round(first_setup_s, 5),
        "iters": r["iters"], "converged": r["converged"], "true_relres": r["true_relres"],
        **bw,
        "fill_factor": round(nnz_pre / nnz_c, 3),
        "interior_fill": round(info["interior_nnz"] / len(v), 2),
        "legs": legs,
        "speedup_vs_plain_f64": round(plain_s / main_t["seconds"], 2) if plain_s else None,
        "interface_forms": forms,
        "cavity512_stretched": big,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, args.coarse, args.ortho)
    print(json.dumps(line))


def bench_large(args, addns, torch, dev):
    """The 512 x 512 stretched workload (785 407 unknowns, 256 subdomains):
    setup, apply bandwidth and the interior solve's roofline with FP32
    factors (the factors, 1.8 GB, exceed the 256 MB last-level cache), and
    FGMRES(50) for a bounded number of iterations, one-level and with the
    coarse correction."""
    import numpy as np

    from workloads.configs import CAVITY512_STRETCHED as wl

    t0 = time.perf_counter()
    rp, ci, v, b, meta = wl.build()
    N = meta["N"]
    part = addns.build_partition(N, rp, ci, v, wl.m, wl.sz)
    t_part = time.perf_counter() - t0
    d_rp, d_ci, d_v = (torch.from_numpy(a).to(dev) for a in (rp, ci, v))
    d_b = torch.from_numpy(b).to(dev)
    out = {"workload": wl.name, "N": N, "subdomains": wl.m, "host_build_and_partition_s": round(t_part, 2)}
    for name, coarse in (("one_level", 0), ("coarse", args.coarse)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pc = addns.setup_precond(part, N, d_rp, d_ci, d_v, interior_prec=addns.F32, schur_prec=addns.F32,
                                 block_sizing=args.block_sizing,
                                 block_mult=1, coarse=coarse)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t1
        info = pc.info()
        n_int = int(part.info()["n_interior"])
        d_y1 = torch.randn(n_int, dtype=torch.float64, device=dev)
        d_z1 = torch.empty_like(d_y1)
        t_int = _events_median_ms(lambda: addns.interior_solve(pc, d_y1, d_z1), 100, torch)
        b_int = info["band_words"] * 4 + 20 * n_int
        d_y = torch.randn(N, dtype=torch.float64, device=dev)
        d_o = torch.empty_like(d_y)
        t_app = _events_median_ms(lambda: addns.apply_precond(pc, d_y, d_o), 100, torch)
        d_x = torch.zeros(N, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        r = addns.gmres_solve(pc, d_b, d_x, restart=wl.restart, maxit=args.large_maxit, tol=wl.tol,
                              flexible=True, ortho=args.ortho)
        torch.cuda.synchronize()
        out[name] = {"setup_s": round(t_setup, 4), "solve_s": round(time.perf_counter() - t2, 4),
                     "iters": r["iters"], "converged": r["converged"], "true_relres": r["true_relres"],
                     "apply_ms": round(t_app, 4),
                     "apply_GBps": round(info["bytes_apply"] / (t_app * 1e-3) / 1e9, 2),
                     "apply_frac_hbm": round(info["bytes_apply"] / (t_app * 1e-3) / PEAK, 4),
                     "interior_solve": {"kernel": "k_chunk_lower + k_chunk_upper + k_chunk_fix"
                                        if info["sweep_chunks"] > 1 else "k_interior_solve",
                                        "launch_ms": round(t_int, 4), "bytes_per_launch": int(b_int),
                                        "achieved_GBps": round(b_int / (t_int * 1e-3) / 1e9, 2),
                                        "frac": round(b_int / (t_int * 1e-3) / PEAK, 4),
                                        "traffic": measured_traffic("cavity512s")},
                     "sweep_chunks": info["sweep_chunks"], "factor_bytes": int(info["factor_bytes"])}
        del pc
    return out


if __name__ == "__main__":
    main()

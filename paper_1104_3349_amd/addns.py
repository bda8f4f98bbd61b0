"""Thin ctypes binding of libaddns (argument marshalling only).

Every function here has the name of the C entry point it wraps, minus the
``addns_`` prefix.  No arithmetic of the method happens in Python: host
arrays are passed as numpy buffers, device arrays as torch CUDA tensors
(their data pointers), streams as torch.cuda.Stream handles.  If the shared
library is missing the import fails loudly; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libaddns.so")

OK, WARN_SHARED_PAIR = 0, 1
ERR_ARG, ERR_SINGULAR, ERR_NOCONV, ERR_HIP, ERR_PARTITION, ERR_NOMEM = -1, -2, -3, -4, -5, -6
SCHUR_MSCN, SCHUR_MSCN_LITERAL, SCHUR_LUM, SCHUR_EXACT_BJ, SCHUR_LEARNED, SCHUR_MSCNR = 0, 1, 2, 3, 4, 5
F64, F32, F16_SCALED = 0, 1, 2

EXPORTED = [
    "addns_build_partition", "addns_partition_info", "addns_partition_export",
    "addns_partition_concat", "addns_partition_coarse_space", "addns_gmres_solve_batched",
    "addns_setup_precond", "addns_apply_precond", "addns_apply_precond_static", "addns_interior_solve", "addns_gmres_solve", "addns_precond_info",
    "addns_precond_schur_blocks", "addns_precond_fill", "addns_partition_destroy", "addns_precond_destroy",
    "addns_last_error", "addns_version",
    "addns_dtn_param_count", "addns_dtn_samples", "addns_dtn_forward", "addns_dtn_grad",
    "addns_dtn_train", "addns_dtn_save", "addns_dtn_load", "addns_gmres_solve_judged",
    "addns_precond_refactor", "addns_release_cached_memory",
]


class AddnsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libaddns error {code}: {msg}")
        self.code = code


class PrecondOpts(C.Structure):
    _fields_ = [("schur", C.c_int32), ("interior_prec", C.c_int32), ("schur_prec", C.c_int32),
                ("row_scale", C.c_int32), ("learned_model", C.POINTER(C.c_float)),
                ("block_mult", C.c_int32), ("learned_bf16", C.c_int32), ("overlap", C.c_int32),
                ("ilu_tol", C.c_double), ("sweep_chunks", C.c_int32), ("coarse", C.c_int32),
                ("sweep_zero_skip", C.c_int32), ("block_sizing", C.c_int32), ("overlap_segment", C.c_int32)]


class GmresOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("maxit", C.c_int32), ("tol", C.c_double),
                ("flexible", C.c_int32), ("use_x0", C.c_int32), ("ortho", C.c_int32)]


class DtnParams(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("seed", C.c_int64), ("init_given", C.c_int32)]


class GmresResult(C.Structure):
    _fields_ = [("iters", C.c_int32), ("cycles", C.c_int32), ("converged", C.c_int32),
                ("true_relres", C.c_double), ("est_relres", C.c_double),
                ("resid_hist", C.POINTER(C.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libaddns.so not built at {LIB_PATH}; run "
                          "`python -m paper_1104_3349_amd.build`")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    i32p, f64p, i64p = C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_int64)
    sig = {
        "addns_build_partition": (C.c_int, [C.c_int32, P, P, P, C.c_int32, C.c_int32, C.POINTER(P)]),
        "addns_partition_info": (C.c_int, [P, i32p, i32p, i32p, i32p, i32p, i32p]),
        "addns_partition_export": (C.c_int, [P, P, P, P, P, P, P, P]),
        "addns_partition_concat": (C.c_int, [C.POINTER(P), C.c_int32, C.POINTER(P)]),
        "addns_partition_coarse_space": (C.c_int, [P, C.c_int32, i32p, i32p, P, P, P, P, P, P]),
        "addns_gmres_solve_batched": (C.c_int, [P, C.c_int32, P, P, P, C.POINTER(GmresOpts),
                                                C.POINTER(GmresResult), P]),
        "addns_setup_precond": (C.c_int, [P, C.c_int32, P, P, P, C.POINTER(PrecondOpts), P,
                                          C.POINTER(P)]),
        "addns_apply_precond": (C.c_int, [P, P, P, P]),
        "addns_apply_precond_static": (C.c_int, [P, P, P, P]),
        "addns_precond_refactor": (C.c_int, [P, P, P, P, P]),
        "addns_interior_solve": (C.c_int, [P, P, P, P]),
        "addns_gmres_solve": (C.c_int, [P, P, P, C.POINTER(GmresOpts), C.POINTER(GmresResult), P]),
        "addns_precond_info": (C.c_int, [P, i32p, i32p, i32p, i32p, i64p, i64p, i64p, i32p, i64p, i32p, i64p, i64p]),
        "addns_precond_schur_blocks": (C.c_int, [P, P, C.c_int64]),
        "addns_precond_fill": (C.c_int, [P, i64p, i64p]),
        "addns_partition_destroy": (None, [P]),
        "addns_precond_destroy": (None, [P]),
        "addns_release_cached_memory": (C.c_int64, []),
        "addns_last_error": (C.c_char_p, []),
        "addns_version": (C.c_char_p, []),
        "addns_dtn_param_count": (C.c_int, []),
        "addns_dtn_samples": (C.c_int, [P, P, P, P, C.c_int64, i64p, P]),
        "addns_dtn_forward": (C.c_int, [P, P, P, C.c_int64, C.c_int32, P]),
        "addns_dtn_grad": (C.c_int, [P, P, P, P, C.c_int64, P, f64p, P]),
        "addns_dtn_train": (C.c_int, [P, P, P, C.c_int64, C.POINTER(DtnParams), P, P, P]),
        "addns_dtn_save": (C.c_int, [C.c_char_p, P]),
        "addns_dtn_load": (C.c_int, [C.c_char_p, P]),
        "addns_gmres_solve_judged": (C.c_int, [P, P, P, P, C.POINTER(GmresOpts), C.POINTER(GmresResult),
                                               i32p, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(code, what):
    if code < 0:
        raise AddnsError(code, f"{what}: {lib().addns_last_error().decode()}")
    return code


def _ptr(a):
    """Data pointer of a numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags.c_contiguous
        return a.ctypes.data
    assert a.is_contiguous()
    return a.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return s.cuda_stream if hasattr(s, "cuda_stream") else s


# --------------------------------------------------------------------------
# partitions
# --------------------------------------------------------------------------

@dataclass
class PartitionArrays:
    perm: np.ndarray
    part: np.ndarray
    int_offsets: np.ndarray
    agg_offsets: np.ndarray
    drange_offsets: np.ndarray
    drange_nodes: np.ndarray
    pair: np.ndarray
    status: int


class Partition:
    def __init__(self, handle, status):
        self.handle = handle
        self.status = status

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.addns_partition_destroy(self.handle)
            self.handle = None

    def info(self):
        v = [C.c_int32() for _ in range(6)]
        _check(lib().addns_partition_info(self.handle, *[C.byref(x) for x in v]), "partition_info")
        return dict(zip(("N", "m", "n_interior", "sep_size", "k", "drange_total"),
                        (x.value for x in v)))

    def export(self) -> PartitionArrays:
        inf = self.info()
        N, m, k = inf["N"], inf["m"], inf["k"]
        arr = dict(perm=np.empty(N, np.int32), part=np.empty(N, np.int32),
                   int_offsets=np.empty(m + 1, np.int32), agg_offsets=np.empty(k + 1, np.int32),
                   drange_offsets=np.empty(k + 1, np.int32),
                   drange_nodes=np.empty(inf["drange_total"], np.int32),
                   pair=np.empty(inf["sep_size"], np.int32))
        _check(lib().addns_partition_export(self.handle, *[_ptr(arr[n]) for n in (
            "perm", "part", "int_offsets", "agg_offsets", "drange_offsets", "drange_nodes",
            "pair")]), "partition_export")
        return PartitionArrays(status=self.status, **arr)

    def coarse_space(self, piece):
        """The coarse space of opts.coarse = piece: (piece_offsets, piece_pos,
        col_piece, col_kind, z0, z1), see addns_partition_coarse_space."""
        npc, nc = C.c_int32(), C.c_int32()
        _check(lib().addns_partition_coarse_space(self.handle, int(piece), C.byref(npc), C.byref(nc),
                                                  None, None, None, None, None, None), "partition_coarse_space")
        inf = self.info()
        ns = inf["sep_size"]
        offs = np.empty(npc.value + 1, np.int32)
        _check(lib().addns_partition_coarse_space(self.handle, int(piece), None, None, _ptr(offs), None, None,
                                                  None, None, None), "partition_coarse_space")
        arr = dict(piece_offsets=offs, piece_pos=np.empty(int(offs[-1]), np.int32),
                   col_piece=np.empty(nc.value, np.int32), col_kind=np.empty(nc.value, np.int32),
                   z0=np.empty(ns, np.float64), z1=np.empty(ns, np.float64))
        _check(lib().addns_partition_coarse_space(self.handle, int(piece), None, None, _ptr(offs),
                                                  *[_ptr(arr[n]) for n in ("piece_pos", "col_piece", "col_kind",
                                                                           "z0", "z1")]),
               "partition_coarse_space")
        return arr


def build_partition(N, rowptr, colidx, vals, m, sz) -> Partition:
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    h = C.c_void_p()
    st = _check(lib().addns_build_partition(int(N), _ptr(rowptr), _ptr(colidx), _ptr(vals),
                                            int(m), int(sz), C.byref(h)), "build_partition")
    return Partition(h, st)


class ConcatPartition(Partition):
    def __init__(self, handle, status, parts):
        super().__init__(handle, status)
        self.parts = parts  # keep the inputs alive with the concatenation


def partition_concat(parts) -> Partition:
    arr = (C.c_void_p * len(parts))(*[p.handle for p in parts])
    h = C.c_void_p()
    _check(lib().addns_partition_concat(arr, len(parts), C.byref(h)), "partition_concat")
    return ConcatPartition(h, max(p.status for p in parts), list(parts))


# --------------------------------------------------------------------------
# preconditioner and solver
# --------------------------------------------------------------------------

class Precond:
    def __init__(self, handle, partition):
        self.handle = handle
        self.partition = partition  # keep alive

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.addns_precond_destroy(self.handle)
            self.handle = None

    def info(self):
        i32 = [C.c_int32() for _ in range(4)]
        i64 = [C.c_int64() for _ in range(3)]
        bm = C.c_int32()
        nz = C.c_int64()
        ch = C.c_int32()
        cb = C.c_int64()
        bw = C.c_int64()
        _check(lib().addns_precond_info(self.handle, *[C.byref(x) for x in i32 + i64], C.byref(bm),
                                        C.byref(nz), C.byref(ch), C.byref(cb), C.byref(bw)), "precond_info")
        d = dict(zip(("kl", "ku", "nb_lower", "nb_upper", "factor_bytes", "bytes_apply",
                      "learned_count"), (x.value for x in i32 + i64)))
        d["block_mult"] = bm.value
        d["interior_nnz"] = nz.value
        d["sweep_chunks"] = ch.value
        d["chunk_bytes"] = cb.value
        d["band_words"] = bw.value
        return d

    def fill(self):
        """(nnz of the preconditioner, nnz of C): the fill factor of section 5
        is their ratio (addns_precond_fill)."""
        a, b = C.c_int64(), C.c_int64()
        _check(lib().addns_precond_fill(self.handle, C.byref(a), C.byref(b)), "precond_fill")
        return a.value, b.value

    def schur_blocks(self, count):
        out = np.empty(int(count), np.float64)
        _check(lib().addns_precond_schur_blocks(self.handle, _ptr(out), int(count)),
               "precond_schur_blocks")
        return out


def setup_precond(partition: Partition, N, d_rowptr, d_colidx, d_vals, schur=SCHUR_MSCN,
                  interior_prec=F64, schur_prec=F64, row_scale=1, learned_model=None,
                  block_mult=1, learned_bf16=True, overlap=0, ilu_tol=0.0, sweep_chunks=0,
                  coarse=0, sweep_zero_skip=0, block_sizing=0, overlap_segment=0, stream=None) -> Precond:
    opts = PrecondOpts(int(schur), int(interior_prec), int(schur_prec), int(row_scale), None,
                       int(block_mult), int(bool(learned_bf16)), int(overlap), float(ilu_tol),
                       int(sweep_chunks), int(coarse), int(sweep_zero_skip), int(block_sizing),
                       int(overlap_segment))
    if learned_model is not None:
        lm = np.ascontiguousarray(learned_model, dtype=np.float32)
        opts.learned_model = lm.ctypes.data_as(C.POINTER(C.c_float))
    h = C.c_void_p()
    _check(lib().addns_setup_precond(partition.handle, int(N), _ptr(d_rowptr), _ptr(d_colidx),
                                     _ptr(d_vals), C.byref(opts), _stream(stream), C.byref(h)),
           "setup_precond")
    return Precond(h, partition)


def refactor_precond(pc: Precond, d_rowptr, d_colidx, d_vals, stream=None):
    """New values on the setup's pattern: every numeric part of the setup is
    recomputed on the handle's plan (addns_precond_refactor)."""
    _check(lib().addns_precond_refactor(pc.handle, _ptr(d_rowptr), _ptr(d_colidx), _ptr(d_vals),
                                        _stream(stream)), "precond_refactor")


def apply_precond(pc: Precond, d_y, d_x, stream=None):
    _check(lib().addns_apply_precond(pc.handle, _ptr(d_y), _ptr(d_x), _stream(stream)),
           "apply_precond")


def apply_precond_static(pc: Precond, d_y, d_x, stream=None):
    """addns_apply_precond_static: the apply with its work vectors in the
    library's static device array (no allocation)."""
    _check(lib().addns_apply_precond_static(pc.handle, _ptr(d_y), _ptr(d_x), _stream(stream)),
           "apply_precond_static")


def interior_solve(pc: Precond, d_y1, d_z1, stream=None):
    _check(lib().addns_interior_solve(pc.handle, _ptr(d_y1), _ptr(d_z1), _stream(stream)),
           "interior_solve")


ORTHO_MGS, ORTHO_CGS2 = 0, 1
_ORTHO = {"mgs": ORTHO_MGS, "cgs2": ORTHO_CGS2}


def _ortho(o):
    """'mgs' / 'cgs2' or the integer code (passed through: the library checks it)."""
    return _ORTHO[o] if isinstance(o, str) else int(o)


def gmres_solve(pc: Precond, d_b, d_x, restart=50, maxit=1000, tol=1e-8, flexible=True,
                use_x0=False, history=False, stream=None, raise_noconv=False, ortho="cgs2"):
    opts = GmresOpts(int(restart), int(maxit), float(tol), int(bool(flexible)), int(bool(use_x0)),
                     _ortho(ortho))
    res = GmresResult()
    hist = None
    if history:
        hist = np.zeros(int(maxit) + 1, np.float64)
        res.resid_hist = hist.ctypes.data_as(C.POINTER(C.c_double))
    code = lib().addns_gmres_solve(pc.handle, _ptr(d_b), _ptr(d_x), C.byref(opts), C.byref(res),
                                   _stream(stream))
    if code < 0 and (code != ERR_NOCONV or raise_noconv):
        _check(code, "gmres_solve")
    out = dict(iters=res.iters, cycles=res.cycles, converged=bool(res.converged),
               true_relres=res.true_relres, est_relres=res.est_relres, code=code)
    if history:
        out["history"] = hist[:res.iters]
    return out


def gmres_solve_batched(pc: Precond, sys_offsets, d_b, d_x, restart=50, maxit=1000, tol=1e-8,
                        use_x0=False, history=False, stream=None):
    offs = np.ascontiguousarray(sys_offsets, dtype=np.int32)
    nsys = len(offs) - 1
    opts = GmresOpts(int(restart), int(maxit), float(tol), 1, int(bool(use_x0)), ORTHO_MGS)
    res = (GmresResult * nsys)()
    hists = []
    if history:
        for q in range(nsys):
            h = np.zeros(int(maxit) + 1, np.float64)
            hists.append(h)
            res[q].resid_hist = h.ctypes.data_as(C.POINTER(C.c_double))
    code = lib().addns_gmres_solve_batched(pc.handle, nsys, _ptr(offs), _ptr(d_b), _ptr(d_x),
                                           C.byref(opts), res, _stream(stream))
    if code < 0 and code != ERR_NOCONV:
        _check(code, "gmres_solve_batched")
    out = []
    for q in range(nsys):
        r = res[q]
        d = dict(iters=r.iters, cycles=r.cycles, converged=bool(r.converged),
                 true_relres=r.true_relres, est_relres=r.est_relres)
        if history:
            d["history"] = hists[q][:r.iters]
        out.append(d)
    return out, code


def _gmres_out(res, code, hist):
    out = dict(iters=res.iters, cycles=res.cycles, converged=bool(res.converged),
               true_relres=res.true_relres, est_relres=res.est_relres, code=code)
    if hist is not None:
        out["history"] = hist[:res.iters]
    return out


def gmres_solve_judged(learned: Precond, plain: Precond, d_b, d_x, restart=50, maxit=1000, tol=1e-8,
                       flexible=True, use_x0=False, history=False, stream=None, ortho="cgs2"):
    opts = GmresOpts(int(restart), int(maxit), float(tol), int(bool(flexible)), int(bool(use_x0)),
                     _ortho(ortho))
    res = GmresResult()
    hist = None
    if history:
        hist = np.zeros(int(maxit) + 1, np.float64)
        res.resid_hist = hist.ctypes.data_as(C.POINTER(C.c_double))
    acc = C.c_int32(0)
    code = lib().addns_gmres_solve_judged(learned.handle, plain.handle, _ptr(d_b), _ptr(d_x),
                                          C.byref(opts), C.byref(res), C.byref(acc), _stream(stream))
    if code < 0 and code != ERR_NOCONV:
        _check(code, "gmres_solve_judged")
    out = _gmres_out(res, code, hist)
    out["accepted"] = bool(acc.value)
    return out


# --------------------------------------------------------------------------
# learned interface correction (extension)
# --------------------------------------------------------------------------

def dtn_param_count() -> int:
    return int(lib().addns_dtn_param_count())


def dtn_samples(pc: Precond, d_X=None, d_Y=None, d_M=None, stream=None) -> int:
    """Sample count; with device tensors X[count,7], Y[count,5], M[count,5]
    (float32) also writes the features, targets and masks."""
    n = C.c_int64(0)
    cap = 0 if d_X is None else int(d_X.shape[0])
    _check(lib().addns_dtn_samples(pc.handle, _ptr(d_X), _ptr(d_Y), _ptr(d_M), cap, C.byref(n),
                                   _stream(stream)), "dtn_samples")
    return int(n.value)


def dtn_forward(weights, d_X, d_P, bf16=False, stream=None):
    w = np.ascontiguousarray(weights, dtype=np.float32)
    _check(lib().addns_dtn_forward(_ptr(w), _ptr(d_X), _ptr(d_P), int(d_X.shape[0]), int(bool(bf16)),
                                   _stream(stream)), "dtn_forward")


def dtn_grad(weights, d_X, d_Y, d_M, stream=None):
    w = np.ascontiguousarray(weights, dtype=np.float32)
    g = np.empty(dtn_param_count(), np.float32)
    loss = C.c_double(0.0)
    _check(lib().addns_dtn_grad(_ptr(w), _ptr(d_X), _ptr(d_Y), _ptr(d_M), int(d_X.shape[0]), _ptr(g),
                                C.byref(loss), _stream(stream)), "dtn_grad")
    return g, loss.value


def dtn_train(d_X, d_Y, d_M, epochs=10, batch=256, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              seed=0, init=None, stream=None):
    hp = DtnParams(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps),
                   int(seed), int(init is not None))
    w = (np.zeros(dtn_param_count(), np.float32) if init is None
         else np.array(init, dtype=np.float32, copy=True))
    loss = np.zeros(max(int(epochs), 1), np.float64)
    _check(lib().addns_dtn_train(_ptr(d_X), _ptr(d_Y), _ptr(d_M), int(d_X.shape[0]), C.byref(hp),
                                 _ptr(w), _ptr(loss), _stream(stream)), "dtn_train")
    return w, loss[:int(epochs)]


def dtn_save(path, weights):
    w = np.ascontiguousarray(weights, dtype=np.float32)
    _check(lib().addns_dtn_save(os.fsencode(path), _ptr(w)), "dtn_save")


def dtn_load(path):
    w = np.empty(dtn_param_count(), np.float32)
    _check(lib().addns_dtn_load(os.fsencode(path), _ptr(w)), "dtn_load")
    return w


def release_cached_memory() -> int:
    """Free the device buffers that released handles left in the library's
    cache; returns the bytes freed."""
    return int(lib().addns_release_cached_memory())


def version() -> str:
    return lib().addns_version().decode()

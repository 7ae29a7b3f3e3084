"""Python binding of libd2d (the C ABI declared in include/d2d.h).

Argument marshalling only: every computation runs in the HIP library.  The
functions carry the C names.  PyTorch supplies device memory and the stream;
the library is loaded from this package directory and its absence is an
error, never a fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libd2d.so")

D2D_OK, D2D_EINVAL, D2D_ENOMEM, D2D_EDEVICE, D2D_ENOCONV, D2D_ESTATE = 0, -1, -2, -3, -4, -5
D2D_FP64, D2D_FP32, D2D_BF16, D2D_BF16X3 = 0, 1, 2, 3
D2D_NPREC = 4
D2D_HEISENBERG, D2D_HUBBARD = 0, 1
D2D_LOG_MAX = 256
D2D_TILE_SPLIT = 1 << 16
D2D_TILE_FUSED = 1 << 17
D2D_TILE_SPLIT4 = 1 << 18
D2D_TILE_XCD = 1 << 19
D2D_TILE_DENSE = 1 << 20
D2D_TILE_ASYM = 1 << 21
D2D_TILE_PERSIST = 1 << 22

_STATUS = {0: "D2D_OK", -1: "D2D_EINVAL", -2: "D2D_ENOMEM", -3: "D2D_EDEVICE", -4: "D2D_ENOCONV",
           -5: "D2D_ESTATE"}

P = C.c_void_p
i64p = C.POINTER(C.c_int64)
f64p = C.POINTER(C.c_double)


class d2d_model(C.Structure):
    _fields_ = [("kind", C.c_int), ("legs", C.c_int), ("t", C.c_double), ("U", C.c_double), ("J", C.c_double)]


class d2d_block_desc(C.Structure):
    _fields_ = [("side", C.c_int), ("ncols", C.c_int), ("nsec", C.c_int), ("sec_qn", i64p), ("sec_dim", i64p),
                ("H", f64p), ("nops", C.c_int), ("op_key", i64p), ("nblk", C.c_int), ("op_blk", i64p),
                ("op_off", i64p), ("op_data", f64p), ("op_data_len", C.c_int64),
                ("H_len", C.c_int64)]


class d2d_sb_info_t(C.Structure):
    _fields_ = [("n", C.c_int64), ("npairs", C.c_int32), ("m", C.c_int32), ("ncol", C.c_int32),
                ("nterms", C.c_int32), ("max_dl", C.c_int32), ("max_dr", C.c_int32),
                ("flops_exec", C.c_double), ("flops_nnz", C.c_double), ("flops_central", C.c_double),
                ("bytes_min_fp64", C.c_double), ("bytes_min_fp32", C.c_double), ("bytes_min_bf16", C.c_double),
                ("op_entries", C.c_int64), ("bytes_min_bf16x3", C.c_double)]


class d2d_lanczos_opts(C.Structure):
    _fields_ = [("prec", C.c_int), ("k_in", C.c_int), ("max_restarts", C.c_int), ("tol_res", C.c_double),
                ("escalate", C.c_double), ("use_graph", C.c_int), ("reorth_window", C.c_int),
                ("separate_central", C.c_int), ("tol_rel_e", C.c_double), ("seed", C.c_uint64),
                ("plain_cgs2", C.c_int), ("basis", C.c_int), ("k_in_bf16", C.c_int),
                ("fixed_cycles", C.c_int), ("one_kernel_step", C.c_int)]


class d2d_lanczos_stats(C.Structure):
    _fields_ = [("restarts", C.c_int), ("hv_count", C.c_int64 * D2D_NPREC), ("residual", C.c_double),
                ("seconds", C.c_double), ("nlog", C.c_int), ("log_t", C.c_double * D2D_LOG_MAX),
                ("log_theta", C.c_double * D2D_LOG_MAX), ("log_rho", C.c_double * D2D_LOG_MAX),
                ("log_prec", C.c_int * D2D_LOG_MAX), ("log_pred", C.c_double * D2D_LOG_MAX),
                ("graph_captures", C.c_int), ("coop_steps", C.c_int64)]


# name -> (restype, argtypes)
_SIGS = {
    "d2d_last_error": (C.c_char_p, []),
    "d2d_version": (C.c_char_p, []),
    "d2d_ctx_create": (C.c_int, [C.c_int, P, C.c_size_t, C.POINTER(P)]),
    "d2d_ctx_destroy": (C.c_int, [P]),
    "d2d_ctx_bytes": (C.c_int, [P, C.POINTER(C.c_size_t)]),
    "d2d_block_import": (C.c_int, [P, C.POINTER(d2d_model), C.POINTER(d2d_block_desc), C.POINTER(P)]),
    "d2d_block_exact": (C.c_int, [P, C.POINTER(d2d_model), C.c_int, C.c_int, C.POINTER(P)]),
    "d2d_block_dims": (C.c_int, [P, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "d2d_block_export": (C.c_int, [P, i64p, i64p, f64p, i64p, i64p, i64p, f64p, i64p]),
    "d2d_block_destroy": (C.c_int, [P]),
    "d2d_sb_create": (C.c_int, [P, P, P, C.POINTER(d2d_model), i64p, C.c_uint, C.POINTER(P)]),
    "d2d_sb_destroy": (C.c_int, [P]),
    "d2d_sb_info": (C.c_int, [P, C.POINTER(d2d_sb_info_t)]),
    "d2d_sb_sectors": (C.c_int, [P, i64p, i64p, i64p, i64p]),
    "d2d_pack": (C.c_int, [P, P, P]),
    "d2d_unpack": (C.c_int, [P, P, P]),
    "d2d_hv": (C.c_int, [P, C.c_int, P, P]),
    "d2d_hv_noalloc": (C.c_int, [P, C.c_int, P, P]),
    "d2d_hv_count": (C.c_int, [P, i64p]),
    "d2d_hv_profile": (C.c_int, [P, C.c_int, P, P, C.c_int, f64p, f64p]),
    "d2d_sb_set_tile": (C.c_int, [P, C.c_int, C.c_int]),
    "d2d_sb_gemm_flops": (C.c_int, [P, C.c_int, f64p]),
    "d2d_batch_gemm_flops": (C.c_int, [P, C.c_int, f64p]),
    "d2d_sb_autotune": (C.c_int, [P, C.c_int, C.c_int, C.POINTER(C.c_int), f64p]),
    "d2d_tile_shapes": (C.c_int, [C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "d2d_lanczos": (C.c_int, [P, C.POINTER(d2d_lanczos_opts), P, f64p, P, C.POINTER(d2d_lanczos_stats)]),
    "d2d_density_matrix": (C.c_int, [P, P, C.c_int, C.c_int, C.POINTER(P), f64p, f64p, i64p]),
    "d2d_column_densities": (C.c_int, [P, P, f64p]),
    "d2d_density_matrix_timed": (C.c_int, [P, P, C.c_int, C.c_int, C.POINTER(P), f64p, f64p, i64p, f64p]),
    "d2d_density_matrix_both": (C.c_int, [P, P, C.c_int, C.POINTER(P), C.POINTER(P), f64p, f64p]),
    "d2d_wavefunction_transform": (C.c_int, [P, P, P, P, C.c_int]),
    "d2d_batch_create": (C.c_int, [P, C.POINTER(P), C.c_int, C.POINTER(P)]),
    "d2d_batch_destroy": (C.c_int, [P]),
    "d2d_batch_hv": (C.c_int, [P, C.c_int, C.POINTER(P), C.POINTER(P)]),
    "d2d_batch_set_tile": (C.c_int, [P, C.c_int, C.c_int]),
    "d2d_batch_autotune": (C.c_int, [P, C.c_int, C.c_int, C.POINTER(C.c_int), f64p]),
    "d2d_batch_lanczos": (C.c_int, [P, C.POINTER(d2d_lanczos_opts), C.POINTER(P), f64p, C.POINTER(P),
                                    C.POINTER(d2d_lanczos_stats)]),
}

EXPORTED = tuple(_SIGS)

_lib = None


def load(path: str = LIB_PATH):
    """Load libd2d.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libd2d is not built ({path} missing): run python -m paper_0707_0159_amd.build")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class D2DError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(st: int, allow=()):
    if st != D2D_OK and st not in allow:
        raise D2DError(st, load().d2d_last_error().decode())
    return st


def d2d_last_error() -> str:
    return load().d2d_last_error().decode()


def d2d_version() -> str:
    return load().d2d_version().decode()


# ------------------------------------------------------------------ objects
@dataclass
class Ctx:
    handle: int
    device: int
    stream: object     # torch.cuda.Stream the library orders its work on


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def d2d_ctx_create(device: int = 0, stream=None, mem_cap: int = 0) -> Ctx:
    import torch
    if stream is None:
        stream = torch.cuda.Stream(device=device)
    h = P()
    _check(load().d2d_ctx_create(device, P(stream.cuda_stream), mem_cap, C.byref(h)))
    return Ctx(h.value, device, stream)


def d2d_ctx_destroy(ctx: Ctx):
    _check(load().d2d_ctx_destroy(P(ctx.handle)))


def d2d_ctx_bytes(ctx: Ctx) -> int:
    v = C.c_size_t()
    _check(load().d2d_ctx_bytes(P(ctx.handle), C.byref(v)))
    return v.value


def make_model(kind, legs, t=1.0, U=0.0, J=1.0) -> d2d_model:
    k = kind if isinstance(kind, int) else (D2D_HUBBARD if kind == "hubbard" else D2D_HEISENBERG)
    return d2d_model(k, int(legs), float(t), float(U), float(J))


def _i64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64).reshape(-1))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))


def d2d_block_import(ctx: Ctx, model: d2d_model, arrays: dict) -> int:
    """Import a block given as the arrays of the frozen block-file layout."""
    keep = {k: (_f64(arrays[k]) if k in ("H", "op_data") else _i64(arrays[k]))
            for k in ("sec_qn", "sec_dim", "H", "op_key", "op_blk", "op_off", "op_data")}
    d = d2d_block_desc()
    d.side = int(arrays["side"])
    d.ncols = int(arrays["ncols"])
    d.nsec = int(keep["sec_dim"].size)
    d.sec_qn = keep["sec_qn"].ctypes.data_as(i64p)
    d.sec_dim = keep["sec_dim"].ctypes.data_as(i64p)
    d.H = keep["H"].ctypes.data_as(f64p)
    d.nops = int(keep["op_key"].size // 3)
    d.op_key = keep["op_key"].ctypes.data_as(i64p)
    d.nblk = int(keep["op_blk"].size // 3)
    d.op_blk = keep["op_blk"].ctypes.data_as(i64p)
    d.op_off = keep["op_off"].ctypes.data_as(i64p)
    d.op_data = keep["op_data"].ctypes.data_as(f64p)
    d.op_data_len = int(keep["op_data"].size)
    d.H_len = int(keep["H"].size)
    h = P()
    _check(load().d2d_block_import(P(ctx.handle), C.byref(model), C.byref(d), C.byref(h)))
    return h.value


def d2d_block_exact(ctx: Ctx, model: d2d_model, ncols: int, side: int) -> int:
    h = P()
    _check(load().d2d_block_exact(P(ctx.handle), C.byref(model), int(ncols), int(side), C.byref(h)))
    return h.value


def d2d_block_dims(block: int):
    m, ns = C.c_int(), C.c_int()
    _check(load().d2d_block_dims(P(block), C.byref(m), C.byref(ns)))
    return m.value, ns.value


def d2d_block_export(block: int) -> dict:
    sizes = np.zeros(5, dtype=np.int64)
    z = None
    _check(load().d2d_block_export(P(block), z, z, z, z, z, z, z, sizes.ctypes.data_as(i64p)))
    ns, hl, nops, nblk, dl = (int(x) for x in sizes)
    out = {"sec_qn": np.zeros(2 * ns, np.int64), "sec_dim": np.zeros(ns, np.int64), "H": np.zeros(hl),
           "op_key": np.zeros(3 * nops, np.int64), "op_blk": np.zeros(3 * nblk, np.int64),
           "op_off": np.zeros(nblk, np.int64), "op_data": np.zeros(dl)}
    _check(load().d2d_block_export(P(block), out["sec_qn"].ctypes.data_as(i64p), out["sec_dim"].ctypes.data_as(i64p),
                                   out["H"].ctypes.data_as(f64p), out["op_key"].ctypes.data_as(i64p),
                                   out["op_blk"].ctypes.data_as(i64p), out["op_off"].ctypes.data_as(i64p),
                                   out["op_data"].ctypes.data_as(f64p), sizes.ctypes.data_as(i64p)))
    out["sec_qn"] = out["sec_qn"].reshape(-1, 2)
    out["op_key"] = out["op_key"].reshape(-1, 3)
    out["op_blk"] = out["op_blk"].reshape(-1, 3)
    return out


def d2d_block_destroy(block: int):
    _check(load().d2d_block_destroy(P(block)))


def d2d_sb_create(ctx: Ctx, b1: int, b4: int, model: d2d_model, target, prec_mask: int = 3) -> int:
    q = _i64(target)
    h = P()
    _check(load().d2d_sb_create(P(ctx.handle), P(b1), P(b4), C.byref(model), q.ctypes.data_as(i64p),
                                C.c_uint(prec_mask), C.byref(h)))
    return h.value


def d2d_sb_destroy(sb: int):
    _check(load().d2d_sb_destroy(P(sb)))


def d2d_sb_info(sb: int) -> dict:
    i = d2d_sb_info_t()
    _check(load().d2d_sb_info(P(sb), C.byref(i)))
    return {name: getattr(i, name) for name, _ in d2d_sb_info_t._fields_}


def d2d_sb_sectors(sb: int):
    n = d2d_sb_info(sb)["npairs"]
    qL = np.zeros(2 * n, np.int64); dL = np.zeros(n, np.int64); dR = np.zeros(n, np.int64)
    off = np.zeros(n, np.int64)
    _check(load().d2d_sb_sectors(P(sb), qL.ctypes.data_as(i64p), dL.ctypes.data_as(i64p),
                                 dR.ctypes.data_as(i64p), off.ctypes.data_as(i64p)))
    return qL.reshape(-1, 2), dL, dR, off


def d2d_pack(sb: int, full, packed):
    """packed <- target-sector elements of the full-space vector (device FP64 tensors)."""
    _check(load().d2d_pack(P(sb), P(_ptr(full)), P(_ptr(packed))))
    return packed


def d2d_unpack(sb: int, packed, full):
    """full-space vector (zero outside the target sector) <- packed (device FP64 tensors)."""
    _check(load().d2d_unpack(P(sb), P(_ptr(packed)), P(_ptr(full))))
    return full


def d2d_hv(sb: int, prec: int, v, w):
    """w = H v on the context stream; v, w torch tensors on the device."""
    _check(load().d2d_hv(P(sb), int(prec), P(_ptr(v)), P(_ptr(w))))
    return w


def d2d_hv_noalloc(sb: int, prec: int, v, w):
    """w = H v as d2d_hv, with the library's static scratch instead of any allocation."""
    _check(load().d2d_hv_noalloc(P(sb), int(prec), P(_ptr(v)), P(_ptr(w))))
    return w


D2D_NOALLOC_SCRATCH_BYTES = 64 << 20


def d2d_hv_profile(sb: int, prec: int, v, w, reps: int = 20):
    """Average (ms_gemm, ms_central) of one Hv, HIP events on the context stream."""
    g, c = C.c_double(), C.c_double()
    _check(load().d2d_hv_profile(P(sb), int(prec), P(_ptr(v)), P(_ptr(w)), int(reps), C.byref(g), C.byref(c)))
    return g.value, c.value


def d2d_hv_count(sb: int):
    c = np.zeros(D2D_NPREC, np.int64)
    _check(load().d2d_hv_count(P(sb), c.ctypes.data_as(i64p)))
    return c


def d2d_sb_set_tile(sb: int, prec: int, tile: int):
    _check(load().d2d_sb_set_tile(P(sb), int(prec), int(tile)))


def d2d_sb_gemm_flops(sb: int, prec: int) -> float:
    f = C.c_double()
    _check(load().d2d_sb_gemm_flops(P(sb), int(prec), C.byref(f)))
    return f.value


def d2d_batch_gemm_flops(b: int, prec: int) -> float:
    f = C.c_double()
    _check(load().d2d_batch_gemm_flops(P(b), int(prec), C.byref(f)))
    return f.value


def d2d_sb_autotune(sb: int, prec: int, reps: int = 20):
    """Time every tile shape of prec, keep the fastest; returns (tile index, ms)."""
    t = C.c_int()
    ms = C.c_double()
    _check(load().d2d_sb_autotune(P(sb), int(prec), int(reps), C.byref(t), C.byref(ms)))
    return t.value, ms.value


def d2d_tile_shapes():
    n = C.c_int()
    _check(load().d2d_tile_shapes(C.byref(n), None))
    desc = (C.c_int * (5 * n.value))()
    _check(load().d2d_tile_shapes(C.byref(n), desc))
    return [tuple(desc[5 * i:5 * i + 5]) for i in range(n.value)]


def lanczos_opts(prec=D2D_FP64, k_in=24, max_restarts=200, tol_res=1e-9, escalate=0.5, use_graph=0,
                 reorth_window=0, separate_central=0, tol_rel_e=0.0, seed=0, plain_cgs2=0, basis=0,
                 k_in_bf16=0, fixed_cycles=0, one_kernel_step=0):
    return d2d_lanczos_opts(int(prec), int(k_in), int(max_restarts), float(tol_res), float(escalate),
                            int(use_graph), int(reorth_window), int(separate_central), float(tol_rel_e),
                            int(seed), int(plain_cgs2), int(basis), int(k_in_bf16), int(fixed_cycles),
                            int(one_kernel_step))


def d2d_lanczos(sb: int, opts: d2d_lanczos_opts, v0, psi=None):
    """Returns (status, energy, stats dict); raises on errors other than D2D_ENOCONV."""
    e = C.c_double()
    st = d2d_lanczos_stats()
    s = _check(load().d2d_lanczos(P(sb), C.byref(opts), P(_ptr(v0)), C.byref(e), P(_ptr(psi)), C.byref(st)),
               allow=(D2D_ENOCONV,))
    n = st.nlog
    stats = {"restarts": st.restarts, "hv_count": list(st.hv_count), "residual": st.residual,
             "seconds": st.seconds, "log_t": list(st.log_t[:n]), "log_theta": list(st.log_theta[:n]),
             "log_rho": list(st.log_rho[:n]), "log_prec": list(st.log_prec[:n]), "log_pred": list(st.log_pred[:n]),
             "graph_captures": st.graph_captures, "coop_steps": st.coop_steps}
    return s, e.value, stats


def d2d_density_matrix(sb: int, psi, side: int, m_keep: int, spectrum_cap: int = 0):
    blk = P()
    te = C.c_double()
    spec = np.zeros(max(spectrum_cap, 1))
    n = np.array([spectrum_cap], dtype=np.int64)
    _check(load().d2d_density_matrix(P(sb), P(_ptr(psi)), int(side), int(m_keep), C.byref(blk), C.byref(te),
                                     spec.ctypes.data_as(f64p) if spectrum_cap else None,
                                     n.ctypes.data_as(i64p)))
    return blk.value, te.value, (spec[: int(n[0])] if spectrum_cap else None)


def d2d_density_matrix_both(sb: int, psi, m_keep: int):
    """Both halves' new blocks at once: (left block, right block, truncation
    errors (2,), milliseconds of the three phases (3,))."""
    bl, br = P(), P()
    te = np.zeros(2)
    ms = np.zeros(3)
    _check(load().d2d_density_matrix_both(P(sb), P(_ptr(psi)), int(m_keep), C.byref(bl), C.byref(br),
                                          te.ctypes.data_as(f64p), ms.ctypes.data_as(f64p)))
    return bl.value, br.value, te, ms


def d2d_density_matrix_timed(sb: int, psi, side: int, m_keep: int, spectrum_cap: int = 0):
    """As d2d_density_matrix, plus the milliseconds of its three phases (formation,
    diagonalisation, renormalisation)."""
    blk = P()
    te = C.c_double()
    spec = np.zeros(max(spectrum_cap, 1))
    n = np.array([spectrum_cap], dtype=np.int64)
    ms = np.zeros(3)
    _check(load().d2d_density_matrix_timed(P(sb), P(_ptr(psi)), int(side), int(m_keep), C.byref(blk), C.byref(te),
                                           spec.ctypes.data_as(f64p) if spectrum_cap else None,
                                           n.ctypes.data_as(i64p), ms.ctypes.data_as(f64p)))
    return blk.value, te.value, (spec[: int(n[0])] if spectrum_cap else None), ms


def d2d_wavefunction_transform(sb_from: int, psi_from, sb_to: int, psi_to, direction: int):
    """Initial guess of the next sweep position: psi_to from psi_from (device FP64)."""
    _check(load().d2d_wavefunction_transform(P(sb_from), P(_ptr(psi_from)), P(sb_to), P(_ptr(psi_to)),
                                             int(direction)))


def d2d_column_densities(sb: int, psi, legs: int):
    """<n_{y,sigma}> on columns 2 and 3: array (2, legs, 2) [column][leg][up, down]."""
    out = np.zeros(4 * legs)
    _check(load().d2d_column_densities(P(sb), P(_ptr(psi)), out.ctypes.data_as(f64p)))
    return out.reshape(2, legs, 2)


def d2d_batch_create(ctx: Ctx, sbs) -> int:
    arr = (P * len(sbs))(*[P(s) for s in sbs])
    h = P()
    _check(load().d2d_batch_create(P(ctx.handle), arr, len(sbs), C.byref(h)))
    return h.value


def d2d_batch_destroy(b: int):
    _check(load().d2d_batch_destroy(P(b)))


def d2d_batch_hv(b: int, prec: int, vs, ws):
    va = (P * len(vs))(*[P(_ptr(v)) for v in vs])
    wa = (P * len(ws))(*[P(_ptr(w)) for w in ws])
    _check(load().d2d_batch_hv(P(b), int(prec), va, wa))


def d2d_batch_set_tile(b: int, prec: int, tile: int):
    _check(load().d2d_batch_set_tile(P(b), int(prec), int(tile)))


def d2d_batch_autotune(b: int, prec: int, reps: int = 20):
    """Time every launch configuration of prec on the batch, keep the fastest;
    returns (tile with flags, ms per batched Hv)."""
    t = C.c_int()
    ms = C.c_double()
    _check(load().d2d_batch_autotune(P(b), int(prec), int(reps), C.byref(t), C.byref(ms)))
    return t.value, ms.value


def d2d_batch_lanczos(b: int, opts: d2d_lanczos_opts, v0s, psis=None, n=None):
    """v0s: device start vectors, or None (seeded start vectors; then n = number of problems)."""
    n = len(v0s) if v0s is not None else int(n)
    va = (P * n)(*[P(_ptr(v)) for v in v0s]) if v0s is not None else None
    pa = (P * n)(*[P(_ptr(p)) for p in psis]) if psis is not None else None
    e = np.zeros(n)
    stats = (d2d_lanczos_stats * n)()
    s = _check(load().d2d_batch_lanczos(P(b), C.byref(opts), va, e.ctypes.data_as(f64p), pa, stats),
               allow=(D2D_ENOCONV,))
    per = [{"restarts": st.restarts, "hv_count": list(st.hv_count), "residual": st.residual,
            "seconds": st.seconds, "log_theta": list(st.log_theta[:st.nlog]),
            "log_rho": list(st.log_rho[:st.nlog]), "log_t": list(st.log_t[:st.nlog]),
            "log_prec": list(st.log_prec[:st.nlog]), "log_pred": list(st.log_pred[:st.nlog]),
            "graph_captures": st.graph_captures, "coop_steps": st.coop_steps} for st in stats]
    return s, e, per

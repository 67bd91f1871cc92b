"""Thin Python binding of libedx (include/edx.h): argument marshalling only.

Every step of the path runs in the HIP library; this module converts Python
dictionaries and torch tensors to the C ABI and raises on every non-OK status.
There is no fallback: importing it without the built library raises.
PyTorch provides device memory and streams only.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # imported before libedx so both share one HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libedx.so")

(EDX_OK, EDX_E_INVALID, EDX_E_NOMEM, EDX_E_DEVICE, EDX_E_NOCONV, EDX_E_DEGENERATE, EDX_E_UNSUPPORTED,
 EDX_PENDING) = range(8)
F64, F32 = 0, 1
WS_LANCZOS, WS_GREEN, WS_LANCZOS_FULL = 0, 1, 2


class EdxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_str(status)}: {msg}")
        self.status = status


class _Model(ctypes.Structure):
    _fields_ = [("norb", ctypes.c_int32), ("nbath", ctypes.c_int32),
                ("eps_imp", ctypes.POINTER(ctypes.c_double)),
                ("eps_bath", ctypes.POINTER(ctypes.c_double)),
                ("vhyb", ctypes.POINTER(ctypes.c_double)),
                ("U", ctypes.c_double), ("Ust", ctypes.c_double),
                ("Jh", ctypes.c_double), ("xmu", ctypes.c_double),
                ("Jx", ctypes.c_double), ("Jp", ctypes.c_double),
                ("nph", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("w0", ctypes.c_double), ("g", ctypes.POINTER(ctypes.c_double))]


class HvPlan(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("col_cols", ctypes.c_int32),
                ("col_threads", ctypes.c_int32), ("row_rows", ctypes.c_int32),
                ("row_cols", ctypes.c_int32), ("col_order", ctypes.c_int32)]


class LanczosOpts(ctypes.Structure):
    _fields_ = [("niter", ctypes.c_int32), ("vtype", ctypes.c_int32),
                ("reorth", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("tol", ctypes.c_double), ("rtol", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("degen_check", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("start", ctypes.c_void_p)]


class LanczosReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("breakdown", ctypes.c_int32), ("degenerate", ctypes.c_int32),
                ("e0", ctypes.c_double), ("e1", ctypes.c_double),
                ("beta_last", ctypes.c_double), ("resid", ctypes.c_double)]


class LowestReport(ctypes.Structure):
    _fields_ = [("nfound", ctypes.c_int32), ("runs", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("verified", ctypes.c_int32),
                ("resid_max", ctypes.c_double)]


class EspaceOpts(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("cutoff", ctypes.c_double),
                ("nstates_sector", ctypes.c_int32), ("nstates_total", ctypes.c_int32),
                ("nstates_step", ctypes.c_int32), ("verify", ctypes.c_int32)]


class ChiReport(ctypes.Structure):
    _fields_ = [("w", ctypes.c_double), ("mean", ctypes.c_double),
                ("n", ctypes.c_int32), ("dropped", ctypes.c_int32)]


class BatchResult(ctypes.Structure):
    _fields_ = [("e0", ctypes.c_double), ("beta_last", ctypes.c_double),
                ("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("breakdown", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class BatchTiles(ctypes.Structure):
    _fields_ = [("lane_wgs", ctypes.c_int32), ("multi_k", ctypes.c_int32),
                ("ccols", ctypes.POINTER(ctypes.c_int32)),
                ("rcols", ctypes.POINTER(ctypes.c_int32)), ("wide_min_dim", ctypes.c_int64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("vtype", ctypes.c_int32), ("ngf", ctypes.c_int32), ("lmats", ctypes.c_int32),
                ("beta", ctypes.c_double), ("lanczos", LanczosOpts)]


class ServerResult(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("e0", ctypes.c_double), ("wp", ctypes.c_double), ("wh", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("footprint", ctypes.c_size_t)]


class GfOpts(ctypes.Structure):
    _fields_ = [("ngf", ctypes.c_int32), ("lmats", ctypes.c_int32),
                ("vtype", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("beta", ctypes.c_double)]


class GfReport(ctypes.Structure):
    _fields_ = [("wp", ctypes.c_double), ("wh", ctypes.c_double),
                ("np", ctypes.c_int32), ("nh", ctypes.c_int32),
                ("alpha_p", ctypes.POINTER(ctypes.c_double)),
                ("beta_p", ctypes.POINTER(ctypes.c_double)),
                ("alpha_h", ctypes.POINTER(ctypes.c_double)),
                ("beta_h", ctypes.POINTER(ctypes.c_double))]


# name -> (restype, argtypes); the C-ABI symbols declared in include/edx.h
_P = ctypes.c_void_p
_SIGS = {
    "edx_build_sector": (ctypes.c_int, [ctypes.POINTER(_Model), ctypes.c_int32, ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "edx_build_sector_orbital": (ctypes.c_int, [ctypes.POINTER(_Model), _P, _P, _P, ctypes.POINTER(_P)]),
    "edx_sector_destroy": (None, [_P]),
    "edx_sector_dims": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "edx_sector_hop_nnz": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]),
    "edx_sector_get_tables": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P]),
    "edx_sector_get_rank": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "edx_sector_ld": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "edx_hv": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_int64, _P]),
    "edx_hv_get_plan": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(HvPlan)]),
    "edx_hv_set_plan": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(HvPlan)]),
    "edx_autotune_hv": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_int64, ctypes.c_int32, _P, ctypes.POINTER(HvPlan), ctypes.POINTER(ctypes.c_double)]),
    "edx_lanczos_default_opts": (None, [ctypes.POINTER(LanczosOpts)]),
    "edx_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "edx_lanczos_ground_state": (ctypes.c_int, [_P, ctypes.POINTER(LanczosOpts), _P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double), _P, ctypes.POINTER(LanczosReport), _P]),
    "edx_lanczos_ground_state_static": (ctypes.c_int, [_P, ctypes.POINTER(LanczosOpts), ctypes.POINTER(ctypes.c_double), _P, ctypes.POINTER(LanczosReport), _P]),
    "edx_lowest_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "edx_lanczos_lowest": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(LanczosOpts), ctypes.c_int32, _P, ctypes.c_size_t, _P, _P, ctypes.POINTER(LowestReport), _P]),
    "edx_espace_default_opts": (None, [ctypes.POINTER(EspaceOpts)]),
    "edx_espace_create": (ctypes.c_int, [ctypes.POINTER(EspaceOpts), ctypes.c_int32, ctypes.POINTER(_P)]),
    "edx_espace_destroy": (None, [_P]),
    "edx_espace_diag_workspace_bytes": (ctypes.c_size_t, [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "edx_espace_diag": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.POINTER(LanczosOpts), _P, ctypes.c_size_t, _P]),
    "edx_espace_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "edx_espace_state": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_P)]),
    "edx_espace_sector": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "edx_espace_green_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int32]),
    "edx_espace_green": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(GfOpts), _P, ctypes.c_size_t, _P, _P]),
    "edx_hv_block": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int32, _P, _P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _P]),
    "edx_hv_multi_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int32, ctypes.c_int32]),
    "edx_hv_multi": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int, _P, _P, _P, ctypes.c_size_t, _P]),
    "edx_transpose": (ctypes.c_int, [ctypes.c_int, _P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_int32, _P]),
    "edx_tridiag_spectrum": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P]),
    "edx_chi": (ctypes.c_int, [_P, _P, ctypes.c_double, _P, _P, ctypes.POINTER(GfOpts), _P, ctypes.c_size_t, _P, ctypes.POINTER(ChiReport), _P]),
    "edx_chi_exciton": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(GfOpts), _P, ctypes.c_size_t, _P, ctypes.POINTER(ChiReport), _P]),
    "edx_chi_pair": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(GfOpts), _P, ctypes.c_size_t, _P, ctypes.POINTER(GfReport), _P]),
    "edx_espace_pair_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int32]),
    "edx_espace_chi_exciton": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(GfOpts), _P, ctypes.c_size_t, _P, _P]),
    "edx_espace_chi_pair": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(GfOpts), _P, ctypes.c_size_t, _P, _P]),
    "edx_espace_chi_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int32]),
    "edx_espace_chi": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(GfOpts), _P, ctypes.c_size_t, _P, _P]),
    "edx_green_cf": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(GfOpts), _P, ctypes.c_size_t, _P, ctypes.POINTER(GfReport), _P]),
    "edx_batch_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64]),
    "edx_batch_ground_state": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(LanczosOpts), ctypes.POINTER(BatchTiles), _P, ctypes.c_size_t, ctypes.POINTER(BatchResult), ctypes.POINTER(ctypes.c_double), _P]),
    "edx_batch_autotune": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(LanczosOpts), _P, ctypes.c_size_t, _P, _P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64), _P]),
    "edx_server_default_opts": (None, [ctypes.POINTER(ServerOpts)]),
    "edx_server_create": (ctypes.c_int, [ctypes.POINTER(ServerOpts), ctypes.POINTER(_P)]),
    "edx_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(_Model), ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "edx_server_poll": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ServerResult), _P]),
    "edx_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_size_t)]),
    "edx_server_clock": (ctypes.c_double, []),
    "edx_server_destroy": (None, [_P]),
    "edx_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "edx_last_error": (ctypes.c_char_p, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2105_06806_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def status_str(st):
    return lib.edx_status_str(st).decode()


def last_error():
    return lib.edx_last_error().decode()


def _check(st, ok=(EDX_OK,)):
    if st not in ok:
        raise EdxError(st, last_error())
    return st


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _vtype_of(t):
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("vectors must be float32 or float64")


def _dtype_of(vtype):
    return torch.float64 if vtype == F64 else torch.float32


def _vt(v):
    if isinstance(v, str):
        return {"f64": F64, "f32": F32}[v]
    return int(v)


class Sector:
    """Owning wrapper of an edx_sector handle."""

    def __init__(self, handle, model, nup, ndw):
        self.handle = handle
        self.model = model
        self.nup, self.ndw = nup, ndw
        dup, ddw, dim = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.edx_sector_dims(handle, ctypes.byref(dup), ctypes.byref(ddw), ctypes.byref(dim)))
        self.dup, self.ddw, self.dim = dup.value, ddw.value, dim.value
        self.dph = self.dim // (self.dup * self.ddw)   # phonon copies (1: none)
        ld = ctypes.c_int64()
        _check(lib.edx_sector_ld(handle, ctypes.byref(ld)))
        self.ld = ld.value   # column stride of the library's own Krylov vectors

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and lib is not None:
            lib.edx_sector_destroy(h)
            self.handle = None

    def hop_nnz(self, spin):
        nnz, mx = ctypes.c_int64(), ctypes.c_int32()
        _check(lib.edx_sector_hop_nnz(self.handle, spin, ctypes.byref(nnz), ctypes.byref(mx)))
        return nnz.value, mx.value

    def tables(self, spin):
        """Host copies of one spin's tables (see edx_sector_get_tables)."""
        D = self.dup if spin == 0 else self.ddw
        nnz, _ = self.hop_nnz(spin)
        out = {
            "map": np.zeros(D, np.uint32), "hop_off": np.zeros(D + 1, np.int64),
            "hop_col": np.zeros(max(nnz, 1), np.int32), "hop_sign": np.zeros(max(nnz, 1), np.int8),
            "hop_amp": np.zeros(max(nnz, 1), np.float64), "diag_e": np.zeros(D, np.float64),
            "diag_p": np.zeros(D, np.uint8),
        }
        p = [out[k].ctypes.data_as(_P) for k in ("map", "hop_off", "hop_col", "hop_sign", "hop_amp", "diag_e", "diag_p")]
        _check(lib.edx_sector_get_tables(self.handle, spin, *p))
        for k in ("hop_col", "hop_sign", "hop_amp"):
            out[k] = out[k][:nnz]
        return out

    def rank(self, spin):
        """Host copy of one spin's inverse map over all 2**Ns strings (see
        edx_sector_get_rank): index in the sector's listing, -1 outside it."""
        out = np.zeros(1 << (int(self.model["norb"]) * (int(self.model["nbath"]) + 1)), np.int32)
        _check(lib.edx_sector_get_rank(self.handle, spin, out.ctypes.data_as(_P)))
        return out


def _model_struct(m):
    keep = []

    def arr(x):
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
        keep.append(a)
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    s = _Model(int(m["norb"]), int(m["nbath"]), arr(m["eps_imp"]), arr(m["eps_bath"]),
               arr(m["vhyb"]), float(m["U"]), float(m["Ust"]), float(m["Jh"]), float(m["xmu"]),
               float(m.get("Jx", 0.0)), float(m.get("Jp", 0.0)), int(m.get("nph", 0)), 0,
               float(m.get("w0", 0.0)),
               arr(m["g"]) if int(m.get("nph", 0)) > 0 else None)
    return s, keep


def build_sector(model, nup, ndw, stream=None):
    ms, keep = _model_struct(model)
    h = _P()
    _check(lib.edx_build_sector(ctypes.byref(ms), int(nup), int(ndw), _stream_ptr(stream), ctypes.byref(h)))
    return Sector(h.value, model, nup, ndw)


def build_sector_orbital(model, nup, ndw, stream=None):
    """Orbital-resolved sector: nup[a], ndw[a] electrons of each spin in
    orbital a (see edx_build_sector_orbital)."""
    norb = int(model["norb"])
    if len(nup) != norb or len(ndw) != norb:
        raise ValueError(f"nup and ndw need {norb} per-orbital counts")
    ms, keep = _model_struct(model)
    cu = (ctypes.c_int32 * norb)(*[int(x) for x in nup])
    cd = (ctypes.c_int32 * norb)(*[int(x) for x in ndw])
    h = _P()
    _check(lib.edx_build_sector_orbital(ctypes.byref(ms), ctypes.cast(cu, _P), ctypes.cast(cd, _P),
                                        _stream_ptr(stream), ctypes.byref(h)))
    s = Sector(h.value, model, sum(nup), sum(ndw))
    s.counts = (tuple(int(x) for x in nup), tuple(int(x) for x in ndw))
    return s


def _vec_len(sector, v, w, ld):
    if v.dtype != w.dtype:
        raise TypeError("v and w must have the same dtype")
    if not (v.is_cuda and w.is_cuda):
        raise ValueError("v and w must be CUDA tensors")
    n = (ld or sector.dup) * sector.ddw * sector.dph
    if v.numel() != n or w.numel() != n or not v.is_contiguous() or not w.is_contiguous():
        raise ValueError(f"v and w must be contiguous with ld * D_dw * D_ph = {n} elements")


def hv(sector, v, w, stream=None, ld=0):
    """w = H v on the device.  ld = 0: dense tensors of sector.dim elements;
    otherwise column stride ld >= D_up (ld * D_dw elements, padding rows of w
    written as zero), e.g. sector.ld."""
    _vec_len(sector, v, w, ld)
    _check(lib.edx_hv(sector.handle, _vtype_of(v), _P(v.data_ptr()), _P(w.data_ptr()), int(ld),
                      _stream_ptr(stream)))
    return w


def hv_multi(sectors, v, w, ws=None, stream=None):
    """w_b = H_b v_b for k = len(sectors) sectors of one shape (edx_hv_multi):
    v, w are device tensors of S.ld * S.ddw * k elements, the k vectors
    interleaved element by element (see interleave)."""
    k = len(sectors)
    vt = _vtype_of(v)
    if w.dtype != v.dtype or v.numel() != sectors[0].ld * sectors[0].ddw * k or w.numel() != v.numel():
        raise ValueError("v, w: k interleaved vectors of the sectors' column stride")
    hs = _handles(sectors)
    if ws is None:
        ws = alloc_workspace(lib.edx_hv_multi_workspace_bytes(hs, k, vt))
    _check(lib.edx_hv_multi(hs, k, vt, _P(v.data_ptr()), _P(w.data_ptr()), _P(ws.data_ptr()),
                            ws.numel(), _stream_ptr(stream)))
    return w


def interleave(sector, xs):
    """k dense vectors (sector.dim each) -> the interleaved padded layout of
    edx_hv_multi (layout only)."""
    k = len(xs)
    out = torch.zeros((sector.ddw, sector.ld, k), dtype=xs[0].dtype, device=xs[0].device)
    for b, x in enumerate(xs):
        out[:, :sector.dup, b] = x.view(sector.ddw, sector.dup)
    return out.view(-1)


def deinterleave(sector, y, k):
    """The inverse of interleave: k dense vectors."""
    t = y.view(sector.ddw, sector.ld, k)
    return [t[:, :sector.dup, b].reshape(-1).clone() for b in range(k)]


def hv_block(sector, part, v, w, ld, c0, c1, stream=None):
    """One GPU's piece of the column-distributed product (see edx_hv_block)."""
    if v.dtype != w.dtype:
        raise TypeError("v and w must have the same dtype")
    cols = sector.ddw if part == 0 else sector.dup
    if not (v.is_cuda and w.is_cuda and v.is_contiguous() and w.is_contiguous()):
        raise ValueError("v and w must be contiguous CUDA tensors")
    if v.numel() < ld * cols or w.numel() < ld * cols:
        raise ValueError(f"v and w need ld * {cols} elements")
    _check(lib.edx_hv_block(sector.handle, _vtype_of(v), int(part), _P(v.data_ptr()), _P(w.data_ptr()),
                            int(ld), int(c0), int(c1), _stream_ptr(stream)))
    return w


def transpose(src, rows, cols, lds, dst, ldd, add=False, stream=None):
    """dst (cols x rows, stride ldd) = src^T (+ dst), device tensors."""
    if src.dtype != dst.dtype:
        raise TypeError("src and dst must have the same dtype")
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous CUDA tensors")
    if src.numel() < lds * cols or dst.numel() < ldd * rows:
        raise ValueError("tensor smaller than its shape and stride")
    _check(lib.edx_transpose(_vtype_of(src), _P(src.data_ptr()), int(rows), int(cols), int(lds),
                             _P(dst.data_ptr()), int(ldd), int(bool(add)), _stream_ptr(stream)))
    return dst


def pad(sector, x, ld=None):
    """Dense vector (D elements) -> column stride ld (default sector.ld), zero padding."""
    ld = sector.ld if ld is None else ld
    nc = sector.ddw * sector.dph
    out = x.new_zeros(ld * nc)
    out.view(nc, ld)[:, :sector.dup] = x.view(nc, sector.dup)
    return out


def unpad(sector, x, ld=None):
    """Column stride ld (default sector.ld) -> dense vector of D elements (a copy)."""
    ld = sector.ld if ld is None else ld
    return x.view(sector.ddw * sector.dph, ld)[:, :sector.dup].reshape(-1).clone()


def _plan_dict(p):
    return {f: getattr(p, f) for f, _ in HvPlan._fields_}


def get_plan(sector, vtype):
    p = HvPlan()
    _check(lib.edx_hv_get_plan(sector.handle, _vt(vtype), ctypes.byref(p)))
    return _plan_dict(p)


def set_plan(sector, vtype, raise_on_error=True, **plan):
    """Replace the sector's H.v launch plan; returns the status."""
    cur = get_plan(sector, vtype)
    cur.update(plan)
    p = HvPlan(*[int(cur[f]) for f, _ in HvPlan._fields_])
    st = lib.edx_hv_set_plan(sector.handle, _vt(vtype), ctypes.byref(p))
    if raise_on_error:
        _check(st)
    return st


def autotune_hv(sector, v, w, reps=5, stream=None, ld=0):
    """Time every candidate plan on (v, w) (column stride ld as for hv) and keep
    the fastest; returns (plan, us)."""
    _vec_len(sector, v, w, ld)
    p = HvPlan()
    us = ctypes.c_double()
    _check(lib.edx_autotune_hv(sector.handle, _vtype_of(v), _P(v.data_ptr()), _P(w.data_ptr()), int(ld),
                               int(reps), _stream_ptr(stream), ctypes.byref(p), ctypes.byref(us)))
    return _plan_dict(p), us.value


def lanczos_opts(**kw):
    o = LanczosOpts()
    lib.edx_lanczos_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "vtype":
            v = _vt(v)
        if k == "start":          # a device tensor (kept alive by the caller) or None
            v = None if v is None else v.data_ptr()
        setattr(o, k, v)
    return o


def _check_start(sector, o, start):
    if start is not None and (start.dtype != _dtype_of(o.vtype) or start.numel() != sector.dim
                              or not start.is_cuda or not start.is_contiguous()):
        raise ValueError("start must be a contiguous device tensor of sector.dim elements of the "
                         "vector type")


def workspace_bytes(sector, what, vtype, n):
    return int(lib.edx_workspace_bytes(sector.handle, what, _vt(vtype), n))


def alloc_workspace(nbytes, device="cuda"):
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def lanczos_ground_state(sector, want_psi=True, ws=None, stream=None, allow=(EDX_OK,), **kw):
    """Returns (e0, psi0 tensor or None, report dict, status)."""
    o = lanczos_opts(**kw)
    _check_start(sector, o, kw.get("start"))
    what = WS_LANCZOS_FULL if o.reorth >= 2 else WS_LANCZOS
    need = workspace_bytes(sector, what, o.vtype, o.niter)
    if ws is None:
        ws = alloc_workspace(need)
    psi = torch.empty(sector.dim, dtype=_dtype_of(o.vtype), device="cuda") if want_psi else None
    e0 = ctypes.c_double()
    rep = LanczosReport()
    st = lib.edx_lanczos_ground_state(sector.handle, ctypes.byref(o), _P(ws.data_ptr()), ws.numel(),
                                      ctypes.byref(e0), _P(psi.data_ptr()) if psi is not None else None,
                                      ctypes.byref(rep), _stream_ptr(stream))
    _check(st, ok=tuple(allow) + (EDX_OK,))
    r = {f: getattr(rep, f) for f, _ in LanczosReport._fields_}
    return e0.value, psi, r, st


def lanczos_ground_state_static(sector, psi=None, stream=None, allow=(EDX_OK,), **kw):
    """edx_lanczos_ground_state_static: the ground state with the library's
    fixed per-device workspace (no device allocation inside the call).  psi:
    a caller-owned device tensor of sector.dim elements of the vector type, or
    None.  Returns (e0, psi, report dict, status)."""
    o = lanczos_opts(**kw)
    _check_start(sector, o, kw.get("start"))
    if psi is not None:
        if psi.dtype != _dtype_of(o.vtype) or psi.numel() != sector.dim or not psi.is_cuda:
            raise ValueError("psi must be a device tensor of sector.dim elements of the vector type")
    e0 = ctypes.c_double()
    rep = LanczosReport()
    st = lib.edx_lanczos_ground_state_static(sector.handle, ctypes.byref(o), ctypes.byref(e0),
                                             _P(psi.data_ptr()) if psi is not None else None,
                                             ctypes.byref(rep), _stream_ptr(stream))
    _check(st, ok=tuple(allow) + (EDX_OK,))
    r = {f: getattr(rep, f) for f, _ in LanczosReport._fields_}
    return e0.value, psi, r, st


def green_cf(sector, psi0, e0, orb=0, spin=0, ngf=200, beta=200.0, lmats=4096, ws=None, stream=None,
             coeffs=False):
    """Impurity G(i w_n) as a complex numpy array, plus the report dict."""
    vtype = _check_state(sector, psi0)
    o = GfOpts(int(ngf), int(lmats), vtype, 0, float(beta))
    need = workspace_bytes(sector, WS_GREEN, vtype, ngf)
    if ws is None:
        ws = alloc_workspace(need)
    g = np.zeros(2 * lmats, np.float64)
    rep = GfReport()
    bufs = {}
    if coeffs:
        for k in ("alpha_p", "beta_p", "alpha_h", "beta_h"):
            bufs[k] = np.zeros(ngf, np.float64)
            setattr(rep, k, bufs[k].ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    _check(lib.edx_green_cf(sector.handle, _P(psi0.data_ptr()), float(e0), int(orb), int(spin), ctypes.byref(o),
                            _P(ws.data_ptr()), ws.numel(), g.ctypes.data_as(_P), ctypes.byref(rep),
                            _stream_ptr(stream)))
    r = {"wp": rep.wp, "wh": rep.wh, "np": rep.np, "nh": rep.nh}
    for k, b in bufs.items():
        n = rep.np if k.endswith("_p") else rep.nh
        r[k] = b[: n if k.startswith("alpha") else max(n - 1, 0)].copy()
    return g[0::2] + 1j * g[1::2], r


def lanczos_lowest(sector, k, verify=1, want_psi=True, ws=None, stream=None, allow=(EDX_OK,), **kw):
    """k lowest eigenpairs: (energies numpy [nfound], psi tensor [nfound, D] or
    None, report dict, status)."""
    o = lanczos_opts(**kw)
    need = int(lib.edx_lowest_workspace_bytes(sector.handle, o.vtype, o.niter, int(k)))
    if need == 0:
        raise ValueError("bad arguments for edx_lowest_workspace_bytes")
    if ws is None:
        ws = alloc_workspace(need)
    kk = min(int(k), sector.dim)
    e = np.zeros(kk, np.float64)
    psi = torch.empty((kk, sector.dim), dtype=_dtype_of(o.vtype), device="cuda") if want_psi else None
    rep = LowestReport()
    st = lib.edx_lanczos_lowest(sector.handle, int(k), ctypes.byref(o), int(verify), _P(ws.data_ptr()),
                                ws.numel(), e.ctypes.data_as(_P),
                                _P(psi.data_ptr()) if psi is not None else None, ctypes.byref(rep),
                                _stream_ptr(stream))
    _check(st, ok=tuple(allow) + (EDX_OK,))
    r = {f: getattr(rep, f) for f, _ in LowestReport._fields_}
    n = r["nfound"]
    return e[:n], (psi[:n] if psi is not None else None), r, st


class Espace:
    """Owning wrapper of an edx_espace (finite-temperature state list)."""

    def __init__(self, nsec, **kw):
        o = EspaceOpts()
        lib.edx_espace_default_opts(ctypes.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        self.opts = o
        h = _P()
        _check(lib.edx_espace_create(ctypes.byref(o), int(nsec), ctypes.byref(h)))
        self.handle = h.value
        self.nsec = int(nsec)
        self.sectors = None
        self.vtype = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and lib is not None:
            lib.edx_espace_destroy(h)
            self.handle = None

    def diag(self, sectors, ws=None, stream=None, **kw):
        o = lanczos_opts(**kw)
        hs = _handles(sectors)
        need = int(lib.edx_espace_diag_workspace_bytes(self.handle, hs, len(sectors), o.vtype, o.niter))
        if need == 0:
            raise ValueError("bad arguments for edx_espace_diag_workspace_bytes")
        if ws is None or ws.numel() < need:
            ws = alloc_workspace(need)
        self.sectors = list(sectors)       # the espace does not own them
        self.vtype = o.vtype
        _check(lib.edx_espace_diag(self.handle, hs, len(sectors), ctypes.byref(o), _P(ws.data_ptr()),
                                   ws.numel(), _stream_ptr(stream)))

    def info(self):
        n, e0, z = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double()
        _check(lib.edx_espace_info(self.handle, ctypes.byref(n), ctypes.byref(e0), ctypes.byref(z)))
        return n.value, e0.value, z.value

    def state(self, i):
        e, sec, w, p = ctypes.c_double(), ctypes.c_int32(), ctypes.c_double(), _P()
        _check(lib.edx_espace_state(self.handle, int(i), ctypes.byref(e), ctypes.byref(sec),
                                    ctypes.byref(w), ctypes.byref(p)))
        return e.value, sec.value, w.value, p.value

    def sector(self, i):
        c, k, nx = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib.edx_espace_sector(self.handle, int(i), ctypes.byref(c), ctypes.byref(k), ctypes.byref(nx)))
        return c.value, k.value, nx.value

    def green(self, orb=0, spin=0, ngf=200, lmats=1024, ws=None, stream=None):
        """Thermal G(i w_n) on the grid of the espace's beta (complex numpy)."""
        o = GfOpts(int(ngf), int(lmats), self.vtype, 0, float(self.opts.beta))
        need = int(lib.edx_espace_green_workspace_bytes(self.handle, int(ngf)))
        if need == 0:
            raise ValueError("no kept states (run diag first)")
        if ws is None or ws.numel() < need:
            ws = alloc_workspace(need)
        g = np.zeros(2 * lmats, np.float64)
        _check(lib.edx_espace_green(self.handle, int(orb), int(spin), ctypes.byref(o), _P(ws.data_ptr()),
                                    ws.numel(), g.ctypes.data_as(_P), _stream_ptr(stream)))
        return g[0::2] + 1j * g[1::2]

    def chi(self, cu, cd, ngf=200, lmats=256, ws=None, stream=None):
        """Thermal density-type susceptibility on the bosonic grid of the espace's beta."""
        norb = int(self.sectors[0].model["norb"])
        cu, cd = _coefs(norb, cu, cd)
        o = GfOpts(int(ngf), int(lmats), self.vtype, 0, float(self.opts.beta))
        need = int(lib.edx_espace_chi_workspace_bytes(self.handle, int(ngf)))
        if need == 0:
            raise ValueError("no kept states (run diag first)")
        if ws is None or ws.numel() < need:
            ws = alloc_workspace(need)
        g = np.zeros(2 * lmats, np.float64)
        _check(lib.edx_espace_chi(self.handle, cu.ctypes.data_as(_P), cd.ctypes.data_as(_P), ctypes.byref(o),
                                  _P(ws.data_ptr()), ws.numel(), g.ctypes.data_as(_P), _stream_ptr(stream)))
        return g[0::2] + 1j * g[1::2]

    def chi_exciton(self, a, b, ngf=200, lmats=256, ws=None, stream=None):
        """Thermal excitonic susceptibility of orbitals a != b (bosonic grid)."""
        o = GfOpts(int(ngf), int(lmats), self.vtype, 0, float(self.opts.beta))
        need = int(lib.edx_espace_chi_workspace_bytes(self.handle, int(ngf)))
        if need == 0:
            raise ValueError("no kept states (run diag first)")
        if ws is None or ws.numel() < need:
            ws = alloc_workspace(need)
        g = np.zeros(2 * lmats, np.float64)
        _check(lib.edx_espace_chi_exciton(self.handle, int(a), int(b), ctypes.byref(o), _P(ws.data_ptr()),
                                          ws.numel(), g.ctypes.data_as(_P), _stream_ptr(stream)))
        return g[0::2] + 1j * g[1::2]

    def chi_pair(self, a, ngf=200, lmats=256, ws=None, stream=None):
        """Thermal pair susceptibility of orbital a (bosonic grid)."""
        o = GfOpts(int(ngf), int(lmats), self.vtype, 0, float(self.opts.beta))
        need = int(lib.edx_espace_pair_workspace_bytes(self.handle, int(ngf)))
        if need == 0:
            raise ValueError("no kept states (run diag first)")
        if ws is None or ws.numel() < need:
            ws = alloc_workspace(need)
        g = np.zeros(2 * lmats, np.float64)
        _check(lib.edx_espace_chi_pair(self.handle, int(a), ctypes.byref(o), _P(ws.data_ptr()),
                                       ws.numel(), g.ctypes.data_as(_P), _stream_ptr(stream)))
        return g[0::2] + 1j * g[1::2]


def _check_state(sector, psi0):
    """A state vector handed to the library: dense, contiguous, on the GPU,
    D elements (the library cannot see the tensor's size)."""
    if not psi0.is_cuda or not psi0.is_contiguous() or psi0.numel() != sector.dim:
        raise ValueError(f"psi0 must be a contiguous CUDA tensor of D = {sector.dim} elements")
    return _vtype_of(psi0)


def tridiag_spectrum(alpha, beta):
    """Eigenvalues and squared first components of the tridiagonal matrix."""
    a = np.ascontiguousarray(alpha, np.float64)
    b = np.ascontiguousarray(beta, np.float64)
    m = a.size
    if b.size != max(m - 1, 0):
        raise ValueError("beta needs len(alpha) - 1 entries")
    th = np.zeros(m)
    w = np.zeros(m)
    _check(lib.edx_tridiag_spectrum(a.ctypes.data_as(_P), b.ctypes.data_as(_P) if m > 1 else None, m,
                                    th.ctypes.data_as(_P), w.ctypes.data_as(_P)))
    return th, w


def _coefs(norb, cu, cd):
    cu = np.ascontiguousarray(cu, np.float64)
    cd = np.ascontiguousarray(cd, np.float64)
    if cu.size != norb or cd.size != norb:
        raise ValueError(f"cu and cd need {norb} coefficients")
    return cu, cd


def chi(sector, psi0, e0, cu, cd, ngf=200, beta=200.0, lmats=1024, ws=None, stream=None):
    """Density-type susceptibility C(i nu_n) (complex numpy; real by symmetry)
    and the report dict."""
    vtype = _check_state(sector, psi0)
    cu, cd = _coefs(int(sector.model["norb"]), cu, cd)
    o = GfOpts(int(ngf), int(lmats), vtype, 0, float(beta))
    need = workspace_bytes(sector, 3, vtype, ngf)
    if ws is None:
        ws = alloc_workspace(need)
    g = np.zeros(2 * lmats, np.float64)
    rep = ChiReport()
    _check(lib.edx_chi(sector.handle, _P(psi0.data_ptr()), float(e0), cu.ctypes.data_as(_P),
                       cd.ctypes.data_as(_P), ctypes.byref(o), _P(ws.data_ptr()), ws.numel(),
                       g.ctypes.data_as(_P), ctypes.byref(rep), _stream_ptr(stream)))
    return g[0::2] + 1j * g[1::2], {f: getattr(rep, f) for f, _ in ChiReport._fields_}


def chi_exciton(sector, psi0, e0, a, b, ngf=200, beta=200.0, lmats=1024, ws=None, stream=None):
    """Excitonic susceptibility of orbitals a != b (complex numpy) and report."""
    vtype = _check_state(sector, psi0)
    o = GfOpts(int(ngf), int(lmats), vtype, 0, float(beta))
    if ws is None:
        ws = alloc_workspace(workspace_bytes(sector, 3, vtype, ngf))
    g = np.zeros(2 * lmats, np.float64)
    rep = ChiReport()
    _check(lib.edx_chi_exciton(sector.handle, _P(psi0.data_ptr()), float(e0), int(a), int(b),
                               ctypes.byref(o), _P(ws.data_ptr()), ws.numel(), g.ctypes.data_as(_P),
                               ctypes.byref(rep), _stream_ptr(stream)))
    return g[0::2] + 1j * g[1::2], {f: getattr(rep, f) for f, _ in ChiReport._fields_}


def chi_pair(sector, psi0, e0, a, ngf=200, beta=200.0, lmats=1024, ws=None, stream=None):
    """Pair susceptibility of orbital a (complex numpy) and report."""
    vtype = _check_state(sector, psi0)
    o = GfOpts(int(ngf), int(lmats), vtype, 0, float(beta))
    if ws is None:
        ws = alloc_workspace(workspace_bytes(sector, 4, vtype, ngf))
    g = np.zeros(2 * lmats, np.float64)
    rep = GfReport()
    _check(lib.edx_chi_pair(sector.handle, _P(psi0.data_ptr()), float(e0), int(a), ctypes.byref(o),
                            _P(ws.data_ptr()), ws.numel(), g.ctypes.data_as(_P), ctypes.byref(rep),
                            _stream_ptr(stream)))
    return g[0::2] + 1j * g[1::2], {"wp": rep.wp, "wh": rep.wh, "np": rep.np, "nh": rep.nh}


def _handles(sectors):
    return (ctypes.c_void_p * len(sectors))(*[s.handle for s in sectors])


def batch_workspace_bytes(sectors, vtype="f64", lane_wgs=8, wide_min_dim=None):
    """Bytes for the batched launch; wide_min_dim None = enough for every
    whole-GPU threshold the autotuner tries."""
    h = _handles(sectors)
    if wide_min_dim is None:
        return max(int(lib.edx_batch_workspace_bytes(h, len(sectors), _vt(vtype), lane_wgs, w))
                   for w in (-1, 250000, 1000000, 2000000, 4000000, 8000000))
    return int(lib.edx_batch_workspace_bytes(h, len(sectors), _vt(vtype), lane_wgs, int(wide_min_dim)))


def batch_autotune(sectors, ws=None, stream=None, **kw):
    """Project autotuner of the batched launch; returns a tiles dict."""
    o = lanczos_opts(**kw)
    n = len(sectors)
    if ws is None:
        ws = alloc_workspace(batch_workspace_bytes(sectors, o.vtype, 8))
    cc = np.zeros(n, np.int32)
    rc = np.zeros(n, np.int32)
    lw = ctypes.c_int32()
    wm = ctypes.c_int64()
    _check(lib.edx_batch_autotune(_handles(sectors), n, ctypes.byref(o), _P(ws.data_ptr()), ws.numel(),
                                  cc.ctypes.data_as(_P), rc.ctypes.data_as(_P), ctypes.byref(lw),
                                  ctypes.byref(wm), _stream_ptr(stream)))
    return {"lane_wgs": lw.value, "ccols": cc, "rcols": rc, "wide_min_dim": wm.value}


def batch_ground_state(sectors, tiles=None, ws=None, stream=None, **kw):
    """Ground energies of many sectors in one persistent launch.
    Returns (list of result dicts, kernel ms)."""
    o = lanczos_opts(**kw)
    n = len(sectors)
    lw = tiles["lane_wgs"] if tiles else 32
    wmin = tiles.get("wide_min_dim", 0) if tiles else 0
    if ws is None:
        ws = alloc_workspace(batch_workspace_bytes(sectors, o.vtype, lw, wmin))
    res = (BatchResult * n)()
    ms = ctypes.c_double()
    tp = None
    if tiles:
        cc = np.ascontiguousarray(tiles["ccols"], np.int32)
        rc = np.ascontiguousarray(tiles["rcols"], np.int32)
        t = BatchTiles(lw, int(tiles.get("multi_k", 0)), cc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                       rc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(wmin))
        tp = ctypes.byref(t)
    _check(lib.edx_batch_ground_state(_handles(sectors), n, ctypes.byref(o), tp, _P(ws.data_ptr()), ws.numel(),
                                      res, ctypes.byref(ms), _stream_ptr(stream)))
    out = [{f: getattr(r, f) for f, _ in BatchResult._fields_ if f != "pad_"} for r in res]
    return out, ms.value


class Server:
    """Continuous-batching request server (edx_server_*)."""

    def __init__(self, hbm_budget=8 << 30, max_slots=8, vtype="f32", ngf=200, lmats=1024, beta=200.0, **lanczos):
        o = ServerOpts()
        lib.edx_server_default_opts(ctypes.byref(o))
        o.hbm_budget = int(hbm_budget)
        o.max_slots = int(max_slots)
        o.vtype = _vt(vtype)
        o.ngf = int(ngf)
        o.lmats = int(lmats)
        o.beta = float(beta)
        lo = lanczos_opts(vtype=o.vtype, **lanczos)
        o.lanczos = lo
        self.opts = o
        h = _P()
        _check(lib.edx_server_create(ctypes.byref(o), ctypes.byref(h)))
        self.handle = h.value

    def submit(self, model, nup, ndw):
        ms, keep = _model_struct(model)
        t = ctypes.c_int64()
        _check(lib.edx_server_submit(self.handle, ctypes.byref(ms), int(nup), int(ndw), ctypes.byref(t)))
        return t.value

    def poll(self, ticket, wait=True):
        """Result dict with "g" (complex array) or None if still pending."""
        r = ServerResult()
        g = np.zeros(2 * max(self.opts.lmats, 1), np.float64)
        st = lib.edx_server_poll(self.handle, int(ticket), 1 if wait else 0, ctypes.byref(r), g.ctypes.data_as(_P))
        if st == EDX_PENDING:
            return None
        _check(st)
        out = {f: getattr(r, f) for f, _ in ServerResult._fields_}
        out["g"] = g[0::2] + 1j * g[1::2]
        return out

    def stats(self):
        p, r, c, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_size_t()
        _check(lib.edx_server_stats(self.handle, ctypes.byref(p), ctypes.byref(r), ctypes.byref(c), ctypes.byref(f)))
        return {"pending": p.value, "running": r.value, "completed": c.value, "largest_free": f.value}

    @staticmethod
    def clock():
        return lib.edx_server_clock()

    def close(self):
        if getattr(self, "handle", None):
            lib.edx_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

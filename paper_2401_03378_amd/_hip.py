"""ctypes binding of libhydro.so (the C ABI in include/hydro.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  There is no fallback; if the library is missing, loading fails
with an error that says how to build it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libhydro.so")

HYDRO_OK, HYDRO_EINVAL, HYDRO_EHIP, HYDRO_ENONPHYS, HYDRO_ENOMEM = 0, -1, -2, -3, -4
MODE_PERSISTENT, MODE_PERBLOCK, MODE_TELESCOPING, MODE_MATERIALISED = 0, 1, 2, 3
TILES = {0: (8, 8), 1: (16, 8), 2: (16, 16)}

EXPORTS = ("hydro_validate", "hydro_create", "hydro_validate_amr", "hydro_create_amr",
           "hydro_set_tuning", "hydro_get_tuning",
           "hydro_fill_guards", "hydro_cfl_dt", "hydro_rk_stage", "hydro_step",
           "hydro_step_vjp", "hydro_step_vjp_stages", "hydro_status", "hydro_last_error", "hydro_destroy",
           "hydro_fp_check", "hydro_cfl_dt_noalloc")
FLAG_LEVEL_BY_LEVEL = 1
FLAG_GRAVITY = 2          # uniform gravitational acceleration (problem attribute grav)
FLAG_SHOCK_DETECT = 4     # shock detector (problem attribute shock_thresh)
HYDRO_DT_FROM_PREVIOUS = 2
HYDRO_DT_RECORD = 3
WENO_EPS = 1e-6          # Jiang & Shu's epsilon, the default of a problem without weno_eps


class HydroError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hydro error {code}: {msg}")
        self.code = code


class Block(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("ng", C.c_int32), ("offset", C.c_int64)]


class Link(C.Structure):
    _fields_ = [("nbr", C.c_int32 * 6)]


class Amr(C.Structure):
    _fields_ = [("level", C.c_int32), ("kind", C.c_int32 * 6), ("nbr", (C.c_int32 * 4) * 6)]


class Params(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("recon", C.c_int32), ("rk", C.c_int32),
                ("flags", C.c_int32), ("gamma", C.c_double), ("cfl", C.c_double),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("weno_eps", C.c_double), ("grav", C.c_double * 3), ("shock_thresh", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("mode", C.c_int32), ("tile", C.c_int32), ("grid", C.c_int32),
                ("zchunk", C.c_int32), ("use_graph", C.c_int32), ("xcd", C.c_int32),
                ("variant", C.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is not built; run `python -m paper_2401_03378_amd.build` "
                               "(or __graft_entry__.build())")
        L = C.CDLL(LIB)
        vp, dp, i32, i64 = C.c_void_p, C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "hydro_validate": (C.c_int, [C.POINTER(Params), C.POINTER(Block), C.POINTER(Link), i32, i64]),
            "hydro_create": (C.c_int, [C.POINTER(Params), C.POINTER(Block), C.POINTER(Link), i32, i64, vp,
                                       C.POINTER(vp)]),
            "hydro_validate_amr": (C.c_int, [C.POINTER(Params), C.POINTER(Block), C.POINTER(Link),
                                             C.POINTER(Amr), i32, i64]),
            "hydro_create_amr": (C.c_int, [C.POINTER(Params), C.POINTER(Block), C.POINTER(Link),
                                           C.POINTER(Amr), i32, i64, vp, C.POINTER(vp)]),
            "hydro_set_tuning": (C.c_int, [vp, C.POINTER(Tuning)]),
            "hydro_get_tuning": (C.c_int, [vp, C.POINTER(Tuning)]),
            "hydro_fill_guards": (C.c_int, [vp, dp]),
            "hydro_cfl_dt": (C.c_int, [vp, dp, dp]),
            "hydro_rk_stage": (C.c_int, [vp, i32, dp, dp, dp, dp]),
            "hydro_step": (C.c_int, [vp, dp, dp, i32]),
            "hydro_step_vjp": (C.c_int, [vp, dp, dp, dp, dp]),
            "hydro_step_vjp_stages": (C.c_int, [vp, dp, C.POINTER(vp), dp, dp, dp]),
            "hydro_status": (C.c_int, [vp, C.POINTER(C.c_int64)]),
            "hydro_last_error": (C.c_char_p, [vp]),
            "hydro_destroy": (None, [vp]),
            "hydro_fp_check": (C.c_int, [dp, dp, dp, dp, dp, dp, i64, vp]),
            "hydro_cfl_dt_noalloc": (C.c_int, [C.POINTER(Params), dp, i32, i64, dp, dp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def tables(prob):
    """ctypes params/blocks/links of a problem description (duck-typed)."""
    blocks = np.ascontiguousarray(prob.blocks)
    links = np.ascontiguousarray(prob.links)
    nb = len(blocks)
    B = (Block * max(nb, 1))()
    L = (Link * max(nb, 1))()
    for i in range(nb):
        b = blocks[i]
        B[i] = Block(int(b["nx"]), int(b["ny"]), int(b["nz"]), int(b["ng"]), int(b["offset"]))
        for f in range(6):
            L[i].nbr[f] = int(links[i]["nbr"][f])
    P = Params(int(prob.ndim), int(prob.recon), int(prob.rk), 0, float(prob.gamma),
               float(prob.cfl), float(prob.dx), float(prob.dy), float(prob.dz),
               float(getattr(prob, "weno_eps", WENO_EPS)))
    grav = getattr(prob, "grav", None)
    if grav is not None:
        g = [float(x) for x in grav] + [0.0] * (3 - len(grav))
        for d in range(3):
            P.grav[d] = g[d]
        P.flags |= FLAG_GRAVITY
    thresh = getattr(prob, "shock_thresh", None)
    if thresh is not None:
        P.shock_thresh = float(thresh)
        P.flags |= FLAG_SHOCK_DETECT
    return P, B, L, nb


def amr_table(prob):
    """ctypes level table of a problem with refinement levels, or None."""
    amr = getattr(prob, "amr", None)
    if amr is None:
        return None
    amr = np.ascontiguousarray(amr)
    A = (Amr * max(len(amr), 1))()
    for i, a in enumerate(amr):
        A[i].level = int(a["level"])
        for f in range(6):
            A[i].kind[f] = int(a["kind"][f])
            for h in range(4):
                A[i].nbr[f][h] = int(a["nbr"][f][h])
    return A


def validate(prob) -> int:
    P, B, L, nb = tables(prob)
    A = amr_table(prob)
    if A is not None:
        return lib().hydro_validate_amr(C.byref(P), B, L, A, nb, int(prob.ncell))
    return lib().hydro_validate(C.byref(P), B, L, nb, int(prob.ncell))


def fp_check(a, b, c, stream=None):
    """Device division, square root and fused multiply-add of float64 CUDA
    tensors of one shape (hydro_fp_check): returns (a / b, sqrt(a),
    fma(a, b, c)) computed by the library's kernel."""
    import torch

    for t in (a, b, c):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.shape != a.shape:
            raise ValueError("fp_check takes contiguous float64 CUDA tensors of one shape")
    quot, root, fmad = torch.empty_like(a), torch.empty_like(a), torch.empty_like(a)
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = lib().hydro_fp_check(a.data_ptr(), b.data_ptr(), c.data_ptr(), quot.data_ptr(), root.data_ptr(),
                              fmad.data_ptr(), a.numel(), C.c_void_p(st.cuda_stream))
    if rc != HYDRO_OK:
        raise HydroError(rc, "hydro_fp_check")
    return quot, root, fmad


def block_table_bytes(prob) -> bytes:
    """The problem's hydro_block_t table as raw bytes (the C layout), for a
    caller that keeps the table in device memory (hydro_cfl_dt_noalloc)."""
    _, B, _, nb = tables(prob)
    return C.string_at(C.addressof(B), C.sizeof(Block) * nb)


def cfl_dt_noalloc(prob, blocks_dev, U, dt, stream=None):
    """hydro_cfl_dt_noalloc: the CFL dt of U into the device double dt,
    with no context and no allocation.  blocks_dev is a CUDA uint8 tensor
    holding block_table_bytes(prob); U and dt are contiguous float64 CUDA
    tensors."""
    import torch

    for t in (U, dt):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("U and dt must be contiguous float64 CUDA tensors")
    if blocks_dev.dtype != torch.uint8 or not blocks_dev.is_cuda or not blocks_dev.is_contiguous():
        raise ValueError("blocks_dev must be a contiguous uint8 CUDA tensor")
    P, _, _, nb = tables(prob)
    if blocks_dev.numel() < C.sizeof(Block) * nb:
        raise ValueError("blocks_dev is smaller than the block table")
    st = stream if stream is not None else torch.cuda.current_stream(U.device)
    rc = lib().hydro_cfl_dt_noalloc(C.byref(P), C.c_void_p(blocks_dev.data_ptr()), nb, int(prob.ncell),
                                    C.c_void_p(U.data_ptr()), C.c_void_p(dt.data_ptr()),
                                    C.c_void_p(st.cuda_stream))
    if rc != HYDRO_OK:
        raise HydroError(rc, lib().hydro_last_error(None).decode())

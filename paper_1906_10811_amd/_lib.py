"""ctypes mirror of include/fd.h and the loader of the in-tree libfd.so.

There is no fallback: if the HIP library is not built, ``load()`` raises.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfd.so")

FD_OK = 0
FD_ERR_ARG = -1
FD_ERR_UNSTABLE = -2
FD_ERR_NOMEM = -3
FD_ERR_DEVICE = -4
FD_ERR_STATE = -5
FD_ERR_TIMEOUT = -6

FD_STORE_F32 = 0
FD_STORE_F16 = 1
FD_STORE_BF16 = 2
FD_STORE_F16_DIFF = 3
FD_STORE_BF16_DIFF = 4

FD_PARAM_F32 = 0
FD_PARAM_Q16 = 1

FD_GRAD_RESIDUAL_GIVEN = 1
FD_GRAD_BINOMIAL = 2
FD_GRAD_VELOCITY = 4

FD_ACT_ADVANCE, FD_ACT_STORE, FD_ACT_RESTORE, FD_ACT_YOUTURN = 1, 2, 3, 4

FD_SERVE_SHARE = 0
FD_SERVE_SHORTEST = 1
FD_SERVE_RATIO = 2

# every symbol include/fd.h declares
EXPORTS = (
    "fd_grid_workspace_bytes", "fd_grid_create", "fd_grid_destroy", "fd_grid_get_info",
    "fd_forward", "fd_adjoint", "fd_gradient_workspace_bytes", "fd_gradient",
    "fd_server_create", "fd_submit", "fd_wait", "fd_request_bytes", "fd_server_stats",
    "fd_server_destroy", "fd_last_error", "fd_diffusion_workspace_bytes", "fd_diffusion_run",
    "fd_checkpoint_schedule", "fd_diffusion_run_noalloc", "fd_diffusion_dt_limit",
)


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("shape", ctypes.c_int * 3),
        ("spacing", ctypes.c_double * 3),
        ("origin", ctypes.c_double * 3),
        ("space_order", ctypes.c_int),
        ("nbl", ctypes.c_int),
        ("damp_max", ctypes.c_double),
        ("storage", ctypes.c_int),
        ("amp_scale", ctypes.c_float),
        ("vp_padded", ctypes.c_int),
        ("max_src", ctypes.c_int),
        ("max_rec", ctypes.c_int),
        ("zchunk", ctypes.c_int),
        ("sinc_radius", ctypes.c_int),
        ("sinc_beta", ctypes.c_double),
        ("tile_x", ctypes.c_int),
        ("time_block", ctypes.c_int),
        ("param_storage", ctypes.c_int),
    ]


class Shot(ctypes.Structure):
    _fields_ = [
        ("nsrc", ctypes.c_int),
        ("src_xyz", ctypes.c_void_p),
        ("src_wavelet", ctypes.c_void_p),
        ("nrec", ctypes.c_int),
        ("rec_xyz", ctypes.c_void_p),
    ]


class FwdOpts(ctypes.Structure):
    _fields_ = [
        ("u0", ctypes.c_void_p),
        ("u_prev", ctypes.c_void_p),
        ("save_u", ctypes.c_void_p),
        ("save_u_prev", ctypes.c_void_p),
    ]


class GridInfo(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("padded", ctypes.c_int * 3),
        ("padded_points", ctypes.c_longlong),
        ("vmax", ctypes.c_double),
        ("critical_dt", ctypes.c_double),
        ("damp_max", ctypes.c_double),
        ("field_bytes", ctypes.c_size_t),
        ("tile", ctypes.c_int * 2),
        ("tile_strip", ctypes.c_int),
        ("zchunk", ctypes.c_int),
        ("time_block", ctypes.c_int),
        ("param_storage", ctypes.c_int),
        ("param_base", ctypes.c_double),
        ("param_step", ctypes.c_double),
    ]


class ServerDesc(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int),
        ("hbm_budget_bytes", ctypes.c_size_t),
        ("max_slots", ctypes.c_int),
        ("steps_per_round", ctypes.c_int),
        ("policy", ctypes.c_int),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("grid", GridDesc),
        ("vp_host", ctypes.c_void_p),
        ("nsrc", ctypes.c_int),
        ("src_xyz", ctypes.c_void_p),
        ("wavelet_host", ctypes.c_void_p),
        ("nrec", ctypes.c_int),
        ("rec_xyz", ctypes.c_void_p),
        ("nt", ctypes.c_int),
        ("dt", ctypes.c_double),
        ("rec_out_host", ctypes.c_void_p),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("t_submit", ctypes.c_double),
        ("t_start", ctypes.c_double),
        ("t_done", ctypes.c_double),
        ("bytes_reserved", ctypes.c_size_t),
    ]


class DiffusionDesc(ctypes.Structure):
    _fields_ = [
        ("shape", ctypes.c_int * 2),
        ("spacing", ctypes.c_double * 2),
        ("space_order", ctypes.c_int),
        ("nu", ctypes.c_double),
        ("time_block", ctypes.c_int),
    ]


class CkptAction(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("step", ctypes.c_int),
        ("count", ctypes.c_int),
        ("slot", ctypes.c_int),
        ("first", ctypes.c_int),
    ]


class FDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libfd error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load the in-tree libfd.so (built by ``python -m paper_1906_10811_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libfd.so is not built (%s); run `python -m paper_1906_10811_amd.build`"
                           % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    PS = ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "fd_grid_workspace_bytes": (I, [ctypes.POINTER(GridDesc), PS]),
        "fd_grid_create": (I, [ctypes.POINTER(GridDesc), P, S, P, P, ctypes.POINTER(P)]),
        "fd_grid_destroy": (I, [P]),
        "fd_grid_get_info": (I, [P, ctypes.POINTER(GridInfo)]),
        "fd_forward": (I, [P, ctypes.POINTER(Shot), I, D, P, ctypes.POINTER(FwdOpts), P]),
        "fd_adjoint": (I, [P, ctypes.POINTER(Shot), I, D, P, P, P]),
        "fd_gradient_workspace_bytes": (I, [P, I, I, I, I, PS]),
        "fd_gradient": (I, [P, ctypes.POINTER(Shot), I, D, P, I, I, P, S, P, P, P, P, P]),
        "fd_server_create": (I, [ctypes.POINTER(ServerDesc), ctypes.POINTER(P)]),
        "fd_submit": (I, [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
        "fd_wait": (I, [P, ctypes.c_uint64, D, ctypes.POINTER(Result)]),
        "fd_request_bytes": (I, [ctypes.POINTER(Request), PS]),
        "fd_server_stats": (I, [P, PS, ctypes.POINTER(ctypes.c_int)]),
        "fd_server_destroy": (I, [P]),
        "fd_last_error": (ctypes.c_char_p, []),
        "fd_diffusion_workspace_bytes": (I, [ctypes.POINTER(DiffusionDesc), PS]),
        "fd_diffusion_run": (I, [ctypes.POINTER(DiffusionDesc), P, S, P, P, I, D, P]),
        "fd_diffusion_run_noalloc": (I, [ctypes.POINTER(DiffusionDesc), P, P, I, D, P]),
        "fd_diffusion_dt_limit": (I, [ctypes.POINTER(DiffusionDesc), ctypes.POINTER(D)]),
        "fd_checkpoint_schedule": (I, [I, I, ctypes.POINTER(CkptAction), I, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_longlong)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != FD_OK:
        msg = load().fd_last_error().decode(errors="replace")
        raise FDError(rc, msg)


def checkpoint_schedule(nt: int, slots: int):
    """fd_checkpoint_schedule as a list of (kind, step, count, slot, first)
    plus the number of forward steps it advances (host only)."""
    lib = load()
    n = ctypes.c_int()
    fwd = ctypes.c_longlong()
    check(lib.fd_checkpoint_schedule(int(nt), int(slots), None, 0, ctypes.byref(n), ctypes.byref(fwd)))
    arr = (CkptAction * max(1, n.value))()
    check(lib.fd_checkpoint_schedule(int(nt), int(slots), arr, n.value, ctypes.byref(n), ctypes.byref(fwd)))
    return [(a.kind, a.step, a.count, a.slot, a.first) for a in arr[:n.value]], fwd.value

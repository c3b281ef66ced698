"""ctypes binding of libcholmod_mi355x.so (argument marshalling only).

Every function here mirrors a C entry point of include/cholmod_mi355x.h.
All arithmetic runs in the HIP kernels of the library; if the library is
missing, loading fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcholmod_mi355x.so")

OK, ERR_ARG, ERR_NOT_PD, ERR_BAD_DIAG, ERR_HIP = 0, -1, -2, -3, -4
FLAG_EXACT, FLAG_BLOCKED, FLAG_ROTATIONS = 1, 2, 4
F64, F32S = 0, 1
INFO_NONE = (1 << 63) - 1

EXPORTS = (
    "cholmod_version", "cholmod_status_string", "cholmod_decode_info",
    "cholmod_workspace_bytes", "cholmod_update", "cholmod_update_async",
    "cholmod_update_ex", "cholmod_update_f32s", "cholmod_update_f32s_async",
    "cholmod_workspace_bytes_batched", "cholmod_update_batched",
    "cholmod_workspace_bytes_ooc", "cholmod_update_ooc",
    "cholmod_batch_graph_create", "cholmod_batch_graph_launch", "cholmod_batch_graph_destroy",
    "cholmod_server_create", "cholmod_server_add_factor", "cholmod_server_submit",
    "cholmod_server_poll", "cholmod_server_drain", "cholmod_server_destroy",
    "cholmod_noalloc_max_bytes", "cholmod_update_noalloc", "cholmod_probe_latency",
    "cholmod_update_batched_plan", "cholmod_set_plan", "cholmod_get_plan", "cholmod_plan_bucket",
    "cholmod_compute_units", "cholmod_update_f32s_ex",
)

SCHED_QUEUED, SCHED_STEPPED = 0, 1
ORDER_BLOCK, ORDER_FACTOR = 0, 1
N_BUCKETS, K_BUCKETS = 5, 4


class ServerCfg(ctypes.Structure):
    """struct cholmod_server_cfg of the header."""
    _fields_ = [("ws_bytes", ctypes.c_size_t), ("max_batch", ctypes.c_int32),
                ("device", ctypes.c_int32), ("streams", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Plan(ctypes.Structure):
    """struct cholmod_plan of the header."""
    _fields_ = [("schedule", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("order", ctypes.c_int32), ("poll", ctypes.c_int32), ("maps", ctypes.c_int32)]


class Desc(ctypes.Structure):
    """struct cholmod_desc of the header."""
    _fields_ = [("L", ctypes.c_void_p), ("V", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("k", ctypes.c_int64), ("ldl", ctypes.c_int64), ("sigma", ctypes.c_int32),
                ("dtype", ctypes.c_int32)]

_lib = None


class LibraryMissing(RuntimeError):
    pass


def load():
    """Load the built library (raises LibraryMissing if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing("%s is not built; run python -m paper_1011_1173_amd.build" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    p, i64, ci, cu, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint,
                          ctypes.c_size_t)
    lib.cholmod_version.argtypes = []
    lib.cholmod_version.restype = ci
    lib.cholmod_status_string.argtypes = [ci]
    lib.cholmod_status_string.restype = ctypes.c_char_p
    lib.cholmod_decode_info.argtypes = [i64, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.cholmod_decode_info.restype = ci
    lib.cholmod_workspace_bytes.argtypes = [i64, i64, ci]
    lib.cholmod_workspace_bytes.restype = sz
    lib.cholmod_update.argtypes = [p, p, i64, i64, i64, ci, p]
    lib.cholmod_update.restype = ci
    lib.cholmod_update_async.argtypes = [p, p, i64, i64, i64, ci, p, sz, p, p]
    lib.cholmod_update_async.restype = ci
    lib.cholmod_update_ex.argtypes = [p, p, i64, i64, i64, ci, cu, p, sz, p, p]
    lib.cholmod_update_ex.restype = ci
    lib.cholmod_noalloc_max_bytes.argtypes = []
    lib.cholmod_noalloc_max_bytes.restype = sz
    lib.cholmod_update_noalloc.argtypes = [p, p, i64, i64, i64, ci, p, p]
    lib.cholmod_update_noalloc.restype = ci
    lib.cholmod_probe_latency.argtypes = [ci, ci, ci, ctypes.POINTER(ctypes.c_double), p]
    lib.cholmod_probe_latency.restype = ci
    lib.cholmod_update_f32s.argtypes = [p, p, i64, i64, i64, ci, p]
    lib.cholmod_update_f32s.restype = ci
    lib.cholmod_update_f32s_async.argtypes = [p, p, i64, i64, i64, ci, p, sz, p, p]
    lib.cholmod_update_f32s_async.restype = ci
    lib.cholmod_update_f32s_ex.argtypes = [p, p, i64, i64, i64, ci, ctypes.c_uint, p, sz, p, p]
    lib.cholmod_update_f32s_ex.restype = ci
    lib.cholmod_workspace_bytes_ooc.argtypes = [i64, i64, ci]
    lib.cholmod_workspace_bytes_ooc.restype = sz
    lib.cholmod_update_ooc.argtypes = [p, p, i64, i64, i64, ci, ci, p, sz,
                                       ctypes.POINTER(i64), p]
    lib.cholmod_update_ooc.restype = ci
    dp = ctypes.POINTER(Desc)
    lib.cholmod_workspace_bytes_batched.argtypes = [dp, i64]
    lib.cholmod_workspace_bytes_batched.restype = sz
    lib.cholmod_update_batched.argtypes = [dp, i64, p, sz, p, p]
    lib.cholmod_batch_graph_create.argtypes = [dp, i64, p, sz, p, ctypes.POINTER(p)]
    lib.cholmod_batch_graph_create.restype = ci
    lib.cholmod_batch_graph_launch.argtypes = [p, p]
    lib.cholmod_batch_graph_launch.restype = ci
    lib.cholmod_batch_graph_destroy.argtypes = [p]
    lib.cholmod_batch_graph_destroy.restype = ci
    lib.cholmod_update_batched.restype = ci
    pp = ctypes.POINTER(Plan)
    lib.cholmod_update_batched_plan.argtypes = [dp, i64, pp, p, sz, p, p]
    lib.cholmod_update_batched_plan.restype = ci
    lib.cholmod_set_plan.argtypes = [ci, ci, ci, pp]
    lib.cholmod_set_plan.restype = ci
    lib.cholmod_get_plan.argtypes = [ci, ci, ci, pp]
    lib.cholmod_get_plan.restype = ci
    lib.cholmod_plan_bucket.argtypes = [i64, i64, ctypes.POINTER(ci), ctypes.POINTER(ci)]
    lib.cholmod_plan_bucket.restype = ci
    lib.cholmod_compute_units.argtypes = []
    lib.cholmod_compute_units.restype = ci
    lib.cholmod_server_create.argtypes = [ctypes.POINTER(ServerCfg), ctypes.POINTER(p)]
    lib.cholmod_server_create.restype = ci
    lib.cholmod_server_add_factor.argtypes = [p, p, i64, i64, ci, ctypes.POINTER(ctypes.c_int32)]
    lib.cholmod_server_add_factor.restype = ci
    lib.cholmod_server_submit.argtypes = [p, ctypes.c_int32, p, i64, ci,
                                          ctypes.POINTER(ctypes.c_uint64)]
    lib.cholmod_server_submit.restype = ci
    lib.cholmod_server_poll.argtypes = [p, ctypes.c_uint64, ctypes.POINTER(ci),
                                        ctypes.POINTER(ctypes.c_double)]
    lib.cholmod_server_poll.restype = ci
    lib.cholmod_server_drain.argtypes = [p]
    lib.cholmod_server_drain.restype = ci
    lib.cholmod_server_destroy.argtypes = [p]
    lib.cholmod_server_destroy.restype = ci
    _lib = lib
    return lib


def status_string(code: int) -> str:
    return load().cholmod_status_string(int(code)).decode()


def decode_info(info: int, k: int):
    row, col = ctypes.c_int64(-1), ctypes.c_int64(-1)
    st = load().cholmod_decode_info(int(info), int(k), ctypes.byref(row), ctypes.byref(col))
    return st, row.value, col.value


def workspace_bytes(n: int, k: int, dtype: int = F64) -> int:
    return int(load().cholmod_workspace_bytes(int(n), int(k), int(dtype)))


def probe_latency(k: int = 16, blocks: int = 200, rounds: int = 2000, stream=None):
    """cholmod_probe_latency: (ns per chain step, ns per 64-row block's chain,
    ns per hand-off across XCDs, ns per hand-off within one XCD)."""
    out = (ctypes.c_double * 4)()
    st = load().cholmod_probe_latency(int(k), int(blocks), int(rounds), out, stream)
    if st != OK:
        raise RuntimeError("cholmod_probe_latency: %s" % status_string(st))
    return tuple(out)

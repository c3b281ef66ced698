"""Rank-k Cholesky modification on AMD Instinct MI355X (gfx950).

Given an upper-triangular factor L with A = L^T L, an n x k matrix V and
sigma = +1 / -1, ``update(L, V, sigma)`` overwrites L in place with the upper
factor of A + sigma V V^T, using the hyperbolic Compute/Apply rotations of
Algorithm 1 (CholeskyModifyB) of Walder 2010, "Rank k Cholesky
Up/Down-dating on the GPU".  All arithmetic runs in the HIP kernels of
``libcholmod_mi355x.so``; PyTorch only supplies device memory and streams.
This module only checks and marshals arguments.
"""
from __future__ import annotations

import ctypes

import torch

from . import _native
from ._native import (ERR_ARG, ERR_BAD_DIAG, ERR_HIP, ERR_NOT_PD, F32S, F64, FLAG_BLOCKED,
                      FLAG_EXACT, INFO_NONE, OK, LibraryMissing)

__all__ = ["update", "update_async", "update_batched", "update_batched_async", "load_plans",
           "update_ooc", "workspace_bytes", "workspace_bytes_ooc", "BatchGraph", "CholmodError", "ArgumentError", "NotPositiveDefinite",
           "BadDiagonal", "HipError", "LibraryMissing", "Pending", "PendingBatch", "Server"]


class CholmodError(RuntimeError):
    status = None


class ArgumentError(CholmodError, ValueError):
    status = ERR_ARG


class HipError(CholmodError):
    status = ERR_HIP


class _NumericalError(CholmodError):
    def __init__(self, row: int, col: int):
        self.row, self.col = row, col
        super().__init__("%s at row %d, column %d" % (self.what, row, col))


class NotPositiveDefinite(_NumericalError):
    """A + sigma V V^T is not positive definite (first failing Compute step)."""
    status = ERR_NOT_PD
    what = "modified matrix is not positive definite"


class BadDiagonal(_NumericalError):
    """The input factor has a diagonal entry that is not > 0."""
    status = ERR_BAD_DIAG
    what = "input factor has a diagonal entry that is not > 0"


def _raise_for(status: int, row: int = -1, col: int = -1):
    if status == OK:
        return
    if status == ERR_NOT_PD:
        raise NotPositiveDefinite(row, col)
    if status == ERR_BAD_DIAG:
        raise BadDiagonal(row, col)
    if status == ERR_ARG:
        raise ArgumentError(_native.status_string(status))
    raise HipError(_native.status_string(status))


def workspace_bytes(n: int, k: int, dtype: int = F64) -> int:
    """Device workspace bytes needed by update_async for an n x k problem."""
    return _native.workspace_bytes(n, k, dtype)


def _factor_args(L: torch.Tensor, V: torch.Tensor):
    if not isinstance(L, torch.Tensor) or not isinstance(V, torch.Tensor):
        raise ArgumentError("L and V must be torch tensors")
    if L.dtype not in (torch.float64, torch.float32) or V.dtype != L.dtype:
        raise ArgumentError("L and V must both be float64, or both float32 (FP32 storage)")
    if L.device.type != "cuda" or V.device != L.device:
        raise ArgumentError("L and V must be on the same GPU")
    if L.dim() != 2 or L.stride(1) != 1 or L.shape[1] < L.shape[0]:
        raise ArgumentError("L must be (n, >= n) with unit column stride")
    n = L.shape[0]
    ldl = L.stride(0) if n > 1 else max(1, L.shape[1])
    if ldl < max(1, n):
        raise ArgumentError("row stride of L must be >= n")
    if V.dim() == 1:
        V = V.view(-1, 1)
    if V.dim() != 2 or V.shape[0] != n:
        raise ArgumentError("V must be (n, k)")
    if not V.is_contiguous():
        raise ArgumentError("V must be contiguous (row-major)")
    return n, V.shape[1], ldl, V


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Pending:
    """An enqueued modification; keeps its workspace alive until checked."""

    def __init__(self, k, ws, info, stream):
        self.k, self._ws, self.info, self.stream = k, ws, info, stream

    def status(self):
        """Wait for the stream and return (status, row, col)."""
        self.stream.synchronize()
        return _native.decode_info(int(self.info.item()), self.k)

    def wait(self):
        """Wait and raise on a numerical failure."""
        st, row, col = self.status()
        _raise_for(st, row, col)


def update_async(L: torch.Tensor, V: torch.Tensor, sigma: int, *, exact: bool = False,
                 blocked: bool = False, rotations: bool = False, stream=None,
                 workspace: torch.Tensor | None = None,
                 info: torch.Tensor | None = None) -> Pending:
    """Enqueue the rank-k modification of L on ``stream``; no host sync.

    float64 tensors use cholmod_update_ex (``exact`` / ``blocked`` select the
    evaluation mode and schedule); float32 tensors use the FP32-storage mode
    cholmod_update_f32s_ex, which has neither option.  ``rotations``: apply
    every block by its rotations (no block maps) in the fast schedule.
    """
    n, k, ldl, V = _factor_args(L, V)
    f32 = L.dtype == torch.float32
    if f32 and (exact or blocked):
        raise ArgumentError("FP32 storage has no exact or blocked mode")
    stream = torch.cuda.current_stream(L.device) if stream is None else stream
    need = workspace_bytes(n, k, F32S if f32 else F64)
    if workspace is None:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=L.device)
    if info is None:
        info = torch.empty(1, dtype=torch.int64, device=L.device)
    lib = _native.load()
    args = (ctypes.c_void_p(L.data_ptr()), ctypes.c_void_p(V.data_ptr()), n, k, ldl, int(sigma))
    tail = (ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
            ctypes.c_void_p(info.data_ptr()), _stream_handle(stream))
    rot = _native.FLAG_ROTATIONS if rotations else 0
    if f32:
        st = lib.cholmod_update_f32s_ex(*args, rot, *tail)
    else:
        flags = (FLAG_EXACT if exact else 0) | (FLAG_BLOCKED if blocked else 0) | rot
        st = lib.cholmod_update_ex(*args, flags, *tail)
    _raise_for(st)
    return Pending(k, workspace, info, stream)


def update(L: torch.Tensor, V: torch.Tensor, sigma: int, *, exact: bool = False,
           blocked: bool = False, rotations: bool = False, stream=None) -> None:
    """Overwrite L (upper, on the GPU; float64, or float32 for FP32 storage)
    with the factor of L^T L + sigma V V^T.

    Raises NotPositiveDefinite / BadDiagonal with the first failing (row,
    column), or ArgumentError for bad shapes and types.
    """
    update_async(L, V, sigma, exact=exact, blocked=blocked, rotations=rotations,
                 stream=stream).wait()


def workspace_bytes_ooc(n: int, k: int, dtype: int = F64) -> int:
    """Device workspace bytes of update_ooc for an n x k problem (O(n (64 + k)))."""
    return int(_native.load().cholmod_workspace_bytes_ooc(n, k, dtype))


def update_ooc(L: torch.Tensor, V: torch.Tensor, sigma: int, *, stream=None,
               workspace: torch.Tensor | None = None) -> None:
    """Out-of-core form (cholmod_update_ooc): L is a HOST tensor (float64, or
    float32 for FP32 storage; pinned memory copies fastest) streamed through
    the GPU in 64-row panels; V is on the GPU.  Synchronous; raises like
    ``update``."""
    if not isinstance(L, torch.Tensor) or not isinstance(V, torch.Tensor):
        raise ArgumentError("L and V must be torch tensors")
    if L.device.type != "cpu":
        raise ArgumentError("L must be a host (CPU) tensor")
    if L.dtype not in (torch.float64, torch.float32) or V.dtype != L.dtype:
        raise ArgumentError("L and V must both be float64, or both float32 (FP32 storage)")
    if V.device.type != "cuda":
        raise ArgumentError("V must be on the GPU")
    if L.dim() != 2 or L.stride(1) != 1 or L.shape[1] < L.shape[0]:
        raise ArgumentError("L must be (n, >= n) with unit column stride")
    n = L.shape[0]
    ldl = L.stride(0) if n > 1 else max(1, L.shape[1])
    if V.dim() == 1:
        V = V.view(-1, 1)
    if V.dim() != 2 or V.shape[0] != n or not V.is_contiguous():
        raise ArgumentError("V must be a contiguous (n, k) tensor")
    k = V.shape[1]
    dtype = F32S if L.dtype == torch.float32 else F64
    stream = torch.cuda.current_stream(V.device) if stream is None else stream
    lib = _native.load()
    ws_ptr, ws_len = None, 0
    if workspace is not None:
        ws_ptr, ws_len = ctypes.c_void_p(workspace.data_ptr()), workspace.numel()
    info = ctypes.c_int64(INFO_NONE)
    st = lib.cholmod_update_ooc(ctypes.c_void_p(L.data_ptr()), ctypes.c_void_p(V.data_ptr()),
                                n, k, ldl, int(sigma), dtype, ws_ptr, ws_len,
                                ctypes.byref(info), _stream_handle(stream))
    if st in (ERR_NOT_PD, ERR_BAD_DIAG):
        _, row, col = _native.decode_info(int(info.value), k)
        _raise_for(st, row, col)
    _raise_for(st)


class PendingBatch:
    """An enqueued batch; keeps its workspace and descriptors alive."""

    def __init__(self, ks, ws, info, stream):
        self.ks, self._ws, self.info, self.stream = ks, ws, info, stream

    def statuses(self):
        """Wait for the stream; (status, row, col) of every factor."""
        self.stream.synchronize()
        raw = self.info.cpu().tolist()
        return [_native.decode_info(int(r), k) for r, k in zip(raw, self.ks)]


def _descs(Ls, Vs, sigmas):
    """Descriptor array of a batch.  The checks of _factor_args, inlined with
    as few tensor queries as possible (a batch has hundreds of factors and
    this runs on the host before every batched call); any factor that fails
    them goes through _factor_args for its error message."""
    count = len(Ls)
    if not (count == len(Vs) == len(sigmas)):
        raise ArgumentError("Ls, Vs and sigmas must have the same length")
    arr = (_native.Desc * max(1, count))()
    ks = [0] * count
    dev = None
    f64, f32, Desc = torch.float64, torch.float32, _native.Desc
    for i in range(count):
        L, V = Ls[i], Vs[i]
        try:
            dt = L.dtype
            d = L.device
            shp, st = L.shape, L.stride()
            if V.dim() == 1:
                V = V.view(-1, 1)
            vs = V.shape
            n = shp[0]
            ldl = st[0] if n > 1 else max(1, shp[1])
            ok = ((dt is f64 or dt is f32) and V.dtype is dt and d.type == "cuda"
                  and V.device == d and len(shp) == 2 and st[1] == 1 and shp[1] >= n
                  and ldl >= max(1, n) and len(vs) == 2 and vs[0] == n and V.is_contiguous())
        except (AttributeError, TypeError, IndexError, RuntimeError):
            ok = False
        if not ok:
            _factor_args(L, V)  # raises ArgumentError with the reason
            raise ArgumentError("factor %d: unsupported L or V" % i)
        if dev is None:
            dev = d
        elif d != dev:
            raise ArgumentError("all factors of a batch must be on one GPU")
        arr[i] = Desc(L.data_ptr(), V.data_ptr(), n, vs[1], ldl, int(sigmas[i]),
                      F32S if dt is f32 else F64)
        ks[i] = vs[1]
    return arr, ks, dev


_plans_loaded = False


def _ensure_plans():
    """Load the shipped plan cache into the library once (before the first
    batched call); without a cache the library's default plan applies."""
    global _plans_loaded
    if not _plans_loaded:
        _plans_loaded = True
        from . import tune
        tune.load_plans()


def update_batched_async(Ls, Vs, sigmas, *, stream=None, workspace: torch.Tensor | None = None,
                         info: torch.Tensor | None = None, plan=None) -> PendingBatch:
    """Enqueue the modification of every factor Ls[i] by (Vs[i], sigmas[i])
    (cholmod_update_batched); float64 and float32 factors may be mixed.
    ``plan``: a launch plan (dict with schedule, grid, order, poll, or a
    _native.Plan) instead of the library's plan table."""
    arr, ks, dev = _descs(Ls, Vs, sigmas)
    count = len(ks)
    if count == 0:
        raise ArgumentError("empty batch")
    stream = torch.cuda.current_stream(dev) if stream is None else stream
    lib = _native.load()
    _ensure_plans()
    need = int(lib.cholmod_workspace_bytes_batched(arr, count))
    if need == 0:
        raise ArgumentError("invalid batch")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    if info is None:
        info = torch.empty(count, dtype=torch.int64, device=dev)
    if plan is not None and not isinstance(plan, _native.Plan):
        plan = _native.Plan(int(plan.get("schedule", 0)), int(plan.get("grid", 0)),
                            int(plan.get("order", 0)), int(plan.get("poll", 2)),
                            int(plan.get("maps", 1)))
    st = lib.cholmod_update_batched_plan(arr, count,
                                         ctypes.byref(plan) if plan is not None else None,
                                         ctypes.c_void_p(workspace.data_ptr()),
                                         workspace.numel(), ctypes.c_void_p(info.data_ptr()),
                                         _stream_handle(stream))
    _raise_for(st)
    return PendingBatch(ks, workspace, info, stream)


def update_batched(Ls, Vs, sigmas, *, stream=None, plan=None):
    """Modify every factor and wait; returns [(status, row, col)] per factor
    (a numerical failure in one factor does not raise and does not affect
    the others)."""
    return update_batched_async(Ls, Vs, sigmas, stream=stream, plan=plan).statuses()


class BatchGraph:
    """A batch captured once as a HIP graph (cholmod_batch_graph_*) and
    replayed by ``launch``: each replay modifies every factor Ls[i] by
    (Vs[i], sigmas[i]) from their current contents.  Keeps the tensors, the
    workspace and the info words alive until ``close``."""

    def __init__(self, Ls, Vs, sigmas):
        arr, ks, dev = _descs(Ls, Vs, sigmas)
        count = len(ks)
        if count == 0:
            raise ArgumentError("empty batch")
        lib = _native.load()
        _ensure_plans()
        need = int(lib.cholmod_workspace_bytes_batched(arr, count))
        if need == 0:
            raise ArgumentError("invalid batch")
        self._keep = (list(Ls), list(Vs))
        self.ks, self.device = ks, dev
        self.workspace = torch.empty(need, dtype=torch.uint8, device=dev)
        self.info = torch.empty(count, dtype=torch.int64, device=dev)
        h = ctypes.c_void_p()
        st = lib.cholmod_batch_graph_create(arr, count, ctypes.c_void_p(self.workspace.data_ptr()),
                                            need, ctypes.c_void_p(self.info.data_ptr()),
                                            ctypes.byref(h))
        _raise_for(st)
        self._h = h

    def launch(self, stream=None):
        """Enqueue one replay on ``stream`` (default: the current stream)."""
        if self._h is None:
            raise ArgumentError("graph closed")
        stream = torch.cuda.current_stream(self.device) if stream is None else stream
        _raise_for(_native.load().cholmod_batch_graph_launch(self._h, _stream_handle(stream)))
        self.stream = stream

    def statuses(self):
        """Wait for the last replay's stream; (status, row, col) per factor."""
        self.stream.synchronize()
        raw = self.info.cpu().tolist()
        return [_native.decode_info(int(r), k) for r, k in zip(raw, self.ks)]

    def close(self):
        if self._h is not None:
            torch.cuda.synchronize(self.device)
            _native.load().cholmod_batch_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Served mode (cholmod_server_*): registered factors, submitted requests,
    continuous batching by a library worker thread: admission by the HBM
    budget ``ws_bytes``, up to ``streams`` batches in flight at once, a
    request complete as soon as its factor is.  The Python object keeps every
    registered factor and every pending V alive."""

    def __init__(self, ws_bytes: int = 1 << 30, max_batch: int = 256, device=None,
                 streams: int = 4):
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        _ensure_plans()
        cfg = _native.ServerCfg(int(ws_bytes), int(max_batch), int(dev.index), int(streams), 0)
        h = ctypes.c_void_p()
        _raise_for(_native.load().cholmod_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h, self.device = h, dev
        self._factors, self._pending = [], {}

    def add_factor(self, L: torch.Tensor) -> int:
        n, _, ldl, _ = _factor_args(L, torch.empty((L.shape[0], 0), dtype=L.dtype,
                                                   device=L.device))
        # the server's stream does not wait for the caller's: L must be written
        torch.cuda.current_stream(L.device).synchronize()
        fid = ctypes.c_int32(-1)
        _raise_for(_native.load().cholmod_server_add_factor(
            self._h, ctypes.c_void_p(L.data_ptr()), n, ldl,
            F32S if L.dtype == torch.float32 else F64, ctypes.byref(fid)))
        self._factors.append((L, L.dtype))
        return fid.value

    def submit(self, fid: int, V: torch.Tensor, sigma: int) -> int:
        if not 0 <= fid < len(self._factors):
            raise ArgumentError("unknown factor")
        L, dt = self._factors[fid]
        if V.dim() == 1:
            V = V.view(-1, 1)
        if V.dtype != dt or V.device != L.device or not V.is_contiguous() or V.shape[0] != L.shape[0]:
            raise ArgumentError("V must be a contiguous (n, k) tensor of the factor's dtype and device")
        # the server's stream does not wait for the caller's: V must be written
        torch.cuda.current_stream(V.device).synchronize()
        t = ctypes.c_uint64(0)
        _raise_for(_native.load().cholmod_server_submit(
            self._h, int(fid), ctypes.c_void_p(V.data_ptr()), V.shape[1], int(sigma),
            ctypes.byref(t)))
        self._pending[t.value] = V
        return t.value

    def poll(self, ticket: int):
        """None while pending, else (status, latency_s)."""
        st, lat = ctypes.c_int(0), ctypes.c_double(0.0)
        rc = _native.load().cholmod_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(st),
                                                ctypes.byref(lat))
        if rc == 1:
            return None
        _raise_for(rc)
        self._pending.pop(ticket, None)
        return st.value, lat.value

    def drain(self):
        _raise_for(_native.load().cholmod_server_drain(self._h))

    def close(self):
        if self._h is not None:
            _raise_for(_native.load().cholmod_server_destroy(self._h))
            self._h = None
            self._pending.clear()

    def __del__(self):
        # a server left open would keep its worker thread (which makes HIP
        # calls) running into interpreter shutdown
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def load_plans(path: str | None = None) -> int:
    """Fill the library's plan table from an autotuner plan cache (JSON, see
    tune.py); default: the cache shipped for this GPU architecture, if any.
    Returns the number of entries set."""
    from . import tune
    return tune.load_plans(path)

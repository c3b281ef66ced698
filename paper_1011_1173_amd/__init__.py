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

__all__ = ["update", "update_async", "workspace_bytes", "CholmodError", "ArgumentError",
           "NotPositiveDefinite", "BadDiagonal", "HipError", "LibraryMissing", "Pending"]


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


def _factor_args(L: torch.Tensor, V: torch.Tensor, dtype: torch.dtype):
    if not isinstance(L, torch.Tensor) or not isinstance(V, torch.Tensor):
        raise ArgumentError("L and V must be torch tensors")
    if L.dtype != dtype or V.dtype != dtype:
        raise ArgumentError("L and V must have dtype %s" % dtype)
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
                 blocked: bool = False, stream=None, workspace: torch.Tensor | None = None,
                 info: torch.Tensor | None = None) -> Pending:
    """Enqueue the rank-k modification of L (FP64) on ``stream``; no host sync."""
    n, k, ldl, V = _factor_args(L, V, torch.float64)
    stream = torch.cuda.current_stream(L.device) if stream is None else stream
    need = workspace_bytes(n, k, F64)
    if workspace is None:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=L.device)
    if info is None:
        info = torch.empty(1, dtype=torch.int64, device=L.device)
    flags = (FLAG_EXACT if exact else 0) | (FLAG_BLOCKED if blocked else 0)
    st = _native.load().cholmod_update_ex(
        ctypes.c_void_p(L.data_ptr()), ctypes.c_void_p(V.data_ptr()), n, k, ldl, int(sigma),
        flags, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
        ctypes.c_void_p(info.data_ptr()), _stream_handle(stream))
    _raise_for(st)
    return Pending(k, workspace, info, stream)


def update(L: torch.Tensor, V: torch.Tensor, sigma: int, *, exact: bool = False,
           blocked: bool = False, stream=None) -> None:
    """Overwrite L (upper, FP64, on the GPU) with the factor of L^T L + sigma V V^T.

    Raises NotPositiveDefinite / BadDiagonal with the first failing (row,
    column), or ArgumentError for bad shapes and types.
    """
    update_async(L, V, sigma, exact=exact, blocked=blocked, stream=stream).wait()

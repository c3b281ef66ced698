"""Seeded synthetic inputs for the rank-k Cholesky modification.

This module only draws random numbers and builds the starting factor with a
library Cholesky; it holds none of the modification's arithmetic, so both
the GPU path and the CPU oracle can be fed from it.

Recipe (the paper's experiments use i.i.d. uniform matrices, Section 5; the
workloads here use the Gaussian recipe stated for them):
  * G is n x n with i.i.d. N(0, 1) entries drawn from ``seed``;
  * A = G^T G + n I  (symmetric positive definite, well conditioned);
  * L is the upper Cholesky factor of A (A = L^T L), from the library
    routine ``torch.linalg.cholesky``;
  * V is n x k with i.i.d. N(0, 1) / sqrt(n) entries from ``seed + 7919``.
The downdate that matches an update by V uses the same V, so the updated
matrix stays positive definite.
"""
from __future__ import annotations

import math

import torch

V_SEED_OFFSET = 7919


def _gen(seed: int, device: str) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def spd_factor(n: int, seed: int, *, device: str = "cpu", ldl: int | None = None,
               dtype: torch.dtype = torch.float64, pad_value: float = 0.0) -> torch.Tensor:
    """Upper Cholesky factor of G^T G + n I as an (n, ldl) row-major tensor.

    G is drawn on ``device``.  The strictly lower triangle is zero and the
    padding columns n..ldl-1 hold ``pad_value``.
    """
    ldl = n if ldl is None else ldl
    if ldl < max(1, n):
        raise ValueError("ldl must be >= max(1, n)")
    out = torch.full((n, ldl), pad_value, dtype=dtype, device=device)
    if n == 0:
        return out
    G = torch.randn(n, n, generator=_gen(seed, device), dtype=torch.float64, device=device)
    A = G.T @ G
    A.diagonal().add_(float(n))
    del G
    U = torch.linalg.cholesky(A, upper=True)
    del A
    out[:, :n] = U.to(dtype)
    if pad_value != 0.0:
        lower = torch.tril(torch.ones(n, n, dtype=torch.bool, device=device), diagonal=-1)
        out[:, :n][lower] = pad_value
    return out


def update_vectors(n: int, k: int, seed: int, *, device: str = "cpu",
                   dtype: torch.dtype = torch.float64) -> torch.Tensor:
    """V of shape (n, k), i.i.d. N(0, 1) / sqrt(n), row-major contiguous."""
    if n == 0 or k == 0:
        return torch.zeros(n, k, dtype=dtype, device=device)
    g = _gen(seed + V_SEED_OFFSET, device)
    V = torch.randn(n, k, generator=g, dtype=torch.float64, device=device)
    V.mul_(1.0 / math.sqrt(n))
    return V.to(dtype).contiguous()


def config_inputs(n: int, k: int, seed: int, *, device: str = "cpu", ldl: int | None = None,
                  dtype: torch.dtype = torch.float64):
    """(L, V) for one synthetic problem of the configured shape."""
    return (spd_factor(n, seed, device=device, ldl=ldl, dtype=dtype),
            update_vectors(n, k, seed, device=device, dtype=dtype))

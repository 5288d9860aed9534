"""Nystrom approximation on the device (Sec. 5, Alg. 2):

    A~ = B C^+ B^T,   B = A Omega,   C = Omega^T B,

for a symmetric positive semidefinite A, with Omega generated from the seed.
The two products are the library's kernels (sketch_gen_matmul for B,
sketch_gen_tmatmul for C, Omega regenerated, never stored).  The pseudo-inverse
of the r x r core and the error check around them use torch's FP64 linear
algebra on the device: they are the application of the sketch, not its path.

Pseudo-inverse tolerance: the paper drops core eigenvalues below 1e-12 of the
largest (Sec. 6.2), which presumes FP64 products.  B and C here carry FP32
rounding (relative error ~ r * 2^-24), so eigenvalues below that level are
noise; the default tolerance is max(1e-12, r * 2^-24).
"""
from __future__ import annotations

import torch

from . import sketch_gen_matmul, sketch_gen_tmatmul


def default_tol(r: int) -> float:
    return max(1e-12, r * 2.0 ** -24)


def core_pinv(C: torch.Tensor, tol: float) -> torch.Tensor:
    """FP64 pseudo-inverse of the symmetric part of C, eigenvalues with
    |lambda| <= tol * max |lambda| treated as zero."""
    S = C.double()
    S = 0.5 * (S + S.t())
    lam, V = torch.linalg.eigh(S)
    keep = lam.abs() > tol * lam.abs().max()
    inv = torch.where(keep, 1.0 / torch.where(keep, lam, torch.ones_like(lam)),
                      torch.zeros_like(lam))
    return (V * inv) @ V.t()


def nystrom(A: torch.Tensor, r: int, seed: int, *, dist="normal", tol: float | None = None,
            stream=None):
    """Factors of the Nystrom approximation of a symmetric FP32 A (n x n, row-major):
    returns (B, C, C_pinv) with B = A Omega (FP32, n x r, rows 16-byte aligned),
    C = Omega^T B (FP32, r x r) and the FP64 pseudo-inverse of C."""
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    ld = (r + 3) // 4 * 4
    B = torch.empty((n, ld), dtype=torch.float32, device=A.device)[:, :r]
    sketch_gen_matmul(A, seed, r, Y=B, stream=stream, dist=dist)
    C = sketch_gen_tmatmul(B, seed, r, stream=stream, dist=dist)
    return B, C, core_pinv(C, default_tol(r) if tol is None else tol)


def reconstruct_rows(B: torch.Tensor, C_pinv: torch.Tensor, rows: slice) -> torch.Tensor:
    """Rows of A~ = B C^+ B^T in FP64."""
    Bd = B.double()
    return (Bd[rows] @ C_pinv) @ Bd.t()


def relative_error(A: torch.Tensor, B: torch.Tensor, C_pinv: torch.Tensor,
                   block_rows: int = 2048) -> float:
    """||A - B C^+ B^T||_F / ||A||_F, accumulated over row blocks in FP64."""
    n = A.shape[0]
    Bd = B.double()
    W = Bd @ C_pinv
    Bt = Bd.t().contiguous()
    num = torch.zeros((), dtype=torch.float64, device=A.device)
    den = torch.zeros((), dtype=torch.float64, device=A.device)
    for i in range(0, n, block_rows):
        blk = A[i:i + block_rows].double()
        diff = blk - W[i:i + block_rows] @ Bt
        num += (diff * diff).sum()
        den += (blk * blk).sum()
    return float((num / den).sqrt())


__all__ = ["nystrom", "core_pinv", "default_tol", "reconstruct_rows", "relative_error"]

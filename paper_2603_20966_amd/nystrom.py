"""Nystrom approximation on the device (Sec. 5, Alg. 2):

    A~ = B C^+ B^T,   B = A Omega,   C = Omega^T B,

for a symmetric positive semidefinite A, with Omega generated from the seed.
Every step is a library call: sketch_gen_matmul for B, sketch_gen_tmatmul for
C (Omega regenerated, never stored), sketch_core_pinv for the FP64
pseudo-inverse of the core (block Jacobi eigensolver, eigenvalues at most tol
times the largest dropped; the paper's tolerance is 1e-12, Sec. 6.2), and
sketch_nystrom_error / sketch_nystrom_rows for the relative Frobenius error of
Table 2 and rows of A~.  torch only provides the device buffers.
"""
from __future__ import annotations

import torch

from . import (sketch_core_pinv, sketch_gen_matmul, sketch_gen_tmatmul, sketch_nystrom_error,
               sketch_nystrom_rows)

PAPER_TOL = 1e-12


def core_pinv(C: torch.Tensor, tol: float = PAPER_TOL, *, max_sweeps: int = 16, stream=None):
    """(C^+, info): FP64 pseudo-inverse of the symmetric part of C; info = device int32
    (sweeps run, converged)."""
    return sketch_core_pinv(C, tol, max_sweeps=max_sweeps, stream=stream)


def nystrom(A: torch.Tensor, r: int, seed: int, *, dist="normal", tol: float = PAPER_TOL,
            max_sweeps: int = 16, stream=None):
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
    Cp, _ = sketch_core_pinv(C, tol, max_sweeps=max_sweeps, stream=stream)
    return B, C, Cp


def reconstruct_rows(B: torch.Tensor, C_pinv: torch.Tensor, rows: slice, stream=None) -> torch.Tensor:
    """Rows of A~ = B C^+ B^T in FP64."""
    start, stop, _ = rows.indices(B.shape[0])
    return sketch_nystrom_rows(B, C_pinv, start, max(stop - start, 0), stream=stream)


def relative_error(A: torch.Tensor, B: torch.Tensor, C_pinv: torch.Tensor, stream=None) -> float:
    """||A - B C^+ B^T||_F / ||A||_F, from the library's FP64 sums."""
    return float(sketch_nystrom_error(A, B, C_pinv, stream=stream)[2].item())


__all__ = ["nystrom", "core_pinv", "reconstruct_rows", "relative_error", "PAPER_TOL"]

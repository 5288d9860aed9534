"""Oracle of the Nystrom approximation (Sec. 5, Alg. 2) -- TEST INFRASTRUCTURE ONLY.

    A~ = (A Omega) (Omega^T A Omega)^+ (A Omega)^T

for a symmetric positive semidefinite A and the generated Omega of the sketch
library's definition (oracle.omega_block).  Plain FP64 numpy: B = A Omega and
C = Omega^T B as FP64 products, the pseudo-inverse of the symmetric core C by
its eigendecomposition, discarding eigenvalues below tol * max|eigenvalue|
(the paper builds the pseudo-inverse with tolerance 1e-12, Sec. 6.2), and the
relative Frobenius error ||A - A~|| / ||A||.
"""
from __future__ import annotations

import numpy as np

from . import omega_block


def core_pinv(C: np.ndarray, tol: float) -> np.ndarray:
    """Pseudo-inverse of the symmetric part of C, eigenvalues with |lambda| <= tol * max|lambda|
    treated as zero."""
    S = 0.5 * (C + C.T)
    lam, V = np.linalg.eigh(S)
    big = np.abs(lam) > tol * np.abs(lam).max() if lam.size else lam
    inv = np.zeros_like(lam)
    inv[big] = 1.0 / lam[big]
    return (V * inv) @ V.T


def nystrom(A: np.ndarray, r: int, seed: int, dist="normal", tol: float = 1e-12):
    """(B, C, A~, relative Frobenius error) for a symmetric n x n A (any float type)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    Om = omega_block(seed, 0, n, 0, r, dist).astype(np.float64)
    B = A @ Om
    C = Om.T @ B
    At = B @ core_pinv(C, tol) @ B.T
    err = np.linalg.norm(A - At) / np.linalg.norm(A)
    return B, C, At, float(err)

"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module draws test data only.  It holds none of the sketch's arithmetic:
the random operand Omega is never produced here (each side generates it from
the seed with its own Philox implementation).

Workload shapes follow the paper's regime (dense A, r << n; Sec. 6.2-6.4)
with iid N(0,1) entries standing in for the paper's datasets, which are not
available.
"""
from __future__ import annotations

import math

import numpy as np


def normal_matrix(m: int, n: int, seed: int, dtype=np.float32) -> np.ndarray:
    """m x n matrix of iid N(0,1) drawn by numpy's PCG64 from `seed`."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, n), dtype=np.float32).astype(dtype, copy=False)


def normal_matrix_device(m: int, n: int, seed: int, device, dtype=None):
    """m x n iid N(0,1) float32 tensor drawn on `device` by torch's own generator."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = torch.empty((m, n), dtype=torch.float32, device=device)
    # fill in row chunks to bound the generator's temporary memory
    step = max(1, (1 << 28) // max(n, 1))
    for r in range(0, m, step):
        out[r:r + step].normal_(generator=g)
    if dtype is not None:
        out = out.to(dtype)
    return out


def selection_matrix(m: int, n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """m x n FP32 matrix with a single 1 per row at a random column; returns (S, cols)."""
    rng = np.random.default_rng(seed)
    cols = rng.integers(0, n, size=m)
    S = np.zeros((m, n), dtype=np.float32)
    S[np.arange(m), cols] = 1.0
    return S, cols


def request_stream(count: int, seed: int, rate_per_s: float, mn_lo: int = 1024,
                   mn_hi: int = 32768, ks=(5, 16, 64)):
    """Poisson stream of sketch requests.

    Returns a list of dicts with arrival time (s), m, n (independent
    log-uniform in [mn_lo, mn_hi]), k (uniform over ks), the seed of A and
    the seed of Omega (distinct per request).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    lo, hi = math.log(mn_lo), math.log(mn_hi)
    for r in range(count):
        t += rng.exponential(1.0 / rate_per_s)
        m = int(round(math.exp(rng.uniform(lo, hi))))
        n = int(round(math.exp(rng.uniform(lo, hi))))
        k = int(ks[rng.integers(0, len(ks))])
        out.append({"id": r, "arrival_s": t, "m": m, "n": n, "k": k,
                    "seed_a": 1_000_000 + r, "seed_omega": 2_000_000 + r})
    return out


def kernel_matrix(kind: str, n: int, seed: int, latent: int = 40, dim: int = 256,
                  noise: float = 0.0, device=None):
    """Synthetic symmetric PSD kernel matrix (stand-in for the paper's CIFAR-10 kernels,
    Sec. 6.2): data X = Z W (+ noise), Z n x latent and W latent x dim iid N(0,1), rows of
    X as samples; kind "linear": A = X X^T (rank <= latent); kind "rbf":
    A_ij = exp(-|x_i - x_j|^2 / (2 sigma^2)) with sigma = ||X||_F / sqrt(n).
    FP32 result; numpy on the host, or torch on `device` (generated there)."""
    if device is None:
        rng = np.random.default_rng(seed)
        Z = rng.standard_normal((n, latent))
        W = rng.standard_normal((latent, dim)) / math.sqrt(latent)
        X = Z @ W
        if noise:
            X += noise * rng.standard_normal((n, dim))
        if kind == "linear":
            return (X @ X.T).astype(np.float32)
        sq = (X * X).sum(1)
        D = np.maximum(sq[:, None] + sq[None, :] - 2.0 * X @ X.T, 0.0)
        sigma2 = (X * X).sum() / n
        return np.exp(-D / (2.0 * sigma2)).astype(np.float32)
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    Z = torch.randn((n, latent), generator=g, device=device, dtype=torch.float32)
    W = torch.randn((latent, dim), generator=g, device=device, dtype=torch.float32) / math.sqrt(latent)
    X = Z @ W
    if noise:
        X += noise * torch.randn((n, dim), generator=g, device=device, dtype=torch.float32)
    if kind == "linear":
        return X @ X.t().contiguous()
    sq = (X * X).sum(1)
    sigma2 = (X * X).sum() / n
    A = X @ X.t().contiguous()
    A.mul_(-2.0).add_(sq[:, None]).add_(sq[None, :]).clamp_(min=0.0)
    return A.mul_(-0.5 / sigma2).exp_()

"""Exact solves with the H^1 Gram operator A (the paper's unperturbed
"Laplace" problem whose inverse the Woodbury formula wraps, Section 3).

dct_solve: A is a Kronecker sum after scaling by W^{-1}:
    W^{-1} A = sum_d (W1^{-1} K1)^(d) + beta*I,
and W1^{-1} K1 has eigenvectors cos(j*pi*i/(n-1)) with eigenvalues
(4/h^2) sin^2(j*pi/(2(n-1))), j = 0..n-1. The type-I DCT maps grid values to
these cosine coefficients, so
    A^{-1} f = IDCT1[ DCT1(W^{-1} f) / (beta + sum_d lambda_{j_d}) ].

lu_solve: scipy's sparse LU of the assembled A (independent route).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.sparse.linalg as spla

from . import operator as op


def eigenvalues_1d(n: int, h: float) -> np.ndarray:
    """lambda_j = (4/h^2) sin^2(j pi / (2(n-1))), j = 0..n-1."""
    j = np.arange(n)
    return 4.0 / h ** 2 * np.sin(j * np.pi / (2 * (n - 1))) ** 2


def _grid(shape, v):
    return np.asarray(v, dtype=np.float64).reshape(tuple(reversed(shape)))


def dct_solve(shape, beta: float, F: np.ndarray, workers: int = -1) -> np.ndarray:
    """X = A^{-1} F for F of shape (N,) or (k, N)."""
    F = np.asarray(F, dtype=np.float64)
    if F.ndim == 2:
        return np.stack([dct_solve(shape, beta, f, workers) for f in F])
    hs = op.spacing(shape)
    Winv = 1.0 / _grid(shape, op.lumped_mass(shape).diagonal())
    g = sfft.dctn(_grid(shape, F) * Winv, type=1, workers=workers)
    denom = np.full(g.shape, beta)
    for d, n in enumerate(shape):       # axis d of the grid array is reversed
        lam = eigenvalues_1d(n, hs[d])
        s = [1] * len(shape)
        s[len(shape) - 1 - d] = n
        denom = denom + lam.reshape(s)
    return sfft.idctn(g / denom, type=1, workers=workers).reshape(-1)


def lu_solve(shape, beta: float, F: np.ndarray) -> np.ndarray:
    """X = A^{-1} F through a sparse LU factorisation of the assembled A."""
    A = op.gram_operator(shape, beta).tocsc()
    lu = spla.splu(A)
    F = np.asarray(F, dtype=np.float64)
    return np.stack([lu.solve(f) for f in F]) if F.ndim == 2 else lu.solve(F)

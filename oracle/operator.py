"""Discrete H^1 Gram operator on a structured vertex-centred grid.

The paper's linearised problem (Section 2.2, eq. (block_primal)) is
(L + (1/beta) J'J) dm = rhs with L the weak Laplacian; the H^1 norm of
Section 2.1 adds the L^2 term. On the unit square / cube with n_d nodes per
axis (h_d = 1/(n_d - 1), x fastest) we use

    A = sum_d  W1 (x) .. (x) K1^(d) (x) .. (x) W1   +   beta * W,     W = (x)_d W1

with the 1D factors
    K1 = h^-2 * tridiag(-1, 2, -1), first and last diagonal entry 1 (Neumann)
    W1 = diag(1/2, 1, ..., 1, 1/2)  (trapezoid weights)

Interior rows are the textbook 5-/7-point -Laplacian + beta; A equals h^-d times
the Q1 Gram matrix of the H^1 inner product with vertex quadrature, so A is
symmetric positive definite with A*1 = beta*W*1 (the natural boundary
condition of Section 2.2 leaves constants in the kernel of the gradient part).
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.sparse as sp


def spacing(shape):
    """Mesh widths h_d = 1/(n_d - 1), one per axis (x first)."""
    return [1.0 / (n - 1) for n in shape]


def trapezoid_1d(n: int) -> np.ndarray:
    """Diagonal of W1: trapezoid-rule weights 1/2, 1, ..., 1, 1/2."""
    w = np.ones(n)
    w[0] = w[-1] = 0.5
    return w


def stiffness_1d(n: int, h: float) -> sp.csr_matrix:
    """K1 = h^-2 tridiag(-1, 2, -1) with Neumann corners (diagonal 1 at both ends)."""
    main = np.full(n, 2.0)
    main[0] = main[-1] = 1.0
    off = -np.ones(n - 1)
    return (sp.diags([off, main, off], [-1, 0, 1], format="csr") / h ** 2).tocsr()


def _kron_axes(factors):
    """Kronecker product with axis 0 (x) fastest: factors listed as [x, y, (z)]."""
    out = sp.csr_matrix(np.ones((1, 1)))
    for f in factors:          # x first ... slowest last: kron(slow, fast)
        out = sp.kron(f, out, format="csr")
    return out


def lumped_mass(shape) -> sp.csr_matrix:
    """W = W1 (x) ... (x) W1 as a diagonal sparse matrix."""
    return _kron_axes([sp.diags(trapezoid_1d(n)) for n in shape])


def gram_operator(shape, beta: float) -> sp.csr_matrix:
    """A = sum_d (K1 on axis d, W1 on the other axes) + beta*W  (CSR, float64).

    The assembled matrix of the last few (shape, beta) pairs is kept (a 257^3
    assembly takes tens of seconds); callers must not modify it."""
    return _gram_operator(tuple(int(n) for n in shape), float(beta))


@functools.lru_cache(maxsize=3)
def _gram_operator(shape, beta):
    hs = spacing(shape)
    A = beta * lumped_mass(shape)
    for d in range(len(shape)):
        fac = [stiffness_1d(n, hs[a]) if a == d else sp.diags(trapezoid_1d(n))
               for a, n in enumerate(shape)]
        A = A + _kron_axes(fac)
    return A.tocsr()


def apply(shape, beta: float, X: np.ndarray) -> np.ndarray:
    """Y = A X for X of shape (N,) or (k, N) (rows are separate vectors)."""
    A = gram_operator(shape, beta)
    X = np.asarray(X, dtype=np.float64)
    return (A @ X.T).T if X.ndim == 2 else A @ X

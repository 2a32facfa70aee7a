"""Textbook symmetric geometric-multigrid V-cycle B ~ A^{-1}.

The paper treats the Laplace solve inside its preconditioner as a black box
(Section 3.2: the Schur-complement approximation is one application of an
algebraic multigrid cycle). Here the same role is played by a geometric V-cycle
on the structured grid; this module is its plain definition, used to check the
GPU's V-cycle operator element by element. Components:

  levels     vertex-centred halving n -> (n-1)/2 + 1 on every axis while all
             n_d >= 5 are odd and the level has more than coarse_max nodes
  A_l        the Gram operator rediscretised on level l (h doubles per level)
  P_l        multilinear interpolation (tensor product of the 1D stencil
             [1/2, 1, 1/2]); restriction R_l = 2^{-d} P_l^T
  smoother   nu Chebyshev-accelerated Jacobi steps x <- x + w_k D^{-1}(f - A x),
             with 1/w_k the roots of the degree-nu Chebyshev polynomial on
             [lo, hi] (k = 0..nu-1 before the coarse correction, k = nu-1..0
             after it, so pre- and post-smoothing are adjoint)
  coarsest   exact dense solve
  start      zero initial guess (B is linear)

With these choices B is symmetric, which conjugate gradients needs.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import operator as op

def level_shapes(shape, coarse_max: int):
    """Grid shapes from fine to coarsest."""
    shapes = [tuple(shape)]
    while True:
        s = shapes[-1]
        if int(np.prod(s)) <= coarse_max:
            break
        if not all(n >= 5 and (n - 1) % 2 == 0 for n in s):
            break
        shapes.append(tuple((n - 1) // 2 + 1 for n in s))
    return shapes


def chebyshev_weights(nu: int, lo: float, hi: float) -> np.ndarray:
    """w_k = 1/theta_k, theta_k = (hi+lo)/2 + (hi-lo)/2 cos(pi (2k+1)/(2 nu))."""
    k = np.arange(nu)
    theta = 0.5 * (hi + lo) + 0.5 * (hi - lo) * np.cos(np.pi * (2 * k + 1) / (2 * nu))
    return 1.0 / theta


def interpolation_1d(nc: int) -> sp.csr_matrix:
    """(2(nc-1)+1) x nc linear interpolation between vertex-centred grids."""
    nf = 2 * (nc - 1) + 1
    rows, cols, vals = [], [], []
    for I in range(nc):
        rows.append(2 * I); cols.append(I); vals.append(1.0)
    for I in range(nc - 1):
        rows += [2 * I + 1, 2 * I + 1]; cols += [I, I + 1]; vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def interpolation(coarse_shape) -> sp.csr_matrix:
    """Tensor-product interpolation, x fastest (kron(slow, fast))."""
    P = sp.csr_matrix(np.ones((1, 1)))
    for nc in coarse_shape:
        P = sp.kron(interpolation_1d(nc), P, format="csr")
    return P


class VCycle:
    """B f for the symmetric V(nu, nu) cycle described in the module docstring.

    Every parameter of B is given by the caller (Section 3.2 leaves the
    Laplace solver open, so none has a value of its own here): nu smoothing
    steps per side, the Chebyshev interval [lo, hi] for eig(D^-1 A), and
    coarse_max, the node count at or below which a level is the coarsest."""

    def __init__(self, shape, beta, *, nu, lo, hi, coarse_max):
        dim = len(shape)
        self.shapes = level_shapes(shape, coarse_max)
        self.dim = dim
        self.weights = chebyshev_weights(nu, lo, hi)
        self.A = [op.gram_operator(s, beta) for s in self.shapes]
        self.Dinv = [1.0 / a.diagonal() for a in self.A]
        self.P = [interpolation(s) for s in self.shapes[1:]]          # P[l]: level l+1 -> l
        self.R = [p.T.tocsr() * 2.0 ** (-dim) for p in self.P]
        self.Acoarse = self.A[-1].toarray()

    @property
    def nlevels(self) -> int:
        return len(self.shapes)

    def _cycle(self, l: int, f: np.ndarray) -> np.ndarray:
        if l == self.nlevels - 1:
            return np.linalg.solve(self.Acoarse, f)
        A, Dinv = self.A[l], self.Dinv[l]
        x = np.zeros_like(f)
        for w in self.weights:                       # pre-smoothing
            x = x + w * Dinv * (f - A @ x)
        r = f - A @ x                                # residual
        e = self._cycle(l + 1, self.R[l] @ r)        # coarse-grid correction
        x = x + self.P[l] @ e
        for w in self.weights[::-1]:                 # post-smoothing (adjoint order)
            x = x + w * Dinv * (f - A @ x)
        return x

    def apply(self, F: np.ndarray) -> np.ndarray:
        """B F for F of shape (N,) or (k, N)."""
        F = np.asarray(F, dtype=np.float64)
        if F.ndim == 2:
            return np.stack([self._cycle(0, f) for f in F])
        return self._cycle(0, F)

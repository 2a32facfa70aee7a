"""The Gauss-Newton linear system and its Woodbury solution.

Notation: the paper's regularisation parameter beta (Section 2.2) is called
alpha here, and its Laplacian L is the Gram operator A (module operator).
Multiplying eq. (block_primal) by alpha gives the system solved here,

    G x = b,    G = alpha*A + J^T J,

with J the dense M x N sensitivity matrix (Section 2.3, the matrix J_m) and,
in the paper's form, b = -alpha*A d - J^T res, d = m - m_ref, res = g - g_obs.
G is symmetric positive definite, so x is unique.

Routes to x (they must agree on small grids):
  solve_dense      Cholesky of the assembled dense G
  solve_augmented  sparse LU of [[alpha*A, J^T], [J, -I]] [x; y] = [b; 0]
                   (eliminating y = J x gives G x = b; the rank-M term stays
                   outside the sparse block as in the mixed system of
                   eq. (block_sol))
  solve_woodbury   the Woodbury identity of Section 3.1 with exact A^{-1}
                   (DCT): Z = A^{-1} J^T, S = alpha*I + J Z,
                   x = (1/alpha)(A^{-1} b - Z S^{-1} J A^{-1} b),
                   then iterative refinement with the same inverse
paper_update: the closed-form update below eq. (woodbury_temp),
    dm = -d + Z S^{-1} (J d - res),
which solves G dm = -alpha*A d - J^T res.
woodbury_precond: the preconditioner of Algorithm 3 written for the primal
system: with y = B r for an approximation B of A^{-1},
    z = (1/alpha)(y - Z S^{-1} J y),  Z = B J^T,  S = alpha*I + J Z,
which is exactly (alpha*B^{-1} + J^T J)^{-1} r.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import operator as op
from . import poisson


def gn_apply(shape, beta, J, alpha, x):
    """G x = alpha*A x + J^T (J x)."""
    A = op.gram_operator(shape, beta)
    return alpha * (A @ x) + J.T @ (J @ x)


def true_relres(shape, beta, J, alpha, b, x) -> float:
    """Euclidean relative residual ||b - G x||_2 / ||b||_2 (the paper's
    stopping quantity, Table 1 caption)."""
    return float(np.linalg.norm(b - gn_apply(shape, beta, J, alpha, x)) / np.linalg.norm(b))


def gn_apply_streamed(shape, beta, row_blocks, alpha, X):
    """G X = alpha*A X + J^T (J X) with J supplied as an iterable of row blocks
    (arrays of shape (rows, N); every row of J exactly once, in any order),
    consumed once: J^T J X is the sum over the blocks of J_b^T (J_b X), so J is
    never held whole (a 1024 x 257^3 J is 139 GB). X: (N,) or (k, N); the
    result has the shape of X."""
    X = np.asarray(X, dtype=np.float64)
    X2 = X.reshape(1, -1) if X.ndim == 1 else X
    out = alpha * op.apply(shape, beta, X2)
    for Jb in row_blocks:
        out += (Jb.T @ (Jb @ X2.T)).T
    return out.reshape(X.shape)


def relres_streamed(shape, beta, row_blocks, alpha, b, X):
    """(relres, floor) for each row x of X (or the single vector X), with J
    streamed as in gn_apply_streamed:
      relres = ||b - G x||_2 / ||b||_2 (the paper's stopping quantity);
      floor  = u || alpha |A||x| + |J|^T (|J||x|) ||_2 / ||b||_2, u = 2^-53,
               the componentwise rounding level of one FP64 product G x, i.e.
               the smallest relative residual an FP64 solve can be expected to
               reach (residual_rounding_floor is 4 sqrt(N) times it).
    Both come from the same single pass over the blocks."""
    X = np.asarray(X, dtype=np.float64)
    X2 = X.reshape(1, -1) if X.ndim == 1 else X
    A = op.gram_operator(shape, beta)
    Gx = alpha * (A @ X2.T).T
    mag = alpha * (abs(A) @ np.abs(X2).T).T
    for Jb in row_blocks:
        Gx += (Jb.T @ (Jb @ X2.T)).T
        aJ = np.abs(Jb)
        mag += (aJ.T @ (aJ @ np.abs(X2).T)).T
    nb = np.linalg.norm(b)
    u = np.finfo(np.float64).eps / 2
    rr = np.linalg.norm(b[None, :] - Gx, axis=1) / nb
    fl = u * np.linalg.norm(mag, axis=1) / nb
    if X.ndim == 1:
        return float(rr[0]), float(fl[0])
    return rr, fl


def residual_rounding_floor(shape, beta, J, alpha, b, x) -> float:
    """Rounding level of an FP64 evaluation of ||b - G x|| / ||b||: with the
    componentwise bound |fl(G x) - G x| <~ u |alpha A| |x| + u |J|^T (|J| |x|)
    per accumulated term and errors that add like a random walk over the
    sqrt(N) terms of the longest sums, two independent evaluations (on the CPU
    and on the GPU) of the relative residual differ by about
    4 sqrt(N) u || |alpha A||x| + |J|^T (|J||x|) || / ||b||."""
    u = np.finfo(np.float64).eps / 2
    A = abs(op.gram_operator(shape, beta))
    ax = np.abs(x)
    mag = alpha * (A @ ax) + (np.abs(J).T @ (np.abs(J) @ ax) if J.shape[0] else 0.0)
    return float(4.0 * np.sqrt(x.size) * u * np.linalg.norm(mag) / np.linalg.norm(b))


def gn_dense(shape, beta, J, alpha) -> np.ndarray:
    A = op.gram_operator(shape, beta).toarray()
    return alpha * A + J.T @ J


def solve_dense(shape, beta, J, alpha, b) -> np.ndarray:
    G = gn_dense(shape, beta, J, alpha)
    return sla.cho_solve(sla.cho_factor(G, lower=True), b)


def solve_augmented(shape, beta, J, alpha, b) -> np.ndarray:
    A = op.gram_operator(shape, beta)
    M = J.shape[0]
    Js = sp.csr_matrix(J)
    K = sp.bmat([[alpha * A, Js.T], [Js, -sp.identity(M)]], format="csc")
    rhs = np.concatenate([b, np.zeros(M)])
    return spla.spsolve(K, rhs)[: A.shape[0]]


def capacitance(shape, beta, J, alpha, Ainv=None):
    """(Z, S): Z = A^{-1} J^T as an M x N array (row i = A^{-1} J_i), S = alpha*I + J Z^T."""
    Ainv = Ainv or (lambda F: poisson.dct_solve(shape, beta, F))
    Z = Ainv(J) if J.shape[0] else np.zeros_like(J)
    S = alpha * np.eye(J.shape[0]) + J @ Z.T
    return Z, S


def solve_woodbury(shape, beta, J, alpha, b, tol=1e-13, maxref=20):
    """Woodbury solve with exact A^{-1} plus iterative refinement to tol."""
    Ainv = lambda F: poisson.dct_solve(shape, beta, F)
    Z, S = capacitance(shape, beta, J, alpha, Ainv)
    lu = sla.lu_factor(S) if J.shape[0] else None

    def Ginv(r):
        y = Ainv(r)
        if lu is None:
            return y / alpha
        return (y - Z.T @ sla.lu_solve(lu, J @ y)) / alpha

    x = Ginv(b)
    nb = np.linalg.norm(b)
    for _ in range(maxref):
        r = b - gn_apply(shape, beta, J, alpha, x)
        if np.linalg.norm(r) <= tol * nb:
            break
        x = x + Ginv(r)
    return x


def paper_rhs(shape, beta, J, alpha, d, res):
    """b = -alpha*A d - J^T res (eq. (block_primal) multiplied by alpha)."""
    return -alpha * op.apply(shape, beta, d) - J.T @ res


def paper_update(shape, beta, J, alpha, d, res):
    """dm = -d + Z S^{-1} (J d - res) with exact Z = A^{-1} J^T (Section 3.1)."""
    Z, S = capacitance(shape, beta, J, alpha)
    return -d + Z.T @ np.linalg.solve(S, J @ d - res)


def woodbury_operator(B, J, alpha, Z=None):
    """The preconditioner apply r -> (1/alpha)(B r - Z S^{-1} J B r) as a
    callable on (N,) vectors, with Z = B J^T (M x N; computed here unless
    given: Z does not depend on alpha) and S = alpha*I + J Z^T factored once."""
    Z = B(J) if Z is None else Z
    S = alpha * np.eye(J.shape[0]) + J @ Z.T
    lu = sla.lu_factor(S)

    def apply(r):
        y = B(r)
        return (y - Z.T @ sla.lu_solve(lu, J @ y)) / alpha
    return apply


def woodbury_precond(B, J, alpha, R):
    """z = (1/alpha)(B r - Z S^{-1} J B r), Z = B J^T, S = alpha*I + J Z^T.

    B: callable applying the Laplace approximation to (k, N) or (N,) arrays.
    R: (N,) or (k, N). Returns the same shape as R.
    """
    R = np.asarray(R, dtype=np.float64)
    Z = B(J)
    S = alpha * np.eye(J.shape[0]) + J @ Z.T
    Y = B(R)
    if Y.ndim == 1:
        return (Y - Z.T @ np.linalg.solve(S, J @ Y)) / alpha
    W = np.linalg.solve(S, J @ Y.T)          # M x k
    return (Y - (Z.T @ W).T) / alpha

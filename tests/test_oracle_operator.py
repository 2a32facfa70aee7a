"""Pins for the oracle's Gram operator and exact Poisson solves (CPU only).

Each check compares against mathematics that is independent of the oracle's
own construction: cosine eigenpairs in closed form, the Neumann null-space
property, the textbook interior stencil, second-order convergence to a smooth
continuous solution, and two different exact solvers.
"""
import numpy as np
import pytest

from oracle import operator as op
from oracle import poisson

pytestmark = pytest.mark.filterwarnings("ignore")


def _cos_mode(shape, js):
    """Tensor product of cos(j_d * pi * i / (n_d - 1)), x fastest."""
    v = None
    for n, j in zip(reversed(shape), reversed(js)):
        c = np.cos(j * np.pi * np.arange(n) / (n - 1))
        v = c if v is None else np.multiply.outer(v, c)
    return np.ascontiguousarray(v).reshape(-1)


@pytest.mark.parametrize("shape", [(9,), (13, 7), (9, 5, 7), (17, 17, 17)])
def test_generalised_eigenpairs(shape):
    # A v = (beta + sum_d (2/h_d^2)(1 - cos(j_d pi/(n_d-1)))) W v  for cosine modes
    beta = 0.37
    if len(shape) == 1:
        A = op.stiffness_1d(shape[0], 1.0 / (shape[0] - 1)) + beta * op.lumped_mass(shape)
    else:
        A = op.gram_operator(shape, beta)
    W = op.lumped_mass(shape)
    rng = np.random.default_rng(5)
    for _ in range(6):
        js = [int(rng.integers(0, n)) for n in shape]
        v = _cos_mode(shape, js)
        lam = beta + sum(2.0 * (n - 1) ** 2 * (1 - np.cos(j * np.pi / (n - 1)))
                         for n, j in zip(shape, js))
        lhs = A @ v
        rhs = lam * (W @ v)
        assert np.linalg.norm(lhs - rhs) <= 1e-12 * max(1.0, np.linalg.norm(rhs))


@pytest.mark.parametrize("shape", [(33, 33), (9, 17, 5)])
def test_neumann_constants_and_symmetry(shape):
    beta = 1e-2
    A = op.gram_operator(shape, beta)
    W = op.lumped_mass(shape)
    one = np.ones(A.shape[0])
    assert np.abs(A @ one - beta * (W @ one)).max() < 1e-9
    assert abs(A - A.T).max() == 0.0
    # positive definite: smallest generalised eigenvalue of (A, W) is beta
    ev = np.linalg.eigvalsh(np.diag(1 / np.sqrt(W.diagonal())) @ A.toarray() @ np.diag(1 / np.sqrt(W.diagonal())))
    assert abs(ev.min() - beta) < 1e-9


def test_interior_rows_are_textbook_stencil():
    shape = (7, 6, 5)
    beta = 0.25
    A = op.gram_operator(shape, beta).toarray()
    nx, ny, nz = shape
    hx, hy, hz = [1.0 / (n - 1) for n in shape]
    i, j, k = 3, 2, 2
    p = i + nx * (j + ny * k)
    row = np.zeros(A.shape[1])
    row[p] = 2 / hx**2 + 2 / hy**2 + 2 / hz**2 + beta
    row[p - 1] = row[p + 1] = -1 / hx**2
    row[p - nx] = row[p + nx] = -1 / hy**2
    row[p - nx * ny] = row[p + nx * ny] = -1 / hz**2
    assert np.allclose(A[p], row, rtol=0, atol=1e-9)
    # a face node (x = 0) carries half the transverse couplings and half the mass
    q = 0 + nx * (j + ny * k)
    assert np.isclose(A[q, q + 1], -1 / hx**2)
    assert np.isclose(A[q, q + nx], -0.5 / hy**2)
    assert np.isclose(A[q, q], 1 / hx**2 + 0.5 * (2 / hy**2 + 2 / hz**2) + 0.5 * beta)


def _manufactured(n, beta, solver):
    # u = cos(pi x) cos(pi y) + x^2 (1-x)^2 has zero normal derivative on the boundary
    x = np.arange(n) / (n - 1)
    X, Y = np.meshgrid(x, x, indexing="xy")  # rows: y, cols: x  -> x fastest
    u = np.cos(np.pi * X) * np.cos(np.pi * Y) + X**2 * (1 - X) ** 2
    f = 2 * np.pi**2 * np.cos(np.pi * X) * np.cos(np.pi * Y) - (2 - 12 * X + 12 * X**2) + beta * u
    shape = (n, n)
    W = op.lumped_mass(shape).diagonal()
    uh = solver(shape, beta, W * f.reshape(-1))
    return np.abs(uh - u.reshape(-1)).max()


@pytest.mark.parametrize("solver", [poisson.dct_solve, poisson.lu_solve])
def test_manufactured_second_order(solver):
    beta = 1.0
    errs = [_manufactured(n, beta, solver) for n in (17, 33, 65)]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.9 < r < 2.1 for r in rates), (errs, rates)


@pytest.mark.parametrize("shape", [(17, 17), (9, 9, 9), (9, 17, 5), (3, 3)])
def test_dct_matches_sparse_lu(shape):
    beta = 1e-2
    rng = np.random.default_rng(1)
    F = rng.standard_normal((3, int(np.prod(shape))))
    X1 = poisson.dct_solve(shape, beta, F)
    X2 = poisson.lu_solve(shape, beta, F)
    assert np.linalg.norm(X1 - X2) <= 1e-11 * np.linalg.norm(X2)
    A = op.gram_operator(shape, beta)
    assert np.linalg.norm(F - (A @ X1.T).T) <= 1e-11 * np.linalg.norm(F)

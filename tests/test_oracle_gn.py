"""Pins for the oracle's GN solves, the paper's update and the Woodbury
preconditioner (CPU only)."""
import numpy as np
import pytest

import h1w_inputs as H
from oracle import gn, multigrid, operator as op, poisson


def _small(shape, m, alpha=1e-3, beta=1e-2, seed=0):
    rng = np.random.default_rng(seed)
    N = int(np.prod(shape))
    J = rng.standard_normal((m, N)) / np.sqrt(N)
    b = rng.standard_normal(N)
    return J, b, alpha, beta


def test_three_routes_agree_square33():
    wl = H.workload("square33")
    J, b = H.j_rows(wl), H.rhs_b(wl)
    s, be, al = wl.shape, wl.beta, wl.alpha
    xs = [gn.solve_dense(s, be, J, al, b), gn.solve_augmented(s, be, J, al, b),
          gn.solve_woodbury(s, be, J, al, b)]
    for x in xs:
        assert gn.true_relres(s, be, J, al, b, x) < 1e-12
    for x in xs[1:]:
        assert np.linalg.norm(x - xs[0]) <= 1e-12 * np.linalg.norm(xs[0])


@pytest.mark.parametrize("name", ["cube17"])
def test_three_routes_agree_3d(name):
    wl = H.workload(name).with_(m=12)
    J, b = H.j_rows(wl), H.rhs_b(wl)
    s, be, al = wl.shape, wl.beta, wl.alpha
    x1 = gn.solve_dense(s, be, J, al, b)
    x2 = gn.solve_augmented(s, be, J, al, b)
    x3 = gn.solve_woodbury(s, be, J, al, b)
    for x in (x2, x3):
        assert np.linalg.norm(x - x1) <= 1e-10 * np.linalg.norm(x1)
    assert gn.true_relres(s, be, J, al, b, x3) < 1e-12


def test_no_rows_reduces_to_scaled_poisson():
    shape = (17, 9)
    J, b, al, be = _small(shape, 0)
    x = gn.solve_woodbury(shape, be, J, al, b)
    assert np.allclose(x, poisson.lu_solve(shape, be, b) / al, rtol=1e-12, atol=0)
    x2 = gn.solve_dense(shape, be, J, al, b)
    # dense Cholesky forward error ~ cond(alpha*A) * eps ~ 2e5 * 1e-16
    assert np.linalg.norm(x - x2) <= 1e-10 * np.linalg.norm(x2)


def test_one_row_sherman_morrison():
    shape = (9, 9, 5)
    J, b, al, be = _small(shape, 1, alpha=1e-4)
    A = op.gram_operator(shape, be).toarray()
    j = J[0]
    Ai = np.linalg.inv(al * A)
    ref = Ai @ b - (Ai @ j) * (j @ Ai @ b) / (1.0 + j @ Ai @ j)
    x = gn.solve_woodbury(shape, be, J, al, b)
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_paper_update_solves_paper_rhs():
    wl = H.workload("square33")
    J = H.j_rows(wl)
    d, res = H.paper_data(wl)
    s, be, al = wl.shape, wl.beta, wl.alpha
    dm = gn.paper_update(s, be, J, al, d, res)
    b = gn.paper_rhs(s, be, J, al, d, res)
    ref = gn.solve_dense(s, be, J, al, b)
    assert np.linalg.norm(dm - ref) <= 1e-10 * np.linalg.norm(ref)
    # b written out from eq. (block_primal) times alpha with the assembled matrix
    A = op.gram_operator(s, be).toarray()
    assert np.allclose(b, -al * A @ d - J.T @ res, rtol=1e-13, atol=1e-12)


def test_woodbury_precond_with_exact_inverse_is_G_inverse():
    shape = (17, 17)
    J, b, al, be = _small(shape, 5, alpha=1e-4)
    B = lambda F: poisson.lu_solve(shape, be, F)
    R = np.random.default_rng(3).standard_normal((2, int(np.prod(shape))))
    Z = gn.woodbury_precond(B, J, al, R)
    G = gn.gn_dense(shape, be, J, al)
    ref = np.linalg.solve(G, R.T).T
    assert np.linalg.norm(Z - ref) <= 1e-10 * np.linalg.norm(ref)


def test_woodbury_precond_identity_with_vcycle():
    # alpha z + B J^T J z = B r  for z = (alpha B^{-1} + J^T J)^{-1} r
    shape = (33, 33)
    J, b, al, be = _small(shape, 7, alpha=1e-3)
    V = multigrid.VCycle(shape, be, nu=2, lo=0.3, hi=2.0, coarse_max=9)
    r = np.random.default_rng(4).standard_normal(int(np.prod(shape)))
    z = gn.woodbury_precond(V.apply, J, al, r)
    lhs = al * z + V.apply(J.T @ (J @ z))
    rhs = V.apply(r)
    assert np.linalg.norm(lhs - rhs) <= 1e-10 * np.linalg.norm(rhs)


def _blocks(J, sizes, order):
    """Rows of J as blocks of the given sizes, handed out in the given order."""
    edges = np.cumsum([0] + list(sizes))
    assert edges[-1] == J.shape[0]
    return (J[edges[k]:edges[k + 1]] for k in order)


def test_streamed_gn_apply_recovers_b_from_dense_solution():
    # G x* = b for x* from the Cholesky factor of the assembled G (another
    # route); J streamed in uneven blocks handed out of order, two vectors at once
    wl = H.workload("cube17").with_(m=12)
    J, b = H.j_rows(wl), H.rhs_b(wl)
    s, be, al = wl.shape, wl.beta, wl.alpha
    xs = gn.solve_dense(s, be, J, al, b)
    X = np.stack([xs, 2.0 * xs])
    GX = gn.gn_apply_streamed(s, be, _blocks(J, [5, 1, 6], [2, 0, 1]), al, X)
    assert np.linalg.norm(GX[0] - b) <= 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(GX[1] - 2.0 * b) <= 2e-12 * np.linalg.norm(b)
    g1 = gn.gn_apply_streamed(s, be, _blocks(J, [12], [0]), al, xs)
    assert g1.shape == xs.shape and np.linalg.norm(g1 - b) <= 1e-12 * np.linalg.norm(b)
    # relres and floor of the exact solution and of a perturbed one
    e = H.rng_for(99, 0).standard_normal(xs.size)
    xp = xs + 1e-6 * np.linalg.norm(xs) / np.linalg.norm(e) * e
    rr, fl = gn.relres_streamed(s, be, _blocks(J, [3, 9], [1, 0]), al, b, np.stack([xs, xp]))
    assert rr[0] <= 1e-12 and rr[1] >= 1e-9
    dense = gn.gn_dense(s, be, J, al)
    assert abs(rr[1] - np.linalg.norm(b - dense @ xp) / np.linalg.norm(b)) <= 1e-6 * rr[1]
    assert np.allclose(fl, [gn.residual_rounding_floor(s, be, J, al, b, v) / (4 * np.sqrt(xs.size))
                            for v in (xs, xp)], rtol=1e-12)


@pytest.mark.parametrize("name", ["square33", "cube17"])
def test_residual_rounding_floor_bounds_fp64_evaluation(name):
    # residual_rounding_floor is a bound on how far an FP64 evaluation of
    # ||b - G x|| / ||b|| lies from the exact value, for x near the solution
    # (where b - G x cancels): checked against the same expression evaluated in
    # x86 extended precision (64-bit significand). The bound is loose (the
    # differences seen here are 2e-17 to 3e-14, about 1/300 of it), and it
    # loosens the comparisons of the GPU's and the oracle's residuals by at most
    # 10% of the FP64 tolerance 1e-10
    wl = H.workload(name)
    if name == "cube17":
        wl = wl.with_(m=12)
    J, b = H.j_rows(wl), H.rhs_b(wl)
    s, be, al = wl.shape, wl.beta, wl.alpha
    xs = gn.solve_dense(s, be, J, al, b)
    e = H.rng_for(98, 0).standard_normal(xs.size)
    ld = np.longdouble
    A = op.gram_operator(s, be).toarray().astype(ld)
    Jl, bl = J.astype(ld), b.astype(ld)
    for scale in (0.0, 1e-11, 1e-9):
        x = xs + scale * np.linalg.norm(xs) / np.linalg.norm(e) * e
        rr64 = gn.true_relres(s, be, J, al, b, x)
        xl = x.astype(ld)
        r = bl - (ld(al) * (A @ xl) + Jl.T @ (Jl @ xl))
        rr_ext = float(np.sqrt(np.sum(r * r)) / np.sqrt(np.sum(bl * bl)))
        floor = gn.residual_rounding_floor(s, be, J, al, b, x)
        assert abs(rr64 - rr_ext) <= floor, (scale, rr64, rr_ext, floor)
        assert floor <= 0.1 * 1e-10

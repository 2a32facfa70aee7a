"""Pins of the oracle's preconditioned CG (oracle/krylov.py).

  * P = G^-1 exactly: one iteration gives x = G^-1 b (up to rounding);
  * CG on a diagonal SPD matrix with k distinct eigenvalues and no
    preconditioner reaches the solution in k iterations (the Krylov space is
    then G-invariant), and not before: a wrong coefficient breaks either;
  * the iterates equal scipy's preconditioned CG iterate by iterate;
  * the flexible (Polak-Ribiere) form gives the PCG iterates for a fixed
    symmetric preconditioner;
  * the G-norm of the error decreases monotonically (CG's minimisation
    property), for the Woodbury preconditioner with the oracle V-cycle on a
    small GN system.
"""
import numpy as np
import scipy.sparse.linalg as spla

import h1w_inputs as H
from oracle import gn, krylov, multigrid as mg, operator as op


def _spd(n, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T


def test_exact_preconditioner_one_iteration():
    G = _spd(60, 1)
    b = np.random.default_rng(2).standard_normal(60)
    Gi = np.linalg.inv(G)
    x, it, hist = krylov.pcg(lambda v: G @ v, lambda v: Gi @ v, b, 1e-10, 50)
    assert it == 1
    assert np.linalg.norm(x - np.linalg.solve(G, b)) <= 1e-10 * np.linalg.norm(x)


def test_distinct_eigenvalues_iteration_count():
    for k in (3, 5, 8):
        ev = np.repeat(np.linspace(1.0, 10.0, k), 7)
        b = np.random.default_rng(k).standard_normal(ev.size)
        x, it, hist = krylov.pcg(lambda v: ev * v, lambda v: v, b, 1e-11, 100)
        assert it == k
        assert hist[k - 1] > 1e-6
        assert np.allclose(x, b / ev, rtol=1e-9, atol=0)


def test_iterates_match_scipy_cg():
    G = _spd(80, 3, cond=1e4)
    b = np.random.default_rng(4).standard_normal(80)
    d = 1.0 / np.diag(G)
    ours, theirs = [], []
    krylov.pcg(lambda v: G @ v, lambda v: d * v, b, 1e-12, 25, callback=lambda x: ours.append(x.copy()))
    M = spla.LinearOperator(G.shape, matvec=lambda v: d * v)
    spla.cg(G, b, x0=np.zeros(80), M=M, rtol=1e-30, maxiter=25, callback=lambda x: theirs.append(x.copy()))
    n = min(len(ours), len(theirs), 20)
    assert n >= 15
    for a, c in zip(ours[:n], theirs[:n]):
        assert np.linalg.norm(a - c) <= 1e-8 * np.linalg.norm(c)


def test_flexible_equals_pcg_for_fixed_preconditioner():
    # preconditioned operator similar to an SPD matrix with eigenvalues in
    # [1, 3]: P^-1 = G^-1/2 C G^-1/2, so both recurrences converge in about
    # 20 iterations, before rounding separates them
    G = _spd(70, 5, cond=1e4)
    b = np.random.default_rng(6).standard_normal(70)
    w, Q = np.linalg.eigh(G)
    Gmh = (Q / np.sqrt(w)) @ Q.T
    Mh = Gmh @ _spd(70, 7, cond=3.0) @ Gmh
    xa, ia, ha = krylov.pcg(lambda v: G @ v, lambda v: Mh @ v, b, 1e-10, 200)
    xb, ib, hb = krylov.pcg(lambda v: G @ v, lambda v: Mh @ v, b, 1e-10, 200, flexible=True)
    assert ia == ib and 10 <= ia <= 30
    assert np.allclose(ha, hb, rtol=1e-9, atol=0)
    assert np.linalg.norm(xa - xb) <= 1e-9 * np.linalg.norm(xa)


def test_woodbury_pcg_error_decreases_in_energy_norm():
    wl = H.workload("square33")
    J, b = H.j_rows(wl), H.rhs_b(wl)
    A = op.gram_operator(wl.shape, wl.beta)
    V = mg.VCycle(wl.shape, wl.beta, nu=2, lo=0.3, hi=2.0, coarse_max=81)
    G = wl.alpha * A.toarray() + J.T @ J
    xs = np.linalg.solve(G, b)
    errs = []
    krylov.pcg(lambda v: G @ v, lambda v: gn.woodbury_precond(V.apply, J, wl.alpha, v), b, 1e-12, 50,
               callback=lambda x: errs.append(float((x - xs) @ G @ (x - xs))))
    assert len(errs) >= 3
    assert all(e1 <= e0 * (1 + 1e-9) for e0, e1 in zip(errs, errs[1:]))
    assert errs[-1] <= 1e-18 * float(xs @ G @ xs)


def test_woodbury_operator_with_exact_inverse_is_g_inverse():
    # with B = A^-1 (DCT solve) the Woodbury apply is exactly G^-1: P^-1 G x = x
    from oracle import poisson
    wl = H.workload("square33")
    J = H.j_rows(wl)
    Ainv = lambda F: poisson.dct_solve(wl.shape, wl.beta, F)
    Pinv = gn.woodbury_operator(Ainv, J, wl.alpha)
    x = np.random.default_rng(9).standard_normal(wl.N)
    y = Pinv(gn.gn_apply(wl.shape, wl.beta, J, wl.alpha, x))
    assert np.linalg.norm(y - x) <= 1e-9 * np.linalg.norm(x)
    # and PCG with it stops after one iteration
    _, it, _ = krylov.pcg(lambda v: gn.gn_apply(wl.shape, wl.beta, J, wl.alpha, v), Pinv, H.rhs_b(wl), 1e-9, 10)
    assert it == 1

"""Pins for the oracle's V-cycle (CPU only): Chebyshev minimax closed form,
interpolation exactness on affine functions, B = A^{-1} when no coarsening
happens, symmetry and positivity, and contraction of the stationary iteration
towards the exact (DCT) solution."""
import numpy as np
import pytest

from oracle import multigrid as mg, operator as op, poisson


def test_chebyshev_polynomial_closed_form():
    for nu, lo, hi in [(1, 0.3, 2.0), (2, 0.3, 2.0), (3, 0.5, 1.9), (4, 0.1, 2.0)]:
        w = mg.chebyshev_weights(nu, lo, hi)
        lam = np.linspace(lo, hi, 101)
        p = np.prod([1 - wk * lam for wk in w], axis=0)
        t = lambda x: np.cosh(nu * np.arccosh(x)) if x >= 1 else np.cos(nu * np.arccos(x))
        ref = np.array([np.cos(nu * np.arccos(np.clip((hi + lo - 2 * l) / (hi - lo), -1, 1))) for l in lam])
        ref = ref / t((hi + lo) / (hi - lo))
        assert np.allclose(p, ref, atol=1e-13)


def test_level_shapes():
    assert mg.level_shapes((129, 129, 129), 729) == [(129,) * 3, (65,) * 3, (33,) * 3, (17,) * 3, (9,) * 3]
    assert mg.level_shapes((193, 193), 9) == [(193, 193), (97, 97), (49, 49), (25, 25), (13, 13), (7, 7), (4, 4)]
    assert mg.level_shapes((33, 33), 289) == [(33, 33), (17, 17)]
    assert mg.level_shapes((9, 17, 5), 1) == [(9, 17, 5), (5, 9, 3)]


@pytest.mark.parametrize("cshape", [(5,), (4, 3), (3, 5, 4)])
def test_interpolation_exact_on_affine(cshape):
    P = mg.interpolation(cshape)
    fshape = tuple(2 * (n - 1) + 1 for n in cshape)

    def affine(shape):
        axes = [np.arange(n) / (n - 1) for n in shape]
        g = np.meshgrid(*reversed(axes), indexing="ij")   # slowest first
        val = 0.3
        for a, G in enumerate(reversed(g)):               # x first
            val = val + (a + 1.7) * G
        return val.reshape(-1)

    assert np.allclose(P @ affine(cshape), affine(fshape), atol=1e-14)


def test_no_coarsening_is_exact_inverse():
    shape = (9, 9)
    V = mg.VCycle(shape, 1e-2, nu=2, lo=0.3, hi=2.0, coarse_max=10**6)
    assert V.nlevels == 1
    f = np.random.default_rng(0).standard_normal(81)
    assert np.allclose(V.apply(f), poisson.dct_solve(shape, 1e-2, f), rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("shape,cmax", [((33, 33), 9), ((17, 17, 17), 27), ((9, 17, 5), 1)])
def test_symmetric_positive(shape, cmax):
    V = mg.VCycle(shape, 1e-2, nu=2, lo=0.3, hi=2.0, coarse_max=cmax)
    rng = np.random.default_rng(2)
    N = int(np.prod(shape))
    for _ in range(4):
        u, v = rng.standard_normal(N), rng.standard_normal(N)
        Bu, Bv = V.apply(u), V.apply(v)
        assert abs(u @ Bv - Bu @ v) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(Bv)
        assert u @ Bu > 0


@pytest.mark.parametrize("shape,cmax,bound", [((65, 65), 9, 0.2), ((33, 33, 33), 27, 0.22)])
def test_vcycle_contraction(shape, cmax, bound):
    beta = 1e-2
    V = mg.VCycle(shape, beta, nu=2, lo=0.3, hi=2.0, coarse_max=cmax)
    A = op.gram_operator(shape, beta)
    f = np.random.default_rng(7).standard_normal(int(np.prod(shape)))
    xs = poisson.dct_solve(shape, beta, f)
    x = np.zeros_like(f)
    errs = []
    for _ in range(8):
        x = x + V.apply(f - A @ x)
        errs.append(np.linalg.norm(x - xs))
    rate = (errs[6] / errs[1]) ** (1 / 5)
    assert rate < bound, rate

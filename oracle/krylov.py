"""Preconditioned conjugate gradients: the Krylov loop of Algorithm 3.

The paper runs MINRES on the symmetric saddle-point system of eq.
(block_sol), preconditioned by the Woodbury-based block diagonal operator of
Section 3.2. For the symmetric positive definite primal system G x = b of
eq. (block_primal) (times alpha), the same preconditioner, applied as
P^-1 = (alpha B^-1 + J^T J)^-1, makes conjugate gradients applicable; this is
that loop written out, from x0 = 0, stopping on the paper's Euclidean
criterion ||b - G x||_2 <= rtol ||b||_2 (Table 1 caption), here on the
recursively updated residual.

pcg       textbook PCG: beta_k = (r_k . z_k) / (r_{k-1} . z_{k-1})
flexible  the Polak-Ribiere form beta_k = z_k . (r_k - r_{k-1}) / (r_{k-1} . z_{k-1}),
          which coincides with PCG for a fixed symmetric preconditioner
          (z_k . r_{k-1} = 0 there) and tolerates a preconditioner that varies
          between applications (an FP32 V-cycle)

Test infrastructure only: plain numpy, FP64, one vector at a time.
"""
from __future__ import annotations

import numpy as np


def pcg(apply_G, apply_P, b, rtol: float, maxit: int, flexible: bool = False, callback=None):
    """(x, iters, relres_history): CG on G x = b preconditioned by z = P^-1 r.

    apply_G, apply_P: callables on (N,) FP64 vectors. iters = number of
    updates of x; relres_history[k] = ||r_k|| / ||b|| (k = 0 .. iters).
    callback(x_k) is called after each update. Stops when the relative
    residual is <= rtol or after maxit updates."""
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    if nb == 0.0:
        return x, 0, [0.0]
    r = b.copy()
    z = apply_P(r)
    p = z.copy()
    rz = float(r @ z)
    hist = [1.0]
    it = 0
    while it < maxit:
        q = apply_G(p)
        a = rz / float(p @ q)
        x = x + a * p
        r_old = r
        r = r - a * q
        it += 1
        hist.append(float(np.linalg.norm(r)) / nb)
        if callback is not None:
            callback(x)
        if hist[-1] <= rtol:
            break
        z = apply_P(r)
        rz_new = float(r @ z)
        beta = (float(z @ (r - r_old)) if flexible else rz_new) / rz
        rz = rz_new
        p = z + beta * p
    return x, it, hist

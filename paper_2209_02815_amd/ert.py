"""ERT forward map and its adjoint behind torch.autograd (thin layer over the
h1w_ert_* entry points of libh1w.so; every step runs in the HIP library).

The voltages g(m) of a pole-pole survey (Section 4, eq. (ert_qoi2) with the
return electrodes at infinity) are a differentiable function of the nodal
log-conductivity m: the backward pass returns J^T gbar from the saved pole
fields by the pairwise-gradient kernel, without forming J (the adjoint field of
a receiver is the source field of that electrode, eq. (ert_qoi_derivative)).
Per-level multigrid state is not saved between forward and backward; the
backward pass sets the conductivity again, which rebuilds it.
"""
from __future__ import annotations

from . import _native as nat
from .solver import Context

__all__ = ["ErtContext", "ert_voltages", "ert_gauss_newton"]


class ErtContext:
    """One ERT grid (unit cube, n_x x n_y x n_z nodes) with a fixed survey.

    src_nodes  node indices of the pole sources (electrodes), x fastest
    pairs      (n_meas, 2) electrode index pairs (a, b): g = k u_a(x_b)
    kgeo       optional geometric factors (default 2 pi |x_a - x_b|)
    """

    def __init__(self, shape, src_nodes, pairs, dirichlet_mask: int = 0, kgeo=None, nu: int = 0,
                 coarse_max: int = 0, stream=None):
        import torch
        self.shape = tuple(shape)
        self.handle = nat.h1w_setup(self.shape, 0.0, nat.H1W_FP64, nu, (0.0, 0.0), coarse_max, 0, stream, 0,
                                    nat.H1W_OP_ERT, dirichlet_mask)
        self.N, self.nlevels = nat.h1w_get_sizes(self.handle)
        dev = torch.device("cuda", torch.cuda.current_device())
        self.src = torch.as_tensor(src_nodes).to(dtype=torch.int32, device=dev).contiguous()
        self.pair = torch.as_tensor(pairs).to(dtype=torch.int32, device=dev).reshape(-1, 2).contiguous()
        self.kgeo = None if kgeo is None else torch.as_tensor(kgeo, dtype=torch.float64, device=dev).contiguous()

    @property
    def n_src(self) -> int:
        return int(self.src.shape[0])

    @property
    def n_meas(self) -> int:
        return int(self.pair.shape[0])

    def close(self):
        if self.handle is not None:
            nat.h1w_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # per-kernel-class event timing, as for the H1 context
    set_kernel_timing = Context.set_kernel_timing
    kernel_timing = Context.kernel_timing
    reset_kernel_timing = Context.reset_kernel_timing

    def set_conductivity(self, logsig):
        nat.h1w_ert_set_conductivity(self.handle, logsig)

    def empty_jacobian(self):
        """An uninitialised n_meas x N FP64 J on the context's device whose rows
        start on 128-byte boundaries (row pitch N rounded up to 16 values): the
        sensitivity kernel writes each row in 512-byte runs, and runs that
        straddle cache lines write J at about half the rate."""
        import torch
        ld = -(-self.N // 16) * 16
        return torch.empty(self.n_meas, ld, dtype=torch.float64, device=self.src.device)[:, :self.N]

    def forward(self, logsig=None, jacobian: bool = False, fields: bool = False, rtol: float = 0.0,
                maxit: int = 0, J_out=None, U_out=None):
        """(g, J or None, U or None, info) for log-conductivity logsig (None:
        the conductivity already set). A J allocated here has the row pitch of
        empty_jacobian()."""
        import torch
        dev = self.src.device
        g = torch.empty(self.n_meas, dtype=torch.float64, device=dev)
        J = J_out if J_out is not None else (self.empty_jacobian() if jacobian else None)
        U = U_out if U_out is not None else (
            torch.empty(self.n_src, self.N, dtype=torch.float64, device=dev) if fields else None)
        info = nat.h1w_ert_sensitivities(self.handle, self.src, self.pair, logsig, self.kgeo, g, J, U,
                                         rtol=rtol, maxit=maxit)
        return g, J, U, info

    def vjp(self, gbar, U=None, grad=None):
        """J^T gbar for the current conductivity and pole fields U."""
        import torch
        grad = torch.empty(self.N, dtype=torch.float64, device=self.src.device) if grad is None else grad
        return nat.h1w_ert_vjp(self.handle, self.pair, gbar, grad, U, self.n_src, self.src, self.kgeo)

    def operator_apply(self, X, Y=None):
        import torch
        Y = torch.empty_like(X) if Y is None else Y
        return nat.h1w_operator_apply(self.handle, X, Y)

    def vcycle(self, F, X=None):
        import torch
        X = torch.empty_like(F) if X is None else X
        nat.h1w_poisson_solve_batched(self.handle, F, X, nat.H1W_VCYCLE_ONCE)
        return X

    def mg_solve(self, F, X=None, rtol=1e-12, maxit=0):
        import torch
        X = torch.empty_like(F) if X is None else X
        info = nat.h1w_poisson_solve_batched(self.handle, F, X, nat.H1W_MG_SOLVE, rtol, maxit)
        return X, info


def _function():
    import torch

    class ErtVoltages(torch.autograd.Function):
        """g = voltages(logsig); d g / d logsig by the adjoint kernel."""

        @staticmethod
        def forward(ctx, logsig, ert, rtol):
            g, _, U, _ = ert.forward(logsig.detach().contiguous(), fields=True, rtol=rtol)
            ctx.ert = ert
            ctx.save_for_backward(logsig.detach(), U)
            return g

        @staticmethod
        def backward(ctx, gbar):
            logsig, U = ctx.saved_tensors
            ert = ctx.ert
            ert.set_conductivity(logsig.contiguous())   # rebuilds the per-level state
            return ert.vjp(gbar.contiguous(), U), None, None

    return ErtVoltages


_FN = None


def ert_voltages(logsig, ert: ErtContext, rtol: float = 1e-12):
    """Differentiable pole-pole voltages of the survey held by `ert`."""
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN.apply(logsig, ert, rtol)


def ert_gauss_newton(ert: ErtContext, h1, m0, m_ref, g_obs, alpha: float, steps: int = 2, rtol: float = 1e-10,
                     maxit: int = 0):
    """Gauss-Newton iterations of Algorithm 2 for the survey held by `ert`
    with the H^1 regulariser of the Context `h1` (same grid): each step is one
    h1w_ert_gn_step call (forward map, J, Woodbury-preconditioned GN solve,
    update). Returns (m, history), history[k] = (misfit ||g(m_k) - g_obs||,
    GN iterations, true relative residual of the GN solve)."""
    import torch
    m = m0.clone()
    dev = m.device
    J = ert.empty_jacobian()
    dm = torch.empty_like(m)
    g = torch.empty(ert.n_meas, dtype=torch.float64, device=dev)
    hist = []
    for _ in range(steps):
        info = nat.h1w_ert_gn_step(ert.handle, h1.handle, m, m_ref, ert.src, ert.pair, g_obs, alpha, J, dm, g,
                                   ert.kgeo, gn_rtol=rtol, gn_maxit=maxit)
        hist.append((float(torch.linalg.norm(g - g_obs)), info.iters, info.relres_true))
    return m, hist

"""Convenience wrapper owning one h1w context (thin layer over _native)."""
from __future__ import annotations

from . import _native as nat


class Context:
    """One grid + multigrid hierarchy on the current CUDA device/stream."""

    def __init__(self, shape, beta: float, precision: str = "fp64", nu: int = 0, cheb=(0.0, 0.0),
                 coarse_max: int = 0, rhs_chunk: int = 0, stream=None, stream_z: bool = False,
                 fused_vcycle: bool = True, graphs: bool = False, vtail: bool = True,
                 cap_fp32_gemm: bool = False):
        prec = {"fp64": nat.H1W_FP64, "mixed": nat.H1W_MIXED}[precision]
        self.shape = tuple(shape)
        self.precision = precision
        self._J = None
        self.handle = nat.h1w_setup(shape, beta, prec, nu, cheb, coarse_max, rhs_chunk, stream,
                                    (nat.H1W_FLAG_STREAM_Z if stream_z else 0)
                                    | (0 if fused_vcycle else nat.H1W_FLAG_UNFUSED_VCYCLE)
                                    | (nat.H1W_FLAG_GRAPH_VCYCLE if graphs else 0)
                                    | (0 if vtail else nat.H1W_FLAG_NO_VTAIL)
                                    | (nat.H1W_FLAG_CAP_FP32_GEMM if cap_fp32_gemm else 0))
        self.N, self.nlevels = nat.h1w_get_sizes(self.handle)

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

    @property
    def vdtype(self):
        import torch
        return torch.float32 if self.precision == "mixed" else torch.float64

    def operator_apply(self, X, Y=None):
        import torch
        Y = torch.empty_like(X) if Y is None else Y
        return nat.h1w_operator_apply(self.handle, X, Y)

    def vcycle(self, F, X=None):
        import torch
        X = torch.empty_like(F) if X is None else X
        nat.h1w_poisson_solve_batched(self.handle, F, X, nat.H1W_VCYCLE_ONCE)
        return X

    def mg_solve(self, F, X=None, rtol=1e-10, maxit=0):
        import torch
        X = torch.empty_like(F) if X is None else X
        info = nat.h1w_poisson_solve_batched(self.handle, F, X, nat.H1W_MG_SOLVE, rtol, maxit)
        return X, info

    def capacitance_build(self, J, alpha, factor=nat.H1W_FACTOR_AUTO, want_S=False, want_Z=False):
        import torch
        m = J.shape[0]
        S = torch.empty((m, m), dtype=torch.float64, device=J.device) if want_S else None
        Z = torch.empty((m, self.N), dtype=self.vdtype, device=J.device) if want_Z else None
        info = nat.h1w_capacitance_build(self.handle, J, alpha, factor, S, Z)
        self._J = J  # the library keeps a pointer to J for later preconditioner applies
        return S, Z, info

    def precond_apply(self, R, out=None, zmode=nat.H1W_Z_AUTO):
        import torch
        out = torch.empty_like(R) if out is None else out
        return nat.h1w_precond_apply(self.handle, R, out, zmode)

    MODES = {"woodbury": 0, "laplace": nat.H1W_SOLVE_LAPLACE_ONLY, "exact": nat.H1W_SOLVE_EXACT_B}

    def gn_solve(self, J, alpha, b=None, d=None, res=None, x=None, rtol=0.0, maxit=0,
                 zmode=nat.H1W_Z_AUTO, factor=nat.H1W_FACTOR_AUTO, mode="woodbury"):
        """mode: 'woodbury' (the method), 'laplace' (B/alpha only, Algorithm 4's
        preconditioner) or 'exact' (B = A^-1 by MG-PCG to 1e-12, Algorithm 1's
        exact Woodbury inverse; FP64 contexts)."""
        import torch
        ref = b if b is not None else d
        x = torch.empty_like(ref) if x is None else x
        info = nat.h1w_gn_solve(self.handle, J, alpha, x, b, d, res, rtol, maxit, zmode, factor,
                                flags=self.MODES[mode])
        self._J = J  # the capacitance left in the context refers to J
        return x, info

    def gn_apply(self, J, alpha, x, y=None):
        import torch
        y = torch.empty_like(x) if y is None else y
        return nat.h1w_gn_apply(self.handle, J, alpha, x, y)

    # ---------------------------------------------------------------- kernel timing
    def set_kernel_timing(self, classes):
        """Time the given kernel classes (names from _native.KCLASS, or 'all'; [] = off)."""
        if classes == "all":
            mask = (1 << len(nat.KCLASS)) - 1
        else:
            mask = 0
            for c in classes:
                mask |= 1 << nat.KCLASS.index(c)
        nat.h1w_set_kernel_timing(self.handle, mask)

    def kernel_timing(self) -> dict:
        return {name: nat.h1w_get_kernel_timing(self.handle, i) for i, name in enumerate(nat.KCLASS)}

    def reset_kernel_timing(self):
        nat.h1w_reset_kernel_timing(self.handle)

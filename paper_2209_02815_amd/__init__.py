"""MI355X library for the Gauss-Newton linear systems of H^1-regularised
parameter identification (Blechta & Ernst, arXiv 2209.02815).

    G x = b,  G = alpha*A + J^T J   (A: H^1 Gram operator on a structured grid)

solved by conjugate gradients with the Woodbury preconditioner around a
batched geometric-multigrid V-cycle, all in the HIP library libh1w.so
(C ABI in include/h1w.h), plus the ERT forward map and its adjoint that
produce J (Section 4). This package is the Python binding: argument
marshalling with torch tensors that live on the GPU.
"""
from ._native import *  # noqa: F401,F403
from ._native import H1WError, h1w_info, lib  # noqa: F401
from .solver import Context  # noqa: F401
from .ert import ErtContext, ert_gauss_newton, ert_voltages  # noqa: F401

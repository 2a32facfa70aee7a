"""Multigrid parameters that tests give to the GPU contexts and to the
oracle's V-cycle alike. Section 3.2 treats the Laplace solve inside the
preconditioner as a black box, so these are parameters of B, chosen here and
passed explicitly on both sides: nu = 2 smoothing steps per side, the
Chebyshev interval [0.3, 2] for eig(D^-1 A), and the coarsest level the first
with at most 729 nodes (3D) or 81 (2D)."""
from oracle import multigrid as mg

MG = {2: dict(nu=2, lo=0.3, hi=2.0, coarse_max=81), 3: dict(nu=2, lo=0.3, hi=2.0, coarse_max=729)}


def params(dim, **over):
    """The parameters for a dim-D grid with the non-None overrides applied."""
    p = dict(MG[dim])
    p.update({k: v for k, v in over.items() if v is not None})
    return p


def vcycle(shape, beta, **over):
    """The oracle's V-cycle with these parameters."""
    return mg.VCycle(shape, beta, **params(len(shape), **over))


def ctx_kw(dim, **over):
    """Keyword arguments of paper_2209_02815_amd.Context for the same parameters."""
    p = params(dim, **over)
    return dict(nu=p["nu"], cheb=(p["lo"], p["hi"]), coarse_max=p["coarse_max"])

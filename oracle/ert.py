"""ERT forward map, pole-pole voltages and their sensitivities (Section 4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Model (Section 4, eq. (model)): -div(sigma grad u) = f in the unit cube, u = 0
on the Dirichlet faces, zero normal flux on the others; the electrodes sit on
the Neumann top face. The conductivity is a nodal field sigma = exp(m) with the
log parametrisation of Section 4, so J has one column per grid node.

Discretisation (our reading; the paper works on unstructured FE meshes): the
vertex-centred finite-volume form of the operator on the structured grid. Each
grid edge (p, q) along axis d carries the conductance

    c_pq = (sigma_p + sigma_q)/2 * (dual-face area) / h_d,

the dual-face area being the product over the other axes of h_e, halved for
every such axis on which the edge lies in a boundary face. The discrete
operator is the quadratic form sum_edges c_pq (u_p - u_q)^2, restricted to the
nodes that are not on a Dirichlet face. A unit pole source at node a is the
nodal load e_a, so u_a = A^{-1} e_a is the potential of a unit current.

Voltages (eq. (ert_qoi2) with the pole-pole limit of eq. (ert_qoi_scaling),
both return electrodes at infinity, as the paper's B electrode):
g_i = k_i u_a(x_b), k_i = 2 pi |x_a - x_b| for pair i = (a, b).

Sensitivities (eq. (ert_qoi_derivative) after the change of variables
m = log sigma; discretely d(A^{-1}) = -A^{-1} dA A^{-1}, and by symmetry of A
the adjoint field of receiver b is the source field u_b):
J[i, j] = -k_i sum_{edges (j, q)} (sigma_j / 2) * (face area / h) *
          (u_a(j) - u_a(q)) (u_b(j) - u_b(q)).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def dirichlet_nodes(shape, mask: int) -> np.ndarray:
    """Boolean (N,) array: nodes on a face whose bit is set in `mask`
    (bits 0..5 = faces x=0, x=1, y=0, y=1, z=0, z=1; x fastest)."""
    idx = np.indices(tuple(reversed(shape)))          # (z, y, x) index grids
    on = np.zeros(tuple(reversed(shape)), dtype=bool)
    for ax in range(len(shape)):
        i = idx[len(shape) - 1 - ax]
        if mask >> (2 * ax) & 1:
            on |= i == 0
        if mask >> (2 * ax + 1) & 1:
            on |= i == shape[ax] - 1
    return on.reshape(-1)


def node_coords(shape) -> np.ndarray:
    """(N, dim) coordinates of the nodes on the unit cube, x fastest."""
    axes = [np.arange(n) / (n - 1) for n in shape]
    grids = np.meshgrid(*reversed(axes), indexing="ij")   # (z, y, x)
    return np.stack([g.reshape(-1) for g in reversed(grids)], axis=1)


def edges(shape):
    """Every grid edge as (p, q, geom) arrays, one triple per axis, with
    geom = dual-face area / edge length (boundary halving as in the module
    docstring)."""
    dim = len(shape)
    h = [1.0 / (n - 1) for n in shape]
    ids = np.arange(int(np.prod(shape))).reshape(tuple(reversed(shape)))
    out = []
    for ax in range(dim):
        arr_ax = dim - 1 - ax
        lo = [slice(None)] * dim
        hi = [slice(None)] * dim
        lo[arr_ax] = slice(0, shape[ax] - 1)
        hi[arr_ax] = slice(1, shape[ax])
        p = ids[tuple(lo)]
        q = ids[tuple(hi)]
        geom = np.full(p.shape, 1.0 / h[ax])
        for other in range(dim):
            if other == ax:
                continue
            w = np.full(shape[other], h[other])
            w[0] *= 0.5
            w[-1] *= 0.5
            view = [1] * dim
            view[dim - 1 - other] = shape[other]
            geom = geom * w.reshape(view)
        out.append((p.reshape(-1), q.reshape(-1), np.broadcast_to(geom, p.shape).reshape(-1).copy()))
    return out


def full_matrix(shape, logsig) -> sp.csr_matrix:
    """The conductance quadratic form on every node (Neumann on all faces)."""
    sig = np.exp(np.asarray(logsig, dtype=np.float64))
    N = sig.size
    rows, cols, vals = [], [], []
    for p, q, geom in edges(shape):
        c = 0.5 * (sig[p] + sig[q]) * geom
        rows += [p, q, p, q]
        cols += [p, q, q, p]
        vals += [c, c, -c, -c]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def operator(shape, logsig, mask: int):
    """(A_free, free): the operator on the non-Dirichlet nodes and their indices."""
    free = np.flatnonzero(~dirichlet_nodes(shape, mask))
    A = full_matrix(shape, logsig)
    return A[free][:, free].tocsc(), free


def fields(shape, logsig, mask: int, src_nodes) -> np.ndarray:
    """U (n_src, N): u_a = A^{-1} e_a for each source node, zero on Dirichlet nodes."""
    Af, free = operator(shape, logsig, mask)
    pos = np.full(int(np.prod(shape)), -1)
    pos[free] = np.arange(free.size)
    src = np.asarray(src_nodes)
    if np.any(pos[src] < 0):
        raise ValueError("a source lies on a Dirichlet face")
    rhs = np.zeros((free.size, src.size))
    rhs[pos[src], np.arange(src.size)] = 1.0
    lu = spla.splu(Af)
    U = np.zeros((src.size, int(np.prod(shape))))
    U[:, free] = lu.solve(rhs).T
    return U


def pole_pole_factors(shape, src_nodes, pairs) -> np.ndarray:
    """k_i = 2 pi |x_a - x_b| (eq. (ert_qoi_scaling), d = 3, x_B and x_N at infinity)."""
    x = node_coords(shape)[np.asarray(src_nodes)]
    pairs = np.asarray(pairs)
    return 2.0 * np.pi * np.linalg.norm(x[pairs[:, 0]] - x[pairs[:, 1]], axis=1)


def measurements(U, src_nodes, pairs, k) -> np.ndarray:
    """g_i = k_i u_a(x_b) for pair i = (a, b) (eq. (ert_qoi2))."""
    pairs = np.asarray(pairs)
    return np.asarray(k) * U[pairs[:, 0], np.asarray(src_nodes)[pairs[:, 1]]]


def jacobian(shape, logsig, U, pairs, k) -> np.ndarray:
    """J (n_meas, N) = d g / d m by the adjoint formula of the module docstring,
    accumulated edge by edge onto both end nodes."""
    sig = np.exp(np.asarray(logsig, dtype=np.float64))
    pairs = np.asarray(pairs)
    Ua, Ub = U[pairs[:, 0]], U[pairs[:, 1]]
    J = np.zeros((len(pairs), sig.size))
    for p, q, geom in edges(shape):
        prod = (Ua[:, p] - Ua[:, q]) * (Ub[:, p] - Ub[:, q]) * geom   # (n_meas, n_edges)
        # d c_pq / d m_p = sigma_p geom / 2, likewise for q
        np.add.at(J.T, p, (prod * (0.5 * sig[p])).T)
        np.add.at(J.T, q, (prod * (0.5 * sig[q])).T)
    return -np.asarray(k)[:, None] * J


def forward(shape, logsig, mask, src_nodes, pairs):
    """(g, U): the voltages and the source fields."""
    U = fields(shape, logsig, mask, src_nodes)
    k = pole_pole_factors(shape, src_nodes, pairs)
    return measurements(U, src_nodes, pairs, k), U

"""Seeded synthetic inputs for the H^1-regularised Gauss-Newton linear solve.

This module only draws numbers: grids, sensitivity rows J_i, right-hand sides b
and the paper-form data (m - m_ref, g - g_obs). It contains none of the
solver's arithmetic and is imported by both the CPU oracle and the GPU path's
tests and benchmark, so that both sides see bit-identical inputs.

The paper's experiments (ERT on unstructured meshes, Section 4) need meshes
and data that are not available; the workloads below are synthetic stand-ins
with the shapes the linear solve of Algorithm 3 sees: a dense M x N
sensitivity matrix (Section 2.3, the matrix J_m) whose rows are smooth,
localised fields, and an N-vector right-hand side.

Seeding: every array is drawn from numpy's PCG64 seeded with
SeedSequence([workload_id, stream, row]); stream 0 = rows of J (noise),
1 = right-hand side b, 2 = bump parameters of the rows of J, 3 = paper-form
data d and res, 4 = instance parameters of an uneven batch, 5 = the white noise
of an ERT conductivity field. Per-row seeds let a large J be regenerated in
row chunks.

ERT surveys (the forward problem of Section 4 that produces J): a structured
grid of the unit cube, a log-conductivity field drawn as a Gaussian random
field, and a lattice of electrodes on the top face (z = 1) whose pole sources
and pole-pole pairs define the measurements. Only the layout and the random
field are drawn here; the forward map, the geometric factors and the
sensitivities belong to the solvers.
"""
from __future__ import annotations

import dataclasses
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "workload", "grid_shape", "num_nodes", "axis_coords",
    "j_rows", "j_row_blocks", "upload_j", "rhs_b", "paper_data", "rng_for", "batch_workloads",
    "ErtSurvey", "ert_survey", "ert_logsig", "ERT_DIRICHLET_DEFAULT",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic GN-system workload.

    shape   nodes per axis, x fastest (len 2 or 3); unit square / cube
    beta    mass weight of the H^1 Gram operator A = K + beta*M
    alpha   regularisation weight in (alpha*A + J^T J) x = b
    m       rows of J
    j_kind  "gauss" (iid N(0,1)/sqrt(N) entries) or "bumps" (sum of Gaussian
            bumps of width `width` with N(0,1) amplitudes plus `noise` white noise)
    wid     integer workload id used in the seed
    """
    name: str
    wid: int
    shape: tuple
    beta: float
    alpha: float
    m: int
    j_kind: str
    nbumps: int = 4
    width: float = 0.05
    noise: float = 1e-3

    @property
    def dim(self) -> int:
        return len(self.shape)

    @property
    def N(self) -> int:
        return num_nodes(self.shape)

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


WORKLOADS = {
    # 2D unit square, 33x33 nodes, J iid Gaussian rows.
    "square33": Workload("square33", 1, (33, 33), 1e-2, 1e-3, 16, "gauss"),
    # 3D unit cube, 129^3 nodes, 512 bump rows.
    "cube129": Workload("cube129", 2, (129, 129, 129), 1e-2, 1e-4, 512, "bumps"),
    # 3D unit cube, 257^3 nodes, 1024 bump rows.
    "cube257": Workload("cube257", 4, (257, 257, 257), 1e-2, 1e-5, 1024, "bumps"),
    # Reduced 3D cases used by parity tests (same recipe as cube129).
    "cube17": Workload("cube17", 12, (17, 17, 17), 1e-2, 1e-4, 24, "bumps"),
    "cube33": Workload("cube33", 13, (33, 33, 33), 1e-2, 1e-4, 64, "bumps"),
    "cube65": Workload("cube65", 14, (65, 65, 65), 1e-2, 1e-4, 128, "bumps"),
    # 2D square with bump rows (shape of one instance of the batched workload).
    "square129": Workload("square129", 15, (129, 129), 1e-2, 1e-4, 64, "bumps"),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


# A batch of independent instances of uneven size: 2D unit squares with sides
# drawn uniformly from `sides`, m uniform in [m_lo, m_hi], log10(alpha) uniform
# in [log10 a_lo, log10 a_hi], beta = 1e-2, bump rows (as cube129, in 2D) and
# b ~ N(0,1). Instance k has workload id batch_id * 100000 + k; the drawing of
# (side, m, alpha) uses stream 4 of batch_id.
BATCH_DEFAULT = dict(count=256, sides=(65, 129, 193, 257), m_lo=16, m_hi=128, a_lo=1e-5, a_hi=1e-2)


def batch_workloads(count: int = 256, batch_id: int = 5, sides=(65, 129, 193, 257), m_lo: int = 16,
                    m_hi: int = 128, a_lo: float = 1e-5, a_hi: float = 1e-2) -> list:
    rng = rng_for(batch_id, 4)
    side = rng.choice(np.asarray(sides), size=count)
    m = rng.integers(m_lo, m_hi + 1, size=count)
    alpha = 10.0 ** rng.uniform(np.log10(a_lo), np.log10(a_hi), size=count)
    return [Workload(f"batch{batch_id}_{k}", batch_id * 100000 + k, (int(side[k]), int(side[k])), 1e-2,
                     float(alpha[k]), int(m[k]), "bumps") for k in range(count)]


def grid_shape(wl: Workload) -> tuple:
    return tuple(wl.shape)


def num_nodes(shape) -> int:
    return int(np.prod(shape))


def axis_coords(n: int) -> np.ndarray:
    """Node coordinates on [0, 1] for n vertex-centred nodes."""
    return np.arange(n, dtype=np.float64) / (n - 1)


def rng_for(wid: int, stream: int, row: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([wid, stream, row])))


def _one_row(wl: Workload, i: int, out: np.ndarray | None = None) -> np.ndarray:
    """Row i of J, written into `out` (length N) when given.

    Bump rows: out = noise * xi + sum_k a_k g_k, with g_k the separable
    Gaussian prod_d exp(-(x_d - c_kd)^2 / (2 w^2)). The bump sum is formed as a
    product with inner dimension nbumps: (slowest-axis factors, n_slow x K)
    times (a_k times the outer product of the other axes' factors, K x rest),
    added slab by slab of the slowest axis, so no N-sized temporary is made."""
    N = wl.N
    if out is None:
        out = np.empty(N, dtype=np.float64)
    if wl.j_kind == "gauss":
        rng_for(wl.wid, 0, i).standard_normal(N, out=out)
        out /= np.sqrt(N)
        return out
    if wl.j_kind != "bumps":
        raise ValueError(f"unknown j_kind {wl.j_kind!r}")
    prm = rng_for(wl.wid, 2, i)
    centres = prm.random((wl.nbumps, wl.dim))
    amps = prm.standard_normal(wl.nbumps)
    rng_for(wl.wid, 0, i).standard_normal(N, out=out)
    out *= wl.noise
    s2 = 2.0 * wl.width ** 2
    g = [[np.exp(-(axis_coords(wl.shape[ax]) - centres[k, ax]) ** 2 / s2) for ax in range(wl.dim)]
         for k in range(wl.nbumps)]
    slow = wl.dim - 1                     # x fastest in memory: the last axis is the slowest
    F = np.stack([g[k][slow] for k in range(wl.nbumps)], axis=1)       # (n_slow, K)
    R = []
    for k in range(wl.nbumps):
        f = None
        for ax in reversed(range(slow)):  # the remaining axes, slowest first
            f = g[k][ax] if f is None else np.multiply.outer(f, g[k][ax])
        R.append(amps[k] * f.ravel())
    R = np.stack(R)                                                     # (K, rest)
    grid = out.reshape(wl.shape[slow], -1)
    step = max(1, (1 << 20) // grid.shape[1])
    for s0 in range(0, grid.shape[0], step):
        grid[s0:s0 + step] += F[s0:s0 + step] @ R
    return out


def j_rows(wl: Workload, i0: int = 0, i1: int | None = None, dtype=np.float64,
           threads: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    """Rows i0..i1-1 of J as a C-contiguous (i1-i0, N) array (row i = sensitivity i).
    `out`, if given, is filled in place (FP64 rows, or any dtype through a
    per-row FP64 buffer). The rows are drawn in parallel on `threads` threads
    with the BLAS of each thread's small products kept single-threaded."""
    i1 = wl.m if i1 is None else i1
    if not (0 <= i0 <= i1 <= wl.m):
        raise ValueError("row range out of bounds")
    if out is None:
        out = np.empty((i1 - i0, wl.N), dtype=dtype)
    threads = threads or min(16, os.cpu_count() or 1)
    direct = out.dtype == np.float64

    def fill(i):
        if direct:
            _one_row(wl, i, out[i - i0])
        else:
            out[i - i0] = _one_row(wl, i)

    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1, user_api="blas"):
        if threads > 1 and i1 - i0 > 1:
            with ThreadPoolExecutor(threads) as ex:
                list(ex.map(fill, range(i0, i1)))
        else:
            for i in range(i0, i1):
                fill(i)
    return out


def j_row_blocks(wl: Workload, block: int = 32, threads: int | None = None):
    """Yield (i0, rows) for consecutive blocks of `block` rows of J, every row
    once, in order. The rows are written into one host buffer that is reused
    for every block, so a consumer must be done with a block before it asks
    for the next (J of the 257^3 workload is 139 GB and is never held whole)."""
    buf = np.empty((min(block, wl.m), wl.N), dtype=np.float64)
    for i0 in range(0, wl.m, block):
        i1 = min(wl.m, i0 + block)
        yield i0, j_rows(wl, i0, i1, threads=threads, out=buf[:i1 - i0])


def upload_j(wl: Workload, Jd, threads: int | None = None, block: int = 32, log=None):
    """Fill the device tensor Jd (m x N, FP64, row-major) with J, block by
    block through two pinned host buffers: a block is drawn into one buffer
    while the previous one is copied to the device, so J is never held whole
    on the host. Returns nothing; the copies have finished on return."""
    import time
    import torch
    rows = min(block, wl.m)
    bufs = [torch.empty((rows, wl.N), dtype=torch.float64, pin_memory=True) for _ in range(2)]
    done = [None, None]
    t0 = time.perf_counter()
    for n, i0 in enumerate(range(0, wl.m, block)):
        i1 = min(wl.m, i0 + block)
        k = n % 2
        if done[k] is not None:
            done[k].synchronize()
        j_rows(wl, i0, i1, threads=threads, out=bufs[k].numpy()[:i1 - i0])
        Jd[i0:i1].copy_(bufs[k][:i1 - i0], non_blocking=True)
        done[k] = torch.cuda.Event()
        done[k].record()
        if log is not None and n % 8 == 0:
            log(f"J rows {i0}..{i1} on the device ({time.perf_counter() - t0:.0f} s)")
    torch.cuda.synchronize()
    del bufs


def rhs_b(wl: Workload, k: int = 1) -> np.ndarray:
    """k right-hand sides b ~ N(0,1), shape (k, N) (k=1 -> shape (N,))."""
    b = np.stack([rng_for(wl.wid, 1, j).standard_normal(wl.N) for j in range(k)])
    return b[0] if k == 1 else b


def paper_data(wl: Workload) -> tuple:
    """(d, res): d = m - m_ref (smooth N-vector), res = g - g_obs (M-vector).

    Used to form the paper's Gauss-Newton right-hand side; d is a low-frequency
    cosine field plus noise so that the regularisation term is O(1).
    """
    g = rng_for(wl.wid, 3, 0)
    amps = g.standard_normal(3)
    d = 0.0
    for k, a in enumerate(amps):
        f = None
        for ax in reversed(range(wl.dim)):
            c = np.cos((k + 1) * np.pi * axis_coords(wl.shape[ax]))
            f = c if f is None else np.multiply.outer(f, c)
        d = d + a * f
    d = np.ascontiguousarray(d).reshape(-1) + 0.1 * g.standard_normal(wl.N)
    res = g.standard_normal(wl.m)
    return d, res


# ---------------------------------------------------------------- ERT surveys

# Faces with u = 0, one bit each: x = 0, x = 1, y = 0, y = 1, z = 0, z = 1.
# Default: every face but the top (z = 1), where the electrodes sit (Neumann).
ERT_DIRICHLET_DEFAULT = 0x1F


@dataclasses.dataclass(frozen=True)
class ErtSurvey:
    """A pole-pole ERT survey on the n^3 unit-cube grid.

    electrodes  node indices (x fastest) of the electrodes on the top face,
                ordered with the lattice's x index fastest
    ex, ey      their lattice node coordinates (ix, iy); iz = n - 1
    pairs       (n_meas, 2) int32, every electrode pair (a, b) with a < b
                (source a, receiver b; the return electrode is at infinity)
    wid         workload id of the conductivity field's seed
    """
    name: str
    wid: int
    shape: tuple
    electrodes: np.ndarray
    ex: np.ndarray
    ey: np.ndarray
    pairs: np.ndarray
    mask: int = ERT_DIRICHLET_DEFAULT
    log10_mean: float = -2.0
    log10_std: float = 0.5
    corr: float = 0.2

    @property
    def N(self) -> int:
        return num_nodes(self.shape)

    @property
    def n_src(self) -> int:
        return len(self.electrodes)

    @property
    def n_meas(self) -> int:
        return len(self.pairs)


def ert_survey(n: int = 65, nex: int = 8, ney: int = 4, spacing: int | None = None, wid: int = 3,
               name: str | None = None) -> ErtSurvey:
    """Centred nex x ney electrode lattice with `spacing` nodes between
    neighbours on the top face of the n^3 grid. n = 65 with the defaults gives
    ix in {11, 17, ..., 53}, iy in {23, 29, 35, 41}: 32 electrodes, 496 pairs."""
    if spacing is None:
        spacing = max(1, round(6 * (n - 1) / 64))
    c = (n - 1) / 2
    ox, oy = c - spacing * (nex - 1) / 2, c - spacing * (ney - 1) / 2
    if ox != int(ox) or oy != int(oy):
        raise ValueError("lattice not centred on nodes: make (nex-1)*spacing and (ney-1)*spacing even")
    ix = int(ox) + spacing * np.arange(nex)
    iy = int(oy) + spacing * np.arange(ney)
    if ix[0] < 1 or iy[0] < 1 or ix[-1] > n - 2 or iy[-1] > n - 2:
        raise ValueError("electrode lattice does not fit inside the top face")
    ex = np.tile(ix, ney)
    ey = np.repeat(iy, nex)
    nodes = ex + n * (ey + n * (n - 1))
    a, b = np.triu_indices(len(nodes), k=1)
    pairs = np.stack([a, b], axis=1).astype(np.int32)
    return ErtSurvey(name or f"ert{n}", wid, (n, n, n), nodes.astype(np.int64), ex, ey, pairs)


def ert_logsig(sv: ErtSurvey) -> np.ndarray:
    """Natural-log conductivity at the nodes (N,), x fastest.

    log10(sigma) is a Gaussian random field with covariance
    0.25 exp(-r^2 / (2 corr^2)) sampled by circulant embedding: the covariance
    is evaluated on a periodic grid of 2 n_d nodes per axis with the grid's
    spacing (wrapped distances), white noise from stream 5 is filtered by the
    square root of its non-negative spectrum, the first n_d nodes per axis
    are kept, and the result is shifted and scaled to the survey's mean and
    standard deviation exactly."""
    shape = sv.shape
    M = [2 * n for n in shape]
    r2 = 0.0
    for ax in range(len(shape)):
        k = np.arange(M[ax])
        dist = np.minimum(k, M[ax] - k) / (shape[ax] - 1)
        # array axes are (z, y, x): axis ax of the grid is array axis -1 - ax
        view = [1] * len(shape)
        view[len(shape) - 1 - ax] = M[ax]
        r2 = r2 + (dist ** 2).reshape(view)
    cov = 0.25 * np.exp(-r2 / (2.0 * sv.corr ** 2))
    lam = np.maximum(np.fft.fftn(cov).real, 0.0)
    noise = rng_for(sv.wid, 5).standard_normal(tuple(reversed(M)))
    field = np.fft.ifftn(np.sqrt(lam) * np.fft.fftn(noise)).real
    crop = field[tuple(slice(0, n) for n in reversed(shape))]
    crop = (crop - crop.mean()) / crop.std()
    log10 = sv.log10_mean + sv.log10_std * crop
    return np.ascontiguousarray(np.log(10.0) * log10).reshape(-1)

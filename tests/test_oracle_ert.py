"""Pins of the ERT oracle (Section 4): the forward operator against the pinned
H^1 stiffness and a manufactured solution, the sensitivities against brute-force
finite differences and the exact homogeneity identity, reciprocity, the sign
structure of the fields and the half-space apparent-resistivity sanity check."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import h1w_inputs as H
from oracle import ert, operator


@pytest.mark.parametrize("shape,mask", [((5, 7, 9), 0x1F), ((9, 5, 6), 0x01), ((6, 6, 5), 0x2A)])
def test_constant_sigma_is_cell_volume_times_h1_stiffness(shape, mask):
    # sigma = 1: every conductance is (face area)/h, i.e. (prod h) times the
    # K part of the Gram operator, whose entries are pinned by its closed-form
    # eigenpairs; sigma = c scales the operator by c
    Af, free = ert.operator(shape, np.zeros(int(np.prod(shape))), mask)
    K = operator.gram_operator(shape, 0.0)
    vol = np.prod([1.0 / (n - 1) for n in shape])
    ref = vol * K[free][:, free]
    assert abs(Af - ref).max() <= 1e-15 * abs(ref).max()
    Ac, _ = ert.operator(shape, np.full(int(np.prod(shape)), np.log(3.0)), mask)
    assert abs(Ac - 3.0 * Af).max() <= 1e-14 * abs(Af).max()


def test_dirichlet_faces():
    on = ert.dirichlet_nodes((4, 5, 6), 0x1F).reshape(6, 5, 4)
    assert on[0].all() and on[:, 0].all() and on[:, -1].all() and on[:, :, 0].all() and on[:, :, -1].all()
    assert not on[-1, 1:-1, 1:-1].any()       # top face interior is Neumann
    assert on.sum() == 4 * 5 * 6 - 2 * 3 * 5


def _manufactured_error(n):
    # u = sin(pi x) sin(pi y) sin(pi z / 2): zero on x = 0, 1, y = 0, 1, z = 0 and
    # zero normal derivative on z = 1; sigma = exp(0.3 x + 0.2 y z);
    # f = -div(sigma grad u) = -sigma (lap u + grad m . grad u)
    shape = (n, n, n)
    x = ert.node_coords(shape)
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    m = 0.3 * X + 0.2 * Y * Z
    pi = np.pi
    s, c = np.sin, np.cos
    u = s(pi * X) * s(pi * Y) * s(pi * Z / 2)
    gu = np.stack([pi * c(pi * X) * s(pi * Y) * s(pi * Z / 2),
                   pi * s(pi * X) * c(pi * Y) * s(pi * Z / 2),
                   0.5 * pi * s(pi * X) * s(pi * Y) * c(pi * Z / 2)], 1)
    gm = np.stack([np.full_like(X, 0.3), 0.2 * Z, 0.2 * Y], 1)
    f = -np.exp(m) * (-2.25 * pi ** 2 * u + (gm * gu).sum(1))
    idx = np.rint(x * (n - 1)).astype(int)
    w = np.where((idx == 0) | (idx == n - 1), 0.5, 1.0).prod(1)
    vol = w / (n - 1) ** 3                       # dual-cell volume
    Af, free = ert.operator(shape, m, 0x1F)
    uh = spla.spsolve(Af, (f * vol)[free])
    return np.abs(uh - u[free]).max()


def test_manufactured_solution_second_order():
    e = [_manufactured_error(n) for n in (9, 17, 33)]
    rates = [np.log2(e[i] / e[i + 1]) for i in range(2)]
    assert all(1.9 <= r <= 2.1 for r in rates), (e, rates)


def _survey(n=9, nex=3, ney=2, s=2):
    sv = H.ert_survey(n, nex, ney, s, wid=31)
    return sv, H.ert_logsig(sv)


def test_homogeneity_row_sums():
    # A_{exp(m + t)} = exp(t) A_{exp(m)} gives g(m + t 1) = exp(-t) g(m), so
    # d/dt at 0: J 1 = -g exactly (a dropped factor 1/2 or a sign fails it)
    for sv, m in (_survey(), _survey(17, 4, 2, 2)):
        g, U = ert.forward(sv.shape, m, sv.mask, sv.electrodes, sv.pairs)
        k = ert.pole_pole_factors(sv.shape, sv.electrodes, sv.pairs)
        J = ert.jacobian(sv.shape, m, U, sv.pairs, k)
        assert np.abs(J.sum(1) + g).max() <= 1e-12 * np.abs(g).max()


def test_bruteforce_fd_jacobian():
    # full central-difference Jacobian, one node at a time, on a 7^3 grid
    sv = H.ert_survey(7, 3, 2, 2, wid=32)
    m = H.ert_logsig(sv)
    g, U = ert.forward(sv.shape, m, sv.mask, sv.electrodes, sv.pairs)
    J = ert.jacobian(sv.shape, m, U, sv.pairs, ert.pole_pole_factors(sv.shape, sv.electrodes, sv.pairs))
    h = 1e-5
    Jfd = np.empty_like(J)
    for j in range(sv.N):
        e = np.zeros(sv.N)
        e[j] = h
        gp, _ = ert.forward(sv.shape, m + e, sv.mask, sv.electrodes, sv.pairs)
        gm, _ = ert.forward(sv.shape, m - e, sv.mask, sv.electrodes, sv.pairs)
        Jfd[:, j] = (gp - gm) / (2 * h)
    assert np.abs(Jfd - J).max() <= 1e-7 * np.abs(J).max()
    # Dirichlet nodes next to free ones carry sensitivity (their sigma sets the
    # conductance of the edges into the domain)
    on = ert.dirichlet_nodes(sv.shape, sv.mask)
    assert np.abs(J[:, on]).max() > 1e-3 * np.abs(J).max()


def test_directional_fd_twenty_directions():
    sv, m = _survey(17, 4, 2, 2)
    g, U = ert.forward(sv.shape, m, sv.mask, sv.electrodes, sv.pairs)
    J = ert.jacobian(sv.shape, m, U, sv.pairs, ert.pole_pole_factors(sv.shape, sv.electrodes, sv.pairs))
    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(20):
        v = rng.standard_normal(sv.N)
        gp, _ = ert.forward(sv.shape, m + h * v, sv.mask, sv.electrodes, sv.pairs)
        gm, _ = ert.forward(sv.shape, m - h * v, sv.mask, sv.electrodes, sv.pairs)
        fd = (gp - gm) / (2 * h)
        assert np.linalg.norm(fd - J @ v) <= 1e-6 * np.linalg.norm(J @ v)


def test_reciprocity_and_sign_structure():
    # u_a(x_b) = u_b(x_a) (Section 4, the first equality of eq. (ert_qoi));
    # a unit positive current gives a potential that vanishes on the Dirichlet
    # faces and is positive at every other node (M-matrix, connected grid)
    sv, m = _survey(17, 4, 2, 2)
    U = ert.fields(sv.shape, m, sv.mask, sv.electrodes)
    V = U[:, sv.electrodes]
    assert np.abs(V - V.T).max() <= 1e-12 * np.abs(V).max()
    on = ert.dirichlet_nodes(sv.shape, sv.mask)
    assert np.all(U[:, on] == 0.0)
    assert np.all(U[:, ~on] > 0.0)
    # each field is the largest at its own source
    assert np.all(np.argmax(U, axis=1) == sv.electrodes)


def test_half_space_apparent_resistivity_sanity():
    # For a homogeneous half space g = 1/sigma0 exactly (footnote to eq.
    # (ert_qoi_scaling)). The unit cube with u = 0 on five faces only lowers
    # the potential, and the grid's pole is accurate to a few per cent at two
    # nodes' distance: a sanity bound, not a pin of the geometric factor's value
    sv = H.ert_survey(17, 4, 2, 2)
    s0 = 1e-2
    g, _ = ert.forward(sv.shape, np.full(sv.N, np.log(s0)), sv.mask, sv.electrodes, sv.pairs)
    k = ert.pole_pole_factors(sv.shape, sv.electrodes, sv.pairs)
    assert np.all(g * s0 > 0.0) and np.all(g * s0 < 1.05)
    near = k <= k.min() * (1 + 1e-12)
    assert np.all(g[near] * s0 > 0.8)


def test_survey_layout_and_field_statistics():
    sv = H.ert_survey()
    assert sv.shape == (65, 65, 65) and sv.n_src == 32 and sv.n_meas == 496
    assert list(sv.ex[:8]) == list(range(11, 54, 6)) and list(sv.ey[::8]) == [23, 29, 35, 41]
    assert np.all(sv.electrodes // (65 * 65) == 64)
    assert not ert.dirichlet_nodes(sv.shape, sv.mask)[sv.electrodes].any()
    assert np.all(sv.pairs[:, 0] < sv.pairs[:, 1])
    m = H.ert_logsig(sv)
    l10 = m / np.log(10.0)
    assert abs(l10.mean() + 2.0) < 1e-12 and abs(l10.std() - 0.5) < 1e-12
    assert np.array_equal(m, H.ert_logsig(sv))

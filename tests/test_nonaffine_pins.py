"""Pins of the oracle's prisms without the affine assumption (Sec. 2.2 takes
F_K affine; here J, det J and J^{-1} of the P1 x P1 vertex map are evaluated
at every quadrature point), against closed forms, exact integrals and
invariants."""
import numpy as np
import pytest

import oracle
from paper_1604_05872_amd import inputs as I
from test_global_pins import global_nodes


def one_prism(heights):
    tri = np.array([[0.1, 0.2], [1.3, 0.4], [0.5, 1.7]])
    bottom = np.concatenate([tri, np.zeros((3, 1))], axis=1)
    top = np.concatenate([tri, np.array(heights, dtype=float)[:, None]], axis=1)
    return np.concatenate([bottom, top])[None]


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_single_prism_volume(p):
    """A vertical prism over a triangle T with edge heights h_i has volume
    |T| (h_0 + h_1 + h_2) / 3; the mass matrix sums to it (partition of unity)."""
    h = [0.7, 1.1, 1.6]
    c = one_prism(h)
    tri = c[0, :3, :2]
    area = 0.5 * abs((tri[1, 0] - tri[0, 0]) * (tri[2, 1] - tri[0, 1]) - (tri[2, 0] - tri[0, 0]) * (tri[1, 1] - tri[0, 1]))
    M, fl = oracle.assemble_pointgeo("mass", p, c)
    assert fl == 0
    assert abs(M.sum() - area * sum(h) / 3) < 1e-14 * area
    # the affine oracle rejects this prism
    _, fl_aff = oracle.assemble("mass", "prism", p, c)
    assert fl_aff == 1


@pytest.mark.parametrize("p", [1, 2, 3])
def test_affine_prisms_reduce_to_affine_oracle(p):
    """With every top face a translate of the bottom the per-point maps are
    the affine map."""
    c, V, cells, h = I.first_elements("prism", 40, 3)
    for form in ("mass", "helmholtz"):
        q = oracle.default_qdeg_pointgeo(form, p)
        A, _ = oracle.assemble(form, "prism", p, c, qdeg=q)
        B, fl = oracle.assemble_pointgeo(form, p, c, qdeg=q)
        assert fl == 0
        assert np.abs(A - B).max() <= 1e-13 * np.abs(A).max()


def zjittered_box(n, p, seed=6):
    V, cells = I.prism_mesh(n, n, seed, zjitter=0.3)
    coords = I.gather(V, cells)
    dofs, N = I.global_dofs("prism", p, cells, n)
    return coords, V, cells, dofs, N


def node_positions_pointgeo(p, coords, dofs, N):
    """Nodes of a non-affine prism: the vertex map at the reference nodes."""
    a = I._node_multi_indices("prism", p).astype(float) / p
    X, Y, Z = a[:, 0], a[:, 1], a[:, 2]
    lam = np.stack([1 - X - Y, X, Y], axis=1)          # [ns][3]
    psi = np.concatenate([lam * (1 - Z)[:, None], lam * Z[:, None]], axis=1)   # [ns][6]
    x = np.einsum("nv,evd->end", psi, coords)
    G = np.full((N, 3), np.nan)
    G[dofs.ravel()] = x.reshape(-1, 3)
    return G, x


@pytest.mark.parametrize("p", [1, 2, 3])
def test_zjittered_box_quadratic_forms(p):
    """The z-jittered prism mesh still fills the unit cube, and x, y, z are in
    the discrete space, so u^T M u = int u^2 and u^T H u = int |grad u|^2 + u^2
    hold exactly (u = 1, x, z); grad z = e_z needs the per-point inverse."""
    n = 2
    coords, V, cells, dofs, N = zjittered_box(n, p)
    G, x = node_positions_pointgeo(p, coords, dofs, N)
    assert np.abs(G[dofs] - x).max() < 1e-14        # shared nodes coincide
    row_ptr, cols = oracle.csr_pattern(dofs, N)
    rows = np.repeat(np.arange(N), np.diff(row_ptr))
    Am, fm = oracle.assemble_pointgeo("mass", p, coords)
    Ah, fh = oracle.assemble_pointgeo("helmholtz", p, coords)
    assert fm == 0 and fh == 0
    vm = oracle.csr_insert(dofs, N, row_ptr, cols, Am)
    vh = oracle.csr_insert(dofs, N, row_ptr, cols, Ah)
    for u, uu, gg in ((np.ones(N), 1.0, 0.0), (G[:, 0], 1 / 3, 1.0), (G[:, 2], 1 / 3, 1.0)):
        qm = float(np.sum(u[rows] * vm * u[cols]))
        qh = float(np.sum(u[rows] * vh * u[cols]))
        assert abs(qm - uu) < 1e-13, (qm, uu)
        assert abs(qh - (uu + gg)) < 1e-12, (qh, uu + gg)


@pytest.mark.parametrize("p", [1, 2])
def test_zjittered_elasticity_rigid_motions(p):
    n = 2
    coords, V, cells, dofs, N = zjittered_box(n, p)
    G, _ = node_positions_pointgeo(p, coords, dofs, N)
    vd = I.vector_dofs(dofs, N, 3)
    lame = I.lame_p1(V.shape[0], cells, 4)
    A, fl = oracle.assemble_pointgeo("elasticity", p, coords, lame)
    assert fl == 0
    row_ptr, cols = oracle.csr_pattern(vd, 3 * N)
    vals = oracle.csr_insert(vd, 3 * N, row_ptr, cols, A)
    rows = np.repeat(np.arange(3 * N), np.diff(row_ptr))
    scale = np.abs(vals).max()
    x, y, z = G[:, 0], G[:, 1], G[:, 2]
    zero = np.zeros(N)
    for U in (np.stack([-y, x, zero], 1), np.stack([zero, -z, y], 1), np.stack([z, zero, -x], 1)):
        u = U.T.ravel()
        r = np.bincount(rows, weights=vals * u[cols], minlength=3 * N)
        assert np.abs(r).max() < 1e-12 * scale


def test_inverted_prism_flagged():
    """A top vertex below the bottom face makes det J change sign inside the
    element: flagged, NaN block."""
    c = one_prism([0.5, 0.8, -0.3])
    A, fl = oracle.assemble_pointgeo("helmholtz", 2, c)
    assert fl == 1 and np.isnan(A).all()

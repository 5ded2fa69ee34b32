"""Pins of the oracle's curved triangles and tetrahedra (Sec. 2.2 takes F_K
affine; here F_K is the isoparametric P2 map through the element's six or
ten P2 nodes, and J, det J and J^{-1} are evaluated at every quadrature
point), against closed forms, exact integrals and invariants that do not
use the oracle's formulas."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import exact_rational as er
import oracle
from paper_1604_05872_amd import inputs as I

SIMPLICES = ["triangle", "tetrahedron"]


def lattice(cell, p):
    return I._node_multi_indices(cell, p).astype(float) / p


def straight_nodes(cell, v):
    """P2 nodes of the straight (affine) element with vertices v."""
    a = lattice(cell, 2)
    d = oracle.TDIM[cell]
    return v[0] + a @ (v[1:d + 1] - v[0])


@pytest.mark.parametrize("cell", SIMPLICES)
@pytest.mark.parametrize("p", [1, 2, 3])
def test_straight_p2_map_reduces_to_affine(cell, p):
    """With every edge node at its edge's midpoint the P2 map is the affine map."""
    x, V, cells, h = I.curved_mesh(cell, 3, 5, bend=0.0)
    coords = V[cells]
    nv = oracle.NVERT[cell]
    for form in ("mass", "helmholtz", "elasticity", "hyperelastic"):
        cf = None
        if form == "elasticity":
            cf = I.lame_p1(V.shape[0], cells, seed=6)
        elif form == "hyperelastic":
            cf = I.displacement_dofs(coords.shape[0], oracle.TDIM[cell], oracle.nbasis(cell, p), h, seed=7,
                                     rel=0.02)
        q = oracle.default_qdeg_curved(form, cell, p)
        A, fa = oracle.assemble(form, cell, p, coords, cf, qdeg=q)
        B, fb = oracle.assemble_curved(form, cell, p, x, cf, qdeg=q)
        assert fa == fb == 0
        assert np.abs(A - B).max() <= 1e-13 * np.abs(A).max(), form
        assert nv == oracle.NVERT[cell]


def _edge_nodes(cell):
    """(P2 lattice index of each edge-midpoint node, its two vertices)."""
    a = I._node_multi_indices(cell, 2)
    d = oracle.TDIM[cell]
    out = []
    for m, idx in enumerate(a):
        bary = np.concatenate([[2 - idx.sum()], idx])
        if bary.max() == 1:
            out.append((m, tuple(np.nonzero(bary)[0])))
    return out


@pytest.mark.parametrize("cell", SIMPLICES)
@pytest.mark.parametrize("p", [1, 2, 3])
def test_one_curved_edge_volume(cell, p):
    """Moving one edge node m (between vertices a, b) by w changes J by the
    rank-one term w (x) grad psi_m, so by the matrix determinant lemma
    det J = det J0 (1 + grad psi_m . J0^{-1} w), affine in X; with
    psi_m = 4 lambda_a lambda_b and int lambda = |K^|/(d+1) the volume is
    |det J0| (|K^| + (J0^{-1} w) . 4 |K^|/(d+1) (grad lambda_a + grad lambda_b)).
    The mass matrix sums to it (partition of unity)."""
    d = oracle.TDIM[cell]
    rng = np.random.default_rng(20 + p)
    v = np.eye(d + 1, d, -1) + rng.uniform(-0.1, 0.1, size=(d + 1, d))
    J0 = (v[1:] - v[0]).T
    Kref = oracle.REF_VOLUME[cell]
    grad_l = np.vstack([-np.ones(d), np.eye(d)])          # reference gradients of the barycentrics
    for m, (a, b) in _edge_nodes(cell):
        w = rng.uniform(-0.08, 0.08, size=d)
        x = straight_nodes(cell, v)
        x[m] += w
        vol = abs(np.linalg.det(J0)) * (Kref + np.linalg.solve(J0, w) @ (4 * Kref / (d + 1) * (grad_l[a] + grad_l[b])))
        M, fl = oracle.assemble_curved("mass", cell, p, x[None])
        assert fl == 0
        assert abs(M.sum() - vol) <= 1e-14 * vol


def _global_curved(cell, n, p, seed=8):
    """Curved mesh of the unit box, global numbering of the degree-p space and
    the positions of its nodes (the P2 map at the reference lattice nodes,
    evaluated with the exact-rational P2 basis)."""
    x2, V, cells, h = I.curved_mesh(cell, n, seed, bend=0.04)
    dofs, N = I.global_dofs(cell, p, cells, n)
    a = I._node_multi_indices(cell, p)
    P2 = np.array([[float(t) for t in er.eval_basis(cell, 2, tuple(Fr(int(c), p) for c in idx))] for idx in a])
    pos = np.einsum("nm,emd->end", P2, x2)                  # [E][n_s][d]
    G = np.full((N, oracle.TDIM[cell]), np.nan)
    G[dofs.ravel()] = pos.reshape(-1, oracle.TDIM[cell])
    assert np.abs(G[dofs] - pos).max() < 1e-13             # shared nodes coincide
    return x2, V, cells, dofs, N, G


def _assembled(form, cell, p, x2, dofs, N, cf=None):
    A, fl = oracle.assemble_curved(form, cell, p, x2, cf)
    assert fl == 0
    row_ptr, cols = oracle.csr_pattern(dofs, N)
    vals = oracle.csr_insert(dofs, N, row_ptr, cols, A)
    rows = np.repeat(np.arange(N), np.diff(row_ptr))
    return rows, cols, vals


def _qform(rows, cols, vals, u, w=None):
    w = u if w is None else w
    return float(np.sum(vals * u[rows] * w[cols]))


@pytest.mark.parametrize("cell,n", [("triangle", 3), ("tetrahedron", 2)])
@pytest.mark.parametrize("p", [2, 3])
def test_curved_box_quadratic_forms(cell, n, p):
    """The curved mesh still fills the unit box and the coordinates x, y (z)
    lie in the isoparametric space (p >= 2), so u^T M u = int u^2 and
    u^T H u = int |grad u|^2 + u^2 hold exactly for u = 1 and each
    coordinate (the default rule integrates u^2 det J exactly); grad x = e_x
    needs each point's own inverse."""
    x2, V, cells, dofs, N, G = _global_curved(cell, n, p)
    rm, cm, vm = _assembled("mass", cell, p, x2, dofs, N)
    rh, ch, vh = _assembled("helmholtz", cell, p, x2, dofs, N)
    one = np.ones(N)
    assert abs(_qform(rm, cm, vm, one) - 1.0) < 1e-13
    assert abs(_qform(rh, ch, vh, one) - 1.0) < 1e-13
    for c in range(oracle.TDIM[cell]):
        u = G[:, c]
        assert abs(_qform(rm, cm, vm, u) - 1.0 / 3.0) < 1e-13
        assert abs(_qform(rh, ch, vh, u) - 4.0 / 3.0) < 1e-13
        assert abs(_qform(rm, cm, vm, u, one) - 0.5) < 1e-13


@pytest.mark.parametrize("cell,n", [("triangle", 3), ("tetrahedron", 2)])
def test_curved_elasticity_rigid_modes(cell, n):
    """Rigid motions lie in the isoparametric P2 space and have zero strain:
    they span the kernel of the assembled elasticity matrix (any positive P1
    Lame fields), and the hyperelastic tangent at u = 0 has them too."""
    p = 2
    x2, V, cells, dofs, N, G = _global_curved(cell, n, p)
    d = oracle.TDIM[cell]
    cf = I.lame_p1(V.shape[0], cells, seed=9)
    vdofs = I.vector_dofs(dofs, N, d)
    r, c, v = _assembled("elasticity", cell, p, x2, vdofs, N * d, cf)
    modes = []
    for k in range(d):
        m = np.zeros(N * d)
        m[k * N:(k + 1) * N] = 1.0
        modes.append(m)
    for a in range(d):
        for b in range(a + 1, d):
            m = np.zeros(N * d)
            m[a * N:(a + 1) * N] = -G[:, b]
            m[b * N:(b + 1) * N] = G[:, a]
            modes.append(m)
    scale = np.abs(v).max()
    for m in modes:
        Am = np.bincount(r, weights=v * m[c], minlength=N * d)
        assert np.abs(Am).max() < 1e-12 * scale * np.abs(m).max()


@pytest.mark.parametrize("cell", SIMPLICES)
def test_inverted_curved_element_flagged(cell):
    """An edge node moved across the element turns det J negative somewhere:
    the element is flagged (NaN block, one count)."""
    d = oracle.TDIM[cell]
    v = np.vstack([np.zeros(d), np.eye(d)])
    x = np.stack([straight_nodes(cell, v)] * 3)
    m, (a, b) = _edge_nodes(cell)[0]
    x[1, m] -= 2.0 * (v[a] + v[b]) / 2 - 3.0 * np.ones(d) / (d + 1)   # far across the element
    A, fl = oracle.assemble_curved("helmholtz", cell, 2, x)
    assert fl == 1 and np.isnan(A[1]).all() and np.isfinite(A[[0, 2]]).all()

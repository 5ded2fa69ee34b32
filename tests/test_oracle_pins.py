"""Pins of the CPU oracle against facts that do not come from the oracle itself:
exact rational integration, closed forms, invariants, special cases and finite
differences.  CPU only."""
import itertools
from fractions import Fraction as Fr

import numpy as np
import pytest

import exact_rational as er
import oracle
from paper_1604_05872_amd import inputs

CELLS = ["triangle", "tetrahedron", "prism"]
REFV = {"triangle": [(0, 0), (1, 0), (0, 1)],
        "tetrahedron": [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)],
        "prism": [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1)]}
# rational affine images (prisms: the top face is the bottom face translated)
IMAGES = {
    "triangle": [[(Fr(1, 3), Fr(1, 5)), (Fr(2), Fr(1, 2)), (Fr(1, 2), Fr(3, 2))],
                 [(Fr(0), Fr(0)), (Fr(-1, 4), Fr(3, 2)), (Fr(2, 3), Fr(1, 3))]],
    "tetrahedron": [[(0, 0, 0), (1, Fr(1, 3), 0), (Fr(1, 4), 1, Fr(1, 5)), (Fr(1, 7), Fr(1, 3), 1)],
                    [(Fr(1, 2), 0, 0), (0, 1, 0), (1, 1, Fr(1, 2)), (Fr(1, 3), Fr(1, 3), Fr(-2, 3))]],
    "prism": [],
}
_pb = [(0, 0, 0), (1, Fr(1, 4), 0), (Fr(1, 3), 1, Fr(1, 6))]
_pt = (Fr(1, 5), Fr(1, 7), Fr(2, 3))
IMAGES["prism"].append(_pb + [tuple(a + b for a, b in zip(v, _pt)) for v in _pb])


def normwise(A, B):
    return float(np.max(np.abs(np.asarray(A, float) - np.asarray(B, float))) / np.max(np.abs(np.asarray(B, float))))


def fverts(v):
    return np.array([[float(c) for c in row] for row in v])


def monomials(cell, D):
    if cell == "triangle":
        return [(a, b) for a in range(D + 1) for b in range(D + 1 - a)]
    if cell == "tetrahedron":
        return [(a, b, c) for a in range(D + 1) for b in range(D + 1 - a) for c in range(D + 1 - a - b)]
    return [(a, b, c) for (a, b) in monomials("triangle", D) for c in range(D + 1)]


# --------------------------------------------------------------------------
# Quadrature (exactness to the stated degree, and not beyond)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("qdeg", list(range(1, 12)))
def test_rule_exact_to_degree(cell, qdeg):
    X, W = oracle.rule(cell, qdeg)
    assert abs(W.sum() - oracle.REF_VOLUME[cell]) < 1e-15
    assert np.all(W > 0)
    for e in monomials(cell, qdeg):
        approx = float(np.sum(W * np.prod(X ** np.array(e), axis=1)))
        exact = float(er.integrate(cell, e))
        assert abs(approx - exact) <= 2e-16 + 1e-14 * exact, (e, approx, exact)


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("qdeg", list(range(1, 12)))
def test_rule_not_exact_beyond(cell, qdeg):
    X, W = oracle.rule(cell, qdeg)
    if cell in ("triangle", "prism") and qdeg <= 2:
        e = (3, 0) if cell == "triangle" else (3, 0, 0)       # 3-point rule: degree 2 only
    else:
        m = (qdeg + 2) // 2
        e = (0, 2 * m) if cell == "triangle" else (0, 0, 2 * m)
    approx = float(np.sum(W * np.prod(X ** np.array(e), axis=1)))
    exact = float(er.integrate(cell, e))
    assert abs(approx - exact) > 1e-8 * exact


# --------------------------------------------------------------------------
# Basis
# --------------------------------------------------------------------------

@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_basis_kronecker_pou_reproduction(cell, p):
    nd = np.array([[float(c) for c in x] for x in er.nodes(cell, p)])
    phi, dphi = oracle.basis(cell, p, nd)
    assert np.max(np.abs(phi - np.eye(len(nd)))) < 1e-13
    rng = np.random.default_rng(7)
    pts = rng.dirichlet(np.ones(4 if cell == "tetrahedron" else 3), size=20)[:, 1:]
    if cell == "prism":
        pts = np.concatenate([rng.dirichlet(np.ones(3), size=20)[:, 1:], rng.uniform(0, 1, (20, 1))], axis=1)
    phi, dphi = oracle.basis(cell, p, pts)
    assert np.max(np.abs(phi.sum(axis=1) - 1)) < 1e-13
    assert np.max(np.abs(dphi.sum(axis=1))) < 1e-11
    for e in er.exponents(cell, p):
        e = np.array(e)
        nodal = np.prod(nd ** e, axis=1)
        val = phi @ nodal
        assert np.max(np.abs(val - np.prod(pts ** e, axis=1))) < 1e-12
        for a in range(len(e)):
            ea = e.copy()
            ea[a] -= 1
            dex = e[a] * np.prod(pts ** np.maximum(ea, 0), axis=1) if e[a] > 0 else 0 * val
            assert np.max(np.abs(dphi[:, :, a] @ nodal - dex)) < 1e-10


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_basis_matches_exact_vandermonde(cell, p):
    rng = np.random.default_rng(p)
    for _ in range(3):
        x = rng.uniform(0, 0.3, size=er.TDIM[cell])
        exact = er.eval_basis(cell, p, tuple(Fr(float(c)) for c in x))
        phi, _ = oracle.basis(cell, p, x[None])
        assert np.max(np.abs(phi[0] - np.array([float(v) for v in exact]))) < 1e-14


def test_geometry_against_linear_algebra():
    rng = np.random.default_rng(3)
    for cell in ["triangle", "tetrahedron"]:
        d = 2 if cell == "triangle" else 3
        for _ in range(20):
            v = rng.normal(size=(d + 1, d))
            J, det, K, bad = oracle.geometry(cell, v)
            Jr = (v[1:] - v[0]).T
            assert not bad
            assert np.allclose(J, Jr, atol=1e-15)
            assert abs(det - np.linalg.det(Jr)) < 1e-13 * abs(np.linalg.det(Jr)) + 1e-15
            assert np.allclose(K, np.linalg.inv(Jr), rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------
# Closed forms
# --------------------------------------------------------------------------

def test_mass_p1_triangle_closed_form():
    """P1 triangle mass = |T|/12 [[2,1,1],[1,2,1],[1,1,2]] on the 4096-element
    jittered 32x64 grid; |T| from the shoelace formula."""
    coords = inputs.mass_tri_workload(seed=1)
    assert coords.shape == (4096, 3, 2)
    A, flagged = oracle.assemble("mass", "triangle", 1, coords, qdeg=2)
    assert flagged == 0
    x, y = coords[..., 0], coords[..., 1]
    area = 0.5 * np.abs((x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0]))
    ref = area[:, None, None] / 12.0 * (np.ones((3, 3)) + np.eye(3))
    err = np.max(np.abs(A - ref), axis=(1, 2)) / np.max(np.abs(ref), axis=(1, 2))
    assert err.max() < 1e-14


def test_mass_p1_tet_closed_form():
    coords, _, _ = inputs.tet_workload(4, seed=2)
    A, _ = oracle.assemble("mass", "tetrahedron", 1, coords)
    e = coords[:, 1:] - coords[:, :1]
    vol = np.abs(np.linalg.det(e)) / 6.0
    ref = vol[:, None, None] / 20.0 * (np.ones((4, 4)) + np.eye(4))
    assert np.max(np.abs(A - ref)) / np.max(ref) < 1e-14


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_mass_and_helmholtz_exact_rational(cell, p):
    for verts in [REFV[cell]] + IMAGES[cell]:
        v = fverts(verts)
        Am, _ = oracle.assemble("mass", cell, p, v[None])
        Ah, _ = oracle.assemble("helmholtz", cell, p, v[None])
        assert normwise(Am[0], er.mass(cell, p, verts)) < 1e-14
        assert normwise(Ah[0], er.helmholtz(cell, p, verts)) < 1e-14


COEF_EXACT = [("triangle", 1, 3), ("triangle", 2, 2), ("triangle", 3, 1), ("tetrahedron", 1, 3),
              ("tetrahedron", 2, 2), ("prism", 1, 2)]


@pytest.mark.parametrize("cell,p,nfmax", COEF_EXACT)
def test_coefficient_fields_exact_rational(cell, p, nfmax):
    """Mass and Helmholtz pre-multiplied by nf coefficient functions of degree
    p (Sec. 7.1): exact integrals of the polynomial weight prod_i f_i."""
    ns = oracle.nbasis(cell, p)
    rng = np.random.default_rng(100 + p)
    verts = IMAGES[cell][0]
    v = fverts(verts)
    for nf in range(1, nfmax + 1):
        fields = [[Fr(int(rng.integers(-3, 6)), int(rng.integers(1, 4))) for _ in range(ns)] for _ in range(nf)]
        cf = np.array([[float(x) for x in f] for f in fields])[None]
        Am, _ = oracle.assemble("mass", cell, p, v[None], cf, nf=nf)
        Ah, _ = oracle.assemble("helmholtz", cell, p, v[None], cf, nf=nf)
        assert normwise(Am[0], er.weighted_mass(cell, p, verts, fields)) < 1e-13
        assert normwise(Ah[0], er.weighted_helmholtz(cell, p, verts, fields)) < 1e-13


def test_coefficient_fields_invariants():
    """Constant fields scale the form by the product of the constants, and a
    field's DOFs enter linearly and symmetrically in the field order."""
    coords = inputs.tet_workload(2, seed=5)[0][:10]
    rng = np.random.default_rng(3)
    for p in (1, 2, 3):
        ns = oracle.nbasis("tetrahedron", p)
        H0, _ = oracle.assemble("helmholtz", "tetrahedron", p, coords)
        const = np.stack([np.full((10, ns), 1.5), np.full((10, ns), -0.5)], axis=1)
        H2, _ = oracle.assemble("helmholtz", "tetrahedron", p, coords, const, nf=2)
        assert np.max(np.abs(H2 + 0.75 * H0)) < 1e-13 * np.max(np.abs(H0))
        f = rng.uniform(0.5, 2.0, size=(10, 2, ns))
        A, _ = oracle.assemble("mass", "tetrahedron", p, coords, f, nf=2)
        B, _ = oracle.assemble("mass", "tetrahedron", p, coords, f[:, ::-1].copy(), nf=2)
        assert np.max(np.abs(A - B)) < 1e-13 * np.max(np.abs(A))
        g = f.copy()
        g[:, 0] *= 3.0
        C, _ = oracle.assemble("mass", "tetrahedron", p, coords, g, nf=2)
        assert np.max(np.abs(C - 3.0 * A)) < 1e-13 * np.max(np.abs(A))


@pytest.mark.parametrize("cell", CELLS)
def test_helmholtz_invariants(cell):
    rng = np.random.default_rng(11)
    d = oracle.TDIM[cell]
    if cell == "prism":
        coords, _, _, _ = inputs.first_elements("prism", 12, seed=3)
    elif cell == "tetrahedron":
        coords = inputs.tet_workload(2, seed=3)[0][:12]
    else:
        coords = inputs.mass_tri_workload(seed=3)[:12]
    for p in [1, 2, 3]:
        M, _ = oracle.assemble("mass", cell, p, coords)
        H, _ = oracle.assemble("helmholtz", cell, p, coords)
        S = H - M
        sc = np.max(np.abs(S), axis=(1, 2))
        assert np.max(np.abs(H - H.transpose(0, 2, 1))) < 1e-15 * np.max(np.abs(H))
        assert np.max(np.abs(S.sum(axis=2)) / sc[:, None]) < 1e-12       # constants in the kernel
        vol = M.sum(axis=(1, 2))
        J = coords[:, 1:d + 1] - coords[:, :1]
        ref_vol = np.abs(np.linalg.det(J)) * oracle.REF_VOLUME[cell]
        assert np.max(np.abs(vol - ref_vol) / ref_vol) < 1e-13
        assert np.max(np.abs(H.sum(axis=2) - M.sum(axis=2)) / sc[:, None]) < 1e-12
        # rigid motion: translation + rotation leaves H unchanged
        Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
        moved = coords @ Q.T + rng.normal(size=d)
        H2, _ = oracle.assemble("helmholtz", cell, p, moved)
        assert np.max(np.abs(H2 - H)) < 1e-12 * np.max(np.abs(H))
        # scaling: mass ~ s^d, stiffness ~ s^(d-2)
        s = 1.7
        M3, _ = oracle.assemble("mass", cell, p, coords * s)
        H3, _ = oracle.assemble("helmholtz", cell, p, coords * s)
        assert np.max(np.abs(M3 - s ** d * M)) < 1e-12 * np.max(M3)
        assert np.max(np.abs((H3 - M3) - s ** (d - 2) * S)) < 1e-12 * np.max(np.abs(S))


# --------------------------------------------------------------------------
# Elasticity
# --------------------------------------------------------------------------

ELAS_EXACT = [("triangle", 1), ("triangle", 2), ("triangle", 3), ("tetrahedron", 1),
              ("tetrahedron", 2), ("prism", 1), ("prism", 2)]


@pytest.mark.parametrize("cell,p", ELAS_EXACT)
def test_elasticity_exact_rational(cell, p):
    nv = oracle.NVERT[cell]
    lam = [Fr(1 + i, 3) for i in range(nv)]
    mu = [Fr(2 + 2 * i, 5) for i in range(nv)]
    for verts in [REFV[cell]] + IMAGES[cell]:
        v = fverts(verts)
        cf = np.array([[float(x) for x in lam], [float(x) for x in mu]])[None]
        A, _ = oracle.assemble("elasticity", cell, p, v[None], cf)
        assert normwise(A[0], er.elasticity(cell, p, verts, lam, mu)) < 1e-14


def _node_coords(cell, p, v):
    nd = np.array([[float(c) for c in x] for x in er.nodes(cell, p)])
    d = oracle.TDIM[cell]
    J = (v[1:d + 1] - v[0]).T
    return v[0] + nd @ J.T


def _rigid_modes(cell, p, v):
    d = oracle.TDIM[cell]
    x = _node_coords(cell, p, v)
    ns = x.shape[0]
    modes = []
    for c in range(d):
        m = np.zeros(d * ns)
        m[c * ns:(c + 1) * ns] = 1.0
        modes.append(m)
    rots = [(0, 1)] if d == 2 else [(0, 1), (1, 2), (0, 2)]
    for a, b in rots:
        m = np.zeros(d * ns)
        m[a * ns:(a + 1) * ns] = -x[:, b]
        m[b * ns:(b + 1) * ns] = x[:, a]
        modes.append(m)
    return modes


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("p", [1, 2, 3])
def test_elasticity_invariants(cell, p):
    rng = np.random.default_rng(5 + p)
    if cell == "prism":
        coords = inputs.first_elements("prism", 6, seed=4)[0]
    elif cell == "tetrahedron":
        coords = inputs.tet_workload(2, seed=4)[0][:6]
    else:
        coords = inputs.mass_tri_workload(seed=4)[:6]
    nv = oracle.NVERT[cell]
    cf = rng.uniform(0.5, 2.0, size=(coords.shape[0], 2, nv))
    A, flagged = oracle.assemble("elasticity", cell, p, coords, cf)
    assert flagged == 0
    for e in range(coords.shape[0]):
        Ae = A[e]
        nrm = np.max(np.abs(Ae))
        assert np.max(np.abs(Ae - Ae.T)) < 1e-15 * nrm
        assert np.linalg.eigvalsh(Ae).min() > -1e-12 * nrm
        for m in _rigid_modes(cell, p, coords[e]):
            assert np.max(np.abs(Ae @ m)) < 1e-11 * nrm * np.max(np.abs(m))
    # the kernel is exactly the rigid modes: rank = n - #modes
    nmodes = 3 if cell == "triangle" else 6
    ev = np.linalg.eigvalsh(A[0])
    assert np.sum(ev > 1e-9 * ev.max()) == A.shape[1] - nmodes


def _textbook_p1(d, v, lam, mu):
    """|T| B^T C B in Voigt notation, re-ordered to component-blocked DOFs."""
    n = d + 1
    M = np.ones((n, n))
    M[:, 1:] = v
    grads = np.linalg.inv(M)[1:, :].T       # rows: grad of the i-th barycentric
    vol = abs(np.linalg.det(M)) / (2 if d == 2 else 6)
    if d == 2:
        B = np.zeros((3, 2 * n))
        for i in range(n):
            bx, by = grads[i]
            B[:, 2 * i:2 * i + 2] = [[bx, 0], [0, by], [by, bx]]
        C = np.array([[lam + 2 * mu, lam, 0], [lam, lam + 2 * mu, 0], [0, 0, mu]])
    else:
        B = np.zeros((6, 3 * n))
        for i in range(n):
            bx, by, bz = grads[i]
            B[:, 3 * i:3 * i + 3] = [[bx, 0, 0], [0, by, 0], [0, 0, bz],
                                     [0, bz, by], [bz, 0, bx], [by, bx, 0]]
        C = lam * np.zeros((6, 6))
        C[:3, :3] = lam
        C[np.arange(3), np.arange(3)] += 2 * mu
        C[np.arange(3, 6), np.arange(3, 6)] = mu
    K = vol * B.T @ C @ B                  # node-interleaved (i, c)
    perm = [i * d + c for c in range(d) for i in range(n)]
    return K[np.ix_(perm, perm)]


@pytest.mark.parametrize("cell", ["triangle", "tetrahedron"])
def test_elasticity_p1_textbook(cell):
    d = oracle.TDIM[cell]
    rng = np.random.default_rng(9)
    for _ in range(5):
        v = rng.normal(size=(d + 1, d))
        lam, mu = 1.3, 0.7
        cf = np.array([[lam] * (d + 1), [mu] * (d + 1)])[None]
        A, _ = oracle.assemble("elasticity", cell, 1, v[None], cf)
        ref = _textbook_p1(d, v, lam, mu)
        assert normwise(A[0], ref) < 1e-13


# --------------------------------------------------------------------------
# Hyperelastic (neo-Hookean tangent)
# --------------------------------------------------------------------------

def _hyper_case(cell, p, seed=0, scale=0.05):
    if cell == "prism":
        coords, _, _, h = inputs.first_elements("prism", 3, seed=seed + 1)
    elif cell == "tetrahedron":
        coords = inputs.tet_workload(2, seed=seed + 1)[0][:3]
        h = 0.5
    else:
        coords = inputs.mass_tri_workload(seed=seed + 1)[:3]
        h = 1.0 / 64
    ns = oracle.nbasis(cell, p)
    d = oracle.TDIM[cell]
    u = inputs.displacement_dofs(coords.shape[0], d, ns, h, seed=seed + 2, rel=scale / p)
    return coords, u


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("p", [1, 2, 3])
def test_hyper_at_zero_is_elasticity(cell, p):
    coords, u = _hyper_case(cell, p)
    nv = oracle.NVERT[cell]
    A, _ = oracle.assemble("hyperelastic", cell, p, coords, np.zeros_like(u), qdeg=4, mu=1.0, lam=10.0)
    cf = np.tile(np.array([[10.0] * nv, [1.0] * nv]), (coords.shape[0], 1, 1))
    B, _ = oracle.assemble("elasticity", cell, p, coords, cf, qdeg=4)
    assert normwise(A, B) < 1e-13


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("p", [1, 2])
def test_hyper_tangent_is_residual_derivative(cell, p):
    coords, u = _hyper_case(cell, p, scale=0.08)
    assert oracle.hyper_min_jf(cell, p, coords, u).min() > 0.2
    A, flagged = oracle.assemble("hyperelastic", cell, p, coords, u, qdeg=4)
    assert flagged == 0
    rng = np.random.default_rng(1)
    delta = rng.normal(size=u.shape) * np.max(np.abs(u))
    errs = []
    for eps in (1e-3, 5e-4):
        Rp, _ = oracle.hyper_residual(cell, p, coords, u + eps * delta)
        Rm, _ = oracle.hyper_residual(cell, p, coords, u - eps * delta)
        fd = (Rp - Rm) / (2 * eps)
        Ad = np.einsum("eij,ej->ei", A, delta)
        errs.append(np.max(np.abs(Ad - fd)) / np.max(np.abs(Ad)))
    assert errs[0] < 1e-4
    assert errs[1] < errs[0] / 3.5 or errs[1] < 1e-10      # second-order convergence


@pytest.mark.parametrize("cell", CELLS)
def test_hyper_residual_is_energy_gradient(cell):
    coords, u = _hyper_case(cell, 2, scale=0.08)
    R, _ = oracle.hyper_residual(cell, 2, coords, u)
    rng = np.random.default_rng(2)
    delta = rng.normal(size=u.shape) * np.max(np.abs(u))
    eps = 1e-4
    _, Ep = oracle.hyper_residual(cell, 2, coords, u + eps * delta)
    _, Em = oracle.hyper_residual(cell, 2, coords, u - eps * delta)
    fd = (Ep - Em) / (2 * eps)
    Rd = np.einsum("ei,ei->e", R, delta)
    assert np.max(np.abs(Rd - fd)) / np.max(np.abs(Rd)) < 1e-6


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("p", [1, 2])
def test_hyper_symmetry_and_translations(cell, p):
    coords, u = _hyper_case(cell, p, scale=0.08)
    A, _ = oracle.assemble("hyperelastic", cell, p, coords, u)
    d = oracle.TDIM[cell]
    ns = oracle.nbasis(cell, p)
    for Ae in A:
        nrm = np.max(np.abs(Ae))
        assert np.max(np.abs(Ae - Ae.T)) < 1e-13 * nrm
        for c in range(d):
            t = np.zeros(d * ns)
            t[c * ns:(c + 1) * ns] = 1
            assert np.max(np.abs(Ae @ t)) < 1e-11 * nrm


@pytest.mark.parametrize("cell", CELLS)
def test_hyper_p1_is_single_point(cell):
    if cell == "prism":
        pytest.skip("P1 x P1 gradients vary on a prism")
    coords, u = _hyper_case(cell, 1, scale=0.08)
    A4, _ = oracle.assemble("hyperelastic", cell, 1, coords, u, qdeg=4)
    A1, _ = oracle.assemble("hyperelastic", cell, 1, coords, u, qdeg=1)
    assert normwise(A4, A1) < 1e-13


# --------------------------------------------------------------------------
# Flagged elements
# --------------------------------------------------------------------------

def test_degenerate_and_nonaffine_flagged():
    v = np.array([[0, 0, 0], [1, 0, 0], [1, 0, 0], [0, 0, 1.0]])
    A, f = oracle.assemble("helmholtz", "tetrahedron", 2, v[None])
    assert f == 1 and np.isnan(A).all()
    pr = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1.1], [0, 1, 1.0]])
    A, f = oracle.assemble("mass", "prism", 1, pr[None])
    assert f == 1 and np.isnan(A).all()
    ref = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    u = np.zeros((2, 12))
    u[1, 1] = -2.0                      # u_x = -2 X on the second element: F_xx = -1
    A, f = oracle.assemble("hyperelastic", "tetrahedron", 1, np.stack([ref, ref]), u)
    assert f == 1 and np.isnan(A[1]).all() and np.isfinite(A[0]).all()


# --------------------------------------------------------------------------
# Seeded inputs
# --------------------------------------------------------------------------

def test_meshes_positive_and_counts():
    c1 = inputs.mass_tri_workload(seed=1)
    x, y = c1[..., 0], c1[..., 1]
    det = (x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0])
    assert c1.shape[0] == 4096 and det.min() > 0.19 * (1 / 32) * (1 / 64)
    c2, V, cells = inputs.tet_workload(10, seed=2)
    assert c2.shape == (6000, 4, 3)
    e = c2[:, 1:] - c2[:, :1]
    dets = np.abs(np.linalg.det(e))
    assert dets.min() > 0.09 * (0.1 ** 3)
    assert abs(dets.sum() / 6 - 1.0) < 1e-12           # the tets tile the unit cube
    pr, _, _, _ = inputs.first_elements("prism", 1000, seed=5)
    J, det, K, bad = oracle.geometry("prism", pr[17])
    assert not bad


@pytest.mark.parametrize("p", [1, 2])
def test_hyperelastic_workload_jf(p):
    """The seeded 55^3 x 6 hyperelastic workload, displacement N(0, (0.05 h)^2)
    per DOF: P1 never inverts; P2 inverts at some quadrature point in exactly
    4,060 of 998,250 elements (0.41%; these take the flagged NaN path on both
    sides), and no element has min J_F within 1e-9 of the J_F = 0 decision
    (float64 rounding of J_F is ~1e-15), so both sides flag the same set."""
    coords, V, cells = inputs.tet_workload(55, seed=4)
    ns = oracle.nbasis("tetrahedron", p)
    u = inputs.displacement_dofs(coords.shape[0], 3, ns, 1.0 / 55, seed=40 + p)
    m = oracle.hyper_min_jf("tetrahedron", p, coords, u)
    assert np.sum(m <= 0) == (0 if p == 1 else 4060)
    assert np.min(np.abs(m)) > 1e-9

"""Pins of the oracle's generic bilinear forms, scalar and vector-valued (the
multilinear operands of sharing elimination, Sec. 3.2), against exact
rational integration on affine elements with rational vertices."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import exact_rational as er
import oracle
from test_oracle_pins import IMAGES, fverts

SYM = {"value": 0, "dx": 1, "dy": 2, "dz": 3}


def _lin(dicts_coeffs):
    out = {}
    for d, c in dicts_coeffs:
        for e, v in d.items():
            out[e] = out.get(e, 0) + c * v
    return out


def symbol_polys(cell, p, K, sym):
    """Polynomial dicts of symbol `sym` of every basis function on the
    reference cell (a physical derivative is K-weighted reference ones)."""
    ex, C = er.lagrange(cell, p)
    if sym == 0:
        return er._val_coeffs(ex, C)
    b = sym - 1
    d = er.TDIM[cell]
    D = [er._deriv_coeffs(ex, C, a) for a in range(d)]
    return [_lin([(D[a][j], K[a][b]) for a in range(d)]) for j in range(len(ex))]


def spec_exact(cell, p, verts, terms, field_vals=None):
    _, adet, K = er.affine(cell, verts)
    n = len(er.lagrange(cell, p)[0])
    A = [[Fr(0)] * n for _ in range(n)]
    psi = er._p1_weights(cell)
    for (ts, rs, f, sc) in terms:
        P = symbol_polys(cell, p, K, SYM[ts])
        Q = symbol_polys(cell, p, K, SYM[rs])
        w = None
        if f >= 0:
            w = _lin([(psi[l], field_vals[f][l]) for l in range(len(psi))])
        B = er._bilinear(cell, P, Q, weight=w)
        for j in range(n):
            for k in range(n):
                A[j][k] += adet * Fr(sc) * B[j][k]
    return np.array([[float(x) for x in r] for r in A])


def rel(A, B):
    return np.abs(A - B).max() / np.abs(B).max()


FORMS = {
    "advection": [("value", "dx", -1, Fr(5, 2)), ("value", "dy", -1, Fr(-1))],
    "anisotropic": [("dx", "dx", -1, Fr(2)), ("dx", "dy", -1, Fr(7, 10)), ("dy", "dx", -1, Fr(7, 10)),
                    ("dy", "dy", -1, Fr(1, 2))],
    "transport_reaction": [("dx", "value", -1, Fr(3, 4)), ("value", "value", -1, Fr(1, 3))],
}


@pytest.mark.parametrize("cell,p", [("triangle", 1), ("triangle", 2), ("triangle", 3), ("tetrahedron", 1),
                                    ("tetrahedron", 2), ("tetrahedron", 3), ("prism", 1), ("prism", 2)])
@pytest.mark.parametrize("name", sorted(FORMS))
def test_spec_constant_terms_exact(cell, p, name):
    verts = IMAGES[cell][0]
    terms = FORMS[name]
    if cell != "triangle":
        terms = terms + [("dz", "value", -1, Fr(-2, 3))]
    A, fl = oracle.assemble_spec([(t[0], t[1], t[2], float(t[3])) for t in terms], cell, p, fverts(verts)[None])
    assert fl == 0
    assert rel(A[0], spec_exact(cell, p, verts, terms)) < 1e-13


@pytest.mark.parametrize("cell", ["triangle", "tetrahedron", "prism"])
@pytest.mark.parametrize("p", [1, 2])
def test_spec_field_terms_exact(cell, p):
    """P1 coefficient fields (Eq. (7)'s coefficient factor) on value and
    derivative symbols."""
    verts = IMAGES[cell][1 if len(IMAGES[cell]) > 1 else 0]
    nv = {"triangle": 3, "tetrahedron": 4, "prism": 6}[cell]
    rng = np.random.default_rng(7)
    fv = [[Fr(int(rng.integers(1, 9)), int(rng.integers(1, 5))) for _ in range(nv)] for _ in range(2)]
    terms = [("value", "value", 0, Fr(1)), ("dx", "dy", 1, Fr(3, 2)), ("dy", "value", 0, Fr(-1, 2))]
    fields = np.array([[float(x) for x in f] for f in fv])[None]
    A, fl = oracle.assemble_spec([(t[0], t[1], t[2], float(t[3])) for t in terms], cell, p, fverts(verts)[None],
                                 fields)
    assert fl == 0
    assert rel(A[0], spec_exact(cell, p, verts, terms, fv)) < 1e-13


@pytest.mark.parametrize("cell", ["triangle", "tetrahedron"])
def test_spec_swapping_test_and_trial_transposes(cell):
    c = fverts(IMAGES[cell][0])[None]
    terms = [("value", "dx", -1, 1.5), ("dy", "value", -1, -0.5), ("dx", "dy", -1, 2.0)]
    swapped = [(t[1], t[0], t[2], t[3]) for t in terms]
    A, _ = oracle.assemble_spec(terms, cell, 2, c)
    B, _ = oracle.assemble_spec(swapped, cell, 2, c)
    assert rel(A[0], B[0].T) < 1e-14
    assert rel(A[0], A[0].T) > 1e-3     # genuinely non-symmetric


# --------------------------------------------------------------------------
# Vector-valued spaces: basis functions phi_j e_c, component-blocked
# (row c * n_s + j); each term couples one test and one trial component.

def vspec_exact(cell, p, verts, terms, n_comp, field_vals=None):
    """Every (test component, trial component) block is the scalar form of
    the terms that couple those components, integrated exactly."""
    ns = len(er.lagrange(cell, p)[0])
    A = np.zeros((n_comp * ns, n_comp * ns))
    for a in range(n_comp):
        for b in range(n_comp):
            sub = [t[:4] for t in terms if t[4] == a and t[5] == b]
            if sub:
                A[a * ns:(a + 1) * ns, b * ns:(b + 1) * ns] = spec_exact(cell, p, verts, sub, field_vals)
    return A


def _random_vector_terms(cell, seed, n_terms=8):
    d = er.TDIM[cell]
    rng = np.random.default_rng(seed)
    names = ["value", "dx", "dy", "dz"][:d + 1]
    terms = [("dx", "dy", -1, Fr(3, 2), 0, 1), ("value", "dx", 0, Fr(-1, 3), 1, 0)]   # non-symmetric blocks
    while len(terms) < n_terms:
        terms.append((names[int(rng.integers(0, d + 1))], names[int(rng.integers(0, d + 1))],
                      int(rng.integers(-1, 2)), Fr(int(rng.integers(-7, 8)) or 1, int(rng.integers(1, 6))),
                      int(rng.integers(0, d)), int(rng.integers(0, d))))
    return terms


@pytest.mark.parametrize("cell,p", [("triangle", 1), ("triangle", 2), ("tetrahedron", 1), ("tetrahedron", 2),
                                    ("prism", 1)])
def test_vspec_blocks_exact(cell, p):
    verts = IMAGES[cell][0]
    d = er.TDIM[cell]
    nv = {"triangle": 3, "tetrahedron": 4, "prism": 6}[cell]
    rng = np.random.default_rng(11)
    fv = [[Fr(int(rng.integers(1, 9)), int(rng.integers(1, 5))) for _ in range(nv)] for _ in range(2)]
    terms = _random_vector_terms(cell, 5 + p)
    fields = np.array([[float(x) for x in f] for f in fv])[None]
    A, fl = oracle.assemble_vspec([(t[0], t[1], t[2], float(t[3]), t[4], t[5]) for t in terms], cell, p,
                                  fverts(verts)[None], fields)
    assert fl == 0 and A.shape == (1, d * len(er.lagrange(cell, p)[0]), d * len(er.lagrange(cell, p)[0]))
    assert rel(A[0], vspec_exact(cell, p, verts, terms, d, fv)) < 1e-13


@pytest.mark.parametrize("cell", ["triangle", "tetrahedron", "prism"])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_vspec_elasticity_is_the_elasticity_form(cell, p):
    """2 mu eps(u):eps(v) + lambda div u div v with P1 Lame fields, written as
    component terms: mu (grad v_a . grad u_a) on the diagonal blocks, mu
    d_b v_a d_a u_b and lambda d_a v_a d_b u_b on every block (a, b), equals
    the oracle's elasticity form (pinned by exact rationals and the P1
    textbook matrix)."""
    d = er.TDIM[cell]
    nv = {"triangle": 3, "tetrahedron": 4, "prism": 6}[cell]
    names = ["dx", "dy", "dz"]
    terms = []
    for a in range(d):
        for b in range(d):
            terms.append((names[b], names[b], 1, 1.0, a, a))
            terms.append((names[b], names[a], 1, 1.0, a, b))
            terms.append((names[a], names[b], 0, 1.0, a, b))
    rng = np.random.default_rng(3 + p)
    c = fverts(IMAGES[cell][0])[None]
    lm = rng.uniform(0.5, 2.0, size=(1, 2, nv))
    A, fl = oracle.assemble_vspec(terms, cell, p, c, lm)
    B, flb = oracle.assemble("elasticity", cell, p, c, lm.reshape(1, -1))
    assert fl == 0 and flb == 0
    assert rel(A[0], B[0]) < 1e-13


@pytest.mark.parametrize("cell", ["triangle", "tetrahedron"])
def test_vspec_one_component_is_the_scalar_form(cell):
    c = fverts(IMAGES[cell][1])[None]
    terms = [("value", "dx", -1, 1.5), ("dy", "value", 0, -0.5), ("dx", "dy", -1, 2.0)]
    fields = np.array([[[1.0, 2.0, 0.5, 3.0][:{"triangle": 3, "tetrahedron": 4}[cell]]]])
    A, _ = oracle.assemble_spec(terms, cell, 2, c, fields)
    B, _ = oracle.assemble_vspec([t + (0, 0) for t in terms], cell, 2, c, fields, n_comp=1)
    assert np.array_equal(A, B)

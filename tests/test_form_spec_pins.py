"""Pins of the oracle's generic scalar bilinear forms (the multilinear
operands of sharing elimination, Sec. 3.2) against exact rational
integration on affine elements with rational vertices."""
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

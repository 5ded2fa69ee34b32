"""Exact rational finite-element tables (test helper, pins the oracle).

Independent of both the oracle and the GPU library:
  * the Lagrange basis is built by inverting the monomial Vandermonde matrix
    over the rationals (not from Silvester's product formula);
  * integrals of monomials use the closed forms
        triangle     int X^a Y^b       = a! b! / (a+b+2)!
        tetrahedron  int X^a Y^b Z^c   = a! b! c! / (a+b+c+3)!
        prism        int X^a Y^b Z^c   = a! b! / (a+b+2)! * 1/(c+1)
so every value is exact.  Node order is the equispaced lattice with the first
index fastest (k, j, i loops), the prism node (t, l) at index l*n_tri + t.
"""
from __future__ import annotations

from fractions import Fraction as Fr
from functools import lru_cache
from math import factorial

CELLS = ("triangle", "tetrahedron", "prism")
TDIM = {"interval": 1, "triangle": 2, "tetrahedron": 3, "prism": 3}


def nodes(cell: str, p: int):
    out = []
    if cell == "interval":
        return [(Fr(l, p),) for l in range(p + 1)]
    if cell == "triangle":
        for j in range(p + 1):
            for i in range(p + 1 - j):
                out.append((Fr(i, p), Fr(j, p)))
    elif cell == "tetrahedron":
        for k in range(p + 1):
            for j in range(p + 1 - k):
                for i in range(p + 1 - j - k):
                    out.append((Fr(i, p), Fr(j, p), Fr(k, p)))
    else:
        tri = nodes("triangle", p)
        for l in range(p + 1):
            for (x, y) in tri:
                out.append((x, y, Fr(l, p)))
    return out


def exponents(cell: str, p: int):
    """Monomial exponents spanning the degree-p space of the cell."""
    if cell == "interval":
        return [(c,) for c in range(p + 1)]
    if cell == "triangle":
        return [(a, b) for a in range(p + 1) for b in range(p + 1 - a)]
    if cell == "tetrahedron":
        return [(a, b, c) for a in range(p + 1) for b in range(p + 1 - a) for c in range(p + 1 - a - b)]
    return [(a, b, c) for (a, b) in exponents("triangle", p) for c in range(p + 1)]


def mono(x, e):
    v = Fr(1)
    for xi, ei in zip(x, e):
        v *= xi ** ei
    return v


def integrate(cell: str, e) -> Fr:
    if cell == "interval":
        return Fr(1, e[0] + 1)
    if cell == "triangle":
        a, b = e
        return Fr(factorial(a) * factorial(b), factorial(a + b + 2))
    if cell == "tetrahedron":
        a, b, c = e
        return Fr(factorial(a) * factorial(b) * factorial(c), factorial(a + b + c + 3))
    a, b, c = e
    return Fr(factorial(a) * factorial(b), factorial(a + b + 2)) * Fr(1, c + 1)


def _solve(M, rhs_cols):
    """Gauss-Jordan over the rationals: returns M^{-1} applied to rhs columns."""
    n = len(M)
    A = [list(M[i]) + list(rhs_cols[i]) for i in range(n)]
    w = len(A[0])
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        inv = 1 / A[col][col]
        A[col] = [v * inv for v in A[col]]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [A[r][k] - f * A[col][k] for k in range(w)]
    return [row[n:] for row in A]


@lru_cache(maxsize=None)
def lagrange(cell: str, p: int):
    """Coefficient matrix C[m][j]: phi_j = sum_m C[m][j] X^{e_m}, from V C = I
    with V[i][m] = (node_i)^{e_m}."""
    ex = exponents(cell, p)
    nd = nodes(cell, p)
    V = [[mono(x, e) for e in ex] for x in nd]
    n = len(ex)
    I = [[Fr(int(i == j)) for j in range(n)] for i in range(n)]
    C = _solve(V, I)
    return ex, C


def eval_basis(cell: str, p: int, x):
    ex, C = lagrange(cell, p)
    mv = [mono(x, e) for e in ex]
    n = len(ex)
    return [sum(C[m][j] * mv[m] for m in range(n) if C[m][j] != 0) for j in range(n)]


def _deriv_coeffs(ex, C, a):
    """Coefficients (in a dict keyed by exponent) of d/dX_a of every basis function."""
    n = len(ex)
    out = []
    for j in range(n):
        d = {}
        for m, e in enumerate(ex):
            if C[m][j] == 0 or e[a] == 0:
                continue
            e2 = tuple(v - (1 if k == a else 0) for k, v in enumerate(e))
            d[e2] = d.get(e2, 0) + C[m][j] * e[a]
        out.append(d)
    return out


def _val_coeffs(ex, C):
    n = len(ex)
    return [{ex[m]: C[m][j] for m in range(n) if C[m][j] != 0} for j in range(n)]


def _bilinear(cell, P, Q, weight=None):
    """[j][k] -> int weight * P_j * Q_k for polynomial dicts."""
    out = []
    wt = weight or {tuple(0 for _ in range(TDIM[cell])): Fr(1)}
    cache = {}

    def I(e):
        if e not in cache:
            cache[e] = integrate(cell, e)
        return cache[e]

    # pre-multiply P by the weight
    PW = []
    for pj in P:
        d = {}
        for e1, c1 in pj.items():
            for e0, c0 in wt.items():
                e = tuple(x + y for x, y in zip(e1, e0))
                d[e] = d.get(e, 0) + c1 * c0
        PW.append(d)
    for pj in PW:
        row = []
        for qk in Q:
            s = Fr(0)
            for e1, c1 in pj.items():
                for e2, c2 in qk.items():
                    s += c1 * c2 * I(tuple(x + y for x, y in zip(e1, e2)))
            row.append(s)
        out.append(row)
    return out


@lru_cache(maxsize=None)
def reference_mass(cell: str, p: int, direct: bool = False):
    if cell == "prism" and not direct:
        Mt, M1 = reference_mass("triangle", p), reference_mass("interval", p)
        return _kron(M1, Mt)
    ex, C = lagrange(cell, p)
    V = _val_coeffs(ex, C)
    return _bilinear(cell, V, V)


def _kron(B1, Bt):
    """[(l,t)][(l',t')] = B1[l][l'] * Bt[t][t'] with index l*nt + t."""
    n1, nt = len(B1), len(Bt)
    return [[B1[i // nt][k // nt] * Bt[i % nt][k % nt] for k in range(n1 * nt)] for i in range(n1 * nt)]


@lru_cache(maxsize=None)
def _mixed(cell: str, p: int):
    """X[a][j][k] = int dphi_j/dX_a phi_k."""
    ex, C = lagrange(cell, p)
    V = _val_coeffs(ex, C)
    return [_bilinear(cell, _deriv_coeffs(ex, C, a), V) for a in range(TDIM[cell])]


@lru_cache(maxsize=None)
def reference_stiffness(cell: str, p: int, direct: bool = False):
    """K[a][b][j][k] = int dphi_j/dX_a dphi_k/dX_b over the reference cell.
    Prisms use the tensor-product factorisation triangle x interval."""
    if cell == "prism" and not direct:
        Mt, M1 = reference_mass("triangle", p), reference_mass("interval", p)
        Kt, K1 = reference_stiffness("triangle", p), reference_stiffness("interval", p)[0][0]
        Xt, X1 = _mixed("triangle", p), _mixed("interval", p)[0]
        X1T = [list(r) for r in zip(*X1)]
        K = [[None] * 3 for _ in range(3)]
        for a in range(2):
            for b in range(2):
                K[a][b] = _kron(M1, Kt[a][b])
            K[a][2] = _kron(X1T, Xt[a])
            K[2][a] = _kron(X1, [list(r) for r in zip(*Xt[a])])
        K[2][2] = _kron(K1, Mt)
        return K
    ex, C = lagrange(cell, p)
    d = TDIM[cell]
    D = [_deriv_coeffs(ex, C, a) for a in range(d)]
    return [[_bilinear(cell, D[a], D[b]) for b in range(d)] for a in range(d)]


def _p1_weights(cell: str):
    ex, C = lagrange(cell, 1)
    return _val_coeffs(ex, C)


@lru_cache(maxsize=None)
def reference_weighted_stiffness(cell: str, p: int):
    """T[l][a][b][j][k] = int psi_l dphi_j/dX_a dphi_k/dX_b, psi the P1 basis."""
    ex, C = lagrange(cell, p)
    d = TDIM[cell]
    D = [_deriv_coeffs(ex, C, a) for a in range(d)]
    return [[[_bilinear(cell, D[a], D[b], weight=w) for b in range(d)] for a in range(d)]
            for w in _p1_weights(cell)]


# ----------------------------------------------------------------------------
# Physical elements with rational vertices
# ----------------------------------------------------------------------------

def _mat_inv(J):
    n = len(J)
    I = [[Fr(int(i == j)) for j in range(n)] for i in range(n)]
    return _solve(J, I)


def _det(J):
    if len(J) == 2:
        return J[0][0] * J[1][1] - J[0][1] * J[1][0]
    return (J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
            - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
            + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]))


def affine(cell: str, verts):
    """J (columns = edge vectors from vertex 0), |det J|, K = J^{-1}."""
    d = TDIM[cell]
    v = [[Fr(c) for c in row] for row in verts]
    J = [[v[a + 1][r] - v[0][r] for a in range(d)] for r in range(d)]
    det = _det(J)
    return J, abs(det), _mat_inv(J)


def mass(cell, p, verts):
    _, adet, _ = affine(cell, verts)
    M = reference_mass(cell, p)
    return [[adet * x for x in row] for row in M]


def stiffness(cell, p, verts):
    d = TDIM[cell]
    _, adet, K = affine(cell, verts)
    G = [[sum(K[a][b] * K[c][b] for b in range(d)) for c in range(d)] for a in range(d)]
    Kr = reference_stiffness(cell, p)
    n = len(Kr[0][0])
    return [[adet * sum(G[a][b] * Kr[a][b][j][k] for a in range(d) for b in range(d))
             for k in range(n)] for j in range(n)]


def helmholtz(cell, p, verts):
    M = mass(cell, p, verts)
    S = stiffness(cell, p, verts)
    return [[M[j][k] + S[j][k] for k in range(len(M))] for j in range(len(M))]


def elasticity(cell, p, verts, lam_dofs, mu_dofs, fields=()):
    """Exact element matrix of int w (2 mu eps(u):eps(v) + lam div u div v)
    with P1 (prism: P1 x P1) Lame fields, from
        mu (delta_cd g_j.g_k + g_jd g_kc) + lam g_jc g_kd,  g = K^T grad_X,
    and w = prod_i f_i of degree-p functions with DOFs `fields` (w = 1 when
    there are none)."""
    d = TDIM[cell]
    _, adet, K = affine(cell, verts)
    if fields:
        ex, C = lagrange(cell, p)
        D = [_deriv_coeffs(ex, C, a) for a in range(d)]
        cw = coefficient_weight(cell, p, fields)
        T = [[[_bilinear(cell, D[a], D[b], weight=_poly_mul(w, cw)) for b in range(d)] for a in range(d)]
             for w in _p1_weights(cell)]
    else:
        T = reference_weighted_stiffness(cell, p)
    ns = len(T[0][0][0])
    lam = [Fr(x) for x in lam_dofs]
    mu = [Fr(x) for x in mu_dofs]
    # W[coef][a][b][j][k] = sum_l coef_l T[l][a][b][j][k]
    def wsum(cf):
        return [[[[sum(cf[l] * T[l][a][b][j][k] for l in range(len(T))) for k in range(ns)]
                  for j in range(ns)] for b in range(d)] for a in range(d)]
    WL, WM = wsum(lam), wsum(mu)
    n = d * ns
    A = [[Fr(0)] * n for _ in range(n)]
    for c in range(d):
        for e in range(d):
            for j in range(ns):
                for k in range(ns):
                    s = Fr(0)
                    for a in range(d):
                        for b in range(d):
                            s += WL[a][b][j][k] * K[a][c] * K[b][e]
                            s += WM[a][b][j][k] * K[a][e] * K[b][c]
                            if c == e:
                                s += WM[a][b][j][k] * sum(K[a][x] * K[b][x] for x in range(d))
                    A[c * ns + j][e * ns + k] = adet * s
    return A


# ----------------------------------------------------------------------------
# Forms pre-multiplied by coefficient functions (Sec. 7.1's nf)
# ----------------------------------------------------------------------------

def _poly_mul(P, Q):
    out = {}
    for e1, c1 in P.items():
        for e2, c2 in Q.items():
            e = tuple(x + y for x, y in zip(e1, e2))
            out[e] = out.get(e, 0) + c1 * c2
    return out


def coefficient_weight(cell: str, p: int, fields):
    """prod_i f_i as a polynomial dict, f_i = sum_l fields[i][l] phi_l (degree p)."""
    ex, C = lagrange(cell, p)
    V = _val_coeffs(ex, C)
    w = {tuple(0 for _ in range(TDIM[cell])): Fr(1)}
    for f in fields:
        fi = {}
        for l, dof in enumerate(f):
            for e, c in V[l].items():
                fi[e] = fi.get(e, 0) + Fr(dof) * c
        w = _poly_mul(w, fi)
    return w


def weighted_mass(cell, p, verts, fields):
    _, adet, _ = affine(cell, verts)
    ex, C = lagrange(cell, p)
    V = _val_coeffs(ex, C)
    M = _bilinear(cell, V, V, weight=coefficient_weight(cell, p, fields))
    return [[adet * x for x in row] for row in M]


def weighted_helmholtz(cell, p, verts, fields):
    d = TDIM[cell]
    _, adet, K = affine(cell, verts)
    ex, C = lagrange(cell, p)
    w = coefficient_weight(cell, p, fields)
    D = [_deriv_coeffs(ex, C, a) for a in range(d)]
    G = [[sum(K[a][b] * K[c][b] for b in range(d)) for c in range(d)] for a in range(d)]
    Kr = [[_bilinear(cell, D[a], D[b], weight=w) for b in range(d)] for a in range(d)]
    M = weighted_mass(cell, p, verts, fields)
    n = len(M)
    return [[M[j][k] + adet * sum(G[a][b] * Kr[a][b][j][k] for a in range(d) for b in range(d))
             for k in range(n)] for j in range(n)]

"""CPU oracle for finite-element local assembly (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never does, and shares no code with it.

The compiled part is ``fe_oracle.c`` (plain C, IEEE double, OpenMP over
elements); this module loads it with ctypes and offers numpy-facing helpers.
It evaluates Eq. (7) of the paper (quadrature mode, Sec. 2.2) as the naive
loop nest of Fig. 1, and the global assembly of Sec. 2 (element matrices summed
into the compressed-row matrix of the continuous space, in element order).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fe_oracle.c")
_LIB = os.environ.get("FE_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

CELL = {"triangle": 0, "tetrahedron": 1, "prism": 2}
FORM = {"mass": 0, "helmholtz": 1, "elasticity": 2, "hyperelastic": 3}
TDIM = {"triangle": 2, "tetrahedron": 3, "prism": 3}
NVERT = {"triangle": 3, "tetrahedron": 4, "prism": 6}
REF_VOLUME = {"triangle": 0.5, "tetrahedron": 1.0 / 6.0, "prism": 0.5}


def build(force: bool = False, out: str | None = None, defines=(), flags=()) -> str:
    """Compile the oracle with gcc (portable flags: it runs on other hosts);
    `flags` adds compiler options (e.g. sanitizers for a test build)."""
    target = out or _LIB
    if force or not os.path.exists(target) or os.path.getmtime(target) < os.path.getmtime(_SRC):
        tmp = target + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", *flags, *[f"-D{d}" for d in defines],
             _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, target)
    return target


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_nbasis.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_rule_size.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_rule.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_basis.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.orc_geometry.argtypes = [ctypes.c_int, dp, dp, dp, dp]
        L.orc_assemble.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int64, dp, dp, ctypes.c_double, ctypes.c_double,
                                   dp, ctypes.c_int]
        L.orc_assemble.restype = ctypes.c_int64
        L.orc_assemble_coef.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int64, dp, dp, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int]
        L.orc_assemble_coef.restype = ctypes.c_int64
        L.orc_hyper_residual.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                         dp, dp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_hyper_residual.restype = ctypes.c_int64
        L.orc_hyper_residual_coef.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                              dp, dp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_hyper_residual_coef.restype = ctypes.c_int64
        L.orc_hyper_min_jf.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                       dp, dp, dp, ctypes.c_int]
        L.orc_hyper_min_jf.restype = ctypes.c_int64
        L.orc_max_threads.restype = ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_assemble_spec.argtypes = [ctypes.c_int, ip, ip, ip, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int64, dp, dp, dp, ctypes.c_int]
        L.orc_assemble_spec.restype = ctypes.c_int64
        L.orc_assemble_vspec.argtypes = [ctypes.c_int, ip, ip, ip, ip, ip, dp, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, dp, dp, dp,
                                         ctypes.c_int]
        L.orc_assemble_vspec.restype = ctypes.c_int64
        L.orc_assemble_pointgeo.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, dp, dp,
                                            ctypes.c_double, ctypes.c_double, dp, ctypes.c_int]
        L.orc_assemble_pointgeo.restype = ctypes.c_int64
        L.orc_assemble_curved.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, dp,
                                          dp, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int]
        L.orc_assemble_curved.restype = ctypes.c_int64
        i32p, i64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
        L.orc_csr_insert.argtypes = [ctypes.c_int64, ctypes.c_int, i32p, ctypes.c_int64, i64p, i32p, dp, dp]
        L.orc_csr_insert.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def nbasis(cell: str, p: int) -> int:
    return lib().orc_nbasis(CELL[cell], p)


def default_qdeg(form: str, cell: str, p: int, nf: int = 0) -> int:
    """Exact quadrature degree for each form (Sec. 7.1 uses exact quadrature):
    mass and Helmholtz 2p; elasticity with P1 Lame fields 2(p-1)+1 on
    simplices and 2p+1 on prisms (tensor-product degree); hyperelastic 4 (its
    integrand is not a polynomial); plus p per pre-multiplying coefficient
    function of degree p."""
    if form in ("mass", "helmholtz"):
        return (2 + nf) * p
    if form == "elasticity":
        return (2 * p + 1 if cell == "prism" else 2 * p - 1) + nf * p
    return 4 + nf * p


def own_coeff(form: str, cell: str, p: int) -> int:
    """The form's own coefficient DOFs per element (before any nf functions)."""
    return {"mass": 0, "helmholtz": 0, "elasticity": 2 * NVERT[cell],
            "hyperelastic": TDIM[cell] * nbasis(cell, p)}[form]


def rule(cell: str, qdeg: int):
    L = lib()
    nq = L.orc_rule_size(CELL[cell], qdeg)
    if nq < 0:
        raise ValueError("bad rule")
    X = np.zeros((nq, TDIM[cell]))
    W = np.zeros(nq)
    L.orc_rule(CELL[cell], qdeg, _p(X), _p(W))
    return X, W


def basis(cell: str, p: int, X):
    X = _f64(np.atleast_2d(X))
    nb = nbasis(cell, p)
    d = TDIM[cell]
    phi = np.zeros((X.shape[0], nb))
    dphi = np.zeros((X.shape[0], nb, d))
    for i in range(X.shape[0]):
        xi = _f64(X[i])
        ph = np.zeros(nb)
        dph = np.zeros((nb, d))
        lib().orc_basis(CELL[cell], p, _p(xi), _p(ph), _p(dph))
        phi[i], dphi[i] = ph, dph
    return phi, dphi


def geometry(cell: str, v):
    d = TDIM[cell]
    v = _f64(v)
    J = np.zeros((d, d))
    K = np.zeros((d, d))
    det = np.zeros(1)
    bad = lib().orc_geometry(CELL[cell], _p(v), _p(J), _p(det), _p(K))
    return J, float(det[0]), K, bool(bad)


def local_dim(form: str, cell: str, p: int) -> int:
    ns = nbasis(cell, p)
    return TDIM[cell] * ns if form in ("elasticity", "hyperelastic") else ns


def assemble(form: str, cell: str, p: int, coords, coeff=None, qdeg=None,
             mu: float = 1.0, lam: float = 10.0, nthreads: int = 0, nf: int = 0):
    """Element matrices [E][n][n] and the number of flagged elements.  For
    mass and Helmholtz, nf > 0 pre-multiplies the form by nf coefficient
    functions of degree p with DOFs coeff [E][nf][n_s]."""
    coords = _f64(coords)
    E = coords.shape[0]
    n = local_dim(form, cell, p)
    if qdeg is None:
        qdeg = default_qdeg(form, cell, p, nf)
    out = np.empty((E, n, n))
    cf = _f64(coeff) if coeff is not None else None
    if nf:
        if cf is None or cf.size != E * (own_coeff(form, cell, p) + nf * nbasis(cell, p)):
            raise ValueError("nf coefficient functions need coeff [E][own + nf * n_s]")
        flagged = lib().orc_assemble_coef(FORM[form], CELL[cell], p, qdeg, nf, E, _p(coords), _p(cf),
                                          mu, lam, _p(out), nthreads)
        if flagged < 0:
            raise ValueError("oracle rejected arguments")
        return out, int(flagged)
    if form in ("elasticity", "hyperelastic") and cf is None:
        raise ValueError("coefficients required")
    flagged = lib().orc_assemble(FORM[form], CELL[cell], p, qdeg, E, _p(coords), _p(cf),
                                 mu, lam, _p(out), nthreads)
    if flagged < 0:
        raise ValueError("oracle rejected arguments")
    return out, int(flagged)


SYMBOLS = {"value": 0, "dx": 1, "dy": 2, "dz": 3}


def assemble_spec(terms, cell: str, p: int, coords, fields=None, qdeg=None, nthreads: int = 0):
    """Element matrices of a generic scalar bilinear form.  terms: list of
    (test_symbol, trial_symbol, field, scale) with symbols from SYMBOLS (or
    their integer codes) and field -1 (constant) or the index of a P1 field
    whose vertex values are fields [E][n_fields][nv].  qdeg defaults to 2p
    plus one per field-weighted term (exact for affine elements)."""
    coords = _f64(coords)
    E = coords.shape[0]
    ns = nbasis(cell, p)
    code = lambda s: SYMBOLS[s] if isinstance(s, str) else int(s)  # noqa: E731
    te = (ctypes.c_int * len(terms))(*[code(t[0]) for t in terms])
    tr = (ctypes.c_int * len(terms))(*[code(t[1]) for t in terms])
    fl = (ctypes.c_int * len(terms))(*[int(t[2]) for t in terms])
    sc = np.array([float(t[3]) for t in terms])
    nfld = 0 if fields is None else np.asarray(fields).shape[1]
    if qdeg is None:
        qdeg = 2 * p + (1 if any(int(t[2]) >= 0 for t in terms) else 0)
        if cell == "prism" and any(int(t[2]) >= 0 for t in terms):
            qdeg = 2 * p + 1
    fd = _f64(fields) if fields is not None else None
    out = np.empty((E, ns, ns))
    flagged = lib().orc_assemble_spec(len(terms), te, tr, fl, _p(sc), nfld, CELL[cell], p, qdeg, E, _p(coords),
                                      _p(fd), _p(out), nthreads)
    if flagged < 0:
        raise ValueError("oracle rejected the form")
    return out, int(flagged)


def assemble_vspec(terms, cell: str, p: int, coords, fields=None, qdeg=None, n_comp=None, nthreads: int = 0):
    """Element matrices of a generic bilinear form on the vector-valued space
    of n_comp components (default: the cell dimension), component-blocked.
    terms: list of (test_symbol, trial_symbol, field, scale, test_comp,
    trial_comp); the rest as for assemble_spec."""
    coords = _f64(coords)
    E = coords.shape[0]
    ns = nbasis(cell, p)
    nc = TDIM[cell] if n_comp is None else int(n_comp)
    code = lambda s: SYMBOLS[s] if isinstance(s, str) else int(s)  # noqa: E731
    arr = lambda xs: (ctypes.c_int * max(1, len(xs)))(*xs)  # noqa: E731
    te = arr([code(t[0]) for t in terms])
    tr = arr([code(t[1]) for t in terms])
    fl = arr([int(t[2]) for t in terms])
    tc = arr([int(t[4]) for t in terms])
    rc = arr([int(t[5]) for t in terms])
    sc = np.array([float(t[3]) for t in terms] or [0.0])
    nfld = 0 if fields is None else np.asarray(fields).shape[1]
    if qdeg is None:
        qdeg = 2 * p + (1 if any(int(t[2]) >= 0 for t in terms) else 0)
    fd = _f64(fields) if fields is not None else None
    out = np.empty((E, nc * ns, nc * ns))
    flagged = lib().orc_assemble_vspec(len(terms), te, tr, tc, rc, fl, _p(sc), nfld, nc, CELL[cell], p, qdeg, E,
                                       _p(coords), _p(fd), _p(out), nthreads)
    if flagged < 0:
        raise ValueError("oracle rejected the form")
    return out, int(flagged)


def assemble_pointgeo(form: str, p: int, coords, coeff=None, qdeg=None, mu: float = 1.0, lam: float = 10.0,
                      nthreads: int = 0):
    """Prism element matrices without the affine assumption: the P1 x P1
    vertex map's J, det J and J^{-1} at every quadrature point.  The default
    rule adds one degree to the affine default (det J varies over the
    element).  Returns (out [E][n][n], flagged)."""
    coords = _f64(coords)
    E = coords.shape[0]
    n = local_dim(form, "prism", p)
    if qdeg is None:
        qdeg = default_qdeg_pointgeo(form, p)
    out = np.empty((E, n, n))
    cf = _f64(coeff) if coeff is not None else None
    if form in ("elasticity", "hyperelastic") and cf is None:
        raise ValueError("coefficients required")
    flagged = lib().orc_assemble_pointgeo(FORM[form], p, qdeg, E, _p(coords), _p(cf), mu, lam, _p(out), nthreads)
    if flagged < 0:
        raise ValueError("oracle rejected arguments")
    return out, int(flagged)


def assemble_curved(form: str, cell: str, p: int, coords, coeff=None, qdeg=None, mu: float = 1.0,
                    lam: float = 10.0, nthreads: int = 0):
    """Element matrices of curved triangles and tetrahedra: the isoparametric
    P2 map through the element's P2 nodes coords [E][n_2][d] (lattice order),
    its J, det J and J^{-1} at every quadrature point.  The default rule adds
    d degrees to the affine default (det J of a P2 map has degree d, so the
    mass form stays exact).  Returns (out [E][n][n], flagged)."""
    coords = _f64(coords)
    E = coords.shape[0]
    n = local_dim(form, cell, p)
    if qdeg is None:
        qdeg = default_qdeg_curved(form, cell, p)
    out = np.empty((E, n, n))
    cf = _f64(coeff) if coeff is not None else None
    if form in ("elasticity", "hyperelastic") and cf is None:
        raise ValueError("coefficients required")
    flagged = lib().orc_assemble_curved(FORM[form], CELL[cell], p, qdeg, E, _p(coords), _p(cf), mu, lam, _p(out),
                                        nthreads)
    if flagged < 0:
        raise ValueError("oracle rejected arguments")
    return out, int(flagged)


def default_qdeg_curved(form: str, cell: str, p: int) -> int:
    return default_qdeg(form, cell, p) + TDIM[cell]


def default_qdeg_pointgeo(form: str, p: int) -> int:
    """Rule degree for non-affine prisms: the affine default plus one, the
    degree det J adds when only the vertex heights vary (det J is then
    linear in X, Y and constant in Z)."""
    return default_qdeg(form, "prism", p) + 1


def hyper_residual(cell: str, p: int, coords, u, qdeg: int = 4, mu: float = 1.0, lam: float = 10.0, nf: int = 0):
    """Residual [E][d n_s] and strain energy [E]; with nf > 0, u holds the
    displacement DOFs then the nf pre-multiplying functions' DOFs per element."""
    coords, u = _f64(coords), _f64(u)
    E = coords.shape[0]
    R = np.zeros((E, TDIM[cell] * nbasis(cell, p)))
    en = np.zeros(E)
    lib().orc_hyper_residual_coef(CELL[cell], p, qdeg, nf, E, _p(coords), _p(u), mu, lam, _p(R), _p(en))
    return R, en


def hyper_min_jf(cell: str, p: int, coords, u, qdeg: int = 4, nthreads: int = 0):
    coords, u = _f64(coords), _f64(u)
    E = coords.shape[0]
    m = np.zeros(E)
    lib().orc_hyper_min_jf(CELL[cell], p, qdeg, E, _p(coords), _p(u), _p(m), nthreads)
    return m


def csr_pattern(dofs, N: int):
    """Compressed-row pattern of the global matrix (Sec. 2, global assembly):
    entry (r, c) is stored when some element holds both global DOFs r and c.
    Columns are sorted within each row.  Returns (row_ptr [N+1] int64,
    cols [nnz] int32)."""
    d = np.asarray(dofs, dtype=np.int64)
    keys = np.unique((d[:, :, None] * N + d[:, None, :]).ravel())
    rows = keys // N
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=N), out=row_ptr[1:])
    return row_ptr, np.ascontiguousarray(keys % N, dtype=np.int32)


def csr_insert(dofs, N: int, row_ptr, cols, A):
    """Values [nnz] of the global matrix: the element matrices A [E][n][n]
    added at (dofs[e][j], dofs[e][k]) in increasing element order."""
    d = np.ascontiguousarray(dofs, dtype=np.int32)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(cols, dtype=np.int32)
    A = _f64(A)
    E, n = d.shape
    if A.shape != (E, n, n) or rp.shape != (N + 1,):
        raise ValueError("shape mismatch")
    vals = np.empty(int(rp[N]))
    i32p, i64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
    rc = lib().orc_csr_insert(E, n, d.ctypes.data_as(i32p), N, rp.ctypes.data_as(i64p), cl.ctypes.data_as(i32p),
                              _p(A), _p(vals))
    if rc != 0:
        raise ValueError("an element entry is missing from the pattern")
    return vals


def csr_row(dofs, r: int, A_of):
    """One row of the global matrix, computed on its own: the elements holding
    DOF r (increasing order), the sorted columns of the row and its values,
    summed in increasing element order.  A_of(elements) returns the element
    matrices [len(elements)][n][n] of those elements."""
    d = np.asarray(dofs)
    els = np.nonzero((d == r).any(axis=1))[0]
    cols = np.unique(d[els].ravel()).astype(np.int64)
    vals = np.zeros(cols.size)
    A = _f64(A_of(els))
    for t, e in enumerate(els):
        j = int(np.nonzero(d[e] == r)[0][0])
        for k in range(d.shape[1]):
            vals[np.searchsorted(cols, d[e, k])] += A[t, j, k]
    return els, cols, vals


def max_threads() -> int:
    return lib().orc_max_threads()

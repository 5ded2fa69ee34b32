"""The float64 matrix-core quadrature kernel of the scalar forms (launch
shape kernel 4 for mass and Helmholtz) against the oracle, with the float64
bar of the other kernels (per element max |A - A_oracle| / max |A_oracle| <=
1e-12): plain rules, coefficient functions with weights of both signs, and
non-affine prisms."""
import sys

import numpy as np
import pytest

import oracle
from paper_1604_05872_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1604_05872_amd import felocal  # noqa: E402

TOL = 1e-12


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def normwise(A, B):
    return np.max(np.abs(A - B), axis=(1, 2)) / np.max(np.abs(B), axis=(1, 2))


def run(form, cell, p, coords, cf=None, **kw):
    n, _ = felocal.fe_local_dims(form, cell, p)
    out = torch.full((len(coords), n, n), float("nan"), dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    felocal.fe_assemble_local(form, cell, p, dev(coords), dev(cf) if cf is not None else None, out, status=st, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy(), int(st.item())


PLAIN = [(f, c, p) for f in ("mass", "helmholtz") for c in ("triangle", "tetrahedron", "prism") for p in (1, 2, 3, 4)
         if not (c == "prism" and p == 4)]


@pytest.mark.parametrize("form,cell,p", PLAIN)
def test_gram_scalar_plain(form, cell, p):
    log(f"gram scalar: {form} {cell} P{p}")
    E = {1: 333, 2: 211, 3: 97, 4: 53}[p]
    coords, V, cells, h = inputs.first_elements(cell, E, 31)
    A, st = run(form, cell, p, coords, mode="quadrature", shape={"kernel": 4})
    B, fl = oracle.assemble(form, cell, p, coords)
    assert st == fl == 0
    assert normwise(A, B).max() <= TOL


COEF = [("mass", "tetrahedron", 2, 1), ("mass", "triangle", 3, 2), ("helmholtz", "tetrahedron", 2, 2),
        ("helmholtz", "tetrahedron", 3, 1), ("helmholtz", "prism", 2, 1), ("mass", "prism", 1, 3),
        ("helmholtz", "triangle", 4, 3)]


@pytest.mark.parametrize("form,cell,p,nf", COEF)
def test_gram_scalar_coefficients(form, cell, p, nf):
    """Coefficient DOFs uniform in [-1, 1]: products of both signs at the
    points, so the signed-root Gram form is exercised."""
    log(f"gram scalar coefficients: {form} {cell} P{p} nf={nf}")
    coords, V, cells, h = inputs.first_elements(cell, 77, 32)
    ns = oracle.nbasis(cell, p)
    cf = np.random.default_rng(33).uniform(-1, 1, size=(len(coords), nf, ns))
    A, st = run(form, cell, p, coords, cf, mode="quadrature", nf=nf, shape={"kernel": 4})
    B, fl = oracle.assemble(form, cell, p, coords, cf, nf=nf)
    assert st == fl == 0
    assert normwise(A, B).max() <= TOL


@pytest.mark.parametrize("form,p", [("mass", 1), ("mass", 3), ("helmholtz", 1), ("helmholtz", 2), ("helmholtz", 3)])
def test_gram_scalar_nonaffine_prisms(form, p):
    log(f"gram scalar non-affine prisms: {form} P{p}")
    coords, V, cells, h = inputs.first_elements("prism", 150, 34, zjitter=0.3)
    A, st = run(form, "prism", p, coords, pointgeo=True, shape={"kernel": 4})
    B, fl = oracle.assemble_pointgeo(form, p, coords)
    assert st == fl == 0
    assert normwise(A, B).max() <= TOL


def test_gram_scalar_flags():
    coords, V, cells, h = inputs.first_elements("tetrahedron", 40, 35)
    coords = coords.copy()
    coords[5, 2] = coords[5, 1]
    A, st = run("helmholtz", "tetrahedron", 2, coords, mode="quadrature", shape={"kernel": 4})
    assert st == 1 and np.isnan(A[5]).all() and not np.isnan(np.delete(A, 5, axis=0)).any()


def test_gram_scalar_against_valu_timing():
    """Both quadrature kernels on the same 82,944 tetrahedra (Helmholtz P3
    and P4, the rule of the Sec. 7.1 sweep with one coefficient function):
    equal within the float64 bar; times are printed for the record."""
    coords, V, cells, h = inputs.first_elements("tetrahedron", 82944, 36)
    for p in (3, 4):
        ns = oracle.nbasis("tetrahedron", p)
        cf = np.random.default_rng(p).uniform(0.5, 1.5, size=(len(coords), 1, ns))
        dc, dcf = dev(coords), dev(cf)
        out = {}
        for k in (3, 4):
            o = torch.empty((len(coords), ns, ns), dtype=torch.float64, device="cuda")
            fn = lambda: felocal.fe_assemble_local("helmholtz", "tetrahedron", p, dc, dcf, o, mode="quadrature",  # noqa
                                                   nf=1, shape={"kernel": k})
            fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(3):
                fn()
            b.record()
            torch.cuda.synchronize()
            out[k] = (a.elapsed_time(b) / 3, o.cpu().numpy())
        log(f"helmholtz tet P{p} nf=1 82944: VALU {out[3][0]:.3f} ms, matrix core {out[4][0]:.3f} ms")
        assert normwise(out[4][1], out[3][1]).max() <= 1e-12

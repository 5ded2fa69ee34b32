"""fe_assemble_csr_noalloc (the one-pass global assembly with its geometry
workspace in the library's file-scope device array, no allocation) against
fe_assemble_csr through the C ABI: the same kernels, so the stored values
must agree bit for bit, on two calls in a row, the second with a smaller
input; sizes beyond the array and tables not yet built are refused."""
import sys

import numpy as np
import pytest

from paper_1604_05872_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1604_05872_amd import felocal  # noqa: E402


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def case(cell, p, n, seed, E=None):
    V, cells = {"triangle": lambda: inputs.triangle_mesh(n, n, seed), "tetrahedron": lambda: inputs.tet_mesh(n, seed),
                "prism": lambda: inputs.prism_mesh(n, n, seed)}[cell]()
    if E is not None:
        cells = cells[:E]
    dofs, N = inputs.global_dofs(cell, p, cells, n)
    return inputs.gather(V, cells), dofs, N


def both(form, cell, p, coords, dofs, N):
    """(fe_assemble_csr values, fe_assemble_csr_noalloc values, status counts)."""
    pat = felocal.CsrPattern(dev(dofs), N)
    nnz = pat.info()["nnz"]
    c = dev(coords)
    ref = torch.full((nnz,), float("nan"), dtype=torch.float64, device="cuda")
    got = torch.full((nnz,), float("nan"), dtype=torch.float64, device="cuda")
    s1 = torch.zeros(1, dtype=torch.int32, device="cuda")
    s2 = torch.zeros(1, dtype=torch.int32, device="cuda")
    pat.assemble(form, cell, p, c, ref, status=s1)
    pat.assemble_noalloc(form, cell, p, c, got, status=s2)
    torch.cuda.synchronize()
    out = ref.cpu().numpy(), got.cpu().numpy(), int(s1.item()), int(s2.item())
    pat.close()
    return out


@pytest.mark.parametrize("form,cell,p", [("helmholtz", "tetrahedron", 2), ("mass", "prism", 3),
                                         ("helmholtz", "triangle", 4)])
def test_noalloc_equals_fe_assemble_csr(form, cell, p):
    """Two calls in a row on one device, the second with fewer elements (the
    array then keeps part of the first call's contents)."""
    n1, n2 = {"triangle": (180, 60), "tetrahedron": (40, 17), "prism": (36, 15)}[cell]
    for n, seed in ((n1, 81), (n2, 82)):
        coords, dofs, N = case(cell, p, n, seed)
        log(f"noalloc {form} {cell} P{p}: {coords.shape[0]} elements, {N} rows")
        ref, got, s1, s2 = both(form, cell, p, coords, dofs, N)
        assert s1 == s2 == 0
        assert np.isfinite(ref).all()
        assert np.array_equal(ref, got)


def test_noalloc_flagged_elements():
    """A degenerate element: NaN in the entries it touches and one count, as
    fe_assemble_csr."""
    coords, dofs, N = case("tetrahedron", 1, 12, 83)
    coords = coords.copy()
    coords[100, 2] = coords[100, 1]
    ref, got, s1, s2 = both("helmholtz", "tetrahedron", 1, coords, dofs, N)
    assert s1 == s2 == 1
    assert np.array_equal(np.isnan(ref), np.isnan(got)) and np.isnan(ref).any()
    assert np.array_equal(ref[~np.isnan(ref)], got[~np.isnan(got)])


def test_noalloc_refusals():
    """More elements than the array holds: FE_ENOMEM before any work.  Tables
    never built on this device (caches released): FE_EINVAL, and the call
    after one fe_assemble_csr succeeds."""
    # 6 * 56^3 = 1,053,696 > 1,048,576 elements
    coords, dofs, N = case("tetrahedron", 1, 56, 84)
    assert coords.shape[0] > 1 << 20
    pat = felocal.CsrPattern(dev(dofs), N)
    vals = torch.zeros(pat.info()["nnz"], dtype=torch.float64, device="cuda")
    with pytest.raises(felocal.FeError) as ei:
        pat.assemble_noalloc("helmholtz", "tetrahedron", 1, dev(coords), vals)
    assert ei.value.code == felocal.FE_ENOMEM
    pat.close()
    coords, dofs, N = case("prism", 2, 9, 85)
    torch.cuda.synchronize()
    felocal.lib().fe_release_caches()
    pat = felocal.CsrPattern(dev(dofs), N)
    vals = torch.full((pat.info()["nnz"],), float("nan"), dtype=torch.float64, device="cuda")
    c = dev(coords)
    with pytest.raises(felocal.FeError) as ei:
        pat.assemble_noalloc("mass", "prism", 2, c, vals)
    assert ei.value.code == felocal.FE_EINVAL
    ref = torch.zeros_like(vals)
    pat.assemble("mass", "prism", 2, c, ref)
    pat.assemble_noalloc("mass", "prism", 2, c, vals)
    torch.cuda.synchronize()
    assert torch.equal(ref, vals)
    pat.close()

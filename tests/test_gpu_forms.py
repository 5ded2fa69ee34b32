"""Generic forms, scalar and on vector-valued spaces, assembled by kernels
generated from Algorithm 1's result (fe_assemble_form, compiled at run time
with hipRTC) against the oracle's naive nest, per element max |A - A_oracle| /
max |A_oracle| <= 1e-12; both the sharing-eliminated and the expanded nests."""
import itertools
import sys

import numpy as np
import pytest

import oracle
from paper_1604_05872_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1604_05872_amd import felocal  # noqa: E402

TOL = 1e-12
D3 = ["dx", "dy", "dz"]


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def normwise(A, B):
    return np.max(np.abs(A - B), axis=(1, 2)) / np.max(np.abs(B), axis=(1, 2))


FORMS = {
    "advection_diffusion_reaction": lambda d: [(a, a, -1, 1.0) for a in D3[:d]] +
                                              [("value", a, -1, 0.3 * (i + 1)) for i, a in enumerate(D3[:d])] +
                                              [("value", "value", 0, 1.0)],
    "full_tensor_diffusion": lambda d: [(a, b, -1, 1.0 + 0.25 * i) for i, (a, b) in
                                        enumerate(itertools.product(D3[:d], D3[:d]))],
    "weighted_transport": lambda d: [("dx", "value", 0, 1.5), ("value", "dy", 1, -0.5), ("value", "value", -1, 2.0)],
}


def run(terms, cell, p, coords, fields, nf, expanded=False):
    n = inputs.n_scalar_dofs(cell, p)
    out = torch.full((len(coords), n, n), float("nan"), dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    felocal.fe_assemble_form(terms, cell, p, dev(coords), dev(fields) if fields is not None else None, out,
                             n_fields=nf, expanded=expanded, status=st)
    torch.cuda.synchronize()
    return out.cpu().numpy(), int(st.item())


# degrees 1-4 (prisms 1-3: P4 has more than 64 basis functions); P4 on
# tetrahedra (35 rows) pads the register tiles past the last row
CASES = [(f, c, p) for f in sorted(FORMS) for c in ("triangle", "tetrahedron", "prism")
         for p in ((1, 2, 3) if c == "prism" else (1, 2, 3, 4))]


@pytest.mark.parametrize("expanded", [False, True])
@pytest.mark.parametrize("name,cell,p", CASES)
def test_generated_form_matches_oracle(name, cell, p, expanded):
    log(f"generated: {name} {cell} P{p} expanded={expanded}")
    d = 2 if cell == "triangle" else 3
    terms = FORMS[name](d)
    coords, V, cells, h = inputs.first_elements(cell, 157, 41)
    nv = inputs.NVERT[cell]
    nf = 2
    fields = np.random.default_rng(42).uniform(0.5, 2.0, size=(len(coords), nf, nv))
    A, st = run(terms, cell, p, coords, fields, nf, expanded)
    B, fl = oracle.assemble_spec(terms, cell, p, coords, fields)
    assert st == fl == 0
    assert normwise(A, B).max() <= TOL


def test_generated_helmholtz_equals_library_form():
    coords, V, cells, h = inputs.first_elements("tetrahedron", 300, 43)
    terms = [("value", "value", -1, 1.0)] + [(a, a, -1, 1.0) for a in D3]
    A, st = run(terms, "tetrahedron", 3, coords, None, 0)
    n = 20
    ref = torch.empty((300, n, n), dtype=torch.float64, device="cuda")
    felocal.fe_assemble_local("helmholtz", "tetrahedron", 3, dev(coords), None, ref)
    torch.cuda.synchronize()
    assert st == 0 and normwise(A, ref.cpu().numpy()).max() <= TOL


def test_generated_flags_and_errors():
    coords, V, cells, h = inputs.first_elements("tetrahedron", 20, 44)
    coords = coords.copy()
    coords[3, 1] = coords[3, 0]
    A, st = run([("dx", "dx", -1, 1.0)], "tetrahedron", 2, coords, None, 0)
    assert st == 1 and np.isnan(A[3]).all() and not np.isnan(np.delete(A, 3, axis=0)).any()
    pc, _, _, _ = inputs.first_elements("prism", 12, 45, zjitter=0.3)
    A, st = run([("value", "value", -1, 1.0)], "prism", 1, pc, None, 0)
    assert st == 12
    out = torch.empty((20, 10, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(felocal.FeError) as ei:   # a field term without fields
        felocal.fe_assemble_form([("value", "value", 0, 1.0)], "tetrahedron", 2, dev(coords), None, out, n_fields=1)
    assert ei.value.code == felocal.FE_EINVAL


def test_sharing_elimination_timing():
    """Full-tensor diffusion on 82,944 tetrahedra: the factorised nest (3
    multiply-adds per (j, k)) against the expanded one (9); printed."""
    coords, V, cells, h = inputs.first_elements("tetrahedron", 82944, 46)
    dc = dev(coords)
    terms = FORMS["full_tensor_diffusion"](3)
    for p in (2, 3, 4):
        n = inputs.n_scalar_dofs("tetrahedron", p)
        out = torch.empty((len(coords), n, n), dtype=torch.float64, device="cuda")
        ms = {}
        for ex in (False, True):
            fn = lambda: felocal.fe_assemble_form(terms, "tetrahedron", p, dc, None, out, expanded=ex)  # noqa
            fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(3):
                fn()
            b.record()
            torch.cuda.synchronize()
            ms[ex] = a.elapsed_time(b) / 3
        pl = felocal.fe_sharing_plan(terms, "tetrahedron", p)
        log(f"full tensor P{p}: factorised {ms[False]:.3f} ms, expanded {ms[True]:.3f} ms, "
            f"theta {pl['theta_se']:.0f} vs {pl['theta_expanded']:.0f}")


# --------------------------------------------------------------------------
# Vector-valued spaces (component-blocked, one loop nest per block)

def elasticity_terms(d):
    t = []
    for a in range(d):
        for b in range(d):
            t.append((D3[b], D3[b], 1, 1.0, a, a))
            t.append((D3[b], D3[a], 1, 1.0, a, b))
            t.append((D3[a], D3[b], 0, 1.0, a, b))
    return t


def advection_diffusion_terms(d):
    """nu grad u : grad v + (w . grad) u . v, velocity w the P1 fields 0..d-1,
    plus a coupling v_1 d_x u_0 (factorised diagonal blocks, one off-diagonal
    block, the others empty)."""
    t = []
    for a in range(d):
        for b in range(d):
            t.append((D3[b], D3[b], -1, 0.1, a, a))
            t.append(("value", D3[b], b, 1.0, a, a))
    return t + [("value", "dx", -1, 0.5, 1, 0)]


def random_vector_terms(d, seed):
    rng = np.random.default_rng(seed)
    syms = ["value"] + D3[:d]
    return [(syms[int(rng.integers(0, d + 1))], syms[int(rng.integers(0, d + 1))], int(rng.integers(-1, 3)),
             float(rng.uniform(-2, 2)), int(rng.integers(0, d)), int(rng.integers(0, d))) for _ in range(14)]


VFORMS = {"elasticity": elasticity_terms, "advection_diffusion": advection_diffusion_terms,
          "random": lambda d: random_vector_terms(d, 7 + d)}
VCASES = [(f, c, p) for f in sorted(VFORMS) for c in ("triangle", "tetrahedron", "prism")
          for p in ((1, 2, 3) if c == "prism" else (1, 2, 3, 4))]


def run_vector(terms, cell, p, coords, fields, nf, expanded=False):
    d = 2 if cell == "triangle" else 3
    n = d * inputs.n_scalar_dofs(cell, p)
    out = torch.full((len(coords), n, n), float("nan"), dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    felocal.fe_assemble_form(terms, cell, p, dev(coords), dev(fields) if fields is not None else None, out,
                             n_fields=nf, expanded=expanded, status=st, n_comp=d)
    torch.cuda.synchronize()
    return out.cpu().numpy(), int(st.item())


@pytest.mark.parametrize("name,cell,p", VCASES)
def test_generated_vector_form_matches_oracle(name, cell, p):
    log(f"generated vector form: {name} {cell} P{p}")
    d = 2 if cell == "triangle" else 3
    terms = VFORMS[name](d)
    coords, V, cells, h = inputs.first_elements(cell, 97, 51)
    nv = inputs.NVERT[cell]
    nf = 3
    fields = np.random.default_rng(52).uniform(0.5, 2.0, size=(len(coords), nf, nv))
    B, fl = oracle.assemble_vspec(terms, cell, p, coords, fields)
    for expanded in ((False, True) if name == "advection_diffusion" else (False,)):
        A, st = run_vector(terms, cell, p, coords, fields, nf, expanded)
        assert st == fl == 0
        assert normwise(A, B).max() <= TOL, expanded


@pytest.mark.parametrize("cell,p", [("triangle", 2), ("tetrahedron", 3), ("prism", 2)])
def test_generated_elasticity_equals_library_form(cell, p):
    """The elasticity form written as component terms, through the generated
    kernel, equals the library's own elasticity kernel (its default plan)."""
    d = 2 if cell == "triangle" else 3
    coords, V, cells, h = inputs.first_elements(cell, 200, 53)
    nv = inputs.NVERT[cell]
    lm = np.random.default_rng(54).uniform(0.5, 2.0, size=(len(coords), 2, nv))
    A, st = run_vector(elasticity_terms(d), cell, p, coords, lm, 2)
    n = A.shape[1]
    ref = torch.empty((len(coords), n, n), dtype=torch.float64, device="cuda")
    felocal.fe_assemble_local("elasticity", cell, p, dev(coords), dev(lm.reshape(len(coords), -1)), ref)
    torch.cuda.synchronize()
    assert st == 0 and normwise(A, ref.cpu().numpy()).max() <= TOL


def test_generated_vector_flags_and_ragged_grid():
    """A degenerate element gets a NaN block over all component blocks, and
    element counts that leave a wavefront partly filled store nothing past
    the end (the output's tail keeps its canary)."""
    coords, V, cells, h = inputs.first_elements("tetrahedron", 37, 55)
    coords = coords.copy()
    coords[5, 2] = coords[5, 0]
    terms = advection_diffusion_terms(3)
    fields = np.random.default_rng(56).uniform(0.5, 2.0, size=(37, 3, 4))
    n = 3 * 10
    out = torch.full((38, n, n), 7.0, dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    felocal.fe_assemble_form(terms, "tetrahedron", 2, dev(coords), dev(fields), out[:37], n_fields=3, status=st,
                             n_comp=3)
    torch.cuda.synchronize()
    A = out.cpu().numpy()
    B, fl = oracle.assemble_vspec(terms, "tetrahedron", 2, coords, fields)
    assert int(st.item()) == fl == 1
    assert np.isnan(A[5]).all() and (A[37] == 7.0).all()
    keep = [i for i in range(37) if i != 5]
    assert normwise(A[keep], B[keep]).max() <= TOL


@pytest.mark.parametrize("name,vector,p", [("full_tensor_diffusion", False, 3), ("advection_diffusion", True, 2),
                                           ("elasticity", True, 2)])
def test_generated_forms_full_size_windows(name, vector, p):
    """82,944 tetrahedra: every wavefront runs the kernel's element loop
    several times (2,048 workgroups of 4 wavefronts).  Three 384-element
    windows (the first, one in the middle, the last, which ends ragged) are
    compared with the oracle element by element."""
    log(f"generated form full size: {name} vector={vector} P{p}")
    E = 82944
    coords, V, cells, h = inputs.first_elements("tetrahedron", E, 57)
    nf = 3
    fields = np.random.default_rng(58).uniform(0.5, 2.0, size=(E, nf, 4))
    if vector:
        terms = VFORMS[name](3)
        A, st = run_vector(terms, "tetrahedron", p, coords, fields, nf)
        ref = lambda sl: oracle.assemble_vspec(terms, "tetrahedron", p, coords[sl], fields[sl])  # noqa: E731
    else:
        terms = FORMS[name](3)
        A, st = run(terms, "tetrahedron", p, coords, fields, nf)
        ref = lambda sl: oracle.assemble_spec(terms, "tetrahedron", p, coords[sl], fields[sl])  # noqa: E731
    assert st == 0 and np.isfinite(A).all()
    for lo in (0, E // 2 - 192, E - 384):
        sl = slice(lo, lo + 384)
        B, fl = ref(sl)
        assert fl == 0
        assert normwise(A[sl], B).max() <= TOL, lo


def test_kernel_cache_keeps_calls_apart():
    """The kernel kept per call signature: alternating forms, degrees, the
    expanded nest, scalar and vector calls and an explicit rule, each result
    still equals the oracle's."""
    coords, V, cells, h = inputs.first_elements("tetrahedron", 61, 62)
    fields = np.random.default_rng(63).uniform(0.5, 2.0, size=(61, 3, 4))
    adv, el = advection_diffusion_terms(3), elasticity_terms(3)
    diff = FORMS["full_tensor_diffusion"](3)
    seq = [("v", adv, 2, False), ("v", el, 2, False), ("s", diff, 2, False), ("v", adv, 3, False),
           ("v", adv, 2, True), ("s", diff, 2, True), ("v", el, 2, False), ("s", diff, 3, False), ("v", adv, 2, False)]
    for kind, terms, p, ex in seq:
        if kind == "v":
            A, st = run_vector(terms, "tetrahedron", p, coords, fields, 3, ex)
            B, fl = oracle.assemble_vspec(terms, "tetrahedron", p, coords, fields)
        else:
            A, st = run(terms, "tetrahedron", p, coords, fields, 3, ex)
            B, fl = oracle.assemble_spec(terms, "tetrahedron", p, coords, fields)
        assert st == fl == 0
        assert normwise(A, B).max() <= TOL, (kind, p, ex)
    # an explicit rule of higher degree is a different call (and still exact)
    n = 3 * 10
    out = torch.full((61, n, n), float("nan"), dtype=torch.float64, device="cuda")
    felocal.fe_assemble_form(adv, "tetrahedron", 2, dev(coords), dev(fields), out, n_fields=3, qdeg=7, n_comp=3)
    torch.cuda.synchronize()
    B, _ = oracle.assemble_vspec(adv, "tetrahedron", 2, coords, fields, qdeg=7)
    assert normwise(out.cpu().numpy(), B).max() <= TOL


def test_generated_vector_form_empty_and_refusals():
    """No elements: nothing launched, no error.  A component count other than
    the cell dimension, a component out of range and a vector matrix too small
    for its output are refused before any launch."""
    coords = np.zeros((0, 4, 3))
    out = torch.empty((0, 30, 30), dtype=torch.float64, device="cuda")
    felocal.fe_assemble_form(advection_diffusion_terms(3), "tetrahedron", 2, dev(coords),
                             dev(np.zeros((0, 3, 4))), out, n_fields=3, n_comp=3)
    c, V, cells, h = inputs.first_elements("tetrahedron", 8, 64)
    f = dev(np.ones((8, 3, 4)))
    o = torch.empty((8, 30, 30), dtype=torch.float64, device="cuda")
    with pytest.raises(felocal.FeError) as ei:
        felocal.fe_assemble_form([("dx", "dx", -1, 1.0, 0, 0)], "tetrahedron", 2, dev(c), f, o, n_fields=3, n_comp=2)
    assert ei.value.code == felocal.FE_EINVAL
    with pytest.raises(felocal.FeError) as ei:
        felocal.fe_assemble_form([("dx", "dx", -1, 1.0, 0, 3)], "tetrahedron", 2, dev(c), f, o, n_fields=3, n_comp=3)
    assert ei.value.code == felocal.FE_EINVAL
    small = torch.empty((8, 10, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        felocal.fe_assemble_form([("dx", "dx", -1, 1.0, 0, 0)], "tetrahedron", 2, dev(c), f, small, n_fields=3,
                                 n_comp=3)


def test_release_caches_unloads_and_recompiles_generated_kernels():
    """After fe_release_caches the generated kernels are compiled again on
    the next call, with the same results bit for bit."""
    coords, V, cells, h = inputs.first_elements("tetrahedron", 45, 66)
    fields = np.random.default_rng(67).uniform(0.5, 2.0, size=(45, 3, 4))
    cases = [([("dx", "dy", -1, 0.5), ("value", "value", 0, 1.0)], 3, False, 1),
             (advection_diffusion_terms(3), 2, True, 3), (elasticity_terms(3), 2, True, 2)]
    def go():
        outs = []
        for terms, p, vec, nf in cases:
            if vec:
                outs.append(run_vector(terms, "tetrahedron", p, coords, fields[:, :nf], nf)[0])
            else:
                outs.append(run(terms, "tetrahedron", p, coords, fields[:, :nf], nf)[0])
        return outs
    first = go()
    torch.cuda.synchronize()
    felocal.lib().fe_release_caches()
    second = go()
    for a, b in zip(first, second):
        assert not np.isnan(a).any() and np.array_equal(a, b)

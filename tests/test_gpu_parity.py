"""Parity of the HIP library (through its C ABI) with the float64 CPU oracle.

Metric: per element, max_jk |A_gpu - A_oracle| / max_jk |A_oracle|; the bars
are 1e-12 for float64, 1e-4 for the bf16x3 split and 2e-6 for the fp32 split
(the bounds stated in include/felocal.h).  Small cases span several tiles and
a ragged tail; the full-size workloads are checked on sampled elements."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1604_05872_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1604_05872_amd import felocal  # noqa: E402

CELLS = ["triangle", "tetrahedron", "prism"]
TOL = {"fp64": 1e-12, "fp32": 2e-6, "bf16x3": 1e-4}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def mesh(cell, E, seed):
    coords, V, cells, h = inputs.first_elements(cell, E, seed)
    return coords, V, cells, h


def coefficients(form, cell, p, E, V, cells, h, seed):
    if form == "elasticity":
        return inputs.lame_p1(V.shape[0], cells, seed)
    if form == "hyperelastic":
        # N(0, 0.05 h) per DOF as the neo-Hookean workload is configured (P1,
        # P2); at P3 and P4 the DOF lattice is finer, and 0.05 h / p keeps
        # inverted elements rare
        rel = 0.05 if p <= 2 else 0.05 / p
        return inputs.displacement_dofs(E, oracle.TDIM[cell], oracle.nbasis(cell, p), h, seed, rel=rel)
    return None


def gpu_assemble(form, cell, p, coords, coeff=None, **kw):
    n, _ = felocal.fe_local_dims(form, cell, p)
    E = coords.shape[0]
    out = torch.full((E, n, n), float("nan"), dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    felocal.fe_assemble_local(form, cell, p, dev(coords), dev(coeff) if coeff is not None else None, out,
                              status=status, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy(), int(status.item())


def normwise(A, B):
    num = np.max(np.abs(A - B), axis=(1, 2))
    den = np.max(np.abs(B), axis=(1, 2))
    return num / den


def oracle_cost(form, cell, p):
    ns = oracle.nbasis(cell, p)
    n = ns * (oracle.TDIM[cell] if form in ("elasticity", "hyperelastic") else 1)
    nq = oracle.rule(cell, oracle.default_qdeg(form, cell, p))[1].size
    per = {"mass": 2, "helmholtz": 8, "elasticity": 60, "hyperelastic": 40}[form]
    return nq * n * n * per


def case_size(form, cell, p, cap=1000):
    return int(max(5, min(cap, 4e9 / oracle_cost(form, cell, p))))


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_tabulation_matches_oracle(cell, p):
    log(f"tabulate {cell} P{p}")
    for qdeg in (2 * p, 7):
        t = felocal.fe_tabulate(cell, p, qdeg)
        phi, dphi = oracle.basis(cell, p, t["points"])
        assert np.max(np.abs(t["phi"] - phi)) < 1e-13
        assert np.max(np.abs(t["dphi"] - dphi)) < 1e-11


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_tabulation_exact_rational(cell, p):
    """The library's basis pinned on its own, not through the oracle: values
    and reference gradients at the rule's points equal the Lagrange basis
    built by Vandermonde inversion over the rationals, evaluated exactly at
    the same float64 points (a construction shared with neither side)."""
    from fractions import Fraction as Fr

    import exact_rational as er
    log(f"tabulate exact {cell} P{p}")
    t = felocal.fe_tabulate(cell, p, 2 * p)
    ex, C = er.lagrange(cell, p)
    d = oracle.TDIM[cell]
    dcs = [er._deriv_coeffs(ex, C, a) for a in range(d)]
    pts = t["points"]
    for q in range(0, pts.shape[0], max(1, pts.shape[0] // 12)):
        x = tuple(Fr(float(c)) for c in pts[q])
        phi = np.array([float(v) for v in er.eval_basis(cell, p, x)])
        dphi = np.array([[float(sum(c * er.mono(x, e) for e, c in dcs[a][j].items())) for a in range(d)]
                         for j in range(len(ex))])
        assert np.max(np.abs(t["phi"][q] - phi)) <= 1e-14
        assert np.max(np.abs(t["dphi"][q] - dphi)) <= 1e-13 * max(1.0, np.abs(dphi).max())


@pytest.mark.parametrize("cell", CELLS)
def test_geometry_matches_oracle(cell):
    log(f"geometry {cell}")
    coords, *_ = mesh(cell, 777, seed=11)
    d = oracle.TDIM[cell]
    det = torch.zeros(coords.shape[0], dtype=torch.float64, device="cuda")
    K = torch.zeros((coords.shape[0], d, d), dtype=torch.float64, device="cuda")
    felocal.fe_geometry(cell, dev(coords), det, K)
    torch.cuda.synchronize()
    det, K = det.cpu().numpy(), K.cpu().numpy()
    for e in range(0, coords.shape[0], 37):
        J, dt, Ko, bad = oracle.geometry(cell, coords[e])
        assert abs(det[e] - dt) <= 1e-14 * abs(dt)
        assert np.max(np.abs(K[e] - Ko)) <= 1e-12 * np.max(np.abs(Ko))


FP64_CASES = [(f, c, p) for f in ("mass", "helmholtz", "elasticity", "hyperelastic") for c in CELLS
              for p in (1, 2, 3, 4)]


@pytest.mark.parametrize("form,cell,p", FP64_CASES)
def test_fp64_parity(form, cell, p):
    E = case_size(form, cell, p)
    log(f"fp64 parity {form} {cell} P{p} E={E}")
    coords, V, cells, h = mesh(cell, E, seed=100 + p)
    cf = coefficients(form, cell, p, E, V, cells, h, seed=200 + p)
    A, st = gpu_assemble(form, cell, p, coords, cf)
    B, fl = oracle.assemble(form, cell, p, coords, cf)
    bad = np.isnan(B[:, 0, 0])
    assert st == fl == bad.sum() and fl <= E // 100
    assert (np.isnan(A[:, 0, 0]) == bad).all() and np.isfinite(A[~bad]).all()
    assert normwise(A[~bad], B[~bad]).max() <= TOL["fp64"]


HELM_MODES = [("tetrahedron", 4, "preeval", 0), ("tetrahedron", 4, "quadrature", 0),
              ("tetrahedron", 4, "auto", 65536), ("prism", 4, "auto", 0), ("prism", 3, "preeval", 0),
              ("triangle", 3, "quadrature", 0), ("prism", 2, "auto", 1000)]


@pytest.mark.parametrize("cell,p,mode,th", HELM_MODES)
def test_helmholtz_modes_agree(cell, p, mode, th):
    """Pre-evaluation, quadrature and both mixed plans give the same matrices."""
    E = case_size("helmholtz", cell, p, cap=600)
    log(f"helmholtz modes {cell} P{p} {mode} th={th} E={E}")
    coords, *_ = mesh(cell, E, seed=7)
    A, st = gpu_assemble("helmholtz", cell, p, coords, mode=mode, th_bytes=th)
    B, _ = oracle.assemble("helmholtz", cell, p, coords)
    assert st == 0 and normwise(A, B).max() <= TOL["fp64"]


# Launch shapes of the pre-evaluated kernels: streaming (kernel 2) with one-step
# and multi-step visits, and tiled (kernel 1), with small persistent grids so
# that every block walks several groups, visits or tiles, ragged element
# counts, a ragged last step and a ragged last visit.
SHAPES = [
    ("mass", "triangle", 1, dict(kernel=2, block=64, epi=64, chunk=64, grid_per_cu=1), 40001),
    ("mass", "triangle", 1, dict(kernel=2, block=64, epi=64, chunk=192, grid_per_cu=1), 40001),
    ("helmholtz", "tetrahedron", 2, dict(kernel=2, block=64, epi=5, chunk=5, grid_per_cu=1), 40003),
    ("helmholtz", "tetrahedron", 2, dict(kernel=2, block=64, epi=5, chunk=35, grid_per_cu=1), 40003),
    ("helmholtz", "tetrahedron", 2, dict(kernel=2, block=512, epi=20, grid_per_cu=1), 30011),
    ("helmholtz", "tetrahedron", 4, dict(kernel=2, block=320, epi=1, chunk=3, grid_per_cu=1), 1501),
    ("helmholtz", "tetrahedron", 4, dict(kernel=2, block=256, epi=1, chunk=1, grid_per_cu=2), 1501),
    ("helmholtz", "prism", 3, dict(kernel=2, block=448, epi=1, chunk=2, grid_per_cu=1), 777),
    ("mass", "prism", 4, dict(kernel=2, block=384, epi=1, grid_per_cu=1), 613),
    ("helmholtz", "tetrahedron", 2, dict(kernel=1, block=256, epi=3, chunk=9, grid_per_cu=1), 5003),
    ("helmholtz", "triangle", 4, dict(kernel=1, block=320, epi=4, chunk=64, grid_per_cu=2), 3001),
    ("helmholtz", "prism", 4, dict(kernel=1, block=512, epi=1, chunk=16, grid_per_cu=1), 555),
]


@pytest.mark.parametrize("form,cell,p,shape,E", SHAPES)
def test_preeval_shapes(form, cell, p, shape, E):
    log(f"pre-evaluated shape {form} {cell} P{p} {shape} E={E}")
    coords, *_ = mesh(cell, E, seed=11 + p)
    A, st = gpu_assemble(form, cell, p, coords, mode="preeval", shape=shape)
    B, fl = oracle.assemble(form, cell, p, coords)
    bad = np.isnan(B[:, 0, 0])
    assert st == fl == bad.sum()
    assert (np.isnan(A[:, 0, 0]) == bad).all() and np.isfinite(A[~bad]).all()
    assert normwise(A[~bad], B[~bad]).max() <= TOL["fp64"]


AUTOTUNE_CASES = [("helmholtz", "tetrahedron", 3, 4001), ("mass", "prism", 2, 3001), ("helmholtz", "prism", 4, 301),
                  ("elasticity", "tetrahedron", 2, 1201), ("hyperelastic", "tetrahedron", 1, 2001),
                  ("elasticity", "tetrahedron", 3, 3001), ("elasticity", "prism", 3, 400)]


@pytest.mark.parametrize("form,cell,p,E", AUTOTUNE_CASES)
def test_autotune_shape_roundtrip(form, cell, p, E):
    """The autotuner's choice is used afterwards, and its reported shape is a
    valid override that gives the same matrices."""
    log(f"autotune {form} {cell} P{p} E={E}")
    coords, V, cells, h = mesh(cell, E, seed=21)
    cf = coefficients(form, cell, p, E, V, cells, h, seed=22)
    n, _ = felocal.fe_local_dims(form, cell, p)
    out = torch.empty((E, n, n), dtype=torch.float64, device="cuda")
    ms, shape = felocal.fe_autotune(form, cell, p, dev(coords), dev(cf) if cf is not None else None, out,
                                    return_shape=True)
    assert ms > 0
    # the shape of the measured faster mode: pre-evaluated (1, 2; 0 for the
    # single pre-evaluated elasticity kernel) or quadrature (3, 4, 5)
    preeval = shape["kernel"] in (0, 1, 2)
    assert form != "hyperelastic" or not preeval
    mode = "preeval" if preeval else "quadrature"
    B, _ = oracle.assemble(form, cell, p, coords, cf)
    A1, st1 = gpu_assemble(form, cell, p, coords, cf)
    shape = {k: v for k, v in shape.items() if v}
    A2, st2 = gpu_assemble(form, cell, p, coords, cf, shape=shape)
    A3, st3 = gpu_assemble(form, cell, p, coords, cf, shape=shape, mode=mode)
    assert st1 == st2 == st3 == 0
    assert np.array_equal(A1, A3) and np.array_equal(A2, A3)   # AUTO now runs the measured mode
    assert normwise(A1, B).max() <= TOL["fp64"]
    felocal.lib().fe_autotune_clear()
    A4, _ = gpu_assemble(form, cell, p, coords, cf)             # Algorithm 3's mode again
    assert normwise(A4, B).max() <= TOL["fp64"]


BAD_SHAPES = [
    ("helmholtz", "tetrahedron", 4, "preeval", dict(kernel=2, block=256, epi=2)),   # 2450 > 8 * 256 slots
    ("helmholtz", "prism", 4, "preeval", dict(kernel=2, block=512, epi=1)),         # 5625 > 8 * 512 slots
    ("helmholtz", "tetrahedron", 2, "preeval", dict(kernel=1, block=256, epi=3, chunk=10)),   # not a multiple
    ("helmholtz", "tetrahedron", 2, "preeval", dict(kernel=2, block=256, epi=3, chunk=10)),   # of epi
    ("helmholtz", "tetrahedron", 2, "preeval", dict(block=1024)),                   # above the kernel's bound
    ("helmholtz", "tetrahedron", 2, "preeval", dict(block=96)),                     # not whole wavefronts
    ("helmholtz", "tetrahedron", 2, "preeval", dict(block=256, epi=300)),           # epi above block
    ("helmholtz", "tetrahedron", 2, "preeval", dict(kernel=1, block=256, epi=1, chunk=100000)),   # LDS limit
    ("elasticity", "tetrahedron", 2, "quadrature", dict(kernel=3, qc=1000)),        # more points than the rule
    ("elasticity", "tetrahedron", 2, "quadrature", dict(kernel=3, eb=100000)),      # LDS above the limit
    ("elasticity", "tetrahedron", 3, "quadrature", dict(kernel=4)),                 # n = 60 > 32
    ("elasticity", "tetrahedron", 2, "quadrature", dict(kernel=2)),                 # a pre-evaluated kernel
    ("helmholtz", "tetrahedron", 2, "preeval", dict(kernel=4)),                     # a quadrature kernel
    ("helmholtz", "prism", 4, "quadrature", dict(kernel=4)),                        # n = 75 > 48
]


@pytest.mark.parametrize("form,cell,p,mode,shape", BAD_SHAPES)
def test_bad_shapes_rejected(form, cell, p, mode, shape):
    log(f"rejected shape {form} {cell} P{p} {mode} {shape}")
    coords, V, cells, h = mesh(cell, 50, seed=3)
    cf = coefficients(form, cell, p, 50, V, cells, h, seed=4)
    n, _ = felocal.fe_local_dims(form, cell, p)
    out = torch.full((50, n, n), float("nan"), dtype=torch.float64, device="cuda")
    with pytest.raises(felocal.FeError):
        felocal.fe_assemble_local(form, cell, p, dev(coords), dev(cf) if cf is not None else None, out,
                                  mode=mode, shape=shape)
    torch.cuda.synchronize()
    assert torch.isnan(out).all()


MFMA_CELLS = [("triangle", 1), ("triangle", 2), ("triangle", 3), ("triangle", 4), ("tetrahedron", 1),
              ("tetrahedron", 2), ("prism", 1)]
VECTOR_MFMA_CASES = [(f, c, p) for f in ("elasticity", "hyperelastic") for (c, p) in MFMA_CELLS]


@pytest.mark.parametrize("kernel", [3, 4])
@pytest.mark.parametrize("form,cell,p", VECTOR_MFMA_CASES)
def test_fp64_vector_kernels(form, cell, p, kernel):
    """Both float64 quadrature kernels of the vector forms: the VALU kernel
    (3) and the matrix-core Gram kernel (4)."""
    E = case_size(form, cell, p, cap=700)
    log(f"fp64 vector kernel {kernel} {form} {cell} P{p} E={E}")
    coords, V, cells, h = mesh(cell, E, seed=300 + p)
    cf = coefficients(form, cell, p, E, V, cells, h, seed=400 + p)
    A, st = gpu_assemble(form, cell, p, coords, cf, shape=dict(kernel=kernel), mode="quadrature")
    B, fl = oracle.assemble(form, cell, p, coords, cf)
    bad = np.isnan(B[:, 0, 0])
    assert st == fl == bad.sum()
    assert (np.isnan(A[:, 0, 0]) == bad).all() and np.isfinite(A[~bad]).all()
    assert normwise(A[~bad], B[~bad]).max() <= TOL["fp64"]


# Pre-evaluated elasticity (the P1 Lame fields expanded, iota = n_c): every
# cell and degree forced into the mode, several 16-element tiles, a
# degenerate element; where Algorithm 3 chooses it the default is the same.
ELAST_PRE = [(c, p) for c in CELLS for p in (1, 2, 3, 4)]


@pytest.mark.parametrize("cell,p", ELAST_PRE)
def test_elasticity_preevaluated(cell, p):
    E = max(5, min(70, case_size("elasticity", cell, p, cap=70)))
    log(f"elasticity pre-evaluated {cell} P{p} E={E}")
    coords, V, cells, h = mesh(cell, E, seed=500 + p)
    coords = coords.copy()
    coords[E // 2, 2] = coords[E // 2, 0]            # degenerate map
    cf = coefficients("elasticity", cell, p, E, V, cells, h, seed=510 + p)
    B, fl = oracle.assemble("elasticity", cell, p, coords, cf)
    bad = np.isnan(B[:, 0, 0])
    assert bad[E // 2] and fl == bad.sum()
    A, st = gpu_assemble("elasticity", cell, p, coords, cf, mode="preeval")
    assert st == fl
    assert (np.isnan(A[:, 0, 0]) == bad).all() and np.isnan(A[bad]).all() and np.isfinite(A[~bad]).all()
    assert normwise(A[~bad], B[~bad]).max() <= TOL["fp64"]
    if felocal.fe_plan("elasticity", cell, p)["mode"] == "preeval":
        A2, _ = gpu_assemble("elasticity", cell, p, coords, cf)
        assert np.array_equal(A2[~bad], A[~bad])


@pytest.mark.parametrize("cell,p,E", [("tetrahedron", 4, 2103), ("prism", 4, 1213), ("triangle", 4, 3005)])
def test_elasticity_preevaluated_many_units(cell, p, E):
    """More units (a few elements and one block row each) than wavefronts,
    so every wavefront takes several, and a ragged last unit: sampled
    elements (every 17th and the last 20) against the oracle, at one and two
    workgroups per CU."""
    log(f"elasticity pre-evaluated, many units: {cell} P{p} E={E}")
    coords, V, cells, h = mesh(cell, E, seed=540)
    cf = coefficients("elasticity", cell, p, E, V, cells, h, seed=541)
    idx = np.unique(np.r_[np.arange(0, E, 17), np.arange(E - 20, E)])
    B, fl = oracle.assemble("elasticity", cell, p, coords[idx], cf[idx])
    assert fl == 0
    for g in (1, 2):
        A, st = gpu_assemble("elasticity", cell, p, coords, cf, mode="preeval", shape={"grid_per_cu": g})
        assert st == 0
        assert np.isfinite(A).all()
        assert normwise(A[idx], B).max() <= TOL["fp64"]


@pytest.mark.parametrize("cell,p", [(c, p) for c in CELLS for p in (1, 4)])
@pytest.mark.parametrize("E", [1, 2, 7])
def test_elasticity_preevaluated_few_elements(cell, p, E):
    """Fewer elements than one unit (triangles take 8 per unit, tetrahedra 5)
    or a single partial unit: most wavefronts of the grid idle, and the
    padding rows of the unit's tiles must not be stored."""
    log(f"elasticity pre-evaluated, few elements: {cell} P{p} E={E}")
    coords, V, cells, h = mesh(cell, E, seed=570 + E)
    cf = coefficients("elasticity", cell, p, E, V, cells, h, seed=571 + E)
    B, fl = oracle.assemble("elasticity", cell, p, coords, cf)
    assert fl == 0
    A, st = gpu_assemble("elasticity", cell, p, coords, cf, mode="preeval")
    assert st == 0 and np.isfinite(A).all()
    assert normwise(A, B).max() <= TOL["fp64"]


# Forced quadrature for elasticity where Algorithm 3 pre-evaluates (P4) or
# where only the VALU kernel serves (n > 32): the float64 VALU kernel.
@pytest.mark.parametrize("cell,p", [("tetrahedron", 4), ("prism", 4), ("triangle", 4), ("prism", 3),
                                    ("tetrahedron", 3)])
def test_elasticity_quadrature_high_degree(cell, p):
    E = case_size("elasticity", cell, p, cap=400)
    log(f"elasticity forced quadrature {cell} P{p} E={E}")
    coords, V, cells, h = mesh(cell, E, seed=560 + p)
    cf = coefficients("elasticity", cell, p, E, V, cells, h, seed=570 + p)
    B, fl = oracle.assemble("elasticity", cell, p, coords, cf)
    assert fl == 0
    A, st = gpu_assemble("elasticity", cell, p, coords, cf, mode="quadrature")
    assert st == 0 and np.isfinite(A).all()
    assert normwise(A, B).max() <= TOL["fp64"]
    A3, _ = gpu_assemble("elasticity", cell, p, coords, cf, mode="quadrature", shape={"kernel": 3})
    assert normwise(A3, B).max() <= TOL["fp64"]


def test_release_caches_then_rebuild():
    """Releasing every cache between calls (reference, coefficient and
    elasticity tables, autotune entries) rebuilds them on the next call with
    the same results."""
    cases = [("helmholtz", "tetrahedron", 2, {}), ("mass", "tetrahedron", 2, {"nf": 1}),
             ("elasticity", "tetrahedron", 4, {"mode": "preeval"}), ("hyperelastic", "tetrahedron", 1, {})]
    runs = []
    for form, cell, p, kw in cases:
        coords, V, cells, h = mesh(cell, 40, seed=530)
        if kw.get("nf"):
            cf = np.random.default_rng(531).uniform(0.5, 1.5, size=(40, 1, oracle.nbasis(cell, p)))
        else:
            cf = coefficients(form, cell, p, 40, V, cells, h, seed=532)
        runs.append((form, cell, p, kw, coords, cf))
    first = [gpu_assemble(form, cell, p, coords, cf, **kw)[0] for form, cell, p, kw, coords, cf in runs]
    torch.cuda.synchronize()
    felocal.lib().fe_release_caches()
    second = [gpu_assemble(form, cell, p, coords, cf, **kw)[0] for form, cell, p, kw, coords, cf in runs]
    for a, b in zip(first, second):
        assert np.array_equal(a, b)


def test_elasticity_preevaluated_refusals():
    coords, V, cells, h = mesh("tetrahedron", 20, seed=520)
    u = coefficients("hyperelastic", "tetrahedron", 2, 20, V, cells, h, seed=521)
    with pytest.raises(felocal.FeError) as ei:
        gpu_assemble("hyperelastic", "tetrahedron", 2, coords, u, mode="preeval")
    assert ei.value.code == felocal.FE_ENOTSUP
    cf = coefficients("elasticity", "tetrahedron", 2, 20, V, cells, h, seed=522)
    for prec in ("fp32", "bf16x3"):
        with pytest.raises(felocal.FeError) as ei:
            gpu_assemble("elasticity", "tetrahedron", 2, coords, cf, mode="preeval", precision=prec)
        assert ei.value.code == felocal.FE_ENOTSUP


# The hoisted degree-1 kernel (shape kernel 5, the default there): several
# 128-element tiles and a ragged tail, degenerate and inverted elements.
@pytest.mark.parametrize("form", ["elasticity", "hyperelastic"])
@pytest.mark.parametrize("cell", ["triangle", "tetrahedron"])
def test_degree1_vector_kernel(form, cell):
    E = 1000
    log(f"degree-1 vector kernel {form} {cell} E={E}")
    coords, V, cells, h = mesh(cell, E, seed=71)
    coords = coords.copy()
    coords[5, 1] = coords[5, 0]                      # degenerate map
    cf = coefficients(form, cell, 1, E, V, cells, h, seed=72)
    if form == "hyperelastic":
        cf = cf.copy()
        cf[[17, 300, 999]] *= 60.0                   # large displacements: inverted F somewhere
    B, fl = oracle.assemble(form, cell, 1, coords, cf)
    bad = np.isnan(B[:, 0, 0])
    assert bad[5] and fl == bad.sum()
    for kw in ({}, {"shape": {"kernel": 5}}, {"shape": {"kernel": 5, "grid_per_cu": 1}}):
        A, st = gpu_assemble(form, cell, 1, coords, cf, **kw)
        assert st == fl
        assert (np.isnan(A[:, 0, 0]) == bad).all() and np.isnan(A[bad]).all() and np.isfinite(A[~bad]).all()
        assert normwise(A[~bad], B[~bad]).max() <= TOL["fp64"]
    # the VALU kernel agrees element by element
    A3, _ = gpu_assemble(form, cell, 1, coords, cf, shape={"kernel": 3})
    assert normwise(A3[~bad], A[~bad]).max() <= 1e-13
    # one element, and the last tile holding a single element
    for n1 in (1, 129):
        A1, st1 = gpu_assemble(form, cell, 1, coords[:n1], cf[:n1], shape={"kernel": 5})
        assert st1 == bad[:n1].sum() and normwise(A1[~bad[:n1]], B[:n1][~bad[:n1]]).max() <= TOL["fp64"]


def test_degree1_vector_kernel_refusals():
    coords, V, cells, h = mesh("tetrahedron", 50, seed=73)
    for form, cell, p, kw in (("elasticity", "tetrahedron", 2, {}), ("hyperelastic", "prism", 1, {}),
                              ("mass", "tetrahedron", 1, {"mode": "quadrature"}),
                              ("hyperelastic", "tetrahedron", 1, {"precision": "bf16x3"})):
        c2, V2, cells2, h2 = mesh(cell, 50, seed=73)
        cf = coefficients(form, cell, p, 50, V2, cells2, h2, seed=74)
        with pytest.raises(felocal.FeError) as ei:
            gpu_assemble(form, cell, p, c2, cf, shape={"kernel": 5}, **kw)
        assert ei.value.code == felocal.FE_EINVAL


# Forms pre-multiplied by nf coefficient functions (the sweep of Sec. 7.1):
# the planner's choice, forced quadrature, and forced pre-evaluation where
# a 16-element tile of the expanded geometry tensor fits in LDS.
NF_CASES = [(f, c, p, nf) for f in ("mass", "helmholtz")
            for (c, p) in [("tetrahedron", 1), ("tetrahedron", 2), ("tetrahedron", 3), ("tetrahedron", 4),
                           ("triangle", 2), ("prism", 1)] for nf in (1, 2, 3)]


def _coef_lds_bytes(form, cell, p, nf):
    from math import comb
    ns = oracle.nbasis(cell, p)
    nr = 1 if form == "mass" else 1 + oracle.TDIM[cell] * (oracle.TDIM[cell] + 1) // 2
    ntp = (nr * comb(ns + nf - 1, nf) + 7) // 8 * 8
    return 8 * 16 * (ntp + nr + nf * ns)


@pytest.mark.parametrize("mode", ["auto", "quadrature", "preeval"])
@pytest.mark.parametrize("form,cell,p,nf", NF_CASES)
def test_coefficient_functions(form, cell, p, nf, mode):
    ns = oracle.nbasis(cell, p)
    nq = oracle.rule(cell, oracle.default_qdeg(form, cell, p, nf))[1].size
    E = int(max(7, min(700, 1.5e9 / (nq * ns * ns * 10))))
    log(f"coefficient functions {form} {cell} P{p} nf={nf} {mode} E={E}")
    coords, *_ = mesh(cell, E, seed=40 + p)
    rng = np.random.default_rng(50 + nf)
    cf = rng.uniform(0.5, 1.5, size=(E, nf, ns))
    lds = _coef_lds_bytes(form, cell, p, nf)
    if mode == "preeval" and lds > 160 * 1024:      # above any LDS per block: rejected up front
        with pytest.raises(felocal.FeError):
            gpu_assemble(form, cell, p, coords, cf, nf=nf, mode=mode)
        return
    try:
        A, st = gpu_assemble(form, cell, p, coords, cf, nf=nf, mode=mode)
    except felocal.FeError:
        assert mode == "preeval" and lds > 64 * 1024   # only where the device's limit decides
        return
    B, fl = oracle.assemble(form, cell, p, coords, cf, nf=nf)
    assert st == fl == 0
    assert normwise(A, B).max() <= TOL["fp64"]


# Mixed Helmholtz plans with coefficient functions: the quadrature kernel
# evaluates one monomial and the coefficient pre-evaluation adds the other.
# `want` is the plan (gradient monomial, mass monomial pre-evaluated); T_H is
# set to the table bytes of the monomials that plan pre-evaluates, so that
# Algorithm 3's step 3 discards every plan with more tables (Constraint 2).
MIXED_NF = [("tetrahedron", 3, 1, (False, True)), ("tetrahedron", 3, 1, (True, False)),
            ("tetrahedron", 1, 1, (False, True)), ("tetrahedron", 2, 2, (False, True)),
            ("triangle", 3, 1, (True, False)), ("triangle", 2, 2, (False, True)),
            ("prism", 2, 1, (False, True)), ("prism", 2, 1, (True, False))]


def mixed_th(cell, p, nf, want):
    """T_H that holds exactly the tables of the wanted monomials."""
    full = felocal.fe_plan("helmholtz", cell, p, nf=nf, th_bytes=1 << 40)
    return sum(b for b, w in zip(full["table_bytes"], want) if w)


@pytest.mark.parametrize("cell,p,nf,want", MIXED_NF)
def test_coefficient_mixed_plans(cell, p, nf, want):
    th = mixed_th(cell, p, nf, want)
    plan = felocal.fe_plan("helmholtz", cell, p, nf=nf, th_bytes=th)
    log(f"mixed plan helmholtz {cell} P{p} nf={nf} th={th}: {plan['preevaluated']}")
    assert tuple(plan["preevaluated"]) == want, plan
    ns = oracle.nbasis(cell, p)
    E = 300
    coords, *_ = mesh(cell, E, seed=60 + p)
    cf = np.random.default_rng(61).uniform(0.5, 1.5, size=(E, nf, ns))
    B, fl = oracle.assemble("helmholtz", cell, p, coords, cf, nf=nf)
    # the quadrature part on both quadrature kernels (VALU, matrix core)
    for kernel in (3, 4):
        log(f"   quadrature kernel {kernel}")
        A, st = gpu_assemble("helmholtz", cell, p, coords, cf, nf=nf, th_bytes=th, shape={"kernel": kernel})
        assert st == fl == 0
        assert normwise(A, B).max() <= TOL["fp64"]


# The vector forms pre-multiplied by nf functions (the Sec. 7.1 matrix for
# Elasticity and Hyperelasticity): Algorithm 3's choice (the hyperelastic
# trace term pre-evaluated by the coefficient kernel on top of the VALU
# kernel where it pays), forced quadrature, and forced pre-evaluation
# (elasticity, where its tile fits the LDS; illegal for the hyperelastic
# terms in F).
VEC_NF_CASES = [(f, c, p, nf) for f in ("elasticity", "hyperelastic")
                for (c, p) in [("tetrahedron", 1), ("tetrahedron", 2), ("tetrahedron", 3), ("triangle", 2),
                               ("triangle", 4), ("prism", 1)] for nf in (1, 2, 3)]


def vec_nf_coeff(form, cell, p, E, V, cells, h, nf, seed):
    own = coefficients(form, cell, p, E, V, cells, h, seed).reshape(E, -1)
    f = np.random.default_rng(seed + 1).uniform(0.5, 1.5, size=(E, nf * oracle.nbasis(cell, p)))
    return np.ascontiguousarray(np.concatenate([own, f], axis=1))


def _elast_coef_lds_bytes(cell, p, nf):
    from math import comb
    ns, nc, d = oracle.nbasis(cell, p), oracle.NVERT[cell], oracle.TDIM[cell]
    iota = comb(ns + nf - 1, nf)
    ntp = (nc * iota * d * d + 7) // 8 * 8
    return 8 * 16 * (ntp + 12 + 2 * nc + nf * ns + iota)


@pytest.mark.parametrize("mode", ["auto", "quadrature", "preeval"])
@pytest.mark.parametrize("form,cell,p,nf", VEC_NF_CASES)
def test_vector_coefficient_functions(form, cell, p, nf, mode):
    ns, d = oracle.nbasis(cell, p), oracle.TDIM[cell]
    nq = oracle.rule(cell, oracle.default_qdeg(form, cell, p, nf))[1].size
    E = int(max(7, min(400, 1.5e9 / (nq * (d * ns) ** 2 * 40))))
    log(f"vector coefficient functions {form} {cell} P{p} nf={nf} {mode} E={E}")
    coords, V, cells, h = mesh(cell, E, seed=90 + p)
    cf = vec_nf_coeff(form, cell, p, E, V, cells, h, nf, seed=95 + nf)
    if mode == "preeval" and form == "hyperelastic":
        with pytest.raises(felocal.FeError) as ei:
            gpu_assemble(form, cell, p, coords, cf, nf=nf, mode=mode)
        assert ei.value.code == felocal.FE_ENOTSUP
        return
    lds = _elast_coef_lds_bytes(cell, p, nf)
    if mode == "preeval" and lds > 160 * 1024:
        with pytest.raises(felocal.FeError):
            gpu_assemble(form, cell, p, coords, cf, nf=nf, mode=mode)
        return
    try:
        A, st = gpu_assemble(form, cell, p, coords, cf, nf=nf, mode=mode)
    except felocal.FeError:
        assert mode == "preeval" and lds > 64 * 1024   # only where the device's limit decides
        return
    B, fl = oracle.assemble(form, cell, p, coords, cf, nf=nf)
    bad = np.isnan(B[:, 0, 0])
    assert st == fl == bad.sum() and fl <= E // 50
    assert (np.isnan(A[:, 0, 0]) == bad).all() and np.isfinite(A[~bad]).all()
    assert normwise(A[~bad], B[~bad]).max() <= TOL["fp64"]


@pytest.mark.parametrize("cell,p,nf", [("tetrahedron", 1, 1), ("tetrahedron", 2, 2), ("triangle", 3, 1),
                                       ("prism", 2, 1)])
def test_hyperelastic_trace_preevaluated(cell, p, nf):
    """A plan that pre-evaluates the hyperelastic trace term with nf
    functions (Algorithm 3 with iota = C(n_s + nf - 1, nf)): the coefficient
    kernel adds it to the diagonal blocks after the VALU kernel, and the
    result equals forced quadrature and the oracle; flagged elements (a
    degenerate map, an inverted point) stay NaN."""
    plan = felocal.fe_plan("hyperelastic", cell, p, nf=nf)
    assert plan["preevaluated"] == [False, True], plan
    E = 300
    log(f"hyperelastic trace pre-evaluated {cell} P{p} nf={nf}")
    coords, V, cells, h = mesh(cell, E, seed=97)
    coords = coords.copy()
    coords[11, 1] = coords[11, 0]
    cf = vec_nf_coeff("hyperelastic", cell, p, E, V, cells, h, nf, seed=98)
    cf[[40, 200], :d_ns(cell, p)] *= 40.0
    B, fl = oracle.assemble("hyperelastic", cell, p, coords, cf, nf=nf)
    bad = np.isnan(B[:, 0, 0])
    assert bad[11] and fl == bad.sum() >= 2
    A, st = gpu_assemble("hyperelastic", cell, p, coords, cf, nf=nf)
    Aq, stq = gpu_assemble("hyperelastic", cell, p, coords, cf, nf=nf, mode="quadrature")
    assert st == stq == fl
    for X in (A, Aq):
        assert (np.isnan(X[:, 0, 0]) == bad).all() and np.isnan(X[bad]).all() and np.isfinite(X[~bad]).all()
        assert normwise(X[~bad], B[~bad]).max() <= TOL["fp64"]


def d_ns(cell, p):
    return oracle.TDIM[cell] * oracle.nbasis(cell, p)


# Indefinite point weights: a Lame field shifted below zero (lambda or mu),
# and a negative hyperelastic lambda, through every precision.
SIGNED_CASES = [("elasticity", "tetrahedron", 2, 0), ("elasticity", "triangle", 3, 0),
                ("elasticity", "tetrahedron", 1, 1), ("elasticity", "prism", 1, 1),
                ("hyperelastic", "tetrahedron", 2, 0), ("hyperelastic", "triangle", 2, 0)]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("form,cell,p,field", SIGNED_CASES)
def test_negative_coefficients(form, cell, p, field, prec):
    E = 300
    log(f"signed weights {form} {cell} P{p} field={field} {prec}")
    coords, V, cells, h = mesh(cell, E, seed=31)
    kw = {}
    if form == "elasticity":
        cf = inputs.lame_p1(V.shape[0], cells, seed=32).copy()
        cf[:, field, :] -= 1.1 if field == 0 else 0.9    # values in [-0.6, 0.9] or [-0.4, 1.1]
    else:
        cf = coefficients(form, cell, p, E, V, cells, h, seed=33)
        kw = dict(mu=1.0, lam=-0.4)
    A, st = gpu_assemble(form, cell, p, coords, cf, precision=prec, **kw)
    B, fl = oracle.assemble(form, cell, p, coords, cf, **kw)
    bad = np.isnan(B[:, 0, 0])
    assert st == fl == bad.sum()
    assert normwise(A[~bad], B[~bad]).max() <= TOL[prec]


SPLIT_CASES = [(f, c, p) for f in ("elasticity", "hyperelastic") for (c, p) in
               [("triangle", 1), ("triangle", 2), ("triangle", 3), ("triangle", 4), ("tetrahedron", 1),
                ("tetrahedron", 2), ("prism", 1)]]


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
@pytest.mark.parametrize("form,cell,p", SPLIT_CASES)
def test_split_parity(form, cell, p, prec):
    E = case_size(form, cell, p, cap=700)
    log(f"split parity {form} {cell} P{p} {prec} E={E}")
    coords, V, cells, h = mesh(cell, E, seed=300 + p)
    cf = coefficients(form, cell, p, E, V, cells, h, seed=400 + p)
    B, fl = oracle.assemble(form, cell, p, coords, cf)
    bad = np.isnan(B[:, 0, 0])          # det F <= 0 somewhere: flagged on both sides
    # degree 1 on a simplex: the default is the float64 hoisted kernel; the
    # matrix-core split kernel stays reachable with shape kernel 4
    runs = [({}, TOL[prec])]
    if p == 1 and cell != "prism":
        runs = [({}, TOL["fp64"]), ({"shape": {"kernel": 4}}, TOL[prec])]
    for kw, tol in runs:
        A, st = gpu_assemble(form, cell, p, coords, cf, precision=prec, **kw)
        assert st == fl == bad.sum() and fl <= E // 100
        assert (np.isnan(A[:, 0, 0]) == bad).all()
        err = normwise(A[~bad], B[~bad])
        log(f"   {kw} max err {err.max():.3e}")
        assert err.max() <= tol


@pytest.mark.parametrize("form", ["mass", "helmholtz", "elasticity", "hyperelastic"])
def test_degenerate_elements_flagged(form):
    log(f"flagged {form}")
    coords, V, cells, h = mesh("tetrahedron", 50, seed=3)
    coords = coords.copy()
    coords[7, 2] = coords[7, 1]            # two coincident vertices
    coords[31, 3] = coords[31, 0]
    cf = coefficients(form, "tetrahedron", 2, 50, V, cells, h, seed=5)
    precs = ["fp64", "bf16x3"] if form in ("elasticity", "hyperelastic") else ["fp64"]
    for prec in precs:
        A, st = gpu_assemble(form, "tetrahedron", 2, coords, cf, precision=prec)
        assert st == 2
        assert np.isnan(A[[7, 31]]).all()
        ok = np.ones(50, bool)
        ok[[7, 31]] = False
        assert np.isfinite(A[ok]).all()


def test_hyperelastic_inverted_points_flagged_like_oracle():
    log("hyperelastic inversion")
    coords, V, cells, h = mesh("tetrahedron", 200, seed=9)
    u = inputs.displacement_dofs(200, 3, 10, h, seed=10, rel=0.3)
    B, fl = oracle.assemble("hyperelastic", "tetrahedron", 2, coords, u)
    bad = np.isnan(B[:, 0, 0])
    assert fl == bad.sum() and 0 < fl < 200
    for prec in ("fp64", "bf16x3", "fp32"):
        A, st = gpu_assemble("hyperelastic", "tetrahedron", 2, coords, u, precision=prec)
        assert st == fl
        assert (np.isnan(A[:, 0, 0]) == bad).all()
        assert normwise(A[~bad], B[~bad]).max() <= TOL[prec]


def test_empty_and_coverage():
    log("empty and coverage")
    coords, *_ = mesh("tetrahedron", 300, seed=4)
    n = 10
    for mode in ("preeval", "quadrature"):
        buf = torch.full((300 * n * n + 64,), float("nan"), dtype=torch.float64, device="cuda")
        buf[-64:] = 12345.0
        out = buf[:300 * n * n].view(300, n, n)
        felocal.fe_assemble_local("helmholtz", "tetrahedron", 2, dev(coords), None, out, mode=mode)
        torch.cuda.synchronize()
        b = buf.cpu().numpy()
        assert np.isfinite(b[:-64]).all()
        assert (b[-64:] == 12345.0).all()
    empty = torch.zeros((0, 4, 3), dtype=torch.float64, device="cuda")
    outE = torch.zeros((0, n, n), dtype=torch.float64, device="cuda")
    felocal.fe_assemble_local("helmholtz", "tetrahedron", 2, empty, None, outE)


def test_nonaffine_prism_rejected_or_flagged():
    log("non-affine prism")
    coords, *_ = mesh("prism", 20, seed=6)
    coords = coords.copy()
    coords[5, 4, 2] += 0.01
    with pytest.raises(felocal.FeError) as ei:
        gpu_assemble("mass", "prism", 1, coords, validate=True)
    assert ei.value.code == felocal.FE_ENONAFFINE
    A, st = gpu_assemble("mass", "prism", 1, coords)
    assert st == 1 and np.isnan(A[5]).all() and np.isfinite(np.delete(A, 5, axis=0)).all()


def test_batch_bitwise_equal_to_separate_calls():
    log("batch vs separate calls")
    rng = np.random.default_rng(5)
    # groups with several sub-batches (mass triangles P1 and P2, Helmholtz
    # tetrahedra P2 and P3, elasticity tetrahedra P2 twice) and an empty one
    specs = [("mass", "triangle", 1, 3000), ("helmholtz", "tetrahedron", 3, 1500), ("elasticity", "prism", 2, 200),
             ("helmholtz", "prism", 4, 60), ("elasticity", "tetrahedron", 2, 999), ("mass", "prism", 3, 0),
             ("helmholtz", "triangle", 4, 777), ("helmholtz", "tetrahedron", 2, 2500), ("mass", "triangle", 2, 1234),
             ("elasticity", "tetrahedron", 2, 321), ("elasticity", "tetrahedron", 4, 45), ("elasticity", "prism", 4, 9)]
    subs, refs = [], []
    for i, (form, cell, p, E) in enumerate(specs):
        coords, V, cells, h = mesh(cell, max(E, 1), seed=20 + i)
        coords = coords[:E]
        cf = coefficients(form, cell, p, E, V, cells[:E], h, seed=30 + i) if E else None
        n, _ = felocal.fe_local_dims(form, cell, p)
        out = torch.full((E, n, n), float("nan"), dtype=torch.float64, device="cuda")
        subs.append(dict(form=form, cell=cell, degree=p, coords=dev(coords),
                         coeff=dev(cf) if cf is not None else None, out=out))
        if E:
            # the batch runs every sub-batch with the kernel and shape of a
            # single call (grouped tiles, single launches, pre-evaluated elasticity)
            ref = gpu_assemble(form, cell, p, coords, cf)[0]
            assert normwise(ref, oracle.assemble(form, cell, p, coords, cf)[0]).max() <= TOL["fp64"]
            refs.append(ref)
        else:
            refs.append(np.zeros((0, n, n)))
    b = felocal.Batch(subs)
    ntiles, grid = b.info()
    assert ntiles >= 0 and grid >= 0
    results = []
    for rep in range(3):
        for s in subs:
            s["out"].fill_(float("nan"))
        b.run()
        torch.cuda.synchronize()
        results.append([s["out"].cpu().numpy() for s in subs])
        _ = torch.ones(1000, device="cuda").sum().item()   # unrelated eager work between replays
    b.close()
    for res in results:
        for got, ref in zip(res, refs):
            assert np.array_equal(got, ref)


# --------------------------------------------------------------------------
# Full-size workloads, sampled elements
# --------------------------------------------------------------------------

def _sample(E, k, seed, window=512):
    """k random elements plus three contiguous windows (the first, a middle
    and the last `window` elements: whole visits of the persistent grids and
    the ragged tail)."""
    rng = np.random.default_rng(seed)
    w = min(window, E)
    mid = max(0, E // 2 - w // 2)
    idx = np.unique(np.concatenate([rng.integers(0, E, size=k), np.arange(w), np.arange(mid, mid + w),
                                    np.arange(E - w, E)]))
    return idx


def _nan_out(E, n):
    return torch.full((E, n, n), float("nan"), dtype=torch.float64, device="cuda")


def _compare_all(A, R, tol, chunk=1 << 14):
    """Every element of A (device) against R (device, float64 GPU output that
    the oracle checks on its samples): the same NaN (flagged) elements, and
    the normwise error of the rest within tol."""
    worst = 0.0
    for s in range(0, A.shape[0], chunk):
        a, r = A[s:s + chunk], R[s:s + chunk]
        bad_r = torch.isnan(r).flatten(1).any(1)
        bad_a = torch.isnan(a).flatten(1).any(1)
        assert torch.equal(bad_a, bad_r), f"flagged sets differ in [{s}, {s + a.shape[0]})"
        ok = ~bad_r
        if ok.any():
            num = (a[ok] - r[ok]).abs().flatten(1).amax(1)
            den = r[ok].abs().flatten(1).amax(1)
            worst = max(worst, float((num / den).max()))
    assert worst <= tol, worst
    return worst


def _full_check(form, cell, p, coords, cf, precs, k=64, extra_idx=None):
    """Full-size run of each precision into a NaN-filled output: sampled
    elements against the oracle; the split precisions also element by element
    against the float64 GPU output of the same launch configuration."""
    n, _ = felocal.fe_local_dims(form, cell, p)
    E = coords.shape[0]
    dc = dev(coords)
    dcf = dev(cf) if cf is not None else None
    idx = _sample(E, k, seed=E)
    if extra_idx is not None:
        idx = np.unique(np.concatenate([idx, extra_idx]))
    B, fl = oracle.assemble(form, cell, p, coords[idx], cf[idx] if cf is not None else None)
    bad = np.isnan(B[:, 0, 0])
    ref = None
    for prec in precs:
        log(f"   {prec}: {E} elements, {idx.size} sampled")
        out = _nan_out(E, n)
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        felocal.fe_assemble_local(form, cell, p, dc, dcf, out, precision=prec, status=status)
        torch.cuda.synchronize()
        A = out[torch.from_numpy(idx).cuda()].cpu().numpy()
        assert (np.isnan(A[:, 0, 0]) == bad).all()
        assert np.isnan(A[bad]).all() and np.isfinite(A[~bad]).all()
        assert normwise(A[~bad], B[~bad]).max() <= TOL[prec]
        if prec == "fp64":
            ref = out
        else:
            assert ref is not None
            log(f"   {prec} vs fp64, every element: {_compare_all(out, ref, TOL[prec]):.3e}")
            del out
        yield int(status.item())
    del ref
    torch.cuda.empty_cache()


def test_full_mass_triangles_4096():
    log("full: mass P1 triangles 4096")
    coords = inputs.mass_tri_workload(seed=1)
    for st in _full_check("mass", "triangle", 1, coords, None, ["fp64"], k=4096):
        assert st == 0


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_full_helmholtz_tets_750k(p):
    log(f"full: helmholtz P{p} 750k tets")
    coords, _, _ = inputs.tet_workload(50, seed=2)
    for st in _full_check("helmholtz", "tetrahedron", p, coords, None, ["fp64"]):
        assert st == 0


def test_full_elasticity_p2_tets_2m():
    log("full: elasticity P2 1.97M tets")
    coords, V, cells = inputs.tet_workload(69, seed=3)
    cf = inputs.lame_p1(V.shape[0], cells, seed=3)
    for st in _full_check("elasticity", "tetrahedron", 2, coords, cf, ["fp64", "fp32", "bf16x3"]):
        assert st == 0


@pytest.mark.parametrize("p", [1, 2])
def test_full_hyperelastic_tets_1m(p):
    log(f"full: hyperelastic P{p} 998k tets")
    coords, V, cells = inputs.tet_workload(55, seed=4)
    u = inputs.displacement_dofs(coords.shape[0], 3, oracle.nbasis("tetrahedron", p), 1.0 / 55, seed=40 + p)
    flagged = np.nonzero(oracle.hyper_min_jf("tetrahedron", p, coords, u) <= 0)[0]
    for st in _full_check("hyperelastic", "tetrahedron", p, coords, u, ["fp64", "fp32", "bf16x3"],
                          extra_idx=flagged):
        assert st == len(flagged)


def test_fe_log_reports_each_dispatch(monkeypatch, capfd):
    """FE_LOG=1: one line on stderr per fe_assemble_local call with the mode,
    precision and launch configuration."""
    c, V, cells, h = inputs.first_elements("tetrahedron", 1000, 61)
    dc = torch.from_numpy(c).cuda()
    out = torch.empty((1000, 10, 10), dtype=torch.float64, device="cuda")
    capfd.readouterr()
    monkeypatch.setenv("FE_LOG", "1")
    felocal.fe_assemble_local("helmholtz", "tetrahedron", 2, dc, None, out)
    felocal.fe_assemble_local("mass", "tetrahedron", 2, dc, None, out, mode="quadrature")
    torch.cuda.synchronize()
    monkeypatch.delenv("FE_LOG")
    felocal.fe_assemble_local("mass", "tetrahedron", 2, dc, None, out)
    torch.cuda.synchronize()
    lines = [l for l in capfd.readouterr().err.splitlines() if l.startswith("felocal: ")]
    assert len(lines) == 2, lines
    assert "helmholtz tetrahedron P2 E=1000" in lines[0] and "mode=preevaluated" in lines[0]
    assert "mass tetrahedron P2 E=1000" in lines[1] and "mode=quadrature" in lines[1] and "precision=fp64" in lines[1]

"""Host-side checks of the HIP library that need no GPU: exported symbols,
dimensions, the library's own quadrature rules, the planner (Algorithm 3 and
the cost function of Sec. 4.2) and synchronous argument errors."""
import ctypes
import json
import math
import os
import re

import numpy as np
import pytest

import exact_rational as er
import oracle
from paper_1604_05872_amd import felocal

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CELLS = ["triangle", "tetrahedron", "prism"]
GOLDEN = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_examples.json")))


def header_functions():
    src = open(os.path.join(ROOT, "include", "felocal.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fe_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = felocal.lib()
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(felocal.EXPORTS)
    assert "gfx950" in felocal.fe_version()


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_local_dims(cell, p):
    ns = oracle.nbasis(cell, p)
    d = oracle.TDIM[cell]
    assert felocal.fe_local_dims("mass", cell, p) == (ns, 0)
    assert felocal.fe_local_dims("helmholtz", cell, p) == (ns, 0)
    assert felocal.fe_local_dims("elasticity", cell, p) == (d * ns, 2 * oracle.NVERT[cell])
    assert felocal.fe_local_dims("hyperelastic", cell, p) == (d * ns, d * ns)


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("qdeg", list(range(0, 13)))
def test_library_rule_exact_and_equal_to_oracle(cell, qdeg):
    r = felocal.fe_tabulate(cell, 1, qdeg, rule_only=True)
    X, W = r["points"], r["weights"]
    assert abs(W.sum() - oracle.REF_VOLUME[cell]) < 1e-15
    D = max(qdeg, 0)
    mons = ([(a, b) for a in range(D + 1) for b in range(D + 1 - a)] if cell == "triangle" else
            [(a, b, c) for a in range(D + 1) for b in range(D + 1 - a) for c in range(D + 1 - a - b)]
            if cell == "tetrahedron" else
            [(a, b, c) for a in range(D + 1) for b in range(D + 1 - a) for c in range(D + 1)])
    for e in mons:
        approx = float(np.sum(W * np.prod(X ** np.array(e), axis=1)))
        assert abs(approx - float(er.integrate(cell, e))) < 2e-16 + 1e-14 * float(er.integrate(cell, e))
    # Gauss rules are unique: same point set and weights as the oracle's Newton construction
    Xo, Wo = oracle.rule(cell, max(qdeg, 0))
    ko = np.lexsort(Xo.T[::-1])
    kl = np.lexsort(X.T[::-1])
    assert np.max(np.abs(Xo[ko] - X[kl])) < 1e-14
    assert np.max(np.abs(Wo[ko] - W[kl])) < 1e-15


def test_planner_matches_paper_examples():
    # rho: mass monomial 1, 2D Poisson 3 (Sec. 4.2)
    pm = felocal.fe_plan("mass", "triangle", 2)
    assert pm["rho"] == [1] and pm["iota"] == [1]
    ph = felocal.fe_plan("helmholtz", "triangle", 2)
    assert ph["rho"][0] == GOLDEN["rho"][1]["value"] and ph["rho"][1] == GOLDEN["rho"][0]["value"]
    # iota = C(n+k-1, k): one P1 coefficient on a triangle (n = 3, k = 1) -> 3
    pe = felocal.fe_plan("elasticity", "triangle", 2)
    assert pe["iota"] == [GOLDEN["iota"][0]["value"]] * 2
    for ex in GOLDEN["iota"]:
        assert math.comb(ex["n"] + ex["k"] - 1, ex["k"]) == ex["value"]
    # Fig. 3: the inner (j,k) body of the sharing-eliminated 2D Poisson is 4 ops per (i,j,k)
    nq = oracle.rule("triangle", 4)[1].size
    ns = oracle.nbasis("triangle", 2)
    assert ph["theta_se"][0] == nq * ns * ns * GOLDEN["fig3_inner_ops_per_IJK"]["after_sharing_elimination_JK_term"]


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_planner_decisions(cell, p):
    big = 1 << 40
    # with no memory bound, the scalar forms pre-evaluate every monomial
    assert felocal.fe_plan("mass", cell, p, th_bytes=big)["mode"] == "preeval"
    assert felocal.fe_plan("helmholtz", cell, p, th_bytes=big)["mode"] == "preeval"
    # elasticity with P1 Lame fields: iota = n_c, rho = d^2 and 2 d^2, one
    # set of tables; pre-evaluated when theta <= 0 for both monomials
    pe = felocal.fe_plan("elasticity", cell, p, th_bytes=big)
    d, nc = (2, 3) if cell == "triangle" else (3, 4) if cell == "tetrahedron" else (3, 6)
    assert pe["iota"] == [nc, nc] and pe["rho"] == [d * d, 2 * d * d]
    both = all(tp <= ts for tp, ts in zip(pe["theta_pre"], pe["theta_se"]))
    assert pe["preevaluated"] == [both, both] and pe["mode"] == ("preeval" if both else "quadrature")
    if (cell, p) == ("tetrahedron", 2):   # the elasticity workload: theta > 0 for both monomials
        assert all(tp > ts for tp, ts in zip(pe["theta_pre"], pe["theta_se"]))
    if (cell, p) == ("tetrahedron", 4):   # 64 points: pre-evaluation pays for both
        assert pe["mode"] == "preeval"
    # tables over T_H: quadrature
    small = felocal.fe_plan("elasticity", cell, p, th_bytes=1024)
    assert small["mode"] == "quadrature" and not any(small["preevaluated"])
    phy = felocal.fe_plan("hyperelastic", cell, p, th_bytes=big)
    assert phy["mode"] == "quadrature" and math.isinf(phy["theta_pre"][0])
    # the trace monomial (constant coefficient) is pre-evaluated: with at least
    # two points its (2 rho + d) ops per pair beat nq * 3d
    d, ns = (2 if cell == "triangle" else 3), oracle.nbasis(cell, p)
    nq = oracle.rule(cell, oracle.default_qdeg("hyperelastic", cell, p))[1].size
    assert phy["n_monomials"] == 2 and phy["preevaluated"] == [False, nq * 3 * d > d * (d + 1) + d]
    assert phy["rho"][1] == d * (d + 1) // 2 and phy["iota"][1] == 1
    assert phy["theta_se"][0] + phy["theta_se"][1] == nq * ns * ns * (4 * d * d + 3 * d)
    assert phy["table_bytes"][1] == d * (d + 1) // 2 * ns * ns * 8


def test_planner_memory_threshold():
    # prism P4 Helmholtz: 6 stiffness tables (270 KB) exceed a 64 KiB T_H, the
    # mass table (45 KB) fits: a mixed plan (Fig. 5's two nests)
    p = felocal.fe_plan("helmholtz", "prism", 4, th_bytes=65536)
    assert p["preevaluated"] == [False, True] and p["mode"] == "quadrature"
    assert p["table_bytes"][0] == 6 * 75 * 75 * 8
    p = felocal.fe_plan("helmholtz", "prism", 4, th_bytes=1 << 30)
    assert p["preevaluated"] == [True, True] and p["mode"] == "preeval"
    p = felocal.fe_plan("helmholtz", "prism", 4, th_bytes=1000)
    assert p["preevaluated"] == [False, False]
    # tet P4 Helmholtz tables (7 x 35^2 x 8 = 68.6 KB) fit 160 KB, not 64 KiB
    assert felocal.fe_plan("helmholtz", "tetrahedron", 4, th_bytes=160 * 1024)["mode"] == "preeval"
    # at 64 KiB the gradient tables (58.8 KB) fit alone: pre-evaluate them, integrate the mass
    assert felocal.fe_plan("helmholtz", "tetrahedron", 4, th_bytes=65536)["preevaluated"] == [True, False]
    assert felocal.fe_plan("helmholtz", "tetrahedron", 4)["th_bytes"] >= 4 << 20   # L2 capacity


def test_planner_coefficient_functions():
    """nf pre-multiplying functions in the test/trial space: iota =
    C(n_s + nf - 1, nf) (Sec. 4.2), tables iota * rho * n_s^2 doubles, and
    Algorithm 3's choices under T_H = 160 KiB follow from theta and T_H."""
    from math import comb
    for p, ns in ((1, 4), (2, 10), (3, 20)):
        for nf in range(4):
            pl = felocal.fe_plan("mass", "tetrahedron", p, nf=nf, th_bytes=160 * 1024)
            assert pl["iota"][0] == comb(ns + nf - 1, nf)
            assert pl["table_bytes"][0] == comb(ns + nf - 1, nf) * ns * ns * 8
    T = 160 * 1024
    # mass P2: nf = 2 fits (44 KB) and pays; nf = 3 (176 KB) exceeds T_H
    assert felocal.fe_plan("mass", "tetrahedron", 2, nf=2, th_bytes=T)["mode"] == "preeval"
    assert felocal.fe_plan("mass", "tetrahedron", 2, nf=3, th_bytes=T)["mode"] == "quadrature"
    # Helmholtz P2 nf = 1: all tables (56 KB) fit; P3 nf = 1: only the mass
    # monomial's (64 KB) fit -> a mixed plan; P4 nf = 1: nothing fits
    assert felocal.fe_plan("helmholtz", "tetrahedron", 2, nf=1, th_bytes=T)["mode"] == "preeval"
    assert felocal.fe_plan("helmholtz", "tetrahedron", 3, nf=1, th_bytes=T)["preevaluated"] == [False, True]
    assert felocal.fe_plan("helmholtz", "tetrahedron", 4, nf=1, th_bytes=T)["preevaluated"] == [False, False]
    # with T_H relaxed the expansion still pays at P3 (theta < 0)
    assert felocal.fe_plan("helmholtz", "tetrahedron", 3, nf=1, th_bytes=1 << 30)["mode"] == "preeval"
    # vector forms: elasticity expands its P1 Lame field and the functions
    # (iota = n_c C(n_s + nf - 1, nf)), the hyperelastic trace term the
    # functions only (iota = C(n_s + nf - 1, nf)); rho as without functions
    pe = felocal.fe_plan("elasticity", "tetrahedron", 2, nf=1)
    assert pe["iota"] == [40, 40] and pe["rho"] == [9, 18]
    assert pe["table_bytes"][0] == 4 * 10 * 9 * 100 * 8
    ph = felocal.fe_plan("hyperelastic", "tetrahedron", 2, nf=2)
    assert ph["iota"] == [0, 55] and ph["rho"] == [0, 6]
    nq = oracle.rule("tetrahedron", oracle.default_qdeg("hyperelastic", "tetrahedron", 2, 2))[1].size
    # trace term: 2 rho iota + d operations per pair against 3 d per pair and point
    assert ph["theta_pre"][1] == (2 * 6 * 55 + 3) * 100 and ph["theta_se"][1] == nq * 100 * 9
    assert ph["preevaluated"] == [False, (2 * 6 * 55 + 3) < nq * 9]


def test_argument_errors_are_synchronous():
    L = felocal.lib()
    o = felocal.fe_options_t()
    L.fe_options_init(ctypes.byref(o))
    assert L.fe_assemble_local(0, 0, 1, 10, None, None, None, ctypes.byref(o)) == felocal.FE_EINVAL
    assert L.fe_assemble_local(0, 0, 5, 10, 8, None, 8, ctypes.byref(o)) == felocal.FE_EINVAL
    assert L.fe_assemble_local(0, 0, 1, -1, 8, None, 8, ctypes.byref(o)) == felocal.FE_EINVAL
    assert L.fe_assemble_local(0, 0, 1, 0, None, None, None, ctypes.byref(o)) == felocal.FE_OK
    assert L.fe_assemble_local(7, 0, 1, 1, 8, None, 8, ctypes.byref(o)) == felocal.FE_EINVAL
    assert L.fe_assemble_local(2, 1, 2, 1, 8, None, 8, ctypes.byref(o)) == felocal.FE_EINVAL   # no coefficients
    o.precision = 2
    assert L.fe_assemble_local(1, 1, 2, 1, 8, None, 8, ctypes.byref(o)) == felocal.FE_ENOTSUP   # split: vector forms
    assert L.fe_assemble_local(2, 1, 3, 1, 8, 8, 8, ctypes.byref(o)) == felocal.FE_ENOTSUP      # n = 60 > 32
    o.precision = 0
    o.mode = 1
    assert L.fe_assemble_local(3, 1, 2, 1, 8, 8, 8, ctypes.byref(o)) == felocal.FE_ENOTSUP      # hyperelastic: no pre-evaluation
    o.qdeg = 99
    o.mode = 0
    assert L.fe_assemble_local(0, 1, 2, 1, 8, None, 8, ctypes.byref(o)) == felocal.FE_EINVAL
    o.qdeg = -1
    o.nf = 4
    assert L.fe_assemble_local(0, 1, 2, 1, 8, 8, 8, ctypes.byref(o)) == felocal.FE_EINVAL     # nf in 0..3
    o.nf = 1
    o.precision = 2
    assert L.fe_assemble_local(2, 1, 2, 1, 8, 8, 8, ctypes.byref(o)) == felocal.FE_ENOTSUP    # float64 only
    o.precision = 0
    assert L.fe_assemble_local(1, 1, 2, 1, 8, None, 8, ctypes.byref(o)) == felocal.FE_EINVAL  # DOFs needed
    o.nf = 0
    for field, bad in (("kernel", 6), ("kernel", -1), ("block", -64), ("epi", -1), ("chunk", -2), ("eb", -1),
                       ("qc", -3), ("grid_per_cu", -1)):
        setattr(o.shape, field, bad)
        assert L.fe_assemble_local(0, 1, 2, 0, None, None, None, ctypes.byref(o)) == felocal.FE_EINVAL
        setattr(o.shape, field, 0)
    o.shape.kernel = 2
    assert L.fe_assemble_local(0, 1, 2, 0, None, None, None, ctypes.byref(o)) == felocal.FE_OK
    assert L.fe_geometry(0, 5, None, None, None, None) == felocal.FE_EINVAL
    assert L.fe_batch_run(None, None) == felocal.FE_EINVAL
    assert L.fe_batch_destroy(None) == felocal.FE_EINVAL
    assert "invalid" in felocal.strerror(felocal.FE_EINVAL)
    info = (ctypes.c_int * 3)()
    assert L.fe_tabulate(1, 4, 8, None, None, None, None, info) == 0 and list(info) == [125, 35, 3]


def test_th_bytes_from_the_environment(monkeypatch):
    """FE_TH_BYTES replaces the device's L2 capacity as T_H where the caller
    passes th_bytes = 0 (Sec. 3.4, Constraint 2): a tiny T_H keeps every
    table-bearing monomial of Helmholtz P4 in quadrature; an explicit
    th_bytes still wins."""
    monkeypatch.setenv("FE_TH_BYTES", "1000")
    p = felocal.fe_plan("helmholtz", "tetrahedron", 4)
    assert p["th_bytes"] == 1000 and not any(p["preevaluated"])
    big = felocal.fe_plan("helmholtz", "tetrahedron", 4, th_bytes=64 << 20)
    assert big["th_bytes"] == 64 << 20 and any(big["preevaluated"])
    monkeypatch.delenv("FE_TH_BYTES")
    assert felocal.fe_plan("helmholtz", "tetrahedron", 4)["th_bytes"] != 1000


def test_generated_form_argument_errors_are_synchronous():
    """fe_assemble_form refuses bad arguments on the host before any launch:
    a negative element count, a launch-shape kernel other than the generated
    nests, curved coordinates, a missing spec, more than 64 scalar basis
    functions (prism P4), a component count other than the cell dimension,
    and missing pointers; no elements is a no-op."""
    L = felocal.lib()
    o = felocal.fe_options_t()
    L.fe_options_init(ctypes.byref(o))
    sp = felocal.form_spec([("dx", "dx", -1, 1.0)])
    tet, prism = felocal.CELLS["tetrahedron"], felocal.CELLS["prism"]
    call = lambda spec, cell, p, E, ptr=8: L.fe_assemble_form(spec, cell, p, E, ptr, None, ptr, ctypes.byref(o))  # noqa
    assert call(ctypes.byref(sp), tet, 2, -1) == felocal.FE_EINVAL
    assert call(None, tet, 2, 1) == felocal.FE_EINVAL
    assert call(ctypes.byref(sp), prism, 4, 1) == felocal.FE_ENOTSUP
    assert call(ctypes.byref(sp), tet, 2, 0, None) == felocal.FE_OK
    assert call(ctypes.byref(sp), tet, 2, 1, None) == felocal.FE_EINVAL
    assert call(ctypes.byref(felocal.form_spec([("dx", "dx", -1, 1.0, 0, 0)], n_comp=2)), tet, 2, 0) == \
        felocal.FE_EINVAL
    assert call(ctypes.byref(felocal.form_spec([("value", "value", 0, 1.0)], n_fields=1)), tet, 2, 1) == \
        felocal.FE_EINVAL   # a field term without fields
    o.shape.kernel = 3
    assert call(ctypes.byref(sp), tet, 2, 1) == felocal.FE_EINVAL
    o.shape.kernel = 0
    o.coord_degree = 2
    assert call(ctypes.byref(sp), tet, 2, 1) == felocal.FE_ENOTSUP

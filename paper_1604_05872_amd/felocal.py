"""ctypes binding of libfelocal.so (include/felocal.h).

Argument marshalling only: every computation runs in the HIP library.  Device
arrays are torch tensors on a ROCm device (float64, contiguous); the stream
defaults to torch's current stream.  When the shared library has not been
built the binding raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfelocal.so")

FE_OK, FE_EINVAL, FE_ENOTSUP, FE_EHIP, FE_ENONAFFINE, FE_ENOMEM = 0, -1, -2, -3, -4, -5
CELLS = {"triangle": 0, "tetrahedron": 1, "prism": 2}
FORMS = {"mass": 0, "helmholtz": 1, "elasticity": 2, "hyperelastic": 3}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
MODES = {"auto": 0, "preeval": 1, "quadrature": 2}
GDIM = {"triangle": 2, "tetrahedron": 3, "prism": 3}
NVERT = {"triangle": 3, "tetrahedron": 4, "prism": 6}


def NBASIS(cell: str, p: int) -> int:
    """Scalar Lagrange P_p basis functions of the cell."""
    return {"triangle": (p + 1) * (p + 2) // 2, "tetrahedron": (p + 1) * (p + 2) * (p + 3) // 6,
            "prism": (p + 1) * (p + 2) // 2 * (p + 1)}[cell]

# every function include/felocal.h declares
EXPORTS = (
    "fe_options_init", "fe_tabulate", "fe_local_dims", "fe_assemble_local", "fe_geometry", "fe_plan",
    "fe_batch_create", "fe_batch_run", "fe_batch_destroy", "fe_batch_info", "fe_autotune", "fe_autotune_clear",
    "fe_strerror", "fe_release_caches", "fe_version",
    "fe_csr_create", "fe_csr_info", "fe_csr_pattern", "fe_csr_insert", "fe_csr_destroy", "fe_assemble_csr",
    "fe_assemble_csr_noalloc",
    "fe_sharing_plan", "fe_form_source", "fe_assemble_form",
)


class FeError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} (code {code})")


class fe_shape_t(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int) for f in ("kernel", "block", "epi", "chunk", "eb", "qc", "grid_per_cu")]


class fe_options_t(ctypes.Structure):
    _fields_ = [
        ("qdeg", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("mode", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("mu", ctypes.c_double),
        ("lambda_", ctypes.c_double),
        ("d_status", ctypes.c_void_p),
        ("th_bytes", ctypes.c_size_t),
        ("validate", ctypes.c_int),
        ("shape", fe_shape_t),
        ("nf", ctypes.c_int),
        ("pointgeo", ctypes.c_int),
        ("coord_degree", ctypes.c_int),
    ]


class fe_plan_t(ctypes.Structure):
    _fields_ = [
        ("n_monomials", ctypes.c_int),
        ("preevaluated", ctypes.c_int * 4),
        ("theta_se", ctypes.c_double * 4),
        ("theta_pre", ctypes.c_double * 4),
        ("iota", ctypes.c_int * 4),
        ("rho", ctypes.c_int * 4),
        ("table_bytes", ctypes.c_size_t * 4),
        ("th_bytes", ctypes.c_size_t),
        ("cost", ctypes.c_double),
        ("mode", ctypes.c_int),
    ]


SYMBOLS = {"value": 0, "dx": 1, "dy": 2, "dz": 3}
MAX_TERMS, MAX_FIELDS, MAX_VERTICES = 64, 4, 72


class fe_term_t(ctypes.Structure):
    _fields_ = [("test", ctypes.c_int), ("trial", ctypes.c_int), ("field", ctypes.c_int), ("scale", ctypes.c_double),
                ("test_comp", ctypes.c_int), ("trial_comp", ctypes.c_int)]


class fe_form_spec_t(ctypes.Structure):
    _fields_ = [("n_terms", ctypes.c_int), ("terms", fe_term_t * MAX_TERMS), ("n_fields", ctypes.c_int),
                ("n_comp", ctypes.c_int)]


class fe_sharing_t(ctypes.Structure):
    _fields_ = [
        ("n_vertices", ctypes.c_int),
        ("vertex_side", ctypes.c_int * MAX_VERTICES),
        ("vertex_symbol", ctypes.c_int * MAX_VERTICES),
        ("factorized", ctypes.c_int * MAX_VERTICES),
        ("n_edges", ctypes.c_int),
        ("edge_test", ctypes.c_int * MAX_TERMS),
        ("edge_trial", ctypes.c_int * MAX_TERMS),
        ("edge_owner", ctypes.c_int * MAX_TERMS),
        ("theta_expanded", ctypes.c_double),
        ("theta_se", ctypes.c_double),
        ("n_comp", ctypes.c_int),
        ("vertex_block", ctypes.c_int * MAX_VERTICES),
    ]


def form_spec(terms, n_fields: int = 0, n_comp: int = 0) -> fe_form_spec_t:
    """terms: list of (test_symbol, trial_symbol, field, scale) or, on a
    vector-valued space (n_comp = the cell dimension), (test_symbol,
    trial_symbol, field, scale, test_comp, trial_comp); symbols are names
    from SYMBOLS or their codes, field -1 for a constant term."""
    if len(terms) > MAX_TERMS:
        raise ValueError(f"at most {MAX_TERMS} terms")
    sp = fe_form_spec_t()
    sp.n_terms = len(terms)
    sp.n_fields = int(n_fields)
    sp.n_comp = int(n_comp)
    code = lambda x: SYMBOLS[x] if isinstance(x, str) else int(x)  # noqa: E731
    for i, t in enumerate(terms):
        te, tr, f, sc = t[:4]
        sp.terms[i].test, sp.terms[i].trial, sp.terms[i].field, sp.terms[i].scale = code(te), code(tr), int(f), float(sc)
        if len(t) > 4:
            sp.terms[i].test_comp, sp.terms[i].trial_comp = int(t[4]), int(t[5])
    return sp


class fe_subbatch_t(ctypes.Structure):
    _fields_ = [
        ("form", ctypes.c_int),
        ("cell", ctypes.c_int),
        ("degree", ctypes.c_int),
        ("qdeg", ctypes.c_int),
        ("n_elems", ctypes.c_int64),
        ("coords", ctypes.c_void_p),
        ("coeff_dofs", ctypes.c_void_p),
        ("out_A", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """The loaded shared library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1604_05872_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        L.fe_options_init.argtypes = [ctypes.POINTER(fe_options_t)]
        L.fe_options_init.restype = None
        L.fe_tabulate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_int)]
        L.fe_local_dims.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int)]
        L.fe_assemble_local.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, vp, vp, vp,
                                        ctypes.POINTER(fe_options_t)]
        L.fe_geometry.argtypes = [ctypes.c_int, ctypes.c_int64, vp, vp, vp, vp]
        L.fe_plan.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_size_t,
                              ctypes.POINTER(fe_plan_t)]
        L.fe_batch_create.argtypes = [ctypes.POINTER(fe_subbatch_t), ctypes.c_int, ctypes.POINTER(fe_options_t),
                                      ctypes.POINTER(vp)]
        L.fe_batch_run.argtypes = [vp, vp]
        L.fe_batch_destroy.argtypes = [vp]
        L.fe_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)]
        L.fe_autotune.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, vp, vp, vp,
                                  ctypes.POINTER(fe_options_t), dp]
        L.fe_strerror.argtypes = [ctypes.c_int]
        L.fe_strerror.restype = ctypes.c_char_p
        L.fe_release_caches.argtypes = []
        L.fe_release_caches.restype = None
        L.fe_autotune_clear.argtypes = []
        L.fe_autotune_clear.restype = None
        L.fe_version.restype = ctypes.c_char_p
        L.fe_csr_create.argtypes = [ctypes.c_int64, ctypes.c_int, vp, ctypes.c_int64, vp, ctypes.POINTER(vp)]
        L.fe_csr_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int)]
        L.fe_csr_pattern.argtypes = [vp, vp, vp, vp]
        L.fe_csr_insert.argtypes = [vp, vp, vp, vp]
        L.fe_csr_destroy.argtypes = [vp]
        L.fe_sharing_plan.argtypes = [ctypes.POINTER(fe_form_spec_t), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(fe_sharing_t)]
        L.fe_form_source.argtypes = [ctypes.POINTER(fe_form_spec_t), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_char_p, ctypes.POINTER(ctypes.c_size_t)]
        L.fe_assemble_form.argtypes = [ctypes.POINTER(fe_form_spec_t), ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                       vp, vp, vp, ctypes.POINTER(fe_options_t)]
        L.fe_assemble_csr.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, vp, vp, vp,
                                      ctypes.POINTER(fe_options_t)]
        L.fe_assemble_csr_noalloc.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, vp, vp, vp,
                                              ctypes.POINTER(fe_options_t)]
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().fe_strerror(int(code)).decode()


def fe_version() -> str:
    return lib().fe_version().decode()


def _check(rc: int, where: str):
    if rc != FE_OK:
        raise FeError(rc, where)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch

        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _f64_dev(t, name):
    if t is None:
        return
    import torch

    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 tensor on the GPU")


def make_options(qdeg=-1, precision="fp64", mode="auto", stream=None, mu=1.0, lam=10.0, status=None,
                 th_bytes=0, validate=False, need_stream=True, shape=None, nf=0, pointgeo=False,
                 coord_degree=1) -> fe_options_t:
    o = fe_options_t()
    lib().fe_options_init(ctypes.byref(o))
    o.qdeg = int(qdeg)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    o.stream = _stream(stream).value if need_stream else None
    o.mu = float(mu)
    o.lambda_ = float(lam)
    o.d_status = status.data_ptr() if status is not None else None
    o.th_bytes = int(th_bytes)
    o.validate = 1 if validate else 0
    for k, v in (shape or {}).items():
        setattr(o.shape, k, int(v))
    o.nf = int(nf)
    o.pointgeo = 1 if pointgeo else 0
    o.coord_degree = int(coord_degree)
    return o


def fe_local_dims(form: str, cell: str, degree: int):
    n, nc = ctypes.c_int(), ctypes.c_int()
    _check(lib().fe_local_dims(FORMS[form], CELLS[cell], int(degree), ctypes.byref(n), ctypes.byref(nc)),
           "fe_local_dims")
    return n.value, nc.value


def fe_tabulate(cell: str, degree: int, qdeg: int, rule_only: bool = False):
    """Quadrature rule and tabulated basis (host arrays).  rule_only needs no GPU."""
    L = lib()
    info = (ctypes.c_int * 3)()
    _check(L.fe_tabulate(CELLS[cell], int(degree), int(qdeg), None, None, None, None, info), "fe_tabulate")
    nq, nb, d = info[0], info[1], info[2]
    X = np.zeros((nq, d))
    W = np.zeros(nq)
    dp = ctypes.POINTER(ctypes.c_double)
    if rule_only:
        _check(L.fe_tabulate(CELLS[cell], int(degree), int(qdeg), X.ctypes.data_as(dp), W.ctypes.data_as(dp),
                             None, None, info), "fe_tabulate")
        return {"points": X, "weights": W}
    phi = np.zeros((nq, nb))
    dphi = np.zeros((nq, nb, d))
    _check(L.fe_tabulate(CELLS[cell], int(degree), int(qdeg), X.ctypes.data_as(dp), W.ctypes.data_as(dp),
                         phi.ctypes.data_as(dp), dphi.ctypes.data_as(dp), info), "fe_tabulate")
    return {"points": X, "weights": W, "phi": phi, "dphi": dphi}


def fe_assemble_local(form: str, cell: str, degree: int, coords, coeff, out, qdeg: int = -1,
                      precision: str = "fp64", mode: str = "auto", stream=None, mu: float = 1.0,
                      lam: float = 10.0, status=None, th_bytes: int = 0, validate: bool = False,
                      shape: dict | None = None, nf: int = 0, pointgeo: bool = False, coord_degree: int = 1):
    """Element matrices of `form` into `out` [E][n][n] (asynchronous on the stream).

    shape: optional launch-shape override, keys of fe_shape_t (kernel: 1 tiled,
    2 streaming pre-evaluated, 3 VALU, 4 matrix-core quadrature, 5 hoisted
    degree-1 vector kernel; block, epi, chunk, eb, qc, grid_per_cu).  nf: the form
    pre-multiplied by nf coefficient functions; an element's coeff record is the
    form's own DOFs followed by the functions' [nf][n_s].
    pointgeo: prisms need not be affine (the vertex map at every point).
    coord_degree 2: curved triangles and tetrahedra, coords [E][n_s(2)][gdim]
    the P2 nodes of each element."""
    _f64_dev(coords, "coords")
    _f64_dev(coeff, "coeff")
    _f64_dev(out, "out")
    E = int(coords.shape[0])
    n, nc = fe_local_dims(form, cell, degree)
    nmap = NBASIS(cell, 2) if coord_degree == 2 else NVERT[cell]
    if tuple(coords.shape) != (E, nmap, GDIM[cell]):
        raise ValueError(f"coords must be [E][{nmap}][{GDIM[cell]}]")
    if tuple(out.shape[-2:]) != (n, n) or out.numel() != E * n * n:
        raise ValueError(f"out must be [E][{n}][{n}]")
    if nf:
        nc += int(nf) * NBASIS(cell, degree)
    if nc and (coeff is None or coeff.numel() != E * nc):
        raise ValueError(f"coeff must hold {nc} values per element")
    o = make_options(qdeg, precision, mode, stream, mu, lam, status, th_bytes, validate, shape=shape, nf=nf,
                     pointgeo=pointgeo, coord_degree=coord_degree)
    _check(lib().fe_assemble_local(FORMS[form], CELLS[cell], int(degree), E, _ptr(coords), _ptr(coeff),
                                   _ptr(out), ctypes.byref(o)), "fe_assemble_local")
    return out


def fe_geometry(cell: str, coords, det, kinv, stream=None):
    _f64_dev(coords, "coords")
    _f64_dev(det, "det")
    _f64_dev(kinv, "kinv")
    _check(lib().fe_geometry(CELLS[cell], int(coords.shape[0]), _ptr(coords), _ptr(det), _ptr(kinv),
                             _stream(stream)), "fe_geometry")


def fe_plan(form: str, cell: str, degree: int, qdeg: int = -1, th_bytes: int = 0, nf: int = 0) -> dict:
    p = fe_plan_t()
    _check(lib().fe_plan(FORMS[form], CELLS[cell], int(degree), int(nf), int(qdeg), int(th_bytes), ctypes.byref(p)),
           "fe_plan")
    m = p.n_monomials
    return {
        "n_monomials": m,
        "preevaluated": [bool(p.preevaluated[i]) for i in range(m)],
        "theta_se": [p.theta_se[i] for i in range(m)],
        "theta_pre": [p.theta_pre[i] for i in range(m)],
        "iota": [p.iota[i] for i in range(m)],
        "rho": [p.rho[i] for i in range(m)],
        "table_bytes": [p.table_bytes[i] for i in range(m)],
        "th_bytes": p.th_bytes,
        "cost": p.cost,
        "mode": {v: k for k, v in MODES.items()}[p.mode],
    }


def fe_autotune(form: str, cell: str, degree: int, coords, coeff, out, qdeg: int = -1,
                precision: str = "fp64", mode: str = "auto", stream=None, mu: float = 1.0, lam: float = 10.0,
                return_shape: bool = False, nf: int = 0):
    """Best time per launch in ms (and, with return_shape, the chosen launch shape as a dict)."""
    _f64_dev(coords, "coords")
    _f64_dev(out, "out")
    o = make_options(qdeg, precision, mode, stream, mu, lam, nf=nf)
    best = ctypes.c_double()
    shape = fe_shape_t()
    _check(lib().fe_autotune(FORMS[form], CELLS[cell], int(degree), int(coords.shape[0]), _ptr(coords),
                             _ptr(coeff), _ptr(out), ctypes.byref(o), ctypes.byref(best), ctypes.byref(shape)),
           "fe_autotune")
    if return_shape:
        return best.value, {f: getattr(shape, f) for f, _ in fe_shape_t._fields_}
    return best.value


class Batch:
    """fe_batch_create / fe_batch_run / fe_batch_destroy.  `subs` is a list of
    dicts with form, cell, degree, coords, coeff (or None), out, qdeg (opt)."""

    def __init__(self, subs, stream=None, status=None):
        arr = (fe_subbatch_t * len(subs))()
        self._keep = []
        for i, s in enumerate(subs):
            _f64_dev(s["coords"], "coords")
            _f64_dev(s["out"], "out")
            arr[i].form = FORMS[s["form"]]
            arr[i].cell = CELLS[s["cell"]]
            arr[i].degree = int(s["degree"])
            arr[i].qdeg = int(s.get("qdeg", -1))
            arr[i].n_elems = int(s["coords"].shape[0])
            arr[i].coords = s["coords"].data_ptr()
            arr[i].coeff_dofs = s["coeff"].data_ptr() if s.get("coeff") is not None else None
            arr[i].out_A = s["out"].data_ptr()
            self._keep.append(s)
        o = make_options(stream=stream, status=status)
        h = ctypes.c_void_p()
        _check(lib().fe_batch_create(arr, len(subs), ctypes.byref(o), ctypes.byref(h)), "fe_batch_create")
        self.handle = h

    def run(self, stream=None):
        _check(lib().fe_batch_run(self.handle, _stream(stream)), "fe_batch_run")

    def info(self):
        nt, g = ctypes.c_int64(), ctypes.c_int()
        _check(lib().fe_batch_info(self.handle, ctypes.byref(nt), ctypes.byref(g)), "fe_batch_info")
        return nt.value, g.value

    def close(self):
        if self.handle:
            _check(lib().fe_batch_destroy(self.handle), "fe_batch_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CsrPattern:
    """Global assembly (fe_csr_create / fe_csr_info / fe_csr_pattern /
    fe_csr_insert / fe_csr_destroy).  cell_dofs: int32 tensor [E][n] on the
    GPU with the global number of every local DOF; n_rows: size of the global
    matrix."""

    def __init__(self, cell_dofs, n_rows: int, stream=None):
        import torch

        if not (isinstance(cell_dofs, torch.Tensor) and cell_dofs.is_cuda and cell_dofs.dtype == torch.int32
                and cell_dofs.is_contiguous() and cell_dofs.dim() == 2):
            raise ValueError("cell_dofs must be a contiguous int32 [E][n] tensor on the GPU")
        h = ctypes.c_void_p()
        self.handle = None
        _check(lib().fe_csr_create(int(cell_dofs.shape[0]), int(cell_dofs.shape[1]), _ptr(cell_dofs), int(n_rows),
                                   _stream(stream), ctypes.byref(h)), "fe_csr_create")
        self.handle = h
        self.n_elems, self.n = int(cell_dofs.shape[0]), int(cell_dofs.shape[1])

    def info(self):
        N, nnz, mr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
        _check(lib().fe_csr_info(self.handle, ctypes.byref(N), ctypes.byref(nnz), ctypes.byref(mr)), "fe_csr_info")
        return {"n_rows": N.value, "nnz": nnz.value, "max_row_len": mr.value}

    def pattern(self, stream=None):
        """(row_ptr int64 [n_rows+1], col_idx int32 [nnz]) as new GPU tensors."""
        import torch

        i = self.info()
        rp = torch.empty(i["n_rows"] + 1, dtype=torch.int64, device="cuda")
        ci = torch.empty(max(i["nnz"], 1), dtype=torch.int32, device="cuda")
        _check(lib().fe_csr_pattern(self.handle, _ptr(rp), _ptr(ci), _stream(stream)), "fe_csr_pattern")
        return rp, ci[: i["nnz"]]

    def insert(self, local_A, values, stream=None):
        """values [nnz] <- element-order sums of local_A [E][n][n] (asynchronous)."""
        _f64_dev(local_A, "local_A")
        _f64_dev(values, "values")
        if local_A.numel() != self.n_elems * self.n * self.n:
            raise ValueError(f"local_A must be [{self.n_elems}][{self.n}][{self.n}]")
        if values.numel() != self.info()["nnz"]:
            raise ValueError("values must hold nnz entries")
        _check(lib().fe_csr_insert(self.handle, _ptr(local_A), _ptr(values), _stream(stream)), "fe_csr_insert")
        return values

    def assemble(self, form: str, cell: str, degree: int, coords, values, qdeg: int = -1, mode: str = "auto",
                 stream=None, status=None, validate: bool = False):
        """values [nnz] <- local and global assembly in one pass (fe_assemble_csr)."""
        _f64_dev(coords, "coords")
        _f64_dev(values, "values")
        if values.numel() != self.info()["nnz"]:
            raise ValueError("values must hold nnz entries")
        o = make_options(qdeg, "fp64", mode, stream, status=status, validate=validate)
        _check(lib().fe_assemble_csr(FORMS[form], CELLS[cell], int(degree), int(coords.shape[0]), _ptr(coords),
                                     self.handle, _ptr(values), ctypes.byref(o)), "fe_assemble_csr")
        return values

    def assemble_noalloc(self, form: str, cell: str, degree: int, coords, values, qdeg: int = -1,
                         mode: str = "auto", stream=None, status=None):
        """As assemble, through fe_assemble_csr_noalloc (no device allocation;
        the reference tables must already be built on this device)."""
        _f64_dev(coords, "coords")
        _f64_dev(values, "values")
        if values.numel() != self.info()["nnz"]:
            raise ValueError("values must hold nnz entries")
        o = make_options(qdeg, "fp64", mode, stream, status=status)
        _check(lib().fe_assemble_csr_noalloc(FORMS[form], CELLS[cell], int(degree), int(coords.shape[0]),
                                             _ptr(coords), self.handle, _ptr(values), ctypes.byref(o)),
               "fe_assemble_csr_noalloc")
        return values

    def close(self):
        if self.handle:
            _check(lib().fe_csr_destroy(self.handle), "fe_csr_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fe_sharing_plan(terms, cell: str, degree: int, qdeg: int = -1, n_fields: int = 0, n_comp: int = 0) -> dict:
    """Algorithm 1 (Sec. 3.2) for a generic form, per component block: the
    factorised symbols and operation counts (host only)."""
    sp = form_spec(terms, n_fields, n_comp)
    pl = fe_sharing_t()
    _check(lib().fe_sharing_plan(ctypes.byref(sp), CELLS[cell], int(degree), int(qdeg), ctypes.byref(pl)),
           "fe_sharing_plan")
    nv, ne = pl.n_vertices, pl.n_edges
    return {
        "n_comp": pl.n_comp,
        "vertices": [(pl.vertex_side[i], pl.vertex_symbol[i]) for i in range(nv)],
        "blocks": [pl.vertex_block[i] for i in range(nv)],
        "factorized": [bool(pl.factorized[i]) for i in range(nv)],
        "edges": [(pl.edge_test[e], pl.edge_trial[e]) for e in range(ne)],
        "owner": [pl.edge_owner[e] for e in range(ne)],
        "theta_expanded": pl.theta_expanded,
        "theta_se": pl.theta_se,
    }


def fe_form_source(terms, cell: str, degree: int, expanded: bool = False, n_fields: int = 0,
                   n_comp: int = 0) -> str:
    sp = form_spec(terms, n_fields, n_comp)
    n = ctypes.c_size_t(0)
    _check(lib().fe_form_source(ctypes.byref(sp), CELLS[cell], int(degree), int(expanded), None, ctypes.byref(n)),
           "fe_form_source")
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().fe_form_source(ctypes.byref(sp), CELLS[cell], int(degree), int(expanded), buf, ctypes.byref(n)),
           "fe_form_source")
    return buf.value.decode()


def fe_assemble_form(terms, cell: str, degree: int, coords, fields, out, n_fields: int = 0, qdeg: int = -1,
                     expanded: bool = False, stream=None, status=None, n_comp: int = 0):
    """Element matrices of a generic form by the generated kernel; out is
    [E][n][n], n = n_comp * n_s on a vector-valued space."""
    _f64_dev(coords, "coords")
    _f64_dev(fields, "fields")
    _f64_dev(out, "out")
    ns = fe_local_dims("mass", cell, degree)[0]
    n = max(1, int(n_comp)) * ns
    if out is not None and coords is not None and out.numel() < int(coords.shape[0]) * n * n:
        raise ValueError(f"out holds fewer than {int(coords.shape[0])} x {n} x {n} values")
    sp = form_spec(terms, n_fields, n_comp)
    o = make_options(qdeg, stream=stream, status=status, shape={"kernel": 5} if expanded else None)
    _check(lib().fe_assemble_form(ctypes.byref(sp), CELLS[cell], int(degree), int(coords.shape[0]), _ptr(coords),
                                  _ptr(fields), _ptr(out), ctypes.byref(o)), "fe_assemble_form")
    return out


def fe_release_caches():
    lib().fe_release_caches()

"""Seeded synthetic inputs for local assembly: jittered meshes and coefficient DOFs.

This module is shared by the tests, the oracle-side checks and the benchmark.  It
holds no finite-element arithmetic: it only lays out vertex lattices, draws random
numbers and gathers vertex data per element.  Nothing here evaluates a basis
function, a Jacobian or an integrand.

Layouts produced (all float64, C-contiguous, element-major):
  coords  [E][nv][gdim]   nv = 3 (triangle), 4 (tetrahedron), 6 (prism)
  elasticity coefficients [E][2][nc]   Lame lambda DOFs, then mu DOFs, P1 per cell vertex
  hyperelastic displacement [E][gdim * n_s]   component-blocked element-local DOFs
  global DOF numbers [E][n_s] int32 (global assembly): the node of local DOF j of
  element e on the refined vertex lattice, shared by every element holding it

Vertex ordering follows the reference cells used throughout the library:
  triangle (0,0),(1,0),(0,1); tetrahedron adds (0,0,1); prism = triangle x [0,1],
  vertices 0..2 on the bottom face and 3..5 = 0..2 + e_z.

Jitter choices (each provably non-inverting, because a simplex volume is
multilinear in the vertex coordinates, so its minimum over a box of per-axis
perturbations is attained at a box corner; the corners were enumerated):
  * triangles, +-0.2 h per axis (h_x, h_y separately): worst area ratio 0.2;
  * Kuhn tetrahedra, +-0.15 h per axis: worst volume ratio 0.10
    (+-0.2 h can invert a Kuhn tetrahedron);
  * prisms: the triangle jitter in x, y only, layers of equal height, so every
    prism is an exact translate-extrusion (affine); optionally each interior
    layer's vertices also move in z by less than half a layer (non-affine
    prisms with positive height everywhere).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

TRI, TET, PRISM = "triangle", "tetrahedron", "prism"
CELLS = (TRI, TET, PRISM)
GDIM = {TRI: 2, TET: 3, PRISM: 3}
NVERT = {TRI: 3, TET: 4, PRISM: 6}

TRI_JITTER = 0.2
TET_JITTER = 0.15


def n_scalar_dofs(cell: str, p: int) -> int:
    """Number of scalar Lagrange DOFs of degree p on a cell (lattice count)."""
    if cell == TRI:
        return (p + 1) * (p + 2) // 2
    if cell == TET:
        return (p + 1) * (p + 2) * (p + 3) // 6
    if cell == PRISM:
        return (p + 1) * (p + 2) // 2 * (p + 1)
    raise ValueError(cell)


def _streams(seed: int, n: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


# ---------------------------------------------------------------------------
# Vertex lattices
# ---------------------------------------------------------------------------

def _jitter_plane(nx: int, ny: int, amp: float, rng) -> np.ndarray:
    """(nx+1)*(ny+1) vertices of the unit square, interior ones jittered per axis."""
    hx, hy = 1.0 / nx, 1.0 / ny
    X, Y = np.meshgrid(np.arange(nx + 1) * hx, np.arange(ny + 1) * hy, indexing="ij")
    V = np.stack([X, Y], axis=-1)  # [nx+1][ny+1][2]
    if amp > 0:
        d = rng.uniform(-amp, amp, size=V.shape)
        d[..., 0] *= hx
        d[..., 1] *= hy
        d[0, :, :] = 0.0
        d[-1, :, :] = 0.0
        d[:, 0, :] = 0.0
        d[:, -1, :] = 0.0
        V = V + d
    return V


def triangle_mesh(nx: int, ny: int, seed: int, jitter: float = TRI_JITTER):
    """Unit square, nx*ny cells, two triangles per cell split along the
    (i,j)->(i+1,j+1) diagonal, counter-clockwise.  Returns (vertices[NV][2],
    cells[E][3]) with E = 2*nx*ny."""
    (rng,) = _streams(seed, 1)
    V = _jitter_plane(nx, ny, jitter, rng).reshape(-1, 2)
    vid = lambda i, j: i * (ny + 1) + j  # noqa: E731
    I, J = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    I, J = I.ravel(), J.ravel()
    a, b, c, d = vid(I, J), vid(I + 1, J), vid(I + 1, J + 1), vid(I, J + 1)
    t1 = np.stack([a, b, c], axis=1)
    t2 = np.stack([a, c, d], axis=1)
    cells = np.stack([t1, t2], axis=1).reshape(-1, 3)
    return V, cells


_KUHN = list(itertools.permutations(range(3)))


def tet_mesh(n: int, seed: int, jitter: float = TET_JITTER):
    """Unit cube, n^3 cubes, 6 Kuhn tetrahedra per cube (one per axis
    permutation, vertex path 0 -> e_s1 -> e_s1+e_s2 -> (1,1,1)).  Interior
    vertices jittered uniformly by +-jitter*h per axis.  Returns
    (vertices[NV][3], cells[E][4]) with E = 6*n^3."""
    (rng,) = _streams(seed, 1)
    h = 1.0 / n
    g = np.arange(n + 1) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    V = np.stack([X, Y, Z], axis=-1)
    if jitter > 0:
        d = rng.uniform(-jitter * h, jitter * h, size=V.shape)
        for ax in range(3):
            sl = [slice(None)] * 3
            sl[ax] = 0
            d[tuple(sl)] = 0.0
            sl[ax] = -1
            d[tuple(sl)] = 0.0
        V = V + d
    V = V.reshape(-1, 3)
    n1 = n + 1
    vid = lambda i, j, k: (i * n1 + j) * n1 + k  # noqa: E731
    I, J, K = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)  # [n^3][3]
    cells = np.empty((base.shape[0], 6, 4), dtype=np.int64)
    for t, perm in enumerate(_KUHN):
        cur = base.copy()
        cells[:, t, 0] = vid(cur[:, 0], cur[:, 1], cur[:, 2])
        for s, ax in enumerate(perm):
            cur = cur.copy()
            cur[:, ax] += 1
            cells[:, t, s + 1] = vid(cur[:, 0], cur[:, 1], cur[:, 2])
    return V, cells.reshape(-1, 4)


def prism_mesh(n: int, nz: int, seed: int, jitter: float = TRI_JITTER, zjitter: float = 0.0):
    """Extruded triangle mesh: n*n*2 triangles (jittered in x, y) times nz
    layers of height 1/nz.  Prism vertices are the bottom triangle then the
    same triangle one layer up, so every prism is affine -- unless zjitter > 0:
    then every vertex of an interior layer moves in z by up to zjitter/nz
    (uniform, per vertex), so a prism's top face is no longer a translate of
    its bottom face (a non-affine prism; its height stays above
    (1 - 2 zjitter)/nz at every point for zjitter < 0.5).  Returns
    (vertices[NV][3], cells[E][6]) with E = 2*n*n*nz."""
    V2, tris = triangle_mesh(n, n, seed, jitter)
    nv2 = V2.shape[0]
    z = np.arange(nz + 1) / nz
    V = np.concatenate(
        [np.concatenate([V2, np.full((nv2, 1), zl)], axis=1) for zl in z], axis=0
    )
    if zjitter > 0:
        if not zjitter < 0.5:
            raise ValueError("zjitter must be below 0.5")
        (rz,) = _streams(seed + 7919, 1)
        dz = rz.uniform(-zjitter / nz, zjitter / nz, size=(nz + 1, nv2))
        dz[0, :] = 0.0
        dz[-1, :] = 0.0
        V[:, 2] += dz.ravel()
    layers = np.arange(nz)
    bot = tris[None, :, :] + (layers * nv2)[:, None, None]
    top = bot + nv2
    cells = np.concatenate([bot, top], axis=2).reshape(-1, 6)
    return V, cells


def _node_multi_indices(cell: str, p: int) -> np.ndarray:
    """Lattice multi-indices of the local nodes in the library's node order:
    triangle (i, j) with i fastest; tetrahedron (i, j, k), loops k, j, i with i
    fastest; prism (i, j, l) for local index l * n_tri + t, t in triangle order.
    A node of a simplex sits at v0 + (i (v1 - v0) + j (v2 - v0) [+ k (v3 - v0)]) / p."""
    if cell == TRI:
        return np.array([(i, j) for j in range(p + 1) for i in range(p + 1 - j)], dtype=np.int64)
    if cell == TET:
        return np.array([(i, j, k) for k in range(p + 1) for j in range(p + 1 - k) for i in range(p + 1 - j - k)],
                        dtype=np.int64)
    tri = _node_multi_indices(TRI, p)
    return np.array([(i, j, l) for l in range(p + 1) for (i, j) in tri], dtype=np.int64)


def global_dofs(cell: str, p: int, cells: np.ndarray, n: int, compact: bool = True):
    """Global numbers of the degree-p Lagrange DOFs of a structured mesh made by
    triangle_mesh(n, n), tet_mesh(n) or prism_mesh(n, n) (possibly truncated to
    its first elements).  Every vertex of these meshes is a point of an integer
    grid (spacing h); the nodes of degree p lie on the grid refined p times, and
    a node shared by several elements has one refined-grid point, so numbering
    the refined grid numbers the DOFs of the continuous space.  With compact,
    the numbers of the nodes in use are renumbered 0..N-1 in increasing order.
    Returns (dofs [E][n_s] int32, N)."""
    cells = np.asarray(cells, dtype=np.int64)
    a = _node_multi_indices(cell, p)
    m = n * p + 1
    if cell == TRI:
        vi = np.stack([cells // (n + 1), cells % (n + 1)], axis=-1)           # [E][3][2]
        X = p * vi[:, None, 0, :] + a[None, :, 0, None] * (vi[:, None, 1, :] - vi[:, None, 0, :]) \
            + a[None, :, 1, None] * (vi[:, None, 2, :] - vi[:, None, 0, :])
        g = X[..., 0] * m + X[..., 1]
    elif cell == TET:
        n1 = n + 1
        vi = np.stack([cells // (n1 * n1), (cells // n1) % n1, cells % n1], axis=-1)   # [E][4][3]
        X = p * vi[:, None, 0, :]
        for c in range(3):
            X = X + a[None, :, c, None] * (vi[:, None, c + 1, :] - vi[:, None, 0, :])
        g = (X[..., 0] * m + X[..., 1]) * m + X[..., 2]
    elif cell == PRISM:
        nv2 = (n + 1) * (n + 1)
        layer, v2 = cells // nv2, cells % nv2
        vi = np.stack([v2 // (n + 1), v2 % (n + 1)], axis=-1)                  # [E][6][2]
        XY = p * vi[:, None, 0, :] + a[None, :, 0, None] * (vi[:, None, 1, :] - vi[:, None, 0, :]) \
            + a[None, :, 1, None] * (vi[:, None, 2, :] - vi[:, None, 0, :])
        Z = p * layer[:, None, 0] + a[None, :, 2]
        g = (XY[..., 0] * m + XY[..., 1]) * m + Z
    else:
        raise ValueError(cell)
    if compact:
        used, inv = np.unique(g, return_inverse=True)
        return np.ascontiguousarray(inv.reshape(g.shape), dtype=np.int32), int(used.size)
    N = m ** (2 if cell == TRI else 3)
    return np.ascontiguousarray(g, dtype=np.int32), int(N)


def vector_dofs(dofs: np.ndarray, N: int, gdim: int) -> np.ndarray:
    """Global numbers of a component-blocked vector space: local DOF c * n_s + j
    of an element maps to c * N + dofs[e][j].  Returns [E][gdim * n_s] int32."""
    return np.ascontiguousarray(np.concatenate([dofs + c * N for c in range(gdim)], axis=1), dtype=np.int32)


def random_local_matrices(E: int, n: int, seed: int) -> np.ndarray:
    """Element matrices [E][n][n] with entries uniform in [-1, 1): synthetic
    input of the insertion step alone."""
    (rng,) = _streams(seed, 1)
    return rng.uniform(-1.0, 1.0, size=(E, n, n))


def gather(V: np.ndarray, cells: np.ndarray) -> np.ndarray:
    """coords[E][nv][gdim] from a vertex array and a connectivity array."""
    return np.ascontiguousarray(V[cells], dtype=np.float64)


# ---------------------------------------------------------------------------
# Coefficient DOFs
# ---------------------------------------------------------------------------

def lame_p1(nverts: int, cells: np.ndarray, seed: int, lo: float = 0.5, hi: float = 2.0):
    """Continuous P1 Lame fields: one lambda and one mu value per mesh vertex,
    uniform in [lo, hi], gathered per element to [E][2][nv]."""
    r_lam, r_mu = _streams(seed, 2)
    lam = r_lam.uniform(lo, hi, size=nverts)
    mu = r_mu.uniform(lo, hi, size=nverts)
    return np.ascontiguousarray(np.stack([lam[cells], mu[cells]], axis=1))


def displacement_dofs(E: int, gdim: int, n_s: int, h: float, seed: int,
                      rel: float = 0.05, clip: float = 3.0) -> np.ndarray:
    """Element-local displacement DOFs [E][gdim*n_s], component-blocked,
    i.i.d. normal with standard deviation rel*h (h the mesh spacing), redrawn
    where beyond clip standard deviations."""
    (rng,) = _streams(seed, 1)
    sig = rel * h
    u = rng.standard_normal(size=(E, gdim * n_s))
    bad = np.abs(u) > clip
    while bad.any():
        u[bad] = rng.standard_normal(size=int(bad.sum()))
        bad = np.abs(u) > clip
    return np.ascontiguousarray(u * sig)


def curved_mesh(cell: str, n: int, seed: int, bend: float = 0.04):
    """Curved triangles or tetrahedra: the P2 nodes of the jittered structured
    mesh (triangle_mesh(n, n) or tet_mesh(n)), laid out per element in the
    library's lattice order, [E][n_s(2)][gdim].  Each node starts on the
    straight element (v0 + (i (v1 - v0) + j (v2 - v0) [+ k (v3 - v0)]) / 2 for
    lattice index (i, j[, k])); every edge-midpoint node strictly inside the
    unit box then moves by U(+-bend h) per axis, drawn once per node, so the
    elements sharing an edge share its curve and the mesh still fills the box
    (boundary edges stay straight).  Returns (coords2, vertices, cells, h)."""
    if cell == TRI:
        V, cells = triangle_mesh(n, n, seed)
    elif cell == TET:
        V, cells = tet_mesh(n, seed)
    else:
        raise ValueError("curved meshes are triangles or tetrahedra")
    d = GDIM[cell]
    a = _node_multi_indices(cell, 2).astype(float) / 2.0               # [n2][d]
    v = V[cells]                                                        # [E][nv][d]
    x = v[:, None, 0, :] + sum(a[None, :, c, None] * (v[:, None, c + 1, :] - v[:, None, 0, :]) for c in range(d))
    g, _ = global_dofs(cell, 2, cells, n, compact=False)                # refined-grid node ids
    m = 2 * n + 1
    if d == 2:
        grid = np.stack([g // m, g % m], axis=-1)
    else:
        grid = np.stack([g // (m * m), (g // m) % m, g % m], axis=-1)
    midpoint = (grid % 2 == 1).any(axis=-1)
    inside = ((grid >= 1) & (grid <= m - 2)).all(axis=-1)
    move = midpoint & inside
    ids, inv = np.unique(g[move], return_inverse=True)
    (rng,) = _streams(seed + 7919, 1)
    disp = rng.uniform(-bend / n, bend / n, size=(ids.size, d))
    x[move] += disp[inv]
    return np.ascontiguousarray(x), V, cells, 1.0 / n


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def mass_tri_workload(seed: int = 1):
    """4096 P1 triangles from a 32 x 64 unit-square grid, +-0.2 h per-axis jitter."""
    V, cells = triangle_mesh(32, 64, seed)
    return gather(V, cells)


def tet_workload(n: int, seed: int):
    V, cells = tet_mesh(n, seed)
    return gather(V, cells), V, cells


def grid_for_count(cell: str, E: int) -> int:
    """Smallest per-side count n whose structured grid holds at least E cells
    (triangle: 2 n^2, tetrahedron: 6 n^3, prism: 2 n^2 * n layers)."""
    per = {TRI: lambda n: 2 * n * n, TET: lambda n: 6 * n ** 3, PRISM: lambda n: 2 * n ** 3}[cell]
    n = max(1, int(math.floor((E / {TRI: 2, TET: 6, PRISM: 2}[cell]) ** (1.0 / (2 if cell == TRI else 3)))))
    while per(n) < E:
        n += 1
    return n


def first_elements(cell: str, E: int, seed: int, zjitter: float = 0.0):
    """The first E elements of the smallest jittered structured grid with at
    least E cells (prisms: non-affine with zjitter > 0, see prism_mesh).
    Returns (coords, vertices, cells[:E], h)."""
    n = grid_for_count(cell, E)
    if cell == TRI:
        V, cells = triangle_mesh(n, n, seed)
    elif cell == TET:
        V, cells = tet_mesh(n, seed)
    else:
        V, cells = prism_mesh(n, n, seed, zjitter=zjitter)
    cells = cells[:E]
    return gather(V, cells), V, cells, 1.0 / n

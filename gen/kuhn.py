"""Structured Kuhn-tetrahedra box meshes and P1 finite element assembly.

Mesh: vertex (i, j, k) of an ``nx x ny x nz`` grid with spacing ``h`` has id
``v = i + nx*(j + ny*k)`` and position ``(i h, j h, k h)``.  Each grid cell with
lower corner ``o`` is split into the six Kuhn tetrahedra
``(o, o+e_p0, o+e_p0+e_p1, o+(1,1,1))``, one per permutation ``p`` of (0,1,2) in
lexicographic order.  Every interior vertex then has 14 neighbours.

Assembly (paper section "fem", Problems prob:gg and prob:epseps): standard conforming P1.
For linear elasticity the bilinear form is ``int 2 mu_L eps(u):eps(v) + lambda div u div v``
(Hooke's law; the paper writes ``mu eps:eps`` with ``mu = 2 mu_L``).  The element matrix
entry for test function ``phi_a e_m`` and trial ``phi_b e_n`` is
``V (mu_L (delta_mn g_a.g_b + g_a[n] g_b[m]) + lambda g_a[m] g_b[n])`` with the constant P1
gradients ``g``.  The matrix is returned without boundary conditions ("A_N"), as a block
CSR with 3x3 (elasticity) or 1x1 (Poisson) row-major blocks, sorted column indices and the
full mesh pattern (a block exists iff the two vertices share a tetrahedron).
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Optional

import numpy as np

_PERMS = list(itertools.permutations(range(3)))


def lame_from_young(E: float, nu: float):
    """Return (mu_L, lambda) from Young's modulus and Poisson ratio."""
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def _tet_offsets() -> np.ndarray:
    """(6, 4, 3) integer vertex offsets (x, y, z) of the six Kuhn tetrahedra of a cell."""
    eye = np.eye(3, dtype=np.int64)
    out = []
    for p in _PERMS:
        out.append(np.stack([np.zeros(3, np.int64), eye[p[0]], eye[p[0]] + eye[p[1]],
                             np.ones(3, np.int64)]))
    return np.array(out)


def _p1_gradients(P: np.ndarray):
    """Gradients (4, 3) of the barycentric functions and the volume of tetrahedron P (4, 3)."""
    X = (P[1:] - P[0]).T
    Xinv = np.linalg.inv(X)
    g = np.empty((4, 3))
    g[1:] = Xinv
    g[0] = -Xinv.sum(axis=0)
    return g, abs(np.linalg.det(X)) / 6.0


def _unit_element_matrices():
    """Per Kuhn tet type, the unit-spacing element matrices.

    Returns (offsets (6,4,3), Kmu (6,12,12), Klam (6,12,12), Klap (6,4,4)), where the
    elasticity element matrix is ``h*(mu_L*Kmu + lambda*Klam)`` and the Laplacian one is
    ``h*Klap`` for spacing ``h`` (gradients scale with 1/h, volume with h^3).
    """
    offs = _tet_offsets()
    Kmu = np.zeros((6, 12, 12))
    Klam = np.zeros((6, 12, 12))
    Klap = np.zeros((6, 4, 4))
    for t in range(6):
        g, vol = _p1_gradients(offs[t].astype(np.float64))
        Klap[t] = vol * g @ g.T
        for a in range(4):
            for b in range(4):
                gg = g[a] @ g[b]
                for m in range(3):
                    for n in range(3):
                        Kmu[t, 3 * a + m, 3 * b + n] = vol * ((m == n) * gg + g[a][n] * g[b][m])
                        Klam[t, 3 * a + m, 3 * b + n] = vol * g[a][m] * g[b][n]
    return offs, Kmu, Klam, Klap


@dataclasses.dataclass
class KuhnMesh:
    nx: int
    ny: int
    nz: int
    h: float

    @property
    def n_vertices(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def cell_shape(self):
        return (self.nz - 1, self.ny - 1, self.nx - 1)

    def coords(self) -> np.ndarray:
        k, j, i = np.meshgrid(np.arange(self.nz), np.arange(self.ny), np.arange(self.nx),
                              indexing="ij")
        return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64) * self.h

    def tet_centroids(self, t: int) -> np.ndarray:
        """Centroids (cells..., 3) of Kuhn tet type t in every cell, array indexed [k, j, i]."""
        off = _tet_offsets()[t].astype(np.float64).mean(axis=0)  # (x, y, z)
        k, j, i = np.meshgrid(np.arange(self.nz - 1), np.arange(self.ny - 1),
                              np.arange(self.nx - 1), indexing="ij")
        return np.stack([(i + off[0]) * self.h, (j + off[1]) * self.h, (k + off[2]) * self.h],
                        axis=-1)


def kuhn_mesh(n: int, ny: Optional[int] = None, nz: Optional[int] = None,
              h: Optional[float] = None) -> KuhnMesh:
    """Box mesh with n (x) by ny by nz vertices; default a unit cube with n vertices per side."""
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    if min(n, ny, nz) < 2:
        raise ValueError("need at least 2 vertices per direction")
    if h is None:
        h = 1.0 / (n - 1)
    return KuhnMesh(n, ny, nz, float(h))


def _shift_slices(shape, d):
    """Slices (target, source) of a (nz, ny, nx) grid such that target[v] = source[v - d] for
    every vertex v with v - d inside the grid; d is an (x, y, z) offset."""
    tgt, src = [], []
    for axis, s in ((0, d[2]), (1, d[1]), (2, d[0])):
        m = shape[axis]
        tgt.append(slice(max(s, 0), m + min(s, 0)))
        src.append(slice(max(-s, 0), m - max(s, 0)))
    return tuple(tgt), tuple(src)


def _assemble(mesh: KuhnMesh, parts):
    """Stencil assembly on the structured Kuhn mesh.

    ``parts`` is a list of ``(coef, K)``: ``coef`` a scalar or a per-(tet type, cell) array
    (6, nz-1, ny-1, nx-1), ``K`` (6, 4 bs, 4 bs) the element matrix of each tet type for a unit
    coefficient.  The element matrix of tet type t in cell c is ``sum_p coef_p[t, c] K_p[t]``.

    The block of vertex v and direction d (a neighbour offset) sums, over the tet types t, the
    one local pair (a, b) of t with offset d, taken in the cell v - offs[t, a].  So the blocks of
    all vertices for the directions d >= 0 (in vertex-id order) are one product of the shifted
    per-cell coefficients (vertices x (part, t, a)) with the matching element blocks; the blocks
    of direction -d are the transposes of those of d at v - d, which keeps A exactly symmetric.
    """
    offs = _tet_offsets()
    bs = parts[0][1].shape[-1] // 4
    nz, ny, nx = mesh.nz, mesh.ny, mesh.nx
    cz, cy, cx = mesh.cell_shape
    n = mesh.n_vertices
    lin = lambda d: int(d[0] + nx * (d[1] + ny * d[2]))
    dset = {tuple(int(x) for x in offs[t, b] - offs[t, a])
            for t in range(6) for a in range(4) for b in range(4)}
    dirs = sorted(dset, key=lin)
    pos = [d for d in dirs if lin(d) >= 0]
    npart = len(parts)
    # shifted coefficients: column (p, t, a) holds coef_p[t] of the cell v - offs[t, a]
    C = np.zeros((npart * 24, nz, ny, nx))
    inside = np.zeros((24, nz, ny, nx), dtype=bool)
    for t in range(6):
        for a in range(4):
            oa = offs[t, a]
            sl = (slice(oa[2], oa[2] + cz), slice(oa[1], oa[1] + cy), slice(oa[0], oa[0] + cx))
            inside[(4 * t + a,) + sl] = True
            for p, (coef, _) in enumerate(parts):
                C[(24 * p + 4 * t + a,) + sl] = coef[t] if np.ndim(coef) else coef
    S = np.zeros((npart * 24, len(pos), bs * bs))
    contrib = [[] for _ in pos]
    for t in range(6):
        for a in range(4):
            for b in range(4):
                d = tuple(int(x) for x in offs[t, b] - offs[t, a])
                if d not in pos:
                    continue
                w = pos.index(d)
                contrib[w].append(4 * t + a)
                for p, (_, K) in enumerate(parts):
                    S[24 * p + 4 * t + a, w] = K[t, bs * a:bs * a + bs, bs * b:bs * b + bs].ravel()
    half = (C.reshape(npart * 24, n).T @ S.reshape(npart * 24, -1)).reshape(nz, ny, nx, len(pos),
                                                                            bs, bs)
    del C
    blocks, touched = {}, {}
    for w, d in enumerate(pos):
        blocks[d] = half[:, :, :, w]
        tw = np.zeros((nz, ny, nx), dtype=bool)
        for ta in contrib[w]:
            tw |= inside[ta]
        touched[d] = tw
    for d in pos:
        if lin(d) == 0:
            continue
        nd = tuple(-x for x in d)
        tgt, src = _shift_slices((nz, ny, nx), d)
        bl = np.zeros((nz, ny, nx, bs, bs))
        bl[tgt] = np.swapaxes(blocks[d][src], -1, -2)
        tw = np.zeros((nz, ny, nx), dtype=bool)
        tw[tgt] = touched[d][src]
        blocks[nd], touched[nd] = bl, tw
    dlin = np.array([lin(d) for d in dirs], dtype=np.int64)
    valid = np.stack([touched[d].ravel() for d in dirs], axis=1)
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    slot = row_ptr[:-1, None] + np.cumsum(valid, axis=1) - 1
    nnzb = int(row_ptr[-1])
    col = np.empty(nnzb, dtype=np.int32)
    vals = np.empty((nnzb, bs, bs))
    vid = np.arange(n, dtype=np.int64)
    for w, d in enumerate(dirs):
        m = valid[:, w]
        at = slot[m, w]
        col[at] = vid[m] + dlin[w]
        vals[at] = blocks[d].reshape(n, bs, bs)[m]
        del blocks[d]
    return row_ptr.astype(np.int32), col, vals


def _coef_array(mesh: KuhnMesh, c):
    """Broadcast a coefficient to per-(tet type, cell) form: scalar or (6, cells...)."""
    c = np.asarray(c, dtype=np.float64)
    if c.ndim == 0:
        return None, float(c)
    if c.shape != (6,) + mesh.cell_shape:
        raise ValueError("coefficient must be scalar or shaped (6, nz-1, ny-1, nx-1)")
    return c, None


def assemble_elasticity(mesh: KuhnMesh, mu, lam):
    """Block CSR (3x3) of the P1 linear elasticity matrix without boundary conditions.

    ``mu`` (= mu_L) and ``lam`` are scalars or per-(tet type, cell) arrays (6, nz-1, ny-1, nx-1).
    """
    _, Kmu, Klam, _ = _unit_element_matrices()
    mu_arr, mu_s = _coef_array(mesh, mu)
    lam_arr, lam_s = _coef_array(mesh, lam)
    h = mesh.h
    return _assemble(mesh, [(mu_arr if mu_arr is not None else mu_s, h * Kmu),
                            (lam_arr if lam_arr is not None else lam_s, h * Klam)])


def assemble_poisson(mesh: KuhnMesh, alpha=1.0):
    """Block CSR (1x1) of the P1 Laplacian ``int alpha grad u . grad v`` without BCs."""
    _, _, _, Klap = _unit_element_matrices()
    al_arr, al_s = _coef_array(mesh, alpha)
    return _assemble(mesh, [(al_arr if al_arr is not None else al_s, mesh.h * Klap)])


def sphere_inclusions(mesh: KuhnMesh, count: int, seed: int, E_host=1.0, nu_host=0.3,
                      E_inc=1.0e4, nu_lo=0.3, nu_hi=0.49, r_lo_cells=2.0, r_hi_cells=6.0):
    """Per-(tet type, cell) (mu_L, lambda) for a host material with random spherical inclusions.

    Sphere centres ~ U[0,1]^3, radii ~ U[r_lo h, r_hi h], inclusion Poisson ratio ~ U[nu_lo, nu_hi],
    all drawn from ``default_rng(seed)`` in that order per sphere.  A tetrahedron takes the
    material of the highest-index sphere containing its centroid.
    """
    rng = np.random.default_rng(seed)
    centres = np.empty((count, 3))
    radii = np.empty(count)
    nus = np.empty(count)
    for s in range(count):
        centres[s] = rng.uniform(0.0, 1.0, 3)
        radii[s] = rng.uniform(r_lo_cells * mesh.h, r_hi_cells * mesh.h)
        nus[s] = rng.uniform(nu_lo, nu_hi)
    mu_h, lam_h = lame_from_young(E_host, nu_host)
    mu = np.full((6,) + mesh.cell_shape, mu_h)
    lam = np.full((6,) + mesh.cell_shape, lam_h)
    for t in range(6):
        cen = mesh.tet_centroids(t)
        for s in range(count):
            inside = ((cen - centres[s]) ** 2).sum(axis=-1) <= radii[s] ** 2
            m, l_ = lame_from_young(E_inc, nus[s])
            mu[t][inside] = m
            lam[t][inside] = l_
    return mu, lam


def eleven_boxes(mesh: KuhnMesh, contrast=1.0e4, lam_over_mu=1.0):
    """Per-(tet type, cell) (mu_L, lambda) of the paper's difficult vector problem: a soft
    material (paper mu = lambda = 1) on the unit cube except the eleven diagonal boxes
    [(i-1)/11, i/11]^3, i = 1..11, which touch at their corners and are `contrast` times stiffer.
    The paper's mu is read as 2 mu_L (Hooke's law), so paper mu = lambda = c gives mu_L = c / 2,
    lambda = c.  A tetrahedron takes the material of the box containing its centroid."""
    mu = np.full((6,) + mesh.cell_shape, 0.5)
    lam = np.full((6,) + mesh.cell_shape, lam_over_mu)
    for t in range(6):
        cen = mesh.tet_centroids(t)
        box = np.floor(cen * 11.0).astype(np.int64)
        inside = (box[..., 0] == box[..., 1]) & (box[..., 1] == box[..., 2]) & (box[..., 0] >= 0) & (box[..., 0] < 11)
        mu[t][inside] = 0.5 * contrast
        lam[t][inside] = lam_over_mu * contrast
    return mu, lam


@dataclasses.dataclass
class KuhnProblem:
    """A generated problem: BC-free block matrix A_N, coordinates, Dirichlet mask, RHS."""
    name: str
    dim: int
    n_vertices: int
    coords: np.ndarray      # (n, 3) float64
    row_ptr: np.ndarray     # (n+1,) int32
    col_idx: np.ndarray     # (nnzb,) int32
    vals: np.ndarray        # (nnzb, dim, dim) float64, row-major blocks
    dirichlet: np.ndarray   # (n,) uint8, 1 = all components clamped
    b: np.ndarray           # (n*dim,) float64, zero at Dirichlet dofs
    meta: dict

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.size)

    @property
    def n_dofs(self) -> int:
        return self.n_vertices * self.dim

    @property
    def n_free_dofs(self) -> int:
        return int((self.dirichlet == 0).sum()) * self.dim


def random_rhs(n_dofs: int, dim: int, dirichlet: np.ndarray, seed) -> np.ndarray:
    """b ~ U[-1, 1] from ``numpy.random.default_rng(seed)`` (PCG64), zero at Dirichlet dofs."""
    b = np.random.default_rng(seed).uniform(-1.0, 1.0, n_dofs)
    b.reshape(-1, dim)[dirichlet.astype(bool)] = 0.0
    return b


def make_problem(n: int, *, kind: str = "elasticity", E: float = 1.0, nu: float = 0.3,
                 seed=0, clamp: str = "x0", inclusions: int = 0, geometry_seed: int = 5,
                 boxes: bool = False,
                 ny: Optional[int] = None, nz: Optional[int] = None, h: Optional[float] = None,
                 name: Optional[str] = None) -> KuhnProblem:
    """Generate a Kuhn box problem.

    kind: "elasticity" (dim 3) or "poisson" (dim 1).
    clamp: "x0" clamps the vertices with x = 0; "all" clamps the whole boundary; "none"
    gives a pure Neumann problem (singular A_N; only meaningful for setup checks).
    boxes: the eleven-box material of the paper's difficult vector problem (E, nu ignored).
    """
    mesh = kuhn_mesh(n, ny, nz, h)
    if kind == "elasticity":
        dim = 3
        if boxes:
            mu, lam = eleven_boxes(mesh)
        elif inclusions:
            mu, lam = sphere_inclusions(mesh, inclusions, geometry_seed, E_host=E, nu_host=nu)
        else:
            mu, lam = lame_from_young(E, nu)
        row_ptr, col, vals = assemble_elasticity(mesh, mu, lam)
    elif kind == "poisson":
        dim = 1
        row_ptr, col, vals = assemble_poisson(mesh, 1.0)
    else:
        raise ValueError(kind)
    coords = mesh.coords()
    nv = mesh.n_vertices
    dirichlet = np.zeros(nv, dtype=np.uint8)
    if clamp == "x0":
        dirichlet[coords[:, 0] == 0.0] = 1
    elif clamp == "all":
        ijk = np.rint(coords / mesh.h).astype(np.int64)
        top = np.array([mesh.nx - 1, mesh.ny - 1, mesh.nz - 1])
        dirichlet[((ijk == 0) | (ijk == top)).any(axis=1)] = 1
    elif clamp != "none":
        raise ValueError(clamp)
    b = random_rhs(nv * dim, dim, dirichlet, seed)
    meta = dict(kind=kind, n=n, ny=mesh.ny, nz=mesh.nz, h=mesh.h, E=E, nu=nu, seed=seed,
                clamp=clamp, inclusions=inclusions, boxes=boxes)
    return KuhnProblem(name or f"{kind}{n}", dim, nv, coords, row_ptr, col, vals, dirichlet, b,
                       meta)


# Named workloads: 3D linear elasticity on the unit cube, clamped at x = 0.
WORKLOADS = {
    # 17^3 vertices = 14,739 dofs, E=1, nu=0.3, RHS seed 0
    "cube17": dict(n=17, E=1.0, nu=0.3, seed=0),
    # 64^3 vertices = 786,432 dofs, same material, RHS seed 1
    "cube64": dict(n=64, E=1.0, nu=0.3, seed=1),
    # 128^3 vertices = 6,291,456 dofs, nu = 0.45, RHS seed 3
    "cube128_nu045": dict(n=128, E=1.0, nu=0.45, seed=3),
    # 96^3 vertices, 200 stiff spherical inclusions (E=1e4), geometry and RHS seed 5
    "spheres96": dict(n=96, E=1.0, nu=0.3, seed=5, inclusions=200, geometry_seed=5),
}

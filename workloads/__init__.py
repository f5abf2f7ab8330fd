"""Seeded synthetic inputs: meshes, the sparse matrices they discretise, and right-hand sides.

This module produces *data only*. It holds none of the solver's arithmetic (no
coarsening, no smoother, no cycle): both the CPU oracle and the GPU path take
their inputs from here and nothing else is shared between them.

The paper's data sets (structured WaterLily problems, unstructured canonical
flows, AirfRANS airfoils; Sec. 4 and App. C) are not available, so every input
is a synthetic stand-in that has the shape, size and value structure of those
workloads: symmetric matrices with a non-positive off-diagonal pattern from a
mesh, zero row sums for all-Neumann problems (the matrix class of Sec. 2.1,
Eq. 1, stored with a positive diagonal), and uniform random right-hand sides.

Every matrix is returned as CSR with int32 ``rowptr``/``col`` (columns sorted
ascending, diagonal stored) and float64 values.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSRMatrix:
    """Square or rectangular CSR matrix: int32 rowptr[n+1], int32 col[nnz], float64 val[nnz]."""

    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    nrows: int
    ncols: int

    @property
    def nnz(self) -> int:
        return int(self.col.size)

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.nrows, self.ncols))


def _from_triplets(rows, cols, vals, n) -> CSRMatrix:
    """CSR from unique (row, col) triplets; columns sorted within each row."""
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order]
    vals = vals[order]
    counts = np.bincount(rows, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return CSRMatrix(rowptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64), n, n)


def _laplacian_from_edges(i, j, w, n) -> CSRMatrix:
    """Symmetric graph Laplacian with off-diagonals -w_ij and diagonal sum_j w_ij.

    ``i < j`` lists each undirected edge once (duplicates allowed: their weights
    are summed in input order). The matrix is bitwise symmetric because each
    edge weight is stored once and mirrored.
    """
    key = i.astype(np.int64) * n + j.astype(np.int64)
    ukey, inv = np.unique(key, return_inverse=True)
    wsum = np.bincount(inv, weights=w)
    ui = (ukey // n).astype(np.int64)
    uj = (ukey % n).astype(np.int64)
    diag = np.bincount(ui, weights=wsum, minlength=n) + np.bincount(uj, weights=wsum, minlength=n)
    rows = np.concatenate([ui, uj, np.arange(n)])
    cols = np.concatenate([uj, ui, np.arange(n)])
    vals = np.concatenate([-wsum, -wsum, diag])
    return _from_triplets(rows, cols, vals, n)


# --------------------------------------------------------------------------------------
# Structured: 2D five-point Poisson (stand-in for the 2D "static" structured problems)
# --------------------------------------------------------------------------------------

def grid5(N: int) -> CSRMatrix:
    """Unscaled 5-point Laplacian on an N x N interior grid, Dirichlet boundary eliminated.

    Diagonal 4, off-diagonals -1, lexicographic order (k = y*N + x). Integer
    valued, hence exact in every precision.
    """
    n = N * N
    idx = np.arange(n).reshape(N, N)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [np.full(n, 4.0)]
    for a, b in ((idx[:, :-1], idx[:, 1:]), (idx[:-1, :], idx[1:, :])):
        rows += [a.ravel(), b.ravel()]
        cols += [b.ravel(), a.ravel()]
        vals += [np.full(a.size, -1.0), np.full(a.size, -1.0)]
    return _from_triplets(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)


# --------------------------------------------------------------------------------------
# Unstructured 2D: P1 finite-element Laplacian on a Delaunay triangulation
# --------------------------------------------------------------------------------------

def morton_order(points: np.ndarray) -> np.ndarray:
    """Stable permutation sorting 2D/3D points in [0,1]^d by their Morton (Z-order) code."""
    d = points.shape[1]
    bits = 21 if d == 3 else 31
    q = np.clip((points * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(points.shape[0], dtype=np.uint64)
    for b in range(bits):
        for k in range(d):
            code |= ((q[:, k] >> b) & 1).astype(np.uint64) << np.uint64(d * b + k)
    return np.argsort(code, kind="stable")


def boundary_points(m: int) -> np.ndarray:
    """4m points evenly spaced on the boundary of the unit square (spacing 1/m, corners included)."""
    t = np.arange(m) / m
    z, o = np.zeros(m), np.ones(m)
    return np.concatenate([np.stack([t, z], 1), np.stack([o, t], 1), np.stack([1 - t, o], 1), np.stack([z, 1 - t], 1)])


def _with_boundary(npts: int):
    """Boundary spacing h = 1/m with m = ceil(sqrt(npts)) (the mean spacing of npts points) and
    the number of interior points; interior points keep a distance of 0.3 h from the boundary so
    that no sliver triangle forms along it."""
    m = max(2, int(np.ceil(np.sqrt(npts))))
    nin = npts - 4 * m
    if nin < 1:
        raise ValueError("too few points for the boundary layout")
    return boundary_points(m), nin, 0.3 / m


def uniform_points(npts: int, seed: int) -> np.ndarray:
    """``npts`` points in the unit square: evenly spaced on the boundary, uniform inside; Morton sorted."""
    bnd, nin, gap = _with_boundary(npts)
    rng = np.random.default_rng(seed)
    p = np.concatenate([gap + (1.0 - 2.0 * gap) * rng.random((nin, 2)), bnd])
    return p[morton_order(p)]


def gmm_points(npts: int, seed: int) -> np.ndarray:
    """Points clustered by a random Gaussian mixture, plus 20% uniform background.

    K ~ U{2..6} components, means in [0.1, 0.9]^2, isotropic sigma ~ U[0.02, 0.15]; samples
    closer than the boundary gap to the border are rejected. Evenly spaced boundary points
    close the domain; the result is Morton sorted.
    """
    bnd, nin, gap = _with_boundary(npts)
    rng = np.random.default_rng(seed)
    K = int(rng.integers(2, 7))
    means = rng.uniform(0.1, 0.9, size=(K, 2))
    sig = rng.uniform(0.02, 0.15, size=K)
    nbg = int(round(0.2 * nin))
    out = [gap + (1.0 - 2.0 * gap) * rng.random((nbg, 2))]
    need = nin - nbg
    while need > 0:
        comp = rng.integers(0, K, size=2 * need)
        cand = means[comp] + sig[comp, None] * rng.standard_normal((2 * need, 2))
        ok = np.all((cand > gap) & (cand < 1.0 - gap), axis=1)
        cand = cand[ok][:need]
        out.append(cand)
        need -= cand.shape[0]
    p = np.concatenate(out + [bnd])
    return p[morton_order(p)]


def delaunay_p1(points: np.ndarray) -> CSRMatrix:
    """P1 (linear triangle) stiffness matrix of -Laplace with natural boundary conditions.

    Off-diagonal a_ij = -1/2 (cot alpha + cot beta), the angles opposite edge ij;
    the diagonal makes every row sum zero, so the matrix is singular with the
    constant vector as null space, like the paper's Poisson class.
    """
    from scipy.spatial import Delaunay

    tri = Delaunay(points).simplices.astype(np.int64)
    n = points.shape[0]
    if np.unique(tri).size != n:
        raise ValueError("triangulation dropped points (duplicates?)")
    i_l, j_l, w_l = [], [], []
    for a, b, c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        pa, pb, pc = points[tri[:, a]], points[tri[:, b]], points[tri[:, c]]
        u = pb - pa
        v = pc - pa
        dot = u[:, 0] * v[:, 0] + u[:, 1] * v[:, 1]
        cross = np.abs(u[:, 0] * v[:, 1] - u[:, 1] * v[:, 0])
        if not np.all(cross > 0):
            raise ValueError("degenerate (zero-area) triangle")
        w = 0.5 * dot / cross  # half the cotangent of the angle at vertex a, for edge (b, c)
        lo = np.minimum(tri[:, b], tri[:, c])
        hi = np.maximum(tri[:, b], tri[:, c])
        i_l.append(lo)
        j_l.append(hi)
        w_l.append(w)
    return _laplacian_from_edges(np.concatenate(i_l), np.concatenate(j_l), np.concatenate(w_l), n)


def rhs_uniform(n: int, seed: int, zero_mean: bool = False) -> np.ndarray:
    """Right-hand side with entries ~ U[-1, 1]; mean removed for all-Neumann problems."""
    f = np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)
    if zero_mean:
        f = f - f.mean()
    return f


# --------------------------------------------------------------------------------------
# Anisotropic 2D: finite-volume Poisson on a C-mesh around a NACA 4-digit airfoil
# (stand-in for airfoil RANS meshes with highly stretched inflation layers)
# --------------------------------------------------------------------------------------

def naca4(code: str, x: np.ndarray):
    """Upper and lower surface points of a NACA 4-digit section (chord 1) at stations x."""
    m, p, t = int(code[0]) / 100.0, int(code[1]) / 10.0, int(code[2:]) / 100.0
    yt = 5 * t * (0.2969 * np.sqrt(x) - 0.1260 * x - 0.3516 * x**2 + 0.2843 * x**3 - 0.1036 * x**4)
    if m == 0.0 or p == 0.0:  # symmetric section (00xx): no camber line
        yc = dy = np.zeros_like(x)
    else:
        yc = np.where(x < p, m / p**2 * (2 * p * x - x**2), m / (1 - p) ** 2 * ((1 - 2 * p) + 2 * p * x - x**2))
        dy = np.where(x < p, 2 * m / p**2 * (p - x), 2 * m / (1 - p) ** 2 * (p - x))
    th = np.arctan(dy)
    return (np.stack([x - yt * np.sin(th), yc + yt * np.cos(th)], 1),
            np.stack([x + yt * np.sin(th), yc - yt * np.cos(th)], 1))


def cmesh_nodes(ni: int, nj: int, code: str = "2412", aspect: float = 1e4, radius: float = 20.0, wake: float = 20.0):
    """Node coordinates [(ni+1), (nj+1), 2] of an algebraic C-mesh.

    i runs along the C: lower wake (downstream to trailing edge), lower surface, upper surface,
    upper wake; j runs away from the wall with geometric stretching whose first cell has a
    height of (mean wall spacing)/aspect, so wall cells reach the given aspect ratio.
    """
    nw = ni // 4                      # cells on each wake branch
    na = ni - 2 * nw                  # cells around the airfoil
    half = na // 2
    beta = np.linspace(0.0, np.pi, half + 1)
    xs = 0.5 * (1.0 - np.cos(beta))   # cosine clustering at both edges
    up, lo = naca4(code, xs)
    surf = np.concatenate([lo[::-1], up[1:]])                         # TE (lower) -> LE -> TE (upper)
    surf = surf[: na + 1] if surf.shape[0] >= na + 1 else np.concatenate([surf, surf[-1:]])
    te = 0.5 * (surf[0] + surf[-1])
    g = np.geomspace(1e-3, 1.0, nw + 1) * wake                       # wake clustered at the trailing edge
    wx = te[0] + np.concatenate([[0.0], g[1:]])
    wake_lo = np.stack([wx[::-1], np.full(nw + 1, te[1])], 1)
    wake_up = np.stack([wx, np.full(nw + 1, te[1])], 1)
    curve = np.concatenate([wake_lo[:-1], surf, wake_up[1:]])        # ni + 1 points
    tang = np.gradient(curve, axis=0)
    tang /= np.linalg.norm(tang, axis=1, keepdims=True)
    normal = np.stack([tang[:, 1], -tang[:, 0]], 1)                  # outward of the C
    normal[: nw] = [0.0, -1.0]
    normal[-nw:] = [0.0, 1.0]
    ds = np.mean(np.linalg.norm(np.diff(surf, axis=0), axis=1))
    h0 = ds / aspect
    r = 1.0 + 1e-3
    for _ in range(200):              # solve h0 (r^nj - 1)/(r - 1) = radius for the growth rate
        r = (1.0 + radius * (r - 1.0) / h0) ** (1.0 / nj)
    d = np.concatenate([[0.0], h0 * (r ** np.arange(1, nj + 1) - 1.0) / (r - 1.0)])
    return curve[:, None, :] + d[None, :, None] * normal[:, None, :]


def cmesh_fv(ni: int, nj: int, code: str = "2412", aspect: float = 1e4) -> CSRMatrix:
    """Cell-centred finite-volume Poisson matrix on the C-mesh (two-point flux |face|/|c_i - c_j|).

    Wall faces are Neumann; the outer C and the two downstream boundaries are Dirichlet p = 0
    (their flux adds to the diagonal), so the matrix is SPD. Across the wake cut, cell (i, 0)
    of the lower branch neighbours cell (ni-1-i, 0) of the upper branch.
    """
    X = cmesh_nodes(ni, nj, code, aspect)
    C = 0.25 * (X[:-1, :-1] + X[1:, :-1] + X[:-1, 1:] + X[1:, 1:])  # cell centres [ni, nj, 2]
    idx = np.arange(ni * nj).reshape(ni, nj)

    def flux(face_a, face_b, ca, cb):
        return np.linalg.norm(face_b - face_a, axis=-1) / np.linalg.norm(cb - ca, axis=-1)

    ii, jj, ww = [], [], []
    # i-direction neighbours: shared face between nodes (i+1, j) and (i+1, j+1)
    w = flux(X[1:-1, :-1], X[1:-1, 1:], C[:-1], C[1:])
    ii.append(idx[:-1].ravel()); jj.append(idx[1:].ravel()); ww.append(w.ravel())
    # j-direction neighbours: shared face between nodes (i, j+1) and (i+1, j+1)
    w = flux(X[:-1, 1:-1], X[1:, 1:-1], C[:, :-1], C[:, 1:])
    ii.append(idx[:, :-1].ravel()); jj.append(idx[:, 1:].ravel()); ww.append(w.ravel())
    # wake cut: lower-branch cell i and upper-branch cell ni-1-i share the j = 0 face
    nw = ni // 4
    lo_i = np.arange(nw)
    up_i = ni - 1 - lo_i
    w = np.linalg.norm(X[lo_i + 1, 0] - X[lo_i, 0], axis=-1) / np.linalg.norm(C[up_i, 0] - C[lo_i, 0], axis=-1)
    ii.append(idx[lo_i, 0]); jj.append(idx[up_i, 0]); ww.append(w)
    i_all = np.concatenate(ii)
    j_all = np.concatenate(jj)
    A = _laplacian_from_edges(np.minimum(i_all, j_all), np.maximum(i_all, j_all), np.concatenate(ww), ni * nj)
    # Dirichlet outer boundary (j = nj - 1 north faces, i = 0 and i = ni - 1 end faces)
    bd = np.zeros(ni * nj)
    far = flux(X[:-1, -1], X[1:, -1], C[:, -1], 2 * 0.5 * (X[:-1, -1] + X[1:, -1]) - C[:, -1])
    bd[idx[:, -1]] += far
    for i_end, node in ((0, 0), (ni - 1, ni)):
        mid = 0.5 * (X[node, :-1] + X[node, 1:])
        bd[idx[i_end]] += flux(X[node, :-1], X[node, 1:], C[i_end], 2 * mid - C[i_end])
    rowid = np.repeat(np.arange(ni * nj), np.diff(A.rowptr))
    isd = A.col == rowid
    A.val[isd] += bd[rowid[isd]]
    return A


def airfoil_cmesh_problem(ni: int = 4096, nj: int = 1024, seed: int = 0):
    """C-mesh FV Poisson around NACA 2412 (wall aspect ratio 1e4), f ~ U[-1, 1]."""
    A = cmesh_fv(ni, nj)
    return A, rhs_uniform(A.nrows, seed + 3000)


# --------------------------------------------------------------------------------------
# 3D: finite-volume Poisson on a random tetrahedral mesh of the unit cube
# --------------------------------------------------------------------------------------

def jittered_lattice(m: int, seed: int, jitter: float = 0.3) -> np.ndarray:
    """m^3 lattice points in the unit cube, interior points moved by U[-jitter h, jitter h]."""
    h = 1.0 / (m - 1)
    g = np.arange(m) * h
    P = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(seed)
    inner = np.all((P > 0.5 * h) & (P < 1 - 0.5 * h), axis=1)
    P[inner] += rng.uniform(-jitter * h, jitter * h, size=(int(inner.sum()), 3))
    return P


def tet_fv(points: np.ndarray) -> CSRMatrix:
    """Cell-centred FV Poisson matrix on the Delaunay tetrahedra of `points`: cells are tets,
    face-neighbours couple with |face| / |centroid distance|; all-Neumann (zero row sums).
    Cells are Morton ordered by centroid."""
    from scipy.spatial import Delaunay

    d = Delaunay(points)
    tets = d.simplices.astype(np.int64)
    cent = points[tets].mean(axis=1)
    vol = np.abs(np.einsum("ij,ij->i", np.cross(points[tets[:, 1]] - points[tets[:, 0]],
                                               points[tets[:, 2]] - points[tets[:, 0]]),
                           points[tets[:, 3]] - points[tets[:, 0]])) / 6.0
    keep = vol > 1e-12 * vol.max()       # drop flat slivers qhull may leave on the boundary
    order = morton_order((cent - cent.min(0)) / (np.ptp(cent, 0) + 1e-300))
    remap = -np.ones(tets.shape[0], np.int64)
    kept = order[keep[order]]
    remap[kept] = np.arange(kept.size)
    nb = d.neighbors.astype(np.int64)
    ii, jj, ww = [], [], []
    for f in range(4):
        other = nb[:, f]
        ok = keep & (other >= 0) & (np.arange(tets.shape[0]) < np.where(other >= 0, other, 0))
        ok &= np.where(other >= 0, keep[np.where(other >= 0, other, 0)], False)
        a = np.nonzero(ok)[0]
        b = other[a]
        face = np.delete(tets[a], f, axis=1)  # the three vertices opposite vertex f
        area = 0.5 * np.linalg.norm(np.cross(points[face[:, 1]] - points[face[:, 0]],
                                             points[face[:, 2]] - points[face[:, 0]]), axis=1)
        dist = np.linalg.norm(cent[a] - cent[b], axis=1)
        ii.append(remap[a]); jj.append(remap[b]); ww.append(area / dist)
    i_all, j_all = np.concatenate(ii), np.concatenate(jj)
    return _laplacian_from_edges(np.minimum(i_all, j_all), np.maximum(i_all, j_all), np.concatenate(ww), kept.size)


def kuhn_tets(m: int, seed: int, jitter: float = 0.15):
    """Tetrahedral mesh of the unit cube: an m^3 lattice, interior points moved by
    U[-jitter h, jitter h], each lattice cube split into the 6 tetrahedra around its main
    diagonal (the Freudenthal/Kuhn split, conforming across cubes). With jitter <= 0.15 every
    tetrahedron keeps its orientation (each vertex-to-face distance is at least h/sqrt(2), and
    a jitter of 0.15 h per coordinate moves a vertex and its opposite face by at most 0.21 h
    each along the face normal). Returns (points[m^3, 3], tets[6 (m-1)^3, 4])."""
    P = jittered_lattice(m, seed, jitter)
    g = np.arange(m - 1)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    base = (I * m * m + J * m + K).ravel().astype(np.int64)
    step = {0: m * m, 1: m, 2: 1}
    tets = []
    for a, b, c in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        v1 = base + step[a]
        v2 = v1 + step[b]
        v3 = v2 + step[c]
        tets.append(np.stack([base, v1, v2, v3], axis=1))
    return P, np.concatenate(tets)


def tet_fv_mesh(points: np.ndarray, tets: np.ndarray) -> CSRMatrix:
    """Cell-centred FV Poisson matrix on a conforming tetrahedral mesh (cells = tets, face
    neighbours couple with |face| / |centroid distance|, all-Neumann), face neighbours found by
    matching the sorted vertex triples of the faces. Cells are Morton ordered by centroid."""
    nt = tets.shape[0]
    npnt = np.int64(points.shape[0])
    cent = points[tets].mean(axis=1)
    order = morton_order((cent - cent.min(0)) / (np.ptp(cent, 0) + 1e-300))
    remap = np.empty(nt, np.int64)
    remap[order] = np.arange(nt)
    keys, owners = [], []
    for f in range(4):
        a, b, c = (tets[:, k] for k in range(4) if k != f)
        lo = np.minimum(np.minimum(a, b), c)
        hi = np.maximum(np.maximum(a, b), c)
        mid = a + b + c - lo - hi
        keys.append((lo * npnt + mid) * npnt + hi)
        owners.append(np.arange(nt, dtype=np.int64))
    key = np.concatenate(keys)
    owner = np.concatenate(owners)
    srt = np.argsort(key)
    ks = key[srt]
    pair = np.nonzero(ks[1:] == ks[:-1])[0]
    a, b = owner[srt[pair]], owner[srt[pair + 1]]
    fk = ks[pair]
    v0, v1, v2 = fk // (npnt * npnt), (fk // npnt) % npnt, fk % npnt
    area = 0.5 * np.linalg.norm(np.cross(points[v1] - points[v0], points[v2] - points[v0]), axis=1)
    dist = np.linalg.norm(cent[a] - cent[b], axis=1)
    i_all, j_all = remap[a], remap[b]
    return _laplacian_from_edges(np.minimum(i_all, j_all), np.maximum(i_all, j_all), area / dist, nt)


def tet_kuhn_problem(m: int, seed: int = 0):
    """3D FV Poisson on the Kuhn tetrahedra of an m^3 jittered lattice (6 (m-1)^3 cells; m = 111
    gives 7,986,000 cells), zero-mean RHS."""
    P, T = kuhn_tets(m, seed)
    A = tet_fv_mesh(P, T)
    return A, rhs_uniform(A.nrows, seed + 5000, zero_mean=True)


def tet_fv_problem(m: int, seed: int = 0):
    """3D FV Poisson on the tetrahedra of an m^3 jittered lattice, zero-mean RHS."""
    A = tet_fv(jittered_lattice(m, seed))
    return A, rhs_uniform(A.nrows, seed + 4000, zero_mean=True)


# --------------------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------------------

def poisson_grid_64(seed: int = 0):
    """64 x 64 Dirichlet 5-point Poisson, 4096 unknowns, f ~ U[-1,1] (seeded)."""
    A = grid5(64)
    return A, rhs_uniform(A.nrows, seed)


def delaunay_p1_problem(npts: int, seed: int = 0):
    """P1 Laplacian on a Delaunay mesh of ``npts`` points (uniform inside, even on the boundary), zero-mean RHS."""
    A = delaunay_p1(uniform_points(npts, seed))
    return A, rhs_uniform(A.nrows, seed + 1000, zero_mean=True)


def training_batch(nmesh: int = 32, seed: int = 0, lo: int = 2000, hi: int = 16000):
    """Batch of Gaussian-mixture-clustered Delaunay P1 meshes with sizes ~ U[lo, hi]."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, size=nmesh)
    out = []
    for m, npts in enumerate(sizes):
        A = delaunay_p1(gmm_points(int(npts), seed * 1000 + m))
        f = rhs_uniform(A.nrows, seed * 1000 + m + 500, zero_mean=True)
        out.append((A, f))
    return out

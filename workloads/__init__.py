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

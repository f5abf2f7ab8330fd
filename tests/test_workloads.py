"""Properties of the synthetic inputs (the matrix class of Sec. 2.1, Eq. 1, in the stored sign)."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W


def _check_csr(A):
    assert A.rowptr[0] == 0 and A.rowptr[-1] == A.col.size
    for i in range(0, A.nrows, max(1, A.nrows // 200)):
        c = A.col[A.rowptr[i]:A.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c


@pytest.mark.parametrize("make", [
    lambda: W.grid5(10),
    lambda: W.delaunay_p1(W.uniform_points(3000, 1)),
    lambda: W.delaunay_p1(W.gmm_points(3000, 2)),
    lambda: W.cmesh_fv(64, 32),
    lambda: W.tet_fv(W.jittered_lattice(9, 3)),
])
def test_matrix_class(make):
    A = make()
    _check_csr(A)
    S = A.to_scipy()
    assert abs(S - S.T).max() == 0.0  # bitwise symmetric
    d = S.diagonal()
    assert np.all(d > 0)
    off = S - sp.diags(d)
    rs = np.asarray(S.sum(axis=1)).ravel()
    assert np.all(rs >= -1e-12 * d)  # weakly diagonally dominant in row sums
    ev = np.linalg.eigvalsh(S.toarray()) if S.shape[0] <= 2500 else None
    if ev is not None:
        assert ev[0] > -1e-10 * ev[-1]  # positive semi-definite


def test_p1_and_tet_are_all_neumann_and_cmesh_is_not():
    for A in (W.delaunay_p1(W.uniform_points(2000, 0)), W.tet_fv(W.jittered_lattice(8, 0))):
        S = A.to_scipy()
        assert np.abs(np.asarray(S.sum(axis=1))).max() <= 1e-12 * S.diagonal().max()
    S = W.cmesh_fv(64, 32).to_scipy()
    rs = np.asarray(S.sum(axis=1)).ravel()
    assert rs.max() > 0.1 * np.median(S.diagonal())  # Dirichlet far field rows


def test_cmesh_wall_cells_reach_target_aspect_ratio():
    X = W.cmesh_nodes(256, 128, aspect=1e4)
    ni = 256
    nw = ni // 4
    wall = slice(nw + 4, ni - nw - 4)  # airfoil cells away from the trailing edge
    along = np.linalg.norm(X[1:, 0] - X[:-1, 0], axis=-1)[wall]
    normal = np.linalg.norm(X[:-1, 1] - X[:-1, 0], axis=-1)[wall]
    ar = along / normal
    assert 1e3 < np.median(ar) < 1e5


def test_row_lengths_match_the_mesh_type():
    A2 = W.delaunay_p1(W.uniform_points(20000, 5))
    assert 6.8 < A2.nnz / A2.nrows < 7.1
    A3 = W.tet_fv(W.jittered_lattice(14, 5))
    assert 4.6 < A3.nnz / A3.nrows <= 5.0
    Ac = W.cmesh_fv(128, 64)
    assert 4.9 < Ac.nnz / Ac.nrows <= 5.0


def test_generators_are_deterministic():
    a = W.delaunay_p1_problem(1500, 3)
    b = W.delaunay_p1_problem(1500, 3)
    assert np.array_equal(a[0].val, b[0].val) and np.array_equal(a[1], b[1])
    t1 = W.tet_fv(W.jittered_lattice(7, 1))
    t2 = W.tet_fv(W.jittered_lattice(7, 1))
    assert np.array_equal(t1.col, t2.col) and np.array_equal(t1.val, t2.val)


def test_kuhn_tetrahedra_keep_orientation_and_fill_the_cube():
    m = 9
    P0, T = W.kuhn_tets(m, 0, jitter=0.0)
    P, T2 = W.kuhn_tets(m, 0, jitter=0.15)
    assert np.array_equal(T, T2) and T.shape == (6 * (m - 1) ** 3, 4)

    def vol(P):
        a, b, c, d = (P[T[:, k]] for k in range(4))
        return np.einsum("ij,ij->i", np.cross(b - a, c - a), d - a) / 6.0

    v0, v = vol(P0), vol(P)
    assert np.all(np.sign(v) == np.sign(v0)) and np.all(np.abs(v) > 0)
    assert abs(np.abs(v0).sum() - 1.0) < 1e-12 and abs(np.abs(v).sum() - 1.0) < 1e-12  # a partition of the cube


def test_tet_fv_mesh_face_neighbours():
    A = W.tet_fv_mesh(*W.kuhn_tets(7, 3))
    deg = np.diff(A.rowptr) - 1
    assert deg.max() == 4 and deg.min() >= 1
    # interior cells have four face neighbours; boundary faces (2 per boundary square) are open
    n_bdry_faces = 6 * 2 * 6 ** 2
    assert (4 * A.nrows - deg.sum()) == n_bdry_faces
    S = A.to_scipy()
    assert abs(S - S.T).max() == 0.0
    assert np.abs(np.asarray(S.sum(axis=1))).max() <= 1e-12 * S.diagonal().max()


def test_symmetric_naca_section_has_no_camber():
    x = np.linspace(0.0, 1.0, 41)
    up, lo = W.naca4("0012", x)
    assert np.allclose(up[:, 0], x) and np.allclose(lo[:, 0], x)
    assert np.allclose(up[:, 1], -lo[:, 1])
    assert abs(up[:, 1].max() - 0.06) < 2e-3  # 12 % thickness, half above the chord

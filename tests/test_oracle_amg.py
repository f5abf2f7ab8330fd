"""Pins of the oracle AMG against closed forms, invariants, library routines and brute force.

Each test names what fixes the expected value independently of the oracle's own code.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as W
from oracle import amg

HERE = os.path.dirname(__file__)


def _grid_eigvec(N, p, q):
    h = 1.0 / (N + 1)
    i = np.arange(1, N + 1)
    vx = np.sin(p * np.pi * i * h)
    vy = np.sin(q * np.pi * i * h)
    return np.outer(vy, vx).ravel()  # index k = y*N + x


def _kappa(N, p, q):
    h = 1.0 / (N + 1)
    return 2 * np.cos(p * np.pi * h) + 2 * np.cos(q * np.pi * h)


# ---------------------------------------------------------------------------------------------
# Smoother (Sec. 3.1, Eq. 5) against the closed-form spectrum of the 5-point Laplacian
# ---------------------------------------------------------------------------------------------


def test_jacobi_smoothing_factor_closed_form():
    """omega-Jacobi on the 5-point grid: mu_pq = 1 - omega + omega/2 (cos p pi h + cos q pi h)."""
    N = 64
    A = amg.to_scipy(W.grid5(N))
    omega = 2.0 / 3.0
    Q = amg.assemble_smoother(A, amg.jacobi_coeffs(omega), 2)
    h = 1.0 / (N + 1)
    for p, q in [(1, 1), (64, 64), (3, 17), (40, 2)]:
        v = _grid_eigvec(N, p, q)
        mu = 1 - omega + omega / 2 * (np.cos(p * np.pi * h) + np.cos(q * np.pi * h))
        out = amg.smooth(A, Q, v, np.zeros_like(v), 1)
        assert np.allclose(out, mu * v, rtol=0, atol=1e-13 * np.abs(v).max())
    # the two numbers quoted for this grid at omega = 2/3
    mu11 = 1 - omega + omega / 2 * 2 * np.cos(np.pi * h)
    mu6464 = 1 - omega + omega / 2 * 2 * np.cos(64 * np.pi * h)
    assert abs(mu11 - 0.999221) < 5e-7 and abs(mu6464 + 0.332555) < 5e-7


@pytest.mark.parametrize("coeffs", [
    [0.5, 0.05, -0.01, 0.3, 0.02],
    [0.9, -0.1, 0.02, -0.4, 0.1],
    [0.7, 0.0, 0.0, 0.25, 0.0],
])
def test_polynomial_smoother_closed_form(coeffs):
    """Unscaled 5-point grid (s = 1): Q = alpha I + beta N with alpha = f_d(4)/4, beta = f_o(-1)/8.

    On eigenvector (p, q): mu = 1 - (alpha + beta kappa)(4 - kappa), kappa = 2 cos p pi h + 2 cos q pi h.
    The polynomials are evaluated here with numpy.polyval (not the oracle's Horner code).
    """
    N = 32
    A = amg.to_scipy(W.grid5(N))
    Q = amg.assemble_smoother(A, coeffs, 2)
    d0, d1, d2, o1, o2 = coeffs
    alpha = np.polyval([d2, d1, d0], 4.0) / 4.0
    beta = np.polyval([o2, o1, 0.0], -1.0) / 8.0
    for p, q in [(1, 1), (32, 32), (5, 9), (20, 3)]:
        v = _grid_eigvec(N, p, q)
        k = _kappa(N, p, q)
        mu = 1 - (alpha + beta * k) * (4 - k)
        out = amg.smooth(A, Q, v, np.zeros_like(v), 1)
        assert np.allclose(out, mu * v, rtol=0, atol=1e-13 * np.abs(v).max())


def test_smoother_scale_invariance_and_symmetry():
    """Scaling A by c rescales s, so Q^{-1} scales by 1/c and Q^{-1} A is unchanged; Q^{-1} is symmetric."""
    A = amg.to_scipy(W.delaunay_p1(W.uniform_points(300, 3)))
    c = [0.6, 0.1, -0.02, 0.2, 0.05]
    Q1 = amg.assemble_smoother(A, c, 2)
    Q2 = amg.assemble_smoother(A * 8.0, c, 2)  # power of two: exact scaling
    assert np.array_equal(Q1.data, Q2.data * 8.0)
    D = Q1.toarray()
    assert np.allclose(D, D.T, rtol=1e-14, atol=0)


def test_smoother_bruteforce_dense():
    """Entry-by-entry construction of Eq. 5 from a dense copy of A, with numpy.polyval."""
    A = amg.to_scipy(W.delaunay_p1(W.gmm_points(60, 5)))
    c = np.array([0.55, 0.07, -0.03, 0.31, -0.04, 0.0, 0.0])[:5]
    Q = amg.assemble_smoother(A, c, 2).toarray()
    M = A.toarray()
    s = np.max(np.abs(M - np.diag(np.diag(M))))
    ref = np.zeros_like(M)
    for i in range(M.shape[0]):
        for j in range(M.shape[1]):
            if i == j:
                ref[i, j] = np.polyval(c[2::-1], M[i, i] / s) / M[i, i]
            elif M[i, j] != 0.0:
                ref[i, j] = np.polyval([c[4], c[3], 0.0], M[i, j] / s) / (M[i, i] + M[j, j])
    assert np.allclose(Q, ref, rtol=1e-14, atol=1e-300)


def test_jacobi_coefficients_give_diagonal_smoother():
    """c = (omega, 0, 0, 0, 0) is exactly omega D^{-1} (Sec. 4 baseline), bit for bit."""
    A = amg.to_scipy(W.delaunay_p1(W.uniform_points(200, 1)))
    Q = amg.assemble_smoother(A, amg.jacobi_coeffs(2 / 3), 2).toarray()
    d = A.diagonal()
    assert np.array_equal(np.diag(Q), (2 / 3) / d)
    off = Q - np.diag(np.diag(Q))
    assert np.all(off == 0.0)


# ---------------------------------------------------------------------------------------------
# Ruge-Stueben setup
# ---------------------------------------------------------------------------------------------


def test_strength_five_point_all_strong():
    A = amg.to_scipy(W.grid5(8))
    S = amg.strength(A, 0.25)
    offdiag = A.copy()
    offdiag.setdiag(0)
    offdiag.eliminate_zeros()
    assert np.array_equal(S.indptr, offdiag.indptr) and np.array_equal(S.indices, offdiag.indices)


def _naive_first_pass(S):
    """Independent quadratic-time statement of the same first pass (scan for max lambda each step)."""
    n = S.shape[0]
    Sd = (S.toarray() != 0)
    state = np.full(n, -1)
    for i in range(n):
        if not Sd[i].any() and not Sd[:, i].any():
            state[i] = 0
    lam = Sd.sum(axis=0).astype(int)  # lambda_i = |{j : i in S_j}|
    while (state == -1).any():
        und = np.where(state == -1)[0]
        i = und[np.argmax(lam[und])]  # argmax returns the first (smallest index) maximum
        state[i] = 1
        newf = [j for j in range(n) if state[j] == -1 and Sd[j, i]]
        for j in newf:
            state[j] = 0
        for j in newf:
            for k in range(n):
                if Sd[j, k] and state[k] == -1:
                    lam[k] += 1
        for k in range(n):
            if Sd[i, k] and state[k] == -1:
                lam[k] -= 1
    return state


@pytest.mark.parametrize("seed", range(6))
def test_cf_split_matches_bruteforce(seed):
    pts = W.gmm_points(30, seed) if seed % 2 else W.uniform_points(30, seed)
    A = amg.to_scipy(W.delaunay_p1(pts))
    S = amg.strength(A, 0.25)
    assert np.array_equal(amg.cf_split(S), _naive_first_pass(S))


def test_cf_split_invariants():
    A = amg.to_scipy(W.delaunay_p1(W.gmm_points(3000, 11)))
    S = amg.strength(A, 0.25)
    st = amg.cf_split(S)
    assert set(np.unique(st)) <= {0, 1}
    for i in range(A.shape[0]):
        if st[i] == 0:
            strong = S.indices[S.indptr[i]:S.indptr[i + 1]]
            has_in = S[:, [i]].nnz > 0
            if strong.size or has_in:
                assert (st[strong] == 1).any(), f"F point {i} lacks a strong C neighbour"


def test_interpolation_preserves_constants_and_injects_c_points():
    """Zero-row-sum rows: P 1 = 1 (direct interpolation reproduces constants); C rows are identity rows."""
    A = amg.to_scipy(W.delaunay_p1(W.uniform_points(2000, 4)))
    S = amg.strength(A, 0.25)
    st = amg.cf_split(S)
    P = amg.direct_interpolation(A, S, st)
    assert np.allclose(P @ np.ones(P.shape[1]), 1.0, rtol=0, atol=1e-14)
    cidx = np.where(st == 1)[0]
    Pc = P[cidx].toarray()
    assert np.array_equal(Pc, np.eye(cidx.size))
    # F rows only interpolate from strong C neighbours
    cid = -np.ones(A.shape[0], int)
    cid[cidx] = np.arange(cidx.size)
    for i in np.where(st == 0)[0][:500]:
        cols = P.indices[P.indptr[i]:P.indptr[i + 1]]
        strong = S.indices[S.indptr[i]:S.indptr[i + 1]]
        assert set(cols) <= set(cid[strong[st[strong] == 1]])


def test_interpolation_weights_five_point_interior():
    """Interior F point of the 5-point grid with all four neighbours C: alpha = 1, weights 1/4."""
    A = amg.to_scipy(W.grid5(16))
    S = amg.strength(A, 0.25)
    st = amg.cf_split(S)
    P = amg.direct_interpolation(A, S, st)
    N = 16
    checked = 0
    for y in range(1, N - 1):
        for x in range(1, N - 1):
            k = y * N + x
            nb = [k - 1, k + 1, k - N, k + N]
            if st[k] == 0 and all(st[j] == 1 for j in nb):
                row = P.data[P.indptr[k]:P.indptr[k + 1]]
                assert np.array_equal(row, np.full(4, 0.25))
                checked += 1
    assert checked > 20


@pytest.mark.parametrize("seed", range(4))
def test_spgemm_vectorised_is_bitwise_loop(seed):
    rng = np.random.default_rng(seed)
    A = sp.random(40, 30, density=0.15, random_state=rng, format="csr")
    B = sp.random(30, 25, density=0.2, random_state=rng, format="csr")
    A.data = rng.standard_normal(A.nnz)
    B.data = rng.standard_normal(B.nnz)
    A.sort_indices()
    B.sort_indices()
    C1 = amg.spgemm_rowwise(A, B)
    C2 = amg.spgemm_rowwise_vec(A, B)
    assert np.array_equal(C1.indptr, C2.indptr)
    assert np.array_equal(C1.indices, C2.indices)
    assert np.array_equal(C1.data, C2.data)
    assert np.allclose(C1.toarray(), A.toarray() @ B.toarray(), rtol=1e-13, atol=1e-13)


def test_galerkin_vectorised_is_bitwise_loop():
    A = amg.to_scipy(W.delaunay_p1(W.gmm_points(800, 2)))
    S = amg.strength(A, 0.25)
    P = amg.direct_interpolation(A, S, amg.cf_split(S))
    G1 = amg.galerkin(A, P, vectorised=False)
    G2 = amg.galerkin(A, P, vectorised=True)
    assert np.array_equal(G1.indptr, G2.indptr) and np.array_equal(G1.indices, G2.indices)
    assert np.array_equal(G1.data, G2.data)


@pytest.mark.parametrize("make", ["grid", "delaunay"])
def test_galerkin_dense_triple_product(make):
    A = amg.to_scipy(W.grid5(20) if make == "grid" else W.delaunay_p1(W.uniform_points(500, 7)))
    h = amg.setup(A, max_levels=4, max_coarse=10)
    for lvl in range(h.nlevels - 1):
        Af = h.levels[lvl].A.toarray()
        P = h.levels[lvl].P.toarray()
        Ac = h.levels[lvl + 1].A.toarray()
        ref = P.T @ Af @ P
        assert np.abs(Ac - ref).max() <= 1e-14 * np.abs(ref).max()
        assert np.abs(Ac - Ac.T).max() <= 1e-14 * np.abs(Ac).max()
        assert np.array_equal(h.levels[lvl].R.toarray(), P.T)
        if make == "delaunay":
            assert np.abs(Ac.sum(axis=1)).max() <= 1e-13 * np.abs(np.diag(Ac)).max()


def test_hierarchy_five_point_sizes():
    """64 x 64 Dirichlet grid, 3 levels: the first pass picks every other point (red-black), n_1 = 2048."""
    A, f, sing = amg.normalize(*W.poisson_grid_64(0))
    assert not sing and A.nnz == 20224
    h = amg.setup(A, max_levels=3)
    assert [L.A.shape[0] for L in h.levels][:2] == [4096, 2048]
    assert h.nlevels == 3


def test_normalize_negated_convention():
    """The paper's negative semi-definite form (-A, -f) gives bitwise the same stored system and solution."""
    A, f = W.delaunay_p1_problem(400, 2)
    A1, f1, s1 = amg.normalize(A, f)
    An = amg.to_scipy(A)
    An = -An
    A2, f2, s2 = amg.normalize(An, -f)
    assert s1 and s2
    assert np.array_equal(A1.data, A2.data) and np.array_equal(f1, f2)


# ---------------------------------------------------------------------------------------------
# Coarse solve and V-cycle
# ---------------------------------------------------------------------------------------------


def test_one_level_vcycle_is_direct_solve():
    A = amg.to_scipy(W.grid5(6))
    f = W.rhs_uniform(36, 3)
    h = amg.setup(A, max_levels=1)
    Qs = amg.smoothers(h, amg.jacobi_coeffs(), 2)
    u = amg.vcycle(h, Qs, np.zeros(36), f)
    ref = sla.solve(A.toarray(), f)
    assert np.allclose(u, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_singular_coarse_solve_zero_mean():
    A = amg.to_scipy(W.delaunay_p1(W.uniform_points(60, 1)))
    f = W.rhs_uniform(A.shape[0], 2, zero_mean=True)
    cs = amg.CoarseSolver(A, singular=True)
    e = cs.solve(f)
    assert abs(e.sum()) <= 1e-12 * np.abs(e).max()
    assert np.linalg.norm(A @ e - f) <= 1e-12 * np.linalg.norm(f)


def _hier(kind, coeffs=None, max_levels=4, max_coarse=20):
    if kind == "grid":
        A = amg.to_scipy(W.grid5(16))
        sing = False
    else:
        A = amg.to_scipy(W.delaunay_p1(W.uniform_points(300, 9)))
        sing = True
    h = amg.setup(A, max_levels=max_levels, max_coarse=max_coarse, singular=sing)
    Qs = amg.smoothers(h, amg.jacobi_coeffs() if coeffs is None else coeffs, 2)
    return A, h, Qs


@pytest.mark.parametrize("kind", ["grid", "delaunay"])
@pytest.mark.parametrize("coeffs", [None, [0.6, 0.05, -0.01, 0.2, 0.03]])
def test_vcycle_linearity(kind, coeffs):
    A, h, Qs = _hier(kind, coeffs)
    n = A.shape[0]
    rng = np.random.default_rng(5)
    u1, u2, f1, f2 = (rng.standard_normal(n) for _ in range(4))
    if h.singular:
        f1 -= f1.mean()
        f2 -= f2.mean()
    a, b = 0.7, -1.3
    lhs = amg.vcycle(h, Qs, a * u1 + b * u2, a * f1 + b * f2, 1, 1)
    rhs = a * amg.vcycle(h, Qs, u1, f1, 1, 1) + b * amg.vcycle(h, Qs, u2, f2, 1, 1)
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(rhs)


@pytest.mark.parametrize("nu", [1, 2])
@pytest.mark.parametrize("coeffs", [None, [0.6, 0.05, -0.01, 0.2, 0.03]])
def test_vcycle_operator_symmetric(nu, coeffs):
    """With nu1 = nu2 and symmetric Q^{-1}, the V-cycle preconditioner M = V(0, .) is symmetric."""
    A, h, Qs = _hier("grid", coeffs)
    n = A.shape[0]
    M = np.column_stack([amg.vcycle(h, Qs, np.zeros(n), e, nu, nu) for e in np.eye(n)])
    assert np.linalg.norm(M - M.T) <= 1e-13 * np.linalg.norm(M)


def test_vcycle_error_propagator_spectrum():
    """omega-Jacobi V(1,1): E = I - M A is A-self-adjoint and A-positive-semidefinite, eigenvalues in [0, 1)."""
    A, h, Qs = _hier("grid")
    n = A.shape[0]
    M = np.column_stack([amg.vcycle(h, Qs, np.zeros(n), e, 1, 1) for e in np.eye(n)])
    E = np.eye(n) - M @ A.toarray()
    ev = np.linalg.eigvals(E)
    assert np.abs(ev.imag).max() < 1e-10
    assert ev.real.min() > -1e-10 and ev.real.max() < 1.0


def test_two_level_without_smoothing_is_projector():
    """nu1 = nu2 = 0 two-level cycle: E = I - P (P^T A P)^{-1} P^T A is an A-orthogonal projector, E^2 = E."""
    A = amg.to_scipy(W.grid5(12))
    h = amg.setup(A, max_levels=2, max_coarse=5)
    assert h.nlevels == 2
    Qs = amg.smoothers(h, amg.jacobi_coeffs(), 2)
    n = A.shape[0]
    M = np.column_stack([amg.vcycle(h, Qs, np.zeros(n), e, 0, 0) for e in np.eye(n)])
    E = np.eye(n) - M @ A.toarray()
    assert np.abs(E @ E - E).max() < 1e-12


@pytest.mark.parametrize("case", ["grid4", "grid8", "delaunay30"])
@pytest.mark.parametrize("method", ["stationary", "fcg", "ir"])
def test_solve_matches_dense_direct(case, method):
    if case.startswith("grid"):
        N = int(case[4:])
        A = amg.to_scipy(W.grid5(N))
        f = W.rhs_uniform(N * N, 1)
        sing = False
    else:
        A = amg.to_scipy(W.delaunay_p1(W.uniform_points(30, 4)))
        f = W.rhs_uniform(A.shape[0], 5, zero_mean=True)
        sing = True
    h = amg.setup(A, max_levels=3, max_coarse=4, singular=sing)
    Qs = amg.smoothers(h, amg.jacobi_coeffs(), 2)
    solve = {"stationary": amg.solve_stationary, "fcg": amg.solve_fcg, "ir": amg.solve_ir}[method]
    res = solve(h, Qs, f, tol=1e-12, maxit=500)
    assert res.converged
    M = A.toarray()
    if sing:
        ref = np.linalg.lstsq(M, f - f.mean(), rcond=None)[0]
        x = res.x - res.x.mean()
        ref = ref - ref.mean()
    else:
        ref = sla.solve(M, f)
        x = res.x
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_grid64_stationary_converges_monotonically():
    A, f, sing = amg.normalize(*W.poisson_grid_64(0))
    h = amg.setup(A, max_levels=3)
    Qs = amg.smoothers(h, amg.jacobi_coeffs(), 2)
    res = amg.solve_stationary(h, Qs, f, tol=1e-8)
    assert res.converged
    hist = np.array(res.history)
    assert np.all(np.diff(hist) < 0)
    assert np.linalg.norm(f - A @ res.x) <= 1e-8 * np.linalg.norm(f)


def test_ir_equals_stationary_in_fp64():
    A, f, sing = amg.normalize(*W.poisson_grid_64(1))
    h = amg.setup(A, max_levels=3)
    Qs = amg.smoothers(h, amg.jacobi_coeffs(), 2)
    a = amg.solve_stationary(h, Qs, f)
    b = amg.solve_ir(h, Qs, f)
    assert a.iterations == b.iterations
    assert np.linalg.norm(a.x - b.x) <= 1e-12 * np.linalg.norm(a.x)


def test_paper_constants_fixture():
    with open(os.path.join(HERE, "golden", "paper_constants.json")) as fh:
        g = json.load(fh)
    assert g["strength_threshold_theta"]["value"] == 0.25
    assert g["jacobi_omega"]["value"] == 2 / 3
    assert np.array_equal(amg.jacobi_coeffs(g["jacobi_omega"]["value"]), [2 / 3, 0, 0, 0, 0])

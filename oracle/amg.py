"""Oracle AMG in plain FP64 NumPy/SciPy: setup, smoother, V-cycle and solves.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the product.

Sign convention. The paper's Poisson matrix is negative semi-definite with zero
row sums (Sec. 2.1, Eq. 1). Ruge-Stueben coarsening is defined for a positive
diagonal, so this oracle stores -A and -f; the solution u is unchanged.

Readings where the paper is silent (each repeated in the design notes):
  * strength of connection: classical negative-coupling form (Sec. 4 names
    classical Ruge-Stueben with theta = 0.25 and nothing more);
  * C/F split: Ruge-Stueben first pass only, ties broken by smallest index;
  * interpolation: direct interpolation, positive couplings lumped on the diagonal;
  * Galerkin product: row-by-row (Gustavson) accumulation in ascending column
    order, exact zeros dropped except on the diagonal;
  * hierarchy ends at max_levels, n <= max_coarse, or when fewer than 10%
    of points are dropped;
  * singular (all-Neumann) coarsest level: factor A_L + alpha 1 1^T with
    alpha = mean(diag A_L)/n_L;
  * smoother scale s is one number per level; polynomial coefficients in the
    monomial basis, order (d0..d_deg, o1..o_deg), evaluated by Horner.
"""
from __future__ import annotations

import heapq
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

# ----------------------------------------------------------------------------
# Input normalisation (Sec. 2.1, Eq. 1)
# ----------------------------------------------------------------------------


def to_scipy(A) -> sp.csr_matrix:
    """CSR copy with sorted column indices; accepts scipy or workloads.CSRMatrix."""
    if not sp.issparse(A):
        A = sp.csr_matrix((np.asarray(A.val, np.float64), np.asarray(A.col), np.asarray(A.rowptr)),
                          shape=(A.nrows, A.ncols))
    A = sp.csr_matrix(A, dtype=np.float64, copy=True)
    A.sort_indices()
    return A


def diagonal_strict(A: sp.csr_matrix) -> np.ndarray:
    """Stored diagonal; raises if a row has no stored diagonal entry."""
    n = A.shape[0]
    d = np.zeros(n)
    found = np.zeros(n, dtype=bool)
    for i in range(n):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        for p in range(lo, hi):
            if A.indices[p] == i:
                d[i] = A.data[p]
                found[i] = True
    if not found.all():
        raise ValueError("diagonal entry missing")
    return d


def normalize(A, f):
    """Return (A, f, singular) with a positive diagonal (Sec. 2.1, Eq. 1).

    A matrix given in the paper's negative semi-definite convention is negated
    together with f. ``singular`` is set when every row sums to zero relative
    to its diagonal (|sum_j a_ij| <= 1e-12 a_ii): the constant null space of the
    all-Neumann Poisson operator.
    """
    A = to_scipy(A)
    f = np.array(f, dtype=np.float64, copy=True)
    d = A.diagonal()
    if np.all(d < 0):
        A = -A
        f = -f
        d = -d
    if np.any(d <= 0):
        raise ValueError("diagonal must be of one strict sign")
    rowsum = np.asarray(A.sum(axis=1)).ravel()
    singular = bool(np.all(np.abs(rowsum) <= 1e-12 * d))
    return A, f, singular


# ----------------------------------------------------------------------------
# Ruge-Stueben setup (Sec. 2.2; Sec. 4: classical RS, theta = 0.25; App. B.1, Tab. 7: <= 10 levels)
# ----------------------------------------------------------------------------


def strength(A: sp.csr_matrix, theta: float) -> sp.csr_matrix:
    """Strong couplings S_i = { j != i : -a_ij >= theta * max_{k != i} (-a_ik) }.

    S_i is empty when row i has no off-diagonal entry or its largest negative
    coupling is not positive. Returned as a 0/1 pattern matrix whose row i lists
    S_i in ascending column order.
    """
    n = A.shape[0]
    rowid = np.repeat(np.arange(n), np.diff(A.indptr))
    off = A.indices != rowid
    neg = -A.data
    m = np.full(n, -np.inf)
    np.maximum.at(m, rowid[off], neg[off])
    keep = off & (m[rowid] > 0) & (neg >= theta * m[rowid])
    rows = rowid[keep]
    cols = A.indices[keep]
    S = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(n, n))
    S.sort_indices()
    return S


UNDECIDED, FPT, CPT = -1, 0, 1


def cf_split(S: sp.csr_matrix) -> np.ndarray:
    """Ruge-Stueben first-pass C/F splitting; returns 1 for C, 0 for F points.

    Points with no strong coupling in either direction are F points with no
    interpolation. The measure lambda_i counts the points that i strongly
    influences. Repeatedly the undecided point of largest lambda (smallest index
    among ties) becomes C; every undecided point it strongly influences becomes
    F; each undecided point that strongly influences such a new F point gains 1;
    each undecided point that strongly influences the new C point loses 1.
    """
    n = S.shape[0]
    ST = S.T.tocsr()
    ST.sort_indices()
    s_len = np.diff(S.indptr)
    st_len = np.diff(ST.indptr)
    state = np.full(n, UNDECIDED, dtype=np.int64)
    state[(s_len == 0) & (st_len == 0)] = FPT
    lam = st_len.astype(np.int64).copy()
    heap = [(-int(lam[i]), i) for i in range(n) if state[i] == UNDECIDED]
    heapq.heapify(heap)
    while heap:
        negl, i = heapq.heappop(heap)
        if state[i] != UNDECIDED or -negl != lam[i]:
            continue
        state[i] = CPT
        new_f = [j for j in ST.indices[ST.indptr[i]:ST.indptr[i + 1]] if state[j] == UNDECIDED]
        for j in new_f:
            state[j] = FPT
        for j in new_f:
            for k in S.indices[S.indptr[j]:S.indptr[j + 1]]:
                if state[k] == UNDECIDED:
                    lam[k] += 1
                    heapq.heappush(heap, (-int(lam[k]), int(k)))
        for k in S.indices[S.indptr[i]:S.indptr[i + 1]]:
            if state[k] == UNDECIDED:
                lam[k] -= 1
                heapq.heappush(heap, (-int(lam[k]), int(k)))
    return state


def direct_interpolation(A: sp.csr_matrix, S: sp.csr_matrix, state: np.ndarray) -> sp.csr_matrix:
    """Direct interpolation P (n x n_c), coarse ids in ascending fine order.

    C row i: P[i, c(i)] = 1. F row i with strong C neighbours C_i = S_i and C:
        at_ii = a_ii + sum_{k != i, a_ik > 0} a_ik
        alpha = (sum_{k != i, a_ik < 0} a_ik) / (sum_{k in C_i} a_ik)
        P[i, c(k)] = -(alpha * a_ik) / at_ii
    every sum taken left to right in ascending column order (at_ii starting
    from a_ii, the others from 0). F rows without strong C neighbours are empty.
    """
    n = A.shape[0]
    cid = np.full(n, -1, dtype=np.int64)
    cmask = state == CPT
    cid[cmask] = np.arange(int(cmask.sum()))
    nc = int(cmask.sum())
    rows, cols, vals = [], [], []
    for i in range(n):
        if state[i] == CPT:
            rows.append(i)
            cols.append(cid[i])
            vals.append(1.0)
            continue
        strong = S.indices[S.indptr[i]:S.indptr[i + 1]]
        ci = set(int(j) for j in strong if state[j] == CPT)
        if not ci:
            continue
        lo, hi = A.indptr[i], A.indptr[i + 1]
        acols = A.indices[lo:hi]
        avals = A.data[lo:hi]
        aii = float(avals[acols == i][0])
        atil = aii
        num = 0.0
        den = 0.0
        for k, a in zip(acols, avals):
            if k == i:
                continue
            if a > 0:
                atil = atil + a
            if a < 0:
                num = num + a
            if int(k) in ci:
                den = den + a
        alpha = num / den
        for k, a in zip(acols, avals):
            if int(k) in ci:
                rows.append(i)
                cols.append(cid[k])
                vals.append(-(alpha * a) / atil)
    P = sp.csr_matrix((np.array(vals), (np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64))),
                      shape=(n, nc))
    P.sort_indices()
    return P


def spgemm_rowwise(A: sp.csr_matrix, B: sp.csr_matrix) -> sp.csr_matrix:
    """C = A B by Gustavson's row-by-row method, written as plain loops.

    For each row i, walk A's entries (j ascending) and for each walk B's row j
    (k ascending), accumulating c_ik = (((0 + a_ij1 b_j1k) + a_ij2 b_j2k) + ...).
    Every structurally generated entry is kept (also exact zeros).
    """
    n = A.shape[0]
    indptr = [0]
    indices, data = [], []
    for i in range(n):
        acc = {}
        for p in range(A.indptr[i], A.indptr[i + 1]):
            j = A.indices[p]
            a = A.data[p]
            for q in range(B.indptr[j], B.indptr[j + 1]):
                k = int(B.indices[q])
                acc[k] = acc.get(k, 0.0) + a * B.data[q]
        for k in sorted(acc):
            indices.append(k)
            data.append(acc[k])
        indptr.append(len(indices))
    return sp.csr_matrix((np.array(data, dtype=np.float64), np.array(indices, dtype=np.int64),
                          np.array(indptr, dtype=np.int64)), shape=(n, B.shape[1]))


def spgemm_rowwise_vec(A: sp.csr_matrix, B: sp.csr_matrix) -> sp.csr_matrix:
    """Same products and the same per-entry summation order as ``spgemm_rowwise``, vectorised.

    All products a_ij * b_jk are listed in the loop order (i, j, k), stably
    grouped by (i, k), and each group summed left to right starting from 0.
    Tests check that the result is bitwise equal to the loop version.
    """
    n, m = A.shape[0], B.shape[1]
    arow = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.indptr))
    acol = A.indices.astype(np.int64)
    blen = np.diff(B.indptr)[acol].astype(np.int64)
    total = int(blen.sum())
    if total == 0:
        return sp.csr_matrix((n, m))
    first = np.cumsum(blen) - blen
    bpos = np.repeat(B.indptr[acol].astype(np.int64), blen) + (np.arange(total) - np.repeat(first, blen))
    prow = np.repeat(arow, blen)
    pcol = B.indices[bpos].astype(np.int64)
    prod = np.repeat(A.data, blen) * B.data[bpos]
    key = prow * m + pcol
    order = np.argsort(key, kind="stable")
    key = key[order]
    prod = prod[order]
    ukey, start, count = np.unique(key, return_index=True, return_counts=True)
    acc = np.zeros(ukey.size)
    for t in range(int(count.max())):
        sel = count > t
        acc[sel] = acc[sel] + prod[start[sel] + t]
    rows = ukey // m
    cols = ukey % m
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=indptr[1:])
    return sp.csr_matrix((acc, cols, indptr), shape=(n, m))


def transpose_exact(P: sp.csr_matrix) -> sp.csr_matrix:
    """R = P^T as CSR with sorted columns (values moved, not recomputed)."""
    R = P.T.tocsr()
    R.sort_indices()
    return R


def galerkin(A: sp.csr_matrix, P: sp.csr_matrix, vectorised: bool | None = None) -> sp.csr_matrix:
    """Coarse operator A_c = P^T (A P) (Sec. 2.2, Galerkin triple product), exact zeros dropped off the diagonal."""
    if vectorised is None:
        vectorised = A.nnz > 20000
    mult = spgemm_rowwise_vec if vectorised else spgemm_rowwise
    AP = mult(A, P)
    Ac = mult(transpose_exact(P), AP)
    rowid = np.repeat(np.arange(Ac.shape[0]), np.diff(Ac.indptr))
    keep = (Ac.data != 0.0) | (Ac.indices == rowid)
    Ac = sp.csr_matrix((Ac.data[keep], (rowid[keep], Ac.indices[keep])), shape=Ac.shape)
    Ac.sort_indices()
    return Ac


@dataclass
class Level:
    A: sp.csr_matrix
    P: sp.csr_matrix | None = None
    R: sp.csr_matrix | None = None
    state: np.ndarray | None = None


@dataclass
class Hierarchy:
    levels: list
    singular: bool
    coarse: "CoarseSolver" = field(default=None)

    @property
    def nlevels(self) -> int:
        return len(self.levels)


def setup(A, theta: float = 0.25, max_levels: int = 10, max_coarse: int = 500,
          singular: bool = False) -> Hierarchy:
    """Ruge-Stueben hierarchy {A_l, P_l, R_l = P_l^T} (Sec. 2.2; Alg. 1, step 2).

    Coarsening stops at ``max_levels`` levels, when a level has at most
    ``max_coarse`` rows, when no C point is found, or when more than 90% of the
    points are C points (10 n_c > 9 n).
    """
    A = to_scipy(A)
    levels = [Level(A)]
    while True:
        A = levels[-1].A
        n = A.shape[0]
        if len(levels) >= max_levels or n <= max_coarse:
            break
        S = strength(A, theta)
        state = cf_split(S)
        nc = int((state == CPT).sum())
        if nc == 0 or 10 * nc > 9 * n:
            break
        P = direct_interpolation(A, S, state)
        levels[-1].P = P
        levels[-1].R = transpose_exact(P)
        levels[-1].state = state
        levels.append(Level(galerkin(A, P)))
    h = Hierarchy(levels, singular)
    h.coarse = CoarseSolver(levels[-1].A, singular)
    return h


# ----------------------------------------------------------------------------
# Coarsest-level direct solve (Sec. 2.2: the coarsest level is solved directly)
# ----------------------------------------------------------------------------


class CoarseSolver:
    """Dense LU with partial pivoting of A_L (LAPACK getrf through SciPy).

    Singular problems factor A_L + alpha 1 1^T, alpha = mean(diag A_L)/n_L, whose
    solution for a consistent right-hand side solves A_L e = f with 1^T e = 0.
    """

    def __init__(self, AL: sp.csr_matrix, singular: bool):
        M = AL.toarray()
        if singular:
            nL = M.shape[0]
            alpha = np.mean(np.diag(M)) / nL
            M = M + alpha * np.ones_like(M)
        self.M = M
        self.lu = sla.lu_factor(M)

    def solve(self, b: np.ndarray) -> np.ndarray:
        if np.iscomplexobj(b):
            return sla.lu_solve(self.lu, b.real) + 1j * sla.lu_solve(self.lu, b.imag)
        return sla.lu_solve(self.lu, b)


# ----------------------------------------------------------------------------
# Sparse pseudo-inverse smoother (Sec. 3.1, Eq. 5)
# ----------------------------------------------------------------------------


def jacobi_coeffs(omega: float = 2.0 / 3.0, degree: int = 2) -> np.ndarray:
    """Coefficients giving f_d = omega, f_o = 0: exactly omega-Jacobi (Sec. 2.3, Eq. 4; Sec. 4, omega = 2/3)."""
    c = np.zeros(2 * degree + 1)
    c[0] = omega
    return c


def offdiag_scale(A: sp.csr_matrix) -> float:
    """s = max |a_ij| over stored off-diagonal entries, one number per level (Sec. 3.1, Eq. 5).

    Reading: Eq. 5 divides by s, which is undefined for a level without a nonzero
    off-diagonal (no stored off-diagonal, or only stored zeros); s = 1 is taken then.
    The off-diagonal part of Q is zero either way, since f_o(0) = 0.
    """
    rowid = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    off = A.indices != rowid
    if not off.any():
        return 1.0
    s = float(np.max(np.abs(A.data[off])))
    return s if s > 0.0 else 1.0


def poly_diag(x, d):
    """f_d(x) = d0 + x (d1 + x (d2 + ...)), Horner, one rounding per operation."""
    t = np.full(np.shape(x), d[-1], dtype=np.result_type(np.asarray(d).dtype, np.asarray(x).dtype))
    for c in d[-2::-1]:
        t = c + x * t
    return t


def poly_off(x, o):
    """f_o(x) = x (o1 + x (o2 + ...)), so that f_o(0) = 0 keeps A's sparsity (Sec. 3.1)."""
    t = np.full(np.shape(x), o[-1], dtype=np.result_type(np.asarray(o).dtype, np.asarray(x).dtype))
    for c in o[-2::-1]:
        t = c + x * t
    return x * t


def assemble_smoother(A: sp.csr_matrix, coeffs, degree: int) -> sp.csr_matrix:
    """Q^{-1} on A's pattern (Sec. 3.1, Eq. 5; Alg. 1, step 8).

    q_ii = f_d(a_ii/s)/a_ii and q_ij = f_o(a_ij/s)/(a_ii + a_jj) with
    coefficients (d0..d_deg, o1..o_deg). Complex coefficients (complex step)
    give a complex Q.
    """
    coeffs = np.asarray(coeffs)
    if coeffs.size != 2 * degree + 1:
        raise ValueError("need 2*degree+1 coefficients")
    d = coeffs[:degree + 1]
    o = coeffs[degree + 1:]
    s = offdiag_scale(A)
    n = A.shape[0]
    rowid = np.repeat(np.arange(n), np.diff(A.indptr))
    diag = A.diagonal()
    x = A.data / s
    isd = A.indices == rowid
    q = np.empty(A.nnz, dtype=np.result_type(coeffs.dtype, np.float64))
    q[isd] = poly_diag(x[isd], d) / A.data[isd]
    q[~isd] = poly_off(x[~isd], o) / (diag[rowid[~isd]] + diag[A.indices[~isd]])
    return sp.csr_matrix((q, A.indices.copy(), A.indptr.copy()), shape=A.shape)


# ----------------------------------------------------------------------------
# Solve phase (Sec. 2.1, Eqs. 2-3; Sec. 2.2; Alg. 1, steps 9-10)
# ----------------------------------------------------------------------------


def smooth(A, Q, u, f, steps: int):
    """``steps`` stationary steps u <- u + Q^{-1} (f - A u) (Sec. 2.1, Eqs. 2-3)."""
    for _ in range(steps):
        r = f - A @ u
        u = u + Q @ r
    return u


def vcycle(h: Hierarchy, Qs, u, f, nu1: int = 1, nu2: int = 1, lvl: int = 0):
    """One V(nu1, nu2) cycle on level ``lvl`` (Sec. 2.2).

    Pre-smooth, restrict the residual with R = P^T, solve the coarse residual
    equation recursively from a zero guess, prolongate and correct, post-smooth.
    The coarsest level is solved directly and ignores u.
    """
    if lvl == h.nlevels - 1:
        return h.coarse.solve(f)
    L = h.levels[lvl]
    u = smooth(L.A, Qs[lvl], u, f, nu1)
    r = f - L.A @ u
    fc = L.R @ r
    ec = vcycle(h, Qs, np.zeros_like(fc), fc, nu1, nu2, lvl + 1)
    u = u + L.P @ ec
    return smooth(L.A, Qs[lvl], u, f, nu2)


def smoothers(h: Hierarchy, coeffs, degree: int):
    """Q^{-1} for every level but the coarsest; ``coeffs`` is one vector or one per level."""
    coeffs = np.asarray(coeffs)
    if coeffs.ndim == 1:
        coeffs = np.tile(coeffs, (h.nlevels, 1))
    return [assemble_smoother(h.levels[l].A, coeffs[l], degree) for l in range(h.nlevels - 1)] + [None]


@dataclass
class SolveResult:
    x: np.ndarray
    iterations: int
    vcycles: int
    converged: bool
    history: list


def solve_stationary(h: Hierarchy, Qs, f, tol=1e-8, maxit=500, nu1=1, nu2=1) -> SolveResult:
    """Repeated V-cycles from u = 0 until ||f - A u|| <= tol ||f|| (Sec. 4: at most 500 iterations)."""
    A = h.levels[0].A
    f = np.asarray(f, dtype=np.float64)
    if h.singular:
        f = f - f.mean()
    nf = np.linalg.norm(f)
    u = np.zeros_like(f)
    hist = [1.0]
    if nf == 0.0:
        return SolveResult(u, 0, 0, True, hist)
    for k in range(1, maxit + 1):
        u = vcycle(h, Qs, u, f, nu1, nu2)
        rel = np.linalg.norm(f - A @ u) / nf
        hist.append(rel)
        if rel <= tol:
            return SolveResult(u, k, k, True, hist)
    return SolveResult(u, maxit, maxit, False, hist)


def solve_fcg(h: Hierarchy, Qs, f, tol=1e-8, maxit=500, nu1=1, nu2=1) -> SolveResult:
    """Flexible preconditioned CG with z = V(0, r) as preconditioner.

    beta_k = z_{k+1}^T (r_{k+1} - r_k) / (z_k^T r_k) (flexible, Polak-Ribiere form);
    stops when the recursively updated residual satisfies ||r|| <= tol ||f||.
    """
    A = h.levels[0].A
    f = np.asarray(f, dtype=np.float64)
    if h.singular:
        f = f - f.mean()
    nf = np.linalg.norm(f)
    x = np.zeros_like(f)
    hist = [1.0]
    if nf == 0.0:
        return SolveResult(x, 0, 0, True, hist)
    r = f.copy()
    z = vcycle(h, Qs, np.zeros_like(r), r, nu1, nu2)
    nv = 1
    p = z.copy()
    gamma = z @ r
    for k in range(1, maxit + 1):
        q = A @ p
        alpha = gamma / (p @ q)
        x = x + alpha * p
        rn = r - alpha * q
        rel = np.linalg.norm(rn) / nf
        hist.append(rel)
        if rel <= tol:
            return SolveResult(x, k, nv, True, hist)
        z = vcycle(h, Qs, np.zeros_like(rn), rn, nu1, nu2)
        nv += 1
        beta = (z @ (rn - r)) / gamma
        gamma = z @ rn
        p = z + beta * p
        r = rn
    return SolveResult(x, maxit, nv, False, hist)


def solve_ir(h: Hierarchy, Qs, f, tol=1e-8, maxit=500, nu1=1, nu2=1) -> SolveResult:
    """Iterative refinement x <- x + V(0, f - A x); with an FP64 cycle this equals ``solve_stationary``."""
    A = h.levels[0].A
    f = np.asarray(f, dtype=np.float64)
    if h.singular:
        f = f - f.mean()
    nf = np.linalg.norm(f)
    x = np.zeros_like(f)
    r = f.copy()
    hist = [1.0]
    if nf == 0.0:
        return SolveResult(x, 0, 0, True, hist)
    for k in range(1, maxit + 1):
        x = x + vcycle(h, Qs, np.zeros_like(r), r, nu1, nu2)
        r = f - A @ x
        rel = np.linalg.norm(r) / nf
        hist.append(rel)
        if rel <= tol:
            return SolveResult(x, k, k, True, hist)
    return SolveResult(x, maxit, maxit, False, hist)

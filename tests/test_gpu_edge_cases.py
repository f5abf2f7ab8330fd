"""Degenerate and boundary inputs of the solve path, GPU against the oracle.

- a hub row with 4,500 entries (longer than a CSR-stream block's LDS buffer: the block falls back
  to per-row loops, and the level's halo is too large for the fused kernels);
- a dense 128-node cluster inside one row block of 256 rows and coupled only within itself
  (16,384 entries in that block: the fused smoothing kernel's own-row products exceed its LDS
  buffer and take its loop path);
- isolated unknowns (rows holding only their diagonal: no strong coupling, F points with an
  empty interpolation row).
Each case: FP64 level operators bitwise equal to the oracle's sparse products on every level the
CSR-stream kernels serve (rows summed in stored order); levels whose mean row length exceeds
about 100 entries (the hub makes its Galerkin products dense) use the lane kernel, whose row
sums combine lane partials in a shuffle tree: there 1e-14 relative. Fused kernels bitwise equal
to separate passes, one FP64 V-cycle within 1e-12, an FP32-cycle / FP64 CG solve to 1e-8 with
the residual recomputed by the oracle.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import amg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()


def _csr(S):
    S = sp.csr_matrix(S)
    S.sort_indices()
    return W.CSRMatrix(S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64),
                       S.shape[0], S.shape[1])


def _laplacian(n, i, j, w, shift):
    """Weighted graph Laplacian (i < j edges, weights w > 0) plus shift * I."""
    L = sp.coo_matrix((np.concatenate([-w, -w]), (np.concatenate([i, j]), np.concatenate([j, i]))), shape=(n, n))
    L = sp.csr_matrix(L)
    L.sum_duplicates()
    d = -np.asarray(L.sum(axis=1)).ravel() + shift
    return _csr(L + sp.diags(d))


def _grid_edges(N):
    idx = np.arange(N * N).reshape(N, N)
    i = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    j = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return i, j


def make(kind):
    rng = np.random.default_rng(7)
    if kind == "hub":
        N = 80
        n = N * N + 1
        i, j = _grid_edges(N)
        hub = n - 1
        nb = np.sort(rng.choice(N * N, 4500, replace=False))
        i = np.concatenate([i, nb])
        j = np.concatenate([j, np.full(nb.size, hub)])
        w = np.concatenate([np.ones(i.size - nb.size), rng.uniform(0.01, 0.05, nb.size)])
        return _laplacian(n, i, j, w, 1e-3)
    if kind == "cluster":
        N = 140
        i, j = _grid_edges(N)
        # a 128-node clique coupled only within itself, inside one row block of the 256-row kernels
        # (its 16k entries exceed the block's product buffer: the fused kernel's loop path)
        c0 = 10 * 256
        out = (i >= c0) & (i < c0 + 128) | (j >= c0) & (j < c0 + 128)
        i, j = i[~out], j[~out]
        a, b = np.triu_indices(128, 1)
        i = np.concatenate([i, c0 + a])
        j = np.concatenate([j, c0 + b])
        w = np.concatenate([np.ones(i.size - a.size), rng.uniform(0.5, 1.5, a.size)])
        return _laplacian(N * N, i, j, w, 0.01)
    if kind == "isolated":
        N = 60
        i, j = _grid_edges(N)
        iso = np.arange(5, N * N, 97)
        keep = ~(np.isin(i, iso) | np.isin(j, iso))
        L = _laplacian(N * N, i[keep], j[keep], np.ones(int(keep.sum())), 0.01).to_scipy()
        return _csr(L + sp.diags(np.where(np.isin(np.arange(N * N), iso), 2.49, 0.0)))
    raise KeyError(kind)


_cache = {}


def _setup(kind):
    if kind not in _cache:
        from paper_2606_19251_amd.solver import DeviceSolver, HostHierarchy

        A = make(kind)
        f = W.rhs_uniform(A.nrows, 11)
        An, fn, sing = amg.normalize(A, f)
        ho = amg.setup(An, singular=sing, max_levels=10, max_coarse=100)
        hp = HostHierarchy.build(A.rowptr, A.col, A.val, max_levels=10, max_coarse=100)
        print(f"[gpu] edge case {kind}: n={A.nrows} nnz={A.nnz} max row {np.diff(A.rowptr).max()} "
              f"levels {[L.n for L in hp.levels]} singular={sing}", flush=True)
        _cache[kind] = (A, fn, ho, hp, DeviceSolver(hp, 0))
    return _cache[kind]


KINDS = ["hub", "cluster", "isolated"]
POLY2 = np.array([0.6, 0.01, -0.001, 0.12, 0.01])


@pytest.mark.parametrize("kind", KINDS)
def test_hierarchy_and_level_operators_bitexact(kind):
    from paper_2606_19251_amd import capi

    A, f, ho, hp, ds = _setup(kind)
    assert hp.nlevels == ho.nlevels
    for l in range(ho.nlevels):
        assert np.array_equal(ho.levels[l].A.indices, hp.levels[l].col)
        assert np.array_equal(_bits(ho.levels[l].A.data), _bits(hp.levels[l].val))
    ds.set_coeffs(POLY2, 2)
    Qs = amg.smoothers(ho, POLY2, 2)
    rng = np.random.default_rng(3)
    for l in range(ho.nlevels - 1):
        L = ho.levels[l]
        n, nc = L.A.shape[0], L.P.shape[1]
        x, fl, y0, xc = rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(nc)
        cases = [(capi.AMGG_OP_RESIDUAL, x, fl, None, fl - L.A @ x, n),
                 (capi.AMGG_OP_SMOOTH, x, None, y0, y0 + Qs[l] @ x, n),
                 (capi.AMGG_OP_RESTRICT, x, None, None, L.R @ x, nc),
                 (capi.AMGG_OP_PROLONG, xc, None, y0, y0 + L.P @ xc, n)]
        for op, xin, fin, yin, ref, m in cases:
            xd = _dev(xin)
            fd = _dev(fin) if fin is not None else xd
            yd = _dev(yin) if yin is not None else torch.zeros(m, dtype=torch.float64, device="cuda")
            capi.amgg_level_apply(ds.ctx, l, op, 64, xd.data_ptr(), yd.data_ptr(), fd.data_ptr(), ds.stream)
            torch.cuda.synchronize()
            got = yd.cpu().numpy()
            rows = {capi.AMGG_OP_RESTRICT: L.R, capi.AMGG_OP_PROLONG: L.P}.get(op, L.A)
            if rows.nnz / rows.shape[0] <= 100:  # CSR-stream kernels: in-order row sums
                assert np.array_equal(_bits(got), _bits(ref)), (kind, l, op)
            else:
                assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref), (kind, l, op)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("cname", ["jacobi", "poly2"])
def test_vcycle_fp64_and_fused_paths(kind, cname):
    A, f, ho, hp, ds = _setup(kind)
    c = amg.jacobi_coeffs() if cname == "jacobi" else POLY2
    ds.set_coeffs(c, 2)
    if kind == "cluster":  # the level with the dense block is fused, its block takes the loop path
        assert ds.level_view(0)["fused_rows"] == 256
    if kind == "hub":  # too large a halo: separate passes
        assert ds.level_view(0)["fused_rows"] == 0
    u0 = np.random.default_rng(5).standard_normal(A.nrows)
    Qs = amg.smoothers(ho, c, 2)
    for nu in [(1, 1), (2, 2)]:
        ref = amg.vcycle(ho, Qs, u0, f, *nu)
        outs = []
        for fuse in (True, False):
            ds.set_fusion(fuse)
            u = _dev(u0)
            ds.vcycle(_dev(f), u, nu[0], nu[1], 64)
            outs.append(u.cpu().numpy())
        ds.set_fusion(True)
        assert np.array_equal(_bits(outs[0]), _bits(outs[1])), (kind, cname, nu)
        err = np.linalg.norm(outs[0] - ref) / np.linalg.norm(ref)
        assert err <= 1e-12, (kind, cname, nu, err)


@pytest.mark.parametrize("kind", KINDS)
def test_fp32_cycle_fcg_reaches_tolerance(kind):
    from paper_2606_19251_amd import capi

    A, f, ho, hp, ds = _setup(kind)
    ds.set_jacobi(2 / 3)
    x, rc, info, _ = ds.solve(_dev(f), outer=capi.AMGG_OUTER_FCG, precision=32, tol=1e-8, fallback=False)
    assert rc == 0, (kind, rc, info.relres)
    fb = f - f.mean() if ho.singular else f
    rel = np.linalg.norm(fb - ho.levels[0].A @ x.cpu().numpy()) / np.linalg.norm(fb)
    assert rel <= 1.01e-8, (kind, rel)


def test_level_with_stored_zero_offdiagonals_gets_unit_scale():
    """A level whose stored off-diagonal entries are all exact zeros has no nonzero off-diagonal,
    so the s of Eq. 5 is taken as 1 (the oracle's reading): the smoother values are finite and
    bitwise the oracle's, on the unbatched level and on the same level inside a batch."""
    from paper_2606_19251_amd.solver import BatchSolver, DeviceSolver, HostHierarchy, HostLevel

    n = 8
    diag = np.arange(2.0, 2.0 + n)
    A0 = sp.csr_matrix(np.diag(diag))
    for i in range(0, n, 2):  # stored zeros on a 2 x 2 block pattern
        A0[i, i + 1] = 0.0
        A0[i + 1, i] = 0.0
    A0 = sp.csr_matrix(A0)
    A0.sort_indices()
    A0.data[A0.indices != np.repeat(np.arange(n), np.diff(A0.indptr))] = 0.0
    assert A0.nnz == 2 * n  # the zeros stay stored
    P0 = sp.csr_matrix(np.kron(np.eye(n // 2), np.ones((2, 1))))
    A1 = sp.csr_matrix(P0.T @ A0 @ P0)
    A1.sort_indices()
    L0 = HostLevel(n, A0.indptr.astype(np.int32), A0.indices.astype(np.int32), A0.data.copy(), n // 2,
                   P0.indptr.astype(np.int32), P0.indices.astype(np.int32), P0.data.copy())
    L1 = HostLevel(n // 2, A1.indptr.astype(np.int32), A1.indices.astype(np.int32), A1.data.copy())
    h = HostHierarchy([L0, L1], False)
    c = np.array([0.5, 0.25, -0.01, 0.3, 0.1])
    ref = amg.assemble_smoother(A0, c, 2)
    assert amg.offdiag_scale(A0) == 1.0 and np.all(np.isfinite(ref.data))
    ds = DeviceSolver(h, 0)
    ds.set_coeffs(c, 2)
    v = ds.level_view(0)
    torch.cuda.synchronize()
    assert float(v["scale"].cpu().numpy()[0]) == 1.0
    assert np.array_equal(_bits(v["q_val"].cpu().numpy()), _bits(ref.data))
    bs = BatchSolver([h, h], 0)
    bs.set_coeffs_device(torch.from_numpy(np.tile(c.astype(np.float32), (4, 1))).cuda(), 2)
    q = bs.ds.level_view(0)["q_val"].cpu().numpy()
    ref32 = amg.assemble_smoother(A0, c.astype(np.float32).astype(np.float64), 2).data
    assert np.array_equal(_bits(q), _bits(np.concatenate([ref32, ref32])))

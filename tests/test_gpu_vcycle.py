"""GPU parity of the solve phase against the CPU oracle, through the C ABI.

Bit-exact: derived hierarchy data (R = P^T, FP32 casts, diagonal, scale) and smoother
values. FP64 V-cycle: one cycle from identical (u, f) within 1e-12 relative. Solves:
cycle counts equal to the oracle's in FP64; the FP32-cycle / FP64-outer solves reach
1e-8 with the residual recomputed by the oracle in FP64.
"""
import numpy as np
import pytest

import workloads as W
from oracle import amg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint64 if a.dtype == np.float64 else np.uint32)


def _make(kind, seed=0):
    if kind == "grid64":
        A, f = W.poisson_grid_64(seed)
        return A, f, dict(max_levels=3, max_coarse=500)
    if kind == "grid64_deep":
        A, f = W.poisson_grid_64(seed)
        return A, f, dict(max_levels=10, max_coarse=30)
    if kind == "delaunay20k":
        A, f = W.delaunay_p1_problem(20000, seed)
        return A, f, dict(max_levels=10, max_coarse=100)
    if kind == "gmm5k":
        A = W.delaunay_p1(W.gmm_points(5003, seed))
        return A, W.rhs_uniform(A.nrows, seed + 7, zero_mean=True), dict(max_levels=10, max_coarse=40)
    if kind == "cmesh32k":
        A, f = W.airfoil_cmesh_problem(256, 128, seed)
        return A, f, dict(max_levels=10, max_coarse=200)
    if kind == "tet30k":
        A, f = W.tet_fv_problem(17, seed)
        return A, f, dict(max_levels=10, max_coarse=100)
    if kind == "tiny":
        A = W.grid5(7)
        return A, W.rhs_uniform(49, seed), dict(max_levels=10, max_coarse=10)
    raise KeyError(kind)


_cache = {}


def _setup(kind, seed=0):
    key = (kind, seed)
    if key not in _cache:
        from paper_2606_19251_amd.solver import DeviceSolver, HostHierarchy

        A, f, kw = _make(kind, seed)
        An, fn, sing = amg.normalize(A, f)
        ho = amg.setup(An, singular=sing, **kw)
        hp = HostHierarchy.build(A.rowptr, A.col, A.val, theta=0.25, **kw)
        print(f"[gpu] setup {kind} seed={seed} n={A.nrows} levels={hp.nlevels}", flush=True)
        ds = DeviceSolver(hp, 0)
        _cache[key] = (A, fn, ho, hp, ds)
    return _cache[key]


def _same_count(got, ref, tol=1e-8):
    """Equal iteration counts, or off by one when the oracle's last ratio is within 1% of tol."""
    if got == ref.iterations:
        return
    near = abs(ref.history[-1] - tol) <= 0.01 * tol or abs(ref.history[-2] - tol) <= 0.01 * tol
    assert abs(got - ref.iterations) == 1 and near, (got, ref.iterations, ref.history[-2:])


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()


@pytest.mark.parametrize("kind", ["grid64", "delaunay20k", "tiny", "cmesh32k", "tet30k"])
def test_derived_hierarchy_bitexact(kind):
    A, f, ho, hp, ds = _setup(kind)
    torch.cuda.synchronize()
    for l in range(ho.nlevels):
        v = ds.level_view(l)
        Ao = ho.levels[l].A
        assert np.array_equal(_bits(v["a_val32"].cpu().numpy()), _bits(Ao.data.astype(np.float32)))
        assert np.array_equal(_bits(v["diag"].cpu().numpy()), _bits(Ao.diagonal()))
        assert np.array_equal(_bits(v["scale"].cpu().numpy()), _bits(np.array([amg.offdiag_scale(Ao)])))
        if l + 1 < ho.nlevels:
            R = ho.levels[l].R
            assert np.array_equal(v["r_rowptr"].cpu().numpy(), R.indptr)
            assert np.array_equal(v["r_col"].cpu().numpy(), R.indices)
            assert np.array_equal(_bits(v["r_val"].cpu().numpy()), _bits(R.data))
            assert np.array_equal(_bits(v["r_val32"].cpu().numpy()), _bits(R.data.astype(np.float32)))
            assert np.array_equal(_bits(v["p_val32"].cpu().numpy()), _bits(ho.levels[l].P.data.astype(np.float32)))
        else:
            assert v["coarse_inv"] is not None


COEFFS = {
    "jacobi": (amg.jacobi_coeffs(), 2),
    # convergent smoothers on the 5-point grid: Q^{-1} eigenvalues alpha + beta kappa stay in
    # (0, 2/(4 - kappa)) (alpha = f_d(4)/4, beta = f_o(-1)/8)
    "poly2": (np.array([0.6, 0.01, -0.001, 0.12, 0.01]), 2),
    "poly3": (np.array([0.6, 0.01, -0.001, 0.0001, 0.12, 0.01, -0.001]), 3),
}


@pytest.mark.parametrize("kind", ["grid64", "delaunay20k"])
@pytest.mark.parametrize("cname", list(COEFFS))
def test_smoother_values_bitexact(kind, cname):
    A, f, ho, hp, ds = _setup(kind)
    c, deg = COEFFS[cname]
    ds.set_coeffs(c, deg)
    torch.cuda.synchronize()
    from paper_2606_19251_amd import capi

    for l in range(ho.nlevels - 1):
        q = amg.assemble_smoother(ho.levels[l].A, c, deg).data
        v = ds.level_view(l)
        assert np.array_equal(_bits(v["q_val"].cpu().numpy()), _bits(q)), f"level {l}"
        assert np.array_equal(_bits(v["q_val32"].cpu().numpy()), _bits(q.astype(np.float32)))
        out = torch.empty(q.size, dtype=torch.float64, device="cuda")
        capi.amgg_get_smoother_values(ds.ctx, l, out.data_ptr(), ds.stream)  # the copy into a caller buffer
        torch.cuda.synchronize()
        assert np.array_equal(_bits(out.cpu().numpy()), _bits(q)), f"level {l}"


@pytest.mark.parametrize("kind", ["grid64", "grid64_deep", "delaunay20k", "gmm5k", "tiny", "cmesh32k", "tet30k"])
@pytest.mark.parametrize("cname", ["jacobi", "poly2", "poly3"])
@pytest.mark.parametrize("nu", [(1, 1), (2, 2), (0, 1), (1, 0)])
def test_vcycle_fp64_matches_oracle(kind, cname, nu):
    A, f, ho, hp, ds = _setup(kind)
    c, deg = COEFFS[cname]
    ds.set_coeffs(c, deg)
    rng = np.random.default_rng(11)
    u0 = rng.standard_normal(A.nrows)
    Qs = amg.smoothers(ho, c, deg)
    ref = amg.vcycle(ho, Qs, u0, f, *nu)
    u = _dev(u0)
    ds.vcycle(_dev(f), u, nu[0], nu[1], 64)
    got = u.cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= 1e-12, err
    # a cycle from zero (the preconditioner form) as well
    ref0 = amg.vcycle(ho, Qs, np.zeros(A.nrows), f, *nu)
    u = _dev(np.zeros(A.nrows))
    ds.vcycle(_dev(f), u, nu[0], nu[1], 64)
    err0 = np.linalg.norm(u.cpu().numpy() - ref0) / np.linalg.norm(ref0)
    assert err0 <= 1e-12, err0


@pytest.mark.parametrize("kind", ["grid64", "delaunay20k"])
def test_vcycle_fp32_close_to_oracle(kind):
    A, f, ho, hp, ds = _setup(kind)
    ds.set_coeffs(*COEFFS["poly2"])
    Qs = amg.smoothers(ho, *COEFFS["poly2"])
    ref = amg.vcycle(ho, Qs, np.zeros(A.nrows), f)
    u = _dev(np.zeros(A.nrows))
    ds.vcycle(_dev(f), u, 1, 1, 32)
    err = np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= 1e-5, err


@pytest.mark.parametrize("seed", [0, 3])
def test_stationary_fp64_same_cycle_count(seed):
    A, f, ho, hp, ds = _setup("grid64", seed)
    ds.set_jacobi(2 / 3)
    res = amg.solve_stationary(ho, amg.smoothers(ho, amg.jacobi_coeffs(), 2), f, tol=1e-8)
    from paper_2606_19251_amd import capi

    x, rc, info, hist = ds.solve(_dev(f), outer=capi.AMGG_OUTER_STATIONARY, precision=64, history_cap=600)
    assert rc == 0 and info.status == 0
    _same_count(info.iterations, res)
    m = min(len(hist), len(res.history))
    assert np.allclose(hist[:m], res.history[:m], rtol=1e-3, atol=1e-10)
    xe = x.cpu().numpy()
    assert np.linalg.norm(xe - res.x) <= 1e-10 * np.linalg.norm(res.x)


@pytest.mark.parametrize("kind", ["grid64", "delaunay20k", "gmm5k", "cmesh32k", "tet30k"])
@pytest.mark.parametrize("outer", ["fcg", "ir"])
@pytest.mark.parametrize("cname", ["jacobi", "poly2"])
def test_fp32_cycle_fp64_outer_reaches_tolerance(kind, outer, cname):
    from paper_2606_19251_amd import capi

    A, f, ho, hp, ds = _setup(kind)
    c, deg = COEFFS[cname]
    ds.set_coeffs(c, deg)
    om = capi.AMGG_OUTER_FCG if outer == "fcg" else capi.AMGG_OUTER_IR
    x, rc, info, hist = ds.solve(_dev(f), outer=om, precision=32, tol=1e-8, history_cap=600, fallback=False)
    assert rc == 0, (rc, info.status, info.relres)
    assert info.fell_back == 0
    xe = x.cpu().numpy()
    An = ho.levels[0].A
    fb = f - f.mean() if ho.singular else f
    rel = np.linalg.norm(fb - An @ xe) / np.linalg.norm(fb)
    assert rel <= 1e-8 * 1.01, rel
    solve = amg.solve_fcg if outer == "fcg" else amg.solve_ir
    ref = solve(ho, amg.smoothers(ho, c, deg), f, tol=1e-8)
    assert abs(info.vcycles - ref.vcycles) <= 2, (info.vcycles, ref.vcycles)
    xr = ref.x - ref.x.mean() if ho.singular else ref.x
    xg = xe - xe.mean() if ho.singular else xe
    assert np.linalg.norm(xg - xr) <= 1e-6 * np.linalg.norm(xr)


def test_fcg_fp64_matches_oracle_iterations():
    from paper_2606_19251_amd import capi

    A, f, ho, hp, ds = _setup("delaunay20k")
    ds.set_coeffs(*COEFFS["poly2"])
    ref = amg.solve_fcg(ho, amg.smoothers(ho, *COEFFS["poly2"]), f, tol=1e-8)
    x, rc, info, hist = ds.solve(_dev(f), outer=capi.AMGG_OUTER_FCG, precision=64, tol=1e-8, history_cap=600)
    assert rc == 0
    _same_count(info.iterations, ref)
    m = min(len(hist), len(ref.history))
    assert np.allclose(hist[:m], ref.history[:m], rtol=1e-3, atol=1e-10)


def test_jacobi_fallback_rescues_divergent_coefficients():
    from paper_2606_19251_amd import capi

    A, f, ho, hp, ds = _setup("grid64")
    ds.set_coeffs([3.0, 0, 0, 0, 0], 2)  # omega = 3 diverges
    x, rc, info, hist = ds.solve(_dev(f), outer=capi.AMGG_OUTER_IR, precision=32, tol=1e-8, fallback=True,
                                 history_cap=600)
    assert rc == 0 and info.fell_back == 1
    ds.set_coeffs([3.0, 0, 0, 0, 0], 2)
    x, rc, info, _ = ds.solve(_dev(f), outer=capi.AMGG_OUTER_IR, precision=32, tol=1e-8, fallback=False)
    assert rc == capi.AMGG_DIVERGED and info.fell_back == 0


def test_maxit_and_errors():
    from paper_2606_19251_amd import capi

    A, f, ho, hp, ds = _setup("grid64")
    ds.set_jacobi()
    x, rc, info, _ = ds.solve(_dev(f), outer=capi.AMGG_OUTER_FCG, precision=32, tol=1e-30, maxit=5)
    assert rc == capi.AMGG_MAXIT and info.iterations == 5
    with pytest.raises(capi.AmggError):
        ds.solve(_dev(f), outer=capi.AMGG_OUTER_STATIONARY, precision=32)
    with pytest.raises(capi.AmggError):
        ds.vcycle(_dev(f), _dev(f), 9, 1, 64)


@pytest.mark.parametrize("outer", ["ir", "fcg"])
def test_truncated_solves_are_prefixes_of_the_full_run(outer):
    """The outer loop enqueues iterations ahead of the one it inspects; none of them may touch the
    result once the iteration limit is reached. A solve stopped after k iterations reports the first
    k + 1 entries of the longer solve's residual history bitwise, returns the same x on a repeat,
    and (iterative refinement, whose history is the true residual) an x whose FP64 residual,
    recomputed on the host, is that history's last entry."""
    from paper_2606_19251_amd import capi

    A, f, ho, hp, ds = _setup("delaunay20k")
    ds.set_jacobi()
    code = capi.AMGG_OUTER_IR if outer == "ir" else capi.AMGG_OUTER_FCG
    kw = dict(outer=code, precision=32, tol=1e-30, fallback=False, history_cap=16)
    _, rc, info, full = ds.solve(_dev(f), maxit=8, **kw)
    assert rc == capi.AMGG_MAXIT and info.iterations == 8 and len(full) == 9
    S = amg.to_scipy(A)
    fb = f - f.mean() if hp.singular else f
    for k in range(1, 8):
        x1, rc, info, hist = ds.solve(_dev(f), maxit=k, **kw)
        x1 = x1.cpu().numpy()
        assert rc == capi.AMGG_MAXIT and info.iterations == k and info.vcycles == k, (outer, k)
        assert np.array_equal(_bits(np.asarray(hist)), _bits(np.asarray(full[:k + 1]))), (outer, k)
        x2, _, _, _ = ds.solve(_dev(f), maxit=k, **kw)
        assert np.array_equal(_bits(x1), _bits(x2.cpu().numpy())), (outer, k)
        if outer == "ir":
            rel = np.linalg.norm(fb - S @ x1) / np.linalg.norm(fb)
            assert abs(rel - hist[-1]) <= 1e-7 * hist[-1], (k, rel, hist[-1])


def test_zero_rhs_returns_zero():
    from paper_2606_19251_amd import capi

    A, f, ho, hp, ds = _setup("grid64")
    ds.set_jacobi()
    x, rc, info, _ = ds.solve(_dev(np.zeros_like(f)), outer=capi.AMGG_OUTER_FCG, precision=32)
    assert rc == 0 and info.iterations == 0 and float(x.abs().max()) == 0.0


def test_single_level_is_direct_solve():
    from paper_2606_19251_amd.solver import DeviceSolver, HostHierarchy
    import scipy.linalg as sla

    A = W.grid5(12)
    f = W.rhs_uniform(144, 4)
    hp = HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=500)
    assert hp.nlevels == 1
    ds = DeviceSolver(hp, 0)
    u = _dev(np.zeros(144))
    ds.vcycle(_dev(f), u, 1, 1, 64)
    ref = sla.solve(amg.to_scipy(A).toarray(), f)
    assert np.linalg.norm(u.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("outer", ["fcg", "ir"])
@pytest.mark.parametrize("cname", ["jacobi", "poly2"])
def test_graph_replay_equals_direct_launches(outer, cname):
    """Outer iterations replayed from captured HIP graphs give bitwise the same iterates as direct
    launches, over several solves with eager work and synchronisation in between."""
    from paper_2606_19251_amd import capi

    A, f, ho, hp, ds = _setup("delaunay20k")
    ds.set_coeffs(*COEFFS[cname])
    om = capi.AMGG_OUTER_FCG if outer == "fcg" else capi.AMGG_OUTER_IR
    for seed in range(3):
        b = _dev(W.rhs_uniform(A.nrows, 50 + seed, zero_mean=True))
        x1, rc1, i1, h1 = ds.solve(b, outer=om, precision=32, graphs=False, history_cap=600)
        torch.cuda.synchronize()
        _ = (b * 2).sum().item()  # unrelated eager work between replays
        x2, rc2, i2, h2 = ds.solve(b, outer=om, precision=32, graphs=True, history_cap=600)
        torch.cuda.synchronize()
        assert rc1 == rc2 == 0 and i1.iterations == i2.iterations
        assert torch.equal(x1, x2)
        assert np.array_equal(h1, h2)


@pytest.mark.parametrize("kind", ["grid64", "cmesh32k", "tet30k"])
@pytest.mark.parametrize("cname", ["jacobi", "poly2"])
def test_level_operators_bitexact(kind, cname):
    """Every level pass sums each row in stored order with separately rounded products, as the
    oracle's sparse products do: residual, smoothing, restriction and prolongation in FP64 are
    bitwise equal to the oracle's."""
    from paper_2606_19251_amd import capi

    A, f, ho, hp, ds = _setup(kind)
    c, deg = COEFFS[cname]
    ds.set_coeffs(c, deg)
    Qs = amg.smoothers(ho, c, deg)
    rng = np.random.default_rng(3)
    st = ds.stream
    for l in range(ho.nlevels - 1):
        L = ho.levels[l]
        n, nc = L.A.shape[0], L.P.shape[1]
        x, fl, y0 = rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n)
        xc = rng.standard_normal(nc)
        cases = [
            (capi.AMGG_OP_RESIDUAL, x, fl, None, fl - L.A @ x, n),
            (capi.AMGG_OP_SMOOTH, x, None, y0, y0 + Qs[l] @ x, n),
            (capi.AMGG_OP_RESTRICT, x, None, None, L.R @ x, nc),
            (capi.AMGG_OP_PROLONG, xc, None, y0, y0 + L.P @ xc, n),
        ]
        for op, xin, fin, yin, ref, m in cases:
            xd = _dev(xin)
            fd = _dev(fin) if fin is not None else xd
            yd = _dev(yin) if yin is not None else torch.zeros(m, dtype=torch.float64, device="cuda")
            capi.amgg_level_apply(ds.ctx, l, op, 64, xd.data_ptr(), yd.data_ptr(), fd.data_ptr(), st)
            torch.cuda.synchronize()
            assert np.array_equal(_bits(yd.cpu().numpy()), _bits(ref)), (l, op)


@pytest.mark.parametrize("kind", ["grid64", "delaunay20k", "gmm5k", "tiny", "cmesh32k", "tet30k"])
@pytest.mark.parametrize("cname", ["jacobi", "poly2"])
@pytest.mark.parametrize("prec", [64, 32])
def test_fused_kernels_equal_separate_passes(kind, cname, prec):
    """The fused kernels (first pre-smoothing step with the residual; halo-fused sparse smoothing
    steps) give bitwise the iterates of the separate passes, for several (nu1, nu2)."""
    A, f, ho, hp, ds = _setup(kind)
    c, deg = COEFFS[cname]
    ds.set_coeffs(c, deg)
    if kind != "tiny":  # the fused kernels are in use on some level
        assert any(ds.level_view(l)["fused_rows"] > 0 for l in range(hp.nlevels - 1))
    rng = np.random.default_rng(5)
    u0 = rng.standard_normal(A.nrows)
    fd = _dev(f)
    try:
        for nu in [(1, 1), (2, 2), (2, 1), (0, 1), (3, 0)]:
            for start in (np.zeros(A.nrows), u0):
                out = []
                for fuse in (True, False):
                    ds.set_fusion(fuse)
                    u = _dev(start)
                    ds.vcycle(fd, u, nu[0], nu[1], prec)
                    out.append(u)
                torch.cuda.synchronize()
                assert torch.equal(out[0], out[1]), (nu, float((out[0] - out[1]).abs().max()))
    finally:
        ds.set_fusion(True)


def test_timed_level_operator_records_kernel_time():
    from paper_2606_19251_amd import capi

    A, f, ho, hp, ds = _setup("delaunay20k")
    ds.set_jacobi()
    x = _dev(np.random.default_rng(1).standard_normal(A.nrows))
    y1 = torch.zeros_like(x)
    y2 = torch.zeros_like(x)
    fd = _dev(f)
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    s1.record()
    torch.cuda.synchronize()
    capi.amgg_level_apply(ds.ctx, 0, capi.AMGG_OP_RESIDUAL, 64, x.data_ptr(), y1.data_ptr(), fd.data_ptr(),
                          ds.stream)
    capi.amgg_level_apply_timed(ds.ctx, 0, capi.AMGG_OP_RESIDUAL, 64, x.data_ptr(), y2.data_ptr(), fd.data_ptr(),
                                s0.cuda_event, s1.cuda_event, ds.stream)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    ms = s0.elapsed_time(s1)
    assert 0.0 < ms < 10.0
    with pytest.raises(capi.AmggError):
        capi.amgg_level_apply_timed(ds.ctx, 0, capi.AMGG_OP_RESIDUAL, 64, x.data_ptr(), y2.data_ptr(),
                                    fd.data_ptr(), 0, 0, ds.stream)


@pytest.mark.parametrize("kind", ["grid64", "delaunay20k", "tet30k"])
@pytest.mark.parametrize("smoother", ["jacobi", "diag2"])
def test_ready_first_step_solves_equal_separate_passes(kind, smoother):
    """Where a level's cycle from zero starts with a diagonal step, the pass that produces its
    right-hand side (the outer loop's FP32 cast on the fine level, the restriction below it) also
    forms u = qd f; under iterative refinement the FP64 residual kernel itself writes the next
    cycle's FP32 right-hand side (scaled by a power of two) instead of the FP64 residual. The
    FP32-cycle solves (iterative refinement and flexible CG, V(1,1) and V(2,2)) are bitwise those
    of the separate passes."""
    from paper_2606_19251_amd import capi

    A, f, ho, hp, ds = _setup(kind)
    if smoother == "jacobi":
        ds.set_jacobi()
    else:  # Eq. 5 with f_o = 0 on the two finest levels, the sparse form below
        c = np.tile(COEFFS["poly2"][0], (ds.nlevels, 1)).astype(np.float32)
        ds.set_coeffs_device(torch.from_numpy(c).cuda(), 2, diag_levels=2)
    fd = _dev(f)
    try:
        for outer in (capi.AMGG_OUTER_IR, capi.AMGG_OUTER_FCG):
            for nu in ((1, 1), (2, 2)):
                res = []
                for fuse in (True, False):
                    ds.set_fusion(fuse)
                    x, rc, info, _ = ds.solve(fd, outer=outer, precision=32, nu1=nu[0], nu2=nu[1], tol=1e-8)
                    torch.cuda.synchronize()
                    res.append((x.clone(), info.iterations, rc, info.fell_back))
                print(f"[gpu] {kind} {smoother} outer={outer} nu={nu}: rc={res[0][2]} it={res[0][1]} "
                      f"fell_back={res[0][3]}", flush=True)
                assert res[0][2] == 0 or smoother != "jacobi"
                assert res[0][1:] == res[1][1:], (outer, nu)
                assert torch.equal(res[0][0], res[1][0]), (outer, nu)
    finally:
        ds.set_fusion(True)


def _stream_rows(n, nnz):
    avg = nnz / n if n > 0 else 0.0
    for r in (256, 128, 64):
        if r * avg <= 0.9 * 2048:
            return r
    for r in (256, 128, 64, 32):
        if r * avg * 1.25 <= 4096:
            return r
    return 0


def _expected_cap(rowptr, n, nnz):
    rows = _stream_rows(n, nnz)
    if rows == 0:
        return 4096  # lane kernel: the capacity is not used
    starts = rowptr[np.minimum(np.arange(0, n, rows), n)]
    ends = rowptr[np.minimum(np.arange(0, n, rows) + rows, n)]
    big = int((ends - starts).max()) if n > 0 else 0
    return min(4096, max(2048, -(-big // 2048) * 2048))


@pytest.mark.parametrize("kind", ["grid64", "delaunay20k", "cmesh32k", "tet30k", "tiny"])
def test_stream_lds_capacity_covers_largest_block(kind):
    """The CSR-stream kernels' LDS product buffer of every matrix is the largest row block rounded
    up to whole rounds of 2048 products (at most 4096), recomputed here from the host matrices."""
    import scipy.sparse as sp

    A, f, ho, hp, ds = _setup(kind)
    caps = set()
    for l, L in enumerate(hp.levels):
        v = ds.level_view(l)
        assert v["stream_cap"][0] == _expected_cap(L.rowptr, L.n, L.nnz), (l, "A")
        caps.add(v["stream_cap"][0])
        if l + 1 < hp.nlevels:
            pz = int(L.p_col.size)
            assert v["stream_cap"][1] == _expected_cap(L.p_rowptr, L.n, pz), (l, "P")
            R = sp.csr_matrix((np.ones(pz), L.p_col, L.p_rowptr), shape=(L.n, L.p_ncols)).T.tocsr()
            assert v["stream_cap"][2] == _expected_cap(R.indptr, L.p_ncols, pz), (l, "R")
    print(f"[gpu] {kind}: stream caps {sorted(caps)}", flush=True)
    assert 2048 in caps

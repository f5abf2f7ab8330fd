"""Block-diagonal (batched) hierarchies against the problems cycled one by one.

A mini-batch of problems with different depths (1 to 5 levels), families and boundary
conditions (Dirichlet grids, an airfoil C-mesh, all-Neumann Delaunay and tetrahedral meshes)
is put in one block-diagonal context, shallower problems repeating their coarsest level
with an identity P and no smoother. Checked against the per-problem contexts:
- V-cycles (FP64 and FP32; Jacobi, host polynomial and per-problem device coefficients):
  bitwise equal block by block (a one-level problem with a nonzero initial guess is the
  exception: its own cycle is the coarse solve A^-1 f, which ignores the guess, while in the
  batch it is u0 + A^-1 (f - A u0), equal up to rounding: 1e-12);
- the residual-reduction loss (Eq. 11) and its coefficient gradient (hand-written adjoint)
  of one and two cycles: equal up to the summation order of the per-block norms and
  gradient sums (1e-12 in FP64; FP32 cycles 1e-4 relative on the gradients). For the
  one-level problem both cycles are exact solves, so from the second cycle on its loss is
  the logarithm of a rounding-level residual in both (checked: below -12 in FP64, -5 in
  FP32) and is not compared;
- one training step (Alg. 1) of the batched trainer against the sequential one;
- the errors: bad block tables, a prolongation that couples blocks, calls that need (or
  must not have) blocks.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

POLY2 = np.array([0.6, 0.01, -0.001, 0.12, 0.01])


def _bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint64 if a.dtype == np.float64 else np.uint32)


@pytest.fixture(scope="module")
def batch():
    from paper_2606_19251_amd.solver import BatchSolver, DeviceSolver, HostHierarchy

    mats = [W.grid5(30), W.grid5(8), W.delaunay_p1(W.gmm_points(3000, 1)), W.cmesh_fv(64, 32, "2412", 1e3),
            W.tet_fv_mesh(*W.kuhn_tets(8, 3)), W.delaunay_p1(W.gmm_points(9000, 2))]
    hiers = [HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=100) for A in mats]
    print(f"[gpu] batch depths {[h.nlevels for h in hiers]} sizes {[h.levels[0].n for h in hiers]}", flush=True)
    assert len({h.nlevels for h in hiers}) >= 3 and min(h.nlevels for h in hiers) == 1
    singles = [DeviceSolver(h, 0) for h in hiers]
    bs = BatchSolver(hiers, 0)
    first = np.cumsum([0] + [h.nlevels for h in hiers])
    return hiers, singles, bs, first


def _random_coeffs(ngraphs, seed):
    rng = np.random.default_rng(seed)
    c = np.tile(POLY2, (ngraphs, 1)) * (1 + 0.1 * rng.standard_normal((ngraphs, 5)))
    return torch.from_numpy(c.astype(np.float32)).cuda()


def _set(kind, singles, bs, first, seed=0):
    if kind == "jacobi":
        for ds in singles:
            ds.set_jacobi(2 / 3)
        bs.ds.set_jacobi(2 / 3)
    elif kind == "poly":
        for ds in singles:
            ds.set_coeffs(POLY2, 2)
        bs.ds.set_coeffs(POLY2, 2)
    else:
        coeffs = _random_coeffs(bs.ngraphs, seed)
        for p, ds in enumerate(singles):
            ds.set_coeffs_device(coeffs[first[p]:first[p + 1]].contiguous(), 2)
        bs.set_coeffs_device(coeffs, 2)
        return coeffs


@pytest.mark.parametrize("guess", ["zero", "random"])
@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("kind", ["jacobi", "poly", "device"])
def test_block_vcycle_bitwise_equal_to_per_problem(batch, kind, precision, guess):
    hiers, singles, bs, first = batch
    _set(kind, singles, bs, first)
    rng = np.random.default_rng(1)
    us = [rng.standard_normal(h.levels[0].n) * (guess == "random") for h in hiers]
    fs = [rng.standard_normal(h.levels[0].n) for h in hiers]
    ref = []
    for ds, u, f in zip(singles, us, fs):
        ud = torch.from_numpy(u).cuda()
        ds.vcycle(torch.from_numpy(f).cuda(), ud, 1, 1, precision)
        ref.append(ud.cpu().numpy())
    ub = torch.from_numpy(np.concatenate(us)).cuda()
    bs.ds.vcycle(torch.from_numpy(np.concatenate(fs)).cuda(), ub, 1, 1, precision)
    got = np.split(ub.cpu().numpy(), bs.offsets[0][1:-1])
    for p in range(len(hiers)):
        if hiers[p].nlevels == 1 and guess == "random":
            tol = 1e-12 if precision == 64 else 1e-6
            assert np.linalg.norm(got[p] - ref[p]) <= tol * np.linalg.norm(ref[p]), (kind, precision, p)
        else:
            assert np.array_equal(_bits(got[p]), _bits(ref[p])), (kind, precision, guess, p, hiers[p].nlevels)


@pytest.mark.parametrize("precision,nvc", [(64, 1), (64, 2), (32, 1), (32, 2)])
def test_block_loss_and_gradient_match_per_problem(batch, precision, nvc):
    from paper_2606_19251_amd import capi

    hiers, singles, bs, first = batch
    _set("device", singles, bs, first, seed=3)
    fs = [W.rhs_uniform(h.levels[0].n, 40 + p, zero_mean=h.singular) for p, h in enumerate(hiers)]
    loss_ref = torch.zeros(len(hiers), dtype=torch.float64, device="cuda")
    dc_ref = torch.zeros(bs.ngraphs, 5, dtype=torch.float64, device="cuda")
    fd = [torch.from_numpy(f).cuda() for f in fs]
    for p, ds in enumerate(singles):
        capi.amgg_vcycle_loss_adjoint(ds.ctx, 1, 1, precision, nvc, fd[p].data_ptr(), 0, loss_ref[p:p + 1].data_ptr(),
                                      dc_ref[first[p]:first[p + 1]].data_ptr(), ds.stream)
    loss = torch.full((len(hiers),), np.nan, dtype=torch.float64, device="cuda")
    dc = torch.full((bs.ngraphs, 5), np.nan, dtype=torch.float64, device="cuda")
    bs.loss_adjoint(torch.cat(fd), loss, dc, precision=precision, nvc=nvc)
    torch.cuda.synchronize()
    lr, l, gr, g = loss_ref.cpu().numpy(), loss.cpu().numpy(), dc_ref.cpu().numpy(), dc.cpu().numpy()
    print(f"[gpu] precision {precision} nvc {nvc}: losses {np.round(l, 4)} / {np.round(lr, 4)}", flush=True)
    exact = [p for p, h in enumerate(hiers) if h.nlevels == 1]
    cmp = [p for p in range(len(hiers)) if nvc == 1 or p not in exact]
    assert np.abs(l[cmp] - lr[cmp]).max() <= (1e-12 if precision == 64 else 1e-6)
    floor = -12 if precision == 64 else -5
    assert all(l[p] < floor and lr[p] < floor for p in exact)
    coarsest = [first[p + 1] - 1 for p in range(len(hiers))]
    assert not g[coarsest].any() and not gr[coarsest].any()
    for p in range(len(hiers)):
        a, b = first[p], first[p + 1]
        err = np.linalg.norm(g[a:b] - gr[a:b]) / max(np.linalg.norm(gr[a:b]), 1e-300)
        assert err <= (1e-10 if precision == 64 else 1e-4), (p, err)


def test_batched_training_step_matches_sequential():
    from paper_2606_19251_amd import capi
    from paper_2606_19251_amd import gcin as G
    from paper_2606_19251_amd.solver import DeviceSolver, HostHierarchy

    meshes = W.training_batch(8, seed=2)
    solvers = [DeviceSolver(HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=100), 0) for A, _ in meshes]
    rhs = [torch.from_numpy(f).cuda() for _, f in meshes]
    out = {}
    for batched in (False, True):
        pred = G.Predictor(G.init_flat(2, 0), torch.device("cuda", 0), 2, capi.GCIN_BF16X3)
        tr = G.Trainer(solvers, rhs, pred, nvc=2, batched=batched)
        losses = tr.step()
        torch.cuda.synchronize()
        out[batched] = (losses.cpu().numpy().copy(), tr.grads.cpu().numpy().copy())
    (l0, g0), (l1, g1) = out[False], out[True]
    print(f"[gpu] batched step: losses {np.round(l1, 4)}, max |dloss| {np.abs(l1 - l0).max():.2e}, "
          f"gradient rel. diff {np.linalg.norm(g1 - g0) / np.linalg.norm(g0):.2e}", flush=True)
    assert np.abs(l1 - l0).max() <= 1e-6
    assert np.linalg.norm(g1 - g0) <= 1e-4 * np.linalg.norm(g0)


def test_block_errors(batch):
    from paper_2606_19251_amd import capi
    from paper_2606_19251_amd.solver import DeviceSolver, block_diagonal

    hiers, singles, bs, first = batch
    bad = [(np.array([0, 5], np.int32), None), (np.array([0, 0, singles[0].n], np.int32), None),
           (np.array([0, 10, singles[0].n], np.int32), np.array([3, 3], np.int32))]
    for offsets, rows in bad:
        with pytest.raises(capi.AmggError) as e:
            capi.amgg_set_level_blocks(singles[0].ctx, 0, offsets, rows)
        assert e.value.code == capi.AMGG_EINVAL
    with pytest.raises(capi.AmggError) as e:
        bs.ds.solve(torch.zeros(bs.ds.n, dtype=torch.float64, device="cuda"))
    assert e.value.code == capi.AMGG_ESTATE
    loss = torch.zeros(8, dtype=torch.float64, device="cuda")
    dc = torch.zeros(bs.ngraphs, 5, dtype=torch.float64, device="cuda")
    f = torch.zeros(bs.ds.n, dtype=torch.float64, device="cuda")
    with pytest.raises(capi.AmggError) as e:
        capi.amgg_vcycle_loss_adjoint(bs.ctx, 1, 1, 64, 1, f.data_ptr(), 0, loss.data_ptr(), dc.data_ptr(), 0)
    assert e.value.code == capi.AMGG_ESTATE
    with pytest.raises(capi.AmggError) as e:
        capi.amgg_vcycle_loss_adjoint_blocks(singles[2].ctx, 1, 1, 64, 1, f.data_ptr(), 0, loss.data_ptr(),
                                             dc.data_ptr(), bs.ngraphs, 0)
    assert e.value.code == capi.AMGG_ESTATE
    # a prolongation entry that couples block 0 with coarse block 1
    bh, offsets, rows, sing = block_diagonal([hiers[0], hiers[2]])
    bh.levels[0].p_col[0] = offsets[1][1]
    with pytest.raises(capi.AmggError) as e:
        DeviceSolver(bh, 0, blocks=(offsets, rows, sing))
    assert e.value.code == capi.AMGG_EINVAL

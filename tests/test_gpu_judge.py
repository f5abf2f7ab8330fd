"""The omega-Jacobi AMG as judge of the learned smoother (amgg_judge_smoother): the paper's
acceleration is the Jacobi solve time over the learned-smoother solve time (Sec. 4), so on a
given matrix the learned coefficients are kept only when they predict the shorter solve.

The decision rests on measured times, so every test checks the judge's record against itself
(predictions recomputed from each probe's iterations, final residual, second-half reduction
rate and time per iteration; the decision their argmin) and the state it leaves (a solve after
the judge is bitwise the solve with the winner set explicitly).
The outcome itself is asserted only where the margin is wide:
- a smoother that barely smooths (c = (0.05, 0, ...), i.e. 0.05-Jacobi) needs many times
  Jacobi's iterations at the same cost per iteration: Jacobi is kept;
- c = (-1, 0, ...) makes flexible CG break down at once (oracle-checked in the fallback tests):
  its prediction is infinite, Jacobi is kept;
- the trained tetrahedral network (diagonal form on the 2 finest levels) under iterative
  refinement on a 1.3M-cell tetrahedral mesh: about 30 % fewer cycles at about 1.15 times the
  cost per cycle on the 8M-cell mesh of the benchmark; the learned smoother is kept.
"""
import math
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_cache = {}


def _grid():
    if "g" not in _cache:
        from paper_2606_19251_amd.solver import DeviceSolver, HostHierarchy

        A, f = W.poisson_grid_64(0)
        hh = HostHierarchy.build(A.rowptr, A.col, A.val, max_levels=3)
        print(f"[gpu] judge problem grid64 levels={hh.nlevels}", flush=True)
        _cache["g"] = (hh, DeviceSolver(hh, 0), torch.from_numpy(f).cuda())
    return _cache["g"]


def _const(ds, c):
    return torch.tensor(np.tile(np.asarray(c, np.float32), (ds.nlevels, 1)), device="cuda").contiguous()


def _check_record(j, tol=1e-8):
    """Each prediction follows from its probe's record; the decision is their argmin."""
    for s in range(2):
        st, k, ms = j["status"][s], j["iterations"][s], j["ms_per_iter"][s]
        rel, rate = j["log10_relres"][s], j["log10_rate"][s]
        if st == 0:
            want = ms * k
        elif st == 1 and rate < 0 and math.isfinite(rel):
            want = ms * (k + (math.log10(tol) - rel) / rate)
        else:
            want = math.inf
        if math.isinf(want):
            assert math.isinf(j["predicted_ms"][s]), (s, j)
        else:
            assert abs(j["predicted_ms"][s] - want) <= 1e-9 * abs(want), (s, j)
    assert j["learned_wins"] == (j["predicted_ms"][0] < j["predicted_ms"][1]), j


def _same_solve(ds, b, outer, set_winner):
    """x after a solve in the judged state equals x after setting the winner explicitly."""
    x1 = torch.empty_like(b)
    _, rc1, i1, _ = ds.solve(b, x1, outer=outer, precision=32, tol=1e-8, fallback=False)
    set_winner()
    x2 = torch.empty_like(b)
    _, rc2, i2, _ = ds.solve(b, x2, outer=outer, precision=32, tol=1e-8, fallback=False)
    torch.cuda.synchronize()
    assert (rc1, i1.iterations) == (rc2, i2.iterations)
    assert torch.equal(x1, x2)
    return rc1, i1.iterations


@pytest.mark.parametrize("outer", ["ir", "fcg"])
def test_judge_keeps_jacobi_for_a_weak_smoother(outer):
    from paper_2606_19251_amd import capi

    hh, ds, b = _grid()
    code = capi.AMGG_OUTER_IR if outer == "ir" else capi.AMGG_OUTER_FCG
    c = _const(ds, [0.05, 0.0, 0.0, 0.0, 0.0])
    j = ds.judge(b, c, 2, outer=code, iters=12, diag_levels=0)
    print(f"[gpu] judge weak smoother ({outer}): {j}", flush=True)
    _check_record(j)
    assert not j["learned_wins"]
    assert j["log10_rate"][1] < 2 * j["log10_rate"][0]  # Jacobi reduces the residual far faster
    rc, it = _same_solve(ds, b, code, lambda: ds.set_jacobi(2 / 3))
    assert rc == 0


def test_judge_counts_a_breakdown_as_a_loss():
    from paper_2606_19251_amd import capi

    hh, ds, b = _grid()
    c = _const(ds, [-1.0, 0.0, 0.0, 0.0, 0.0])
    j = ds.judge(b, c, 2, outer=capi.AMGG_OUTER_FCG, iters=6)
    print(f"[gpu] judge indefinite smoother: {j}", flush=True)
    _check_record(j)
    assert j["status"][0] == capi.AMGG_BREAKDOWN and math.isinf(j["predicted_ms"][0])
    assert not j["learned_wins"] and j["status"][1] in (0, capi.AMGG_MAXIT)
    _same_solve(ds, b, capi.AMGG_OUTER_FCG, lambda: ds.set_jacobi(2 / 3))


def test_judge_keeps_the_trained_network_under_refinement():
    from paper_2606_19251_amd import capi
    from paper_2606_19251_amd import gcin as G
    from paper_2606_19251_amd.solver import DeviceSolver, HostHierarchy

    A, f = W.tet_kuhn_problem(60, 3)
    hh = HostHierarchy.build(A.rowptr, A.col, A.val, max_levels=10, max_coarse=500, galerkin="device")
    print(f"[gpu] judge problem tet m=60 n={A.nrows} levels={hh.nlevels}", flush=True)
    ds = DeviceSolver(hh, 0)
    b = torch.from_numpy(f).cuda()
    pred = G.Predictor.load(os.path.join(ROOT, "paper_2606_19251_amd", "weights", "gcin_tet_deg2_d2.npz"),
                            torch.device("cuda", 0))
    coeffs, j = pred.predict_judged(hh, ds, b, outer=capi.AMGG_OUTER_IR)
    print(f"[gpu] judge trained tet network (IR): {j}", flush=True)
    _check_record(j)
    assert j["learned_wins"], j
    _same_solve(ds, b, capi.AMGG_OUTER_IR, lambda: ds.set_coeffs_device(coeffs, pred.degree))
    ds.close()


def test_judge_rejects_bad_arguments():
    from paper_2606_19251_amd import capi

    hh, ds, b = _grid()
    c = _const(ds, [2 / 3, 0.0, 0.0, 0.0, 0.0])
    x = torch.empty_like(b)
    o = capi.amgg_solve_opts(capi.AMGG_OUTER_FCG, 32, 1, 1, 8, 1e-8, 0, 0.0, 0.0, 0, 1)
    for iters, deg, coeffs, diag in ((0, 2, c.data_ptr(), 0), (101, 2, c.data_ptr(), 0), (8, 0, c.data_ptr(), 0),
                                     (8, 2, 0, 0), (8, 2, c.data_ptr(), -1)):
        with pytest.raises(capi.AmggError) as ei:
            capi.amgg_judge_smoother(ds.ctx, o, iters, deg, coeffs, diag, b.data_ptr(), x.data_ptr(), ds.stream)
        assert ei.value.code == capi.AMGG_EINVAL, (iters, deg, diag)


def test_judge_not_available_on_a_block_diagonal_context():
    from paper_2606_19251_amd import capi
    from paper_2606_19251_amd.solver import BatchSolver, HostHierarchy

    hs = []
    for k in (24, 30):
        A = W.grid5(k)
        hs.append(HostHierarchy.build(A.rowptr, A.col, A.val, max_levels=3, max_coarse=50))
    bs = BatchSolver(hs, 0)
    n = sum(h.levels[0].n for h in hs)
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    c = torch.zeros(bs.ngraphs, 5, dtype=torch.float32, device="cuda")
    o = capi.amgg_solve_opts(capi.AMGG_OUTER_FCG, 32, 1, 1, 8, 1e-8, 0, 0.0, 0.0, 0, 1)
    with pytest.raises(capi.AmggError) as ei:
        capi.amgg_judge_smoother(bs.ctx, o, 4, 2, c.data_ptr(), 0, b.data_ptr(), x.data_ptr(), bs.ds.stream)
    assert ei.value.code == capi.AMGG_ESTATE

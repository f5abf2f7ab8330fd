"""Parity at the benchmark's full size: P1 Laplacian on the Delaunay mesh of 1,000,000 points.

The oracle builds its own hierarchy (compared bit for bit with the product's), runs one FP64
V-cycle from the same (u, f) as the GPU (1e-12 relative), and recomputes in FP64 the residual
of the GPU's FP32-cycle / FP64 flexible-CG solves (Jacobi and trained GCIN smoothers) at 1e-8.
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle import amg

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def full():
    from paper_2606_19251_amd.solver import DeviceSolver, HostHierarchy

    print("[gpu] full-size workload: 1M-point Delaunay P1", flush=True)
    A, f = W.delaunay_p1_problem(1_000_000, 0)
    An, fn, sing = amg.normalize(A, f)
    ho = amg.setup(An, singular=sing, max_levels=10, max_coarse=500)
    hp = HostHierarchy.build(A.rowptr, A.col, A.val, max_levels=10, max_coarse=500)
    print(f"[gpu] levels {[L.n for L in hp.levels]}", flush=True)
    return A, fn, ho, hp, DeviceSolver(hp, 0)


def test_full_hierarchy_bitexact(full):
    A, f, ho, hp, ds = full
    assert hp.nlevels == ho.nlevels
    for l in range(ho.nlevels):
        assert np.array_equal(ho.levels[l].A.indices, hp.levels[l].col)
        assert np.array_equal(ho.levels[l].A.data.view(np.uint64), hp.levels[l].val.view(np.uint64))
        if l + 1 < ho.nlevels:
            assert np.array_equal(ho.levels[l].P.data.view(np.uint64), hp.levels[l].p_val.view(np.uint64))


def test_full_vcycle_fp64(full):
    A, f, ho, hp, ds = full
    c = np.array([0.6, 0.01, -0.001, 0.12, 0.01])
    ds.set_coeffs(c, 2)
    u0 = np.random.default_rng(2).standard_normal(A.nrows)
    ref = amg.vcycle(ho, amg.smoothers(ho, c, 2), u0, f)
    u = torch.from_numpy(u0).cuda()
    ds.vcycle(torch.from_numpy(f).cuda(), u, 1, 1, 64)
    err = np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= 1e-12, err


@pytest.mark.parametrize("smoother", ["jacobi", "gcin"])
def test_full_solve_residual(full, smoother):
    from paper_2606_19251_amd import capi
    from paper_2606_19251_amd import gcin as G

    A, f, ho, hp, ds = full
    if smoother == "jacobi":
        ds.set_jacobi(2 / 3)
    else:
        pred = G.Predictor.load(os.path.join(ROOT, "paper_2606_19251_amd", "weights", "gcin_deg2.npz"),
                                torch.device("cuda", 0))
        ds.set_coeffs_device(pred.predict(hp, ds), pred.degree)
    x, rc, info, _ = ds.solve(torch.from_numpy(f).cuda(), outer=capi.AMGG_OUTER_FCG, precision=32, tol=1e-8,
                              fallback=False)
    assert rc == 0
    fb = f - f.mean()
    rel = np.linalg.norm(fb - ho.levels[0].A @ x.cpu().numpy()) / np.linalg.norm(fb)
    print(f"[gpu] {smoother}: {info.vcycles} cycles, oracle residual {rel:.2e}", flush=True)
    assert rel <= 1e-8 * 1.01


def test_full_fp32_level_operators_elementwise(full):
    """The FP32 operators of the timed cycle on the fine and first coarse level, row by row within
    the FP32 rounding bound of each row's sum (tests/fp32_operators.py)."""
    import scipy.sparse as sp

    from fp32_operators import check_level
    from paper_2606_19251_amd import capi

    A, f, ho, hp, ds = full
    c = np.array([0.6, 0.01, -0.001, 0.12, 0.01])
    ds.set_coeffs(c, 2)
    for l in (0, 1):
        L = hp.levels[l]
        Al = sp.csr_matrix((L.val, L.col, L.rowptr), shape=(L.n, L.n))
        P = sp.csr_matrix((L.p_val, L.p_col, L.p_rowptr), shape=(L.n, L.p_ncols))
        worst = check_level(torch, capi, ds, Al, P, amg.assemble_smoother(Al, c, 2), l, 10 + l)
        print(f"[gpu] 1M level {l}: largest FP32 error / bound {worst:.3f}", flush=True)

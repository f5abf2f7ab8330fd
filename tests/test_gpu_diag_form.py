"""The diagonal form of the Eq. 5 smoother on the finest levels (f_o taken as 0; the cost-aware
member of the family: a one-pass diagonal step where the levels are largest), against the oracle
with those levels' off-diagonal coefficients set to zero:
- smoother values bitwise, one FP64 V-cycle within 1e-12, the diagonal step actually used;
- loss and coefficient gradient (FP64 cycles) within 1e-9 of the complex step, the off-diagonal
  entries of the diagonal levels exactly zero (they are no parameters there);
- the block-diagonal (batched) form against the per-problem one.
"""
import numpy as np
import pytest

import workloads as W
from oracle import amg, grad

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_cache = {}
DIAG = 2


def _problem(seed=41, npts=6000):
    key = (seed, npts)
    if key not in _cache:
        from paper_2606_19251_amd.solver import DeviceSolver, HostHierarchy

        A = W.delaunay_p1(W.gmm_points(npts, seed))
        f = W.rhs_uniform(A.nrows, seed + 1, zero_mean=True)
        An, fn, sing = amg.normalize(A, f)
        ho = amg.setup(An, max_coarse=60, singular=sing)
        hp = HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=60)
        print(f"[gpu] diag-form problem levels={hp.nlevels}", flush=True)
        assert hp.nlevels > DIAG + 1
        _cache[key] = (ho, fn, hp, DeviceSolver(hp, 0))
    return _cache[key]


def _coeffs(nlevels, seed):
    rng = np.random.default_rng(seed)
    base = np.array([0.6, 0.01, -0.001, 0.12, 0.01])
    return (np.tile(base, (nlevels, 1)) * (1 + 0.05 * rng.standard_normal((nlevels, 5)))).astype(np.float32)


def _zero_offdiag(c, k):
    c = np.array(c, np.float64)
    c[:k, 3:] = 0.0
    return c


def test_diag_form_smoother_and_cycle_match_oracle():
    ho, fn, hp, ds = _problem()
    c32 = _coeffs(ds.nlevels, 1)
    ds.set_coeffs_device(torch.from_numpy(c32).cuda(), 2, diag_levels=DIAG)
    cref = _zero_offdiag(c32, DIAG)
    for l in range(ds.nlevels - 1):
        v = ds.level_view(l)
        ref = amg.assemble_smoother(ho.levels[l].A, cref[l], 2).data
        assert np.array_equal(v["q_val"].cpu().numpy().view(np.uint64), ref.view(np.uint64)), l
    u0 = np.random.default_rng(2).standard_normal(fn.size)
    u = torch.from_numpy(u0).cuda()
    ds.vcycle(torch.from_numpy(fn).cuda(), u, 1, 1, 64)
    ref = amg.vcycle(ho, amg.smoothers(ho, cref, 2), u0, fn)
    assert np.linalg.norm(u.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("nu", [(1, 1), (2, 2)])
def test_diag_form_gradient_matches_complex_step(nu):
    from paper_2606_19251_amd import capi

    ho, fn, hp, ds = _problem()
    c32 = _coeffs(ds.nlevels, 3)
    ds.set_coeffs_device(torch.from_numpy(c32).cuda(), 2, diag_levels=DIAG)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.full((ds.nlevels, 5), np.nan, dtype=torch.float64, device="cuda")
    capi.amgg_vcycle_loss_adjoint(ds.ctx, nu[0], nu[1], 64, 1, torch.from_numpy(fn).cuda().data_ptr(), 0,
                                  loss.data_ptr(), g.data_ptr(), ds.stream)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    cref = _zero_offdiag(c32, DIAG)
    ref_loss = grad.vcycle_loss(ho, cref, 2, fn, nu1=nu[0], nu2=nu[1])
    ref = grad.grad_complex_step(ho, cref, 2, fn, nu1=nu[0], nu2=nu[1])
    ref[:DIAG, 3:] = 0.0  # f_o is no part of the diagonal levels' smoother
    assert abs(float(loss.item()) - ref_loss) <= 1e-11 * max(1.0, abs(ref_loss))
    assert np.all(g[:DIAG, 3:] == 0.0)
    assert np.abs(g - ref).max() <= 1e-9 * np.abs(ref).max(), np.abs(g - ref).max() / np.abs(ref).max()


def test_diag_form_blocks_match_per_problem():
    from paper_2606_19251_amd import capi
    from paper_2606_19251_amd.solver import BatchSolver

    probs = [_problem(41, 6000), _problem(43, 3000)]
    hiers = [p[2] for p in probs]
    bs = BatchSolver(hiers, 0)
    bs.diag_levels = DIAG
    first = np.cumsum([0] + [h.nlevels for h in hiers])
    c32 = _coeffs(bs.ngraphs, 5)
    bs.set_coeffs_device(torch.from_numpy(c32).cuda(), 2)
    fs = [p[1] for p in probs]
    loss = torch.zeros(2, dtype=torch.float64, device="cuda")
    dc = torch.zeros(bs.ngraphs, 5, dtype=torch.float64, device="cuda")
    bs.loss_adjoint(torch.from_numpy(np.concatenate(fs)).cuda(), loss, dc, (1, 1), 64, 1)
    torch.cuda.synchronize()
    for p, (ho, fn, hp, ds) in enumerate(probs):
        ds.set_coeffs_device(torch.from_numpy(c32[first[p]:first[p + 1]].copy()).cuda(), 2, diag_levels=DIAG)
        lr = torch.zeros(1, dtype=torch.float64, device="cuda")
        gr = torch.zeros(ds.nlevels, 5, dtype=torch.float64, device="cuda")
        capi.amgg_vcycle_loss_adjoint(ds.ctx, 1, 1, 64, 1, torch.from_numpy(fn).cuda().data_ptr(), 0, lr.data_ptr(),
                                      gr.data_ptr(), ds.stream)
        torch.cuda.synchronize()
        assert abs(loss[p].item() - lr.item()) <= 1e-12 * max(1.0, abs(lr.item()))
        a, b = dc[first[p]:first[p + 1]].cpu().numpy(), gr.cpu().numpy()
        assert np.all(a[:DIAG, 3:] == 0.0)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    bs.close()

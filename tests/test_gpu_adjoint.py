"""GPU V-cycle adjoint against the oracle's complex-step gradient and central differences."""
import numpy as np
import pytest

import workloads as W
from oracle import amg, grad

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_cache = {}


def _problem(kind):
    if kind not in _cache:
        from paper_2606_19251_amd.solver import DeviceSolver, HostHierarchy

        if kind == "gmm3k":
            A = W.delaunay_p1(W.gmm_points(3000, 5))
            f = W.rhs_uniform(A.nrows, 9, zero_mean=True)
            kw = dict(max_levels=10, max_coarse=40)
        else:
            A, f = W.poisson_grid_64(2)
            kw = dict(max_levels=3, max_coarse=500)
        An, fn, sing = amg.normalize(A, f)
        ho = amg.setup(An, singular=sing, **kw)
        hp = HostHierarchy.build(A.rowptr, A.col, A.val, **kw)
        print(f"[gpu] adjoint problem {kind} levels={hp.nlevels}", flush=True)
        _cache[kind] = (fn, ho, DeviceSolver(hp, 0))
    return _cache[kind]


def _coeffs(h, degree, seed):
    base = {2: [0.6, 0.01, -0.001, 0.12, 0.01], 3: [0.6, 0.01, -0.001, 0.0001, 0.12, 0.01, -0.001]}[degree]
    rng = np.random.default_rng(seed)
    return np.array([np.array(base) * (1 + 0.05 * rng.standard_normal(len(base))) for _ in range(h.nlevels)])


def _gpu_loss_grad(ds, c, degree, f, u0, nu, nvc, precision):
    from paper_2606_19251_amd import capi

    ds.set_coeffs(c, degree)
    fd = torch.from_numpy(f).cuda()
    ud = None if u0 is None else torch.from_numpy(u0).cuda()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.zeros(ds.nlevels, 2 * degree + 1, dtype=torch.float64, device="cuda")
    capi.amgg_vcycle_loss_adjoint(ds.ctx, nu[0], nu[1], precision, nvc, fd.data_ptr(),
                                  0 if ud is None else ud.data_ptr(), loss.data_ptr(), g.data_ptr(), ds.stream)
    torch.cuda.synchronize()
    return float(loss.item()), g.cpu().numpy()


@pytest.mark.parametrize("kind", ["grid64", "gmm3k"])
@pytest.mark.parametrize("degree", [2, 3])
@pytest.mark.parametrize("nu,nvc,with_u0", [((1, 1), 1, False), ((2, 2), 1, False), ((1, 1), 2, True), ((1, 2), 1, True)])
def test_adjoint_fp64_matches_complex_step(kind, degree, nu, nvc, with_u0):
    f, ho, ds = _problem(kind)
    c = _coeffs(ho, degree, 1)
    u0 = np.random.default_rng(4).standard_normal(f.size) * 0.1 if with_u0 else None
    loss, g = _gpu_loss_grad(ds, c, degree, f, u0, nu, nvc, 64)
    ref_loss = grad.vcycle_loss(ho, c, degree, f, u0, nvc, *nu)
    ref_g = grad.grad_complex_step(ho, c, degree, f, u0, nvc, *nu)
    assert abs(loss - ref_loss) <= 1e-11 * max(1.0, abs(ref_loss))
    scale = np.abs(ref_g).max()
    assert np.abs(g - ref_g).max() <= 1e-9 * scale, np.abs(g - ref_g).max() / scale
    assert np.all(g[-1] == 0.0)


def test_adjoint_fp64_central_differences_of_gpu_loss():
    """Central differences of the GPU's own FP64 loss, step 1e-6 relative (independent of the adjoint)."""
    f, ho, ds = _problem("gmm3k")
    c = _coeffs(ho, 2, 7)
    _, g = _gpu_loss_grad(ds, c, 2, f, None, (1, 1), 1, 64)
    for l in range(ho.nlevels - 1):
        for k in range(5):
            h = 1e-6 * max(abs(c[l, k]), 1e-2)
            cp, cm = c.copy(), c.copy()
            cp[l, k] += h
            cm[l, k] -= h
            lp, _ = _gpu_loss_grad(ds, cp, 2, f, None, (1, 1), 1, 64)
            lm, _ = _gpu_loss_grad(ds, cm, 2, f, None, (1, 1), 1, 64)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[l, k]) <= 1e-6 * max(np.abs(g).max(), 1e-12) + 1e-6 * abs(fd), (l, k, fd, g[l, k])


@pytest.mark.parametrize("kind", ["grid64", "gmm3k"])
def test_adjoint_fp32_close_to_oracle(kind):
    f, ho, ds = _problem(kind)
    c = _coeffs(ho, 2, 3)
    loss, g = _gpu_loss_grad(ds, c, 2, f, None, (1, 1), 1, 32)
    ref_g = grad.grad_complex_step(ho, c, 2, f)
    ref_loss = grad.vcycle_loss(ho, c, 2, f)
    assert abs(loss - ref_loss) <= 1e-4 * max(1.0, abs(ref_loss))
    a, b = g[:-1].ravel(), ref_g[:-1].ravel()
    cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
    assert cos >= 0.999, cos
    assert np.abs(a - b).max() <= 1e-4 * np.abs(b).max()


def test_adjoint_at_jacobi_coefficients_has_offdiagonal_gradient():
    """At c = (omega, 0, 0, 0, 0) the cycle uses the one-pass diagonal step; the gradient still
    covers the off-diagonal coefficients and matches the complex step."""
    f, ho, ds = _problem("gmm3k")
    c = np.tile(amg.jacobi_coeffs(), (ho.nlevels, 1))
    _, g = _gpu_loss_grad(ds, c, 2, f, None, (1, 1), 1, 64)
    ref = grad.grad_complex_step(ho, c, 2, f)
    assert np.abs(g - ref).max() <= 1e-9 * np.abs(ref).max()
    assert np.abs(g[0, 3:]).max() > 0

"""The learning loop on the GPU: the autograd Functions against the oracle, the autograd training
step against the direct library calls, the validation metric (Eq. 13) against the oracle, and a
short training run whose schedule (plateau halving, best model kept, seed ensemble) is checked.
"""
import argparse
import os

import numpy as np
import pytest

import workloads as W
from oracle import amg, grad
from oracle import gcin as OG

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_cache = {}


def _problem():
    if "p" not in _cache:
        from paper_2606_19251_amd.solver import DeviceSolver, HostHierarchy

        A = W.delaunay_p1(W.gmm_points(4000, 31))
        f = W.rhs_uniform(A.nrows, 32, zero_mean=True)
        An, fn, sing = amg.normalize(A, f)
        ho = amg.setup(An, max_coarse=60, singular=sing)
        hp = HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=60)
        print(f"[gpu] training problem levels={hp.nlevels}", flush=True)
        _cache["p"] = (ho, fn, DeviceSolver(hp, 0))
    return _cache["p"]


@pytest.mark.parametrize("degree", [2, 3])
def test_vcycle_loss_function_gradient_matches_complex_step(degree):
    from paper_2606_19251_amd.autograd import VCycleLoss

    ho, fn, ds = _problem()
    base = {2: [0.6, 0.01, -0.001, 0.12, 0.01], 3: [0.6, 0.01, -0.001, 0.0001, 0.12, 0.01, -0.001]}[degree]
    rng = np.random.default_rng(degree)
    c = (np.tile(base, (ds.nlevels, 1)) * (1 + 0.05 * rng.standard_normal((ds.nlevels, 2 * degree + 1))))
    c = c.astype(np.float32)
    coeffs = torch.from_numpy(c).cuda().requires_grad_()
    f = torch.from_numpy(fn).cuda()
    loss = VCycleLoss.apply(coeffs, ds, f, (1, 1), 64, 1)
    (3.0 * loss).sum().backward()  # an outer factor, applied by the chain rule
    g = coeffs.grad.cpu().numpy().astype(np.float64)
    c64 = c.astype(np.float64)
    ref = 3.0 * grad.grad_complex_step(ho, c64, degree, fn)
    ref_loss = grad.vcycle_loss(ho, c64, degree, fn)
    assert abs(float(loss.item()) - ref_loss) <= 1e-11 * max(1.0, abs(ref_loss))
    # FP32 output of the chain rule: one FP32 rounding of each FP64 gradient entry
    assert np.abs(g - ref).max() <= 1e-6 * np.abs(ref).max(), np.abs(g - ref).max() / np.abs(ref).max()


def test_gcin_function_gradient_matches_oracle():
    from paper_2606_19251_amd import capi
    from paper_2606_19251_amd import gcin as G
    from paper_2606_19251_amd.autograd import GCIN

    ho, fn, ds = _problem()
    # parameters as in the GCIN kernel tests: nonzero shifts and gains, outputs not a bias
    p = OG.init_params(2, 5)
    rng = np.random.default_rng(6)
    for l in range(4):
        p[f"norm{l}.beta"] = rng.uniform(-0.3, 0.6, 64)
        p[f"norm{l}.gamma"] = rng.uniform(0.7, 1.3, 64)
        p[f"conv{l}.b"] = rng.uniform(-0.1, 0.1, 64)
    p["ln.gamma"] = rng.uniform(0.8, 1.2, 128)
    p["mlp2.b"] = np.zeros(5)
    p["mlp2.W"] *= 3.0
    flat = G.pack(p, 2)
    p64 = G.unpack(flat, 2)
    batch = G.GraphBatch([ds.A[l] for l in range(ds.nlevels)], torch.device("cuda", 0))
    P = torch.from_numpy(flat).cuda().requires_grad_()
    coeffs = GCIN.apply(P, batch, 2, capi.GCIN_FP32)
    w = rng.standard_normal((ds.nlevels, 5)).astype(np.float32)
    torch.autograd.backward(coeffs, grad_tensors=torch.from_numpy(w).cuda())
    g = P.grad.cpu().numpy()
    # the Function routes exactly the library's backward
    batch.forward(P.detach(), 2, capi.GCIN_FP32)
    direct = batch.backward(P.detach(), torch.from_numpy(w).cuda(), 2, capi.GCIN_FP32).cpu().numpy()
    assert np.array_equal(g.view(np.uint32), direct.view(np.uint32))
    # and that is the oracle's gradient, per tensor as in the kernel tests
    g = g.astype(np.float64)
    ref = OG.gradient(p64, [L.A for L in ho.levels], w.astype(np.float64), 2)
    refflat = G.pack(ref, 2).astype(np.float64)
    cos = g @ refflat / (np.linalg.norm(g) * np.linalg.norm(refflat))
    assert cos >= 0.99999, cos
    gd = G.unpack(g, 2)
    for name, r in ref.items():
        err = np.linalg.norm(gd[name] - r) / max(np.linalg.norm(r), 1e-3 * np.linalg.norm(refflat))
        assert err <= 2e-3, (name, err)
    # a backward after another forward of the same batch is refused
    coeffs = GCIN.apply(P, batch, 2, capi.GCIN_FP32)
    batch.forward(P.detach(), 2, capi.GCIN_FP32)
    with pytest.raises(RuntimeError):
        coeffs.sum().backward()


def _batch_meshes(k=3, seed=3):
    from paper_2606_19251_amd.solver import DeviceSolver, HostHierarchy

    meshes = W.training_batch(k, seed=seed, lo=2000, hi=5000)
    return [DeviceSolver(HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=100), 0) for A, _ in meshes], \
        [torch.from_numpy(f).cuda() for _, f in meshes]


def test_autograd_step_equals_direct_library_calls():
    """The batched training step through GCIN / VCycleLoss gives bitwise the gradient of the direct
    calls (forward, block adjoint, cast with 1/|batch|, GCIN backward)."""
    from paper_2606_19251_amd import capi
    from paper_2606_19251_amd import gcin as G

    solvers, rhs = _batch_meshes()
    dev = torch.device("cuda", 0)
    pred = G.Predictor(G.init_flat(3, 1), dev, 3, capi.GCIN_BF16X3)
    tr = G.Trainer(solvers, rhs, pred, lr=0.0)  # lr 0: the step leaves the parameters unchanged
    tr.step()
    torch.cuda.synchronize()
    # the direct calls on the same state
    tr.loss_and_grad()
    g_direct = tr.batch.backward(pred.params, tr.dc32, 3, capi.GCIN_BF16X3).cpu().numpy()
    P = pred.params.detach().requires_grad_()
    from paper_2606_19251_amd.autograd import GCIN, VCycleLoss

    coeffs = GCIN.apply(P, tr.batch, 3, capi.GCIN_BF16X3)
    losses = VCycleLoss.apply(coeffs, tr.bsolver, tr.f_cat, (1, 1), 32, 1)
    torch.autograd.backward(losses, grad_tensors=tr.wmean)
    g_auto = P.grad.cpu().numpy()
    assert np.array_equal(g_auto.view(np.uint32), g_direct.view(np.uint32))
    assert np.array_equal(losses.detach().cpu().numpy(), tr.losses.cpu().numpy())


def test_validation_metric_matches_oracle():
    """Eq. 13 formed on the device (mean over held-out meshes of the learned minus the Jacobi loss
    after nvc cycles, FP64 cycles here) against the oracle's metric mesh by mesh."""
    from paper_2606_19251_amd import gcin as G
    from paper_2606_19251_amd.train import Validator

    solvers, rhs = _batch_meshes(2, seed=5)
    dev = torch.device("cuda", 0)
    flat = G.init_flat(2, 3)
    rng = np.random.default_rng(9)
    flat[-5:] = np.array([0.55, 0.02, -0.002, 0.1, 0.01], np.float32)  # mlp2 bias: away from Jacobi
    pred = G.Predictor(flat, dev, 2)
    v = Validator(solvers, rhs, pred, (1, 1), 2, cycle_precision=64)
    got = v()
    coeffs = v.tr.batch.forward(pred.params, 2, pred.precision).cpu().numpy().astype(np.float64)
    ref = []
    row = 0
    for ds, f in zip(solvers, rhs):
        hh = ds.hier
        A = W.CSRMatrix(hh.levels[0].rowptr, hh.levels[0].col, hh.levels[0].val, ds.n, ds.n)
        An, fn, sing = amg.normalize(A, f.cpu().numpy())
        ho = amg.setup(An, max_coarse=100, singular=sing)
        ref.append(grad.validation_metric(ho, coeffs[row:row + ds.nlevels], 2, fn, ncycles=2))
        row += ds.nlevels
    print(f"[gpu] validation metric {got:.6f}, oracle {np.mean(ref):.6f} ({ref})", flush=True)
    assert abs(got - float(np.mean(ref))) <= 1e-9 * max(1.0, abs(float(np.mean(ref))))


def _args(**kw):
    a = dict(degree=2, hidden=64, batch=3, lr=0.05, nu=1, nvc=1, plateau_patience=1, plateau_factor=0.5,
             min_lr=1e-5, steps=12, val_every=1)
    a.update(kw)
    return argparse.Namespace(**a)


def test_training_run_schedule_best_model_and_ensemble(tmp_path):
    from paper_2606_19251_amd import gcin as G
    from paper_2606_19251_amd import train as T

    dev = torch.device("cuda", 0)
    trn = T.build_problems("delaunay", 100, 3, dev)
    val = T.build_problems("delaunay", 900, 2, dev)
    args = _args()
    best, flat, hist = T.train_one(args, 0, trn, val, dev)
    vals = [h["val"] for h in hist]
    lrs = [h["lr"] for h in hist]
    # the schedule replayed on the recorded metrics gives the recorded rates; it halved at least once
    s = T.Plateau(args.lr, args.plateau_patience, args.plateau_factor, args.min_lr)
    for v, lr in zip(vals, lrs):
        s.update(v)
        assert s.lr == lr
    assert min(lrs) < args.lr, lrs
    # the returned model is the best one: its metric is the minimum, and re-validating it gives it again
    assert best == min(vals)
    pred = G.Predictor(flat, dev, 2, G.capi.GCIN_BF16X3)
    again = T.Validator(val, T.seeded_rhs(val, T.VAL_RHS_SEED, dev), pred, (1, 1), 1)()
    assert again == best, (again, best)
    # seed ensemble: the saved model is the argmin of the members' best metrics
    out = str(tmp_path / "w.npz")
    T.main(["--out", out, "--steps", "3", "--val-every", "1", "--seeds", "2", "--train-meshes", "3",
            "--val-meshes", "2", "--batch", "3", "--nvc", "1", "--lr", "0.02"])
    z = np.load(out, allow_pickle=False)
    ens = z["ensemble_val"]
    assert ens.shape == (2,)
    val2 = T.build_problems("delaunay", 900, 2, dev)
    pred = G.Predictor(z["params"], dev, 2, G.capi.GCIN_BF16X3)
    again = T.Validator(val2, T.seeded_rhs(val2, T.VAL_RHS_SEED, dev), pred, (1, 1), 1)()
    assert again == ens[T.best_run(ens)], (again, ens)
    for ds in trn + val + val2:
        ds.close()

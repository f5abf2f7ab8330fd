"""Pins of the oracle GCIN predictor and of the oracle loss gradient."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import workloads as W
from oracle import amg, gcin, grad

HERE = os.path.dirname(__file__)


def _golden():
    with open(os.path.join(HERE, "golden", "paper_constants.json")) as fh:
        return json.load(fh)


def test_parameter_count_matches_paper():
    g = _golden()
    assert gcin.param_count(2) == g["gcin_trainable_parameters"]["value"] == 55045
    assert gcin.param_count(3) == 55175
    shapes = dict(gcin.param_shapes(2))
    assert shapes["conv0.W"] == (g["gcin_input_features"]["value"], g["gcin_hidden"]["value"])
    assert shapes["mlp2.W"][1] == g["coefficients_out"]["value"]
    assert shapes["mlp0.W"][1] == g["mlp_hidden"]["value"]
    assert sum(1 for k, _ in gcin.param_shapes(2) if k.startswith("conv") and k.endswith(".W")) == g["gcin_layers"]["value"]


def _torus(N):
    n = N * N
    idx = np.arange(n).reshape(N, N)
    rows, cols = [], []
    for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        rows.append(idx.ravel())
        cols.append(np.roll(np.roll(idx, dy, 0), dx, 1).ravel())
    A = sp.csr_matrix((np.full(4 * n, -1.0), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    A = A + sp.eye(n) * 4.0
    A = sp.csr_matrix(A)
    A.sort_indices()
    return A


def _mats(seed=0):
    A = amg.to_scipy(W.delaunay_p1(W.gmm_points(400, seed)))
    h = amg.setup(A, max_coarse=20)
    return [L.A for L in h.levels]


def test_permutation_invariance():
    p = gcin.init_params(2, 1)
    A = amg.to_scipy(W.delaunay_p1(W.uniform_points(150, 3)))
    perm = np.random.default_rng(0).permutation(A.shape[0])
    Ap = A[perm][:, perm]
    Ap.sort_indices()
    c1 = gcin.forward_np(p, [A])
    c2 = gcin.forward_np(p, [Ap])
    assert np.allclose(c1, c2, rtol=1e-12, atol=1e-12)


def test_batch_independence():
    p = gcin.init_params(2, 2)
    mats = _mats(1) + _mats(2)
    together = gcin.forward_np(p, mats)
    alone = np.concatenate([gcin.forward_np(p, [M]) for M in mats])
    assert np.allclose(together, alone, rtol=1e-12, atol=1e-12)


def test_vertex_transitive_graph_ignores_conv_weights():
    """On a torus every node is alike, so InstanceNorm maps each layer to beta: the output cannot depend on Theta."""
    A = _torus(6)
    p = gcin.init_params(2, 3)
    for l in range(4):
        p[f"norm{l}.beta"] = np.random.default_rng(l).uniform(-0.5, 1.0, 64)
    c1 = gcin.forward_np(p, [A])
    q = dict(p)
    for l in range(4):
        q[f"conv{l}.W"] = p[f"conv{l}.W"] * 3.0 + 0.1
    c2 = gcin.forward_np(q, [A])
    assert np.allclose(c1, c2, rtol=1e-10, atol=1e-10)
    # and changing a norm shift does change it
    q = dict(p)
    q["norm3.beta"] = p["norm3.beta"] + 0.3
    assert not np.allclose(gcin.forward_np(q, [A]), c1)


def test_gcin_gradient_central_fd():
    p = gcin.init_params(2, 4)
    for l in range(4):
        p[f"norm{l}.beta"] = np.random.default_rng(10 + l).uniform(-0.2, 0.4, 64)
    mats = _mats(3)
    w = np.random.default_rng(5).standard_normal((len(mats), 5))
    g = gcin.gradient(p, mats, w)
    rng = np.random.default_rng(6)
    for name in ["conv0.W", "conv2.W", "norm1.gamma", "readout3.W", "ln.gamma", "mlp0.W", "mlp2.b", "conv1.b"]:
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in p[name].shape)
            h = 1e-6
            pp = {k: v.copy() for k, v in p.items()}
            pm = {k: v.copy() for k, v in p.items()}
            pp[name][idx] += h
            pm[name][idx] -= h
            fd = (np.sum(gcin.forward_np(pp, mats) * w) - np.sum(gcin.forward_np(pm, mats) * w)) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, g[name][idx])


# ---------------------------------------------------------------------------------------------
# Loss (Eq. 11) and its gradient
# ---------------------------------------------------------------------------------------------


def _small_problem():
    A, f = W.delaunay_p1_problem(700, 7)
    A, f, sing = amg.normalize(A, f)
    h = amg.setup(A, max_coarse=40, singular=sing)
    return h, f


def test_loss_telescopes():
    h, f = _small_problem()
    c = np.tile([0.6, 0.04, -0.01, 0.2, 0.02], (h.nlevels, 1))
    l3 = grad.vcycle_loss(h, c, 2, f, nvc=3)
    Qs = amg.smoothers(h, c, 2)
    u = np.zeros_like(f)
    for _ in range(3):
        u = amg.vcycle(h, Qs, u, f)
    ref = np.log10(np.linalg.norm(f - h.levels[0].A @ u) / np.linalg.norm(f))
    assert abs(l3 - ref) < 1e-12


def test_validation_metric_zero_for_jacobi():
    h, f = _small_problem()
    c = np.tile(amg.jacobi_coeffs(), (h.nlevels, 1))
    assert grad.validation_metric(h, c, 2, f) == 0.0


@pytest.mark.parametrize("degree", [2, 3])
def test_complex_step_matches_central_fd(degree):
    h, f = _small_problem()
    base = [0.6, 0.04, -0.01, 0.0, 0.2, 0.02, 0.0][: degree + 1] + [0.2, 0.02, 0.001][:degree]
    rng = np.random.default_rng(3)
    c = np.array([np.array(base) + 0.01 * rng.standard_normal(2 * degree + 1) for _ in range(h.nlevels)])
    gcs = grad.grad_complex_step(h, c, degree, f)
    gfd = grad.grad_central_fd(h, c, degree, f)
    scale = np.abs(gcs).max()
    assert np.abs(gcs - gfd).max() <= 1e-6 * scale
    assert np.all(gcs[-1] == 0.0)  # the coarsest level has no smoother

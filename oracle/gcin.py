"""Oracle GCIN coefficient predictor in FP64 PyTorch CPU ops (gradient by autograd).

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product.

Architecture (Sec. 3.2, Eqs. 6-10; App. A.1, Tab. 5):
  * graph of a level matrix A: nodes = rows, node features x_i = [a_ii, deg(i)]
    (Eq. 6; deg = number of stored off-diagonal entries), edge weight w_ij = a_ij;
  * 4 GCIN layers (Eqs. 7-8): H = A_hat X with A_hat = (A - D) + I (added
    self-loops, no GCN normalisation), then a linear map Theta_l (+ bias),
    InstanceNorm per graph (biased variance, eps = 1e-5, affine), ReLU;
  * readout (Eq. 9) per layer: [mean_i x_i, max_i x_i] (128 values) followed by
    a Linear(128 -> 32); the four results are concatenated (Eq. 10, 128 values);
  * LayerNorm(128, eps = 1e-5, affine), sigmoid, then the predictive MLP
    Linear(128,128)-ReLU-Linear(128,64)-ReLU-Linear(64, 2d+1) giving the raw
    smoother coefficients (d0..d_d, o1..o_d) of one level.

Reading: the paper's text gives several incompatible sizes for the head. This
one has the 55,045 trainable parameters the paper states (App. A.1) for d = 2
(55,175 for d = 3), an MLP hidden width of 128 (Tab. 5) and the LayerNorm and
sigmoid of App. A.1. The readout uses layers 1..4 (not the raw input layer 0),
which the parameter count requires. Self-loop weight is 1.
"""
from __future__ import annotations

import numpy as np
import torch

HIDDEN = 64
LAYERS = 4
READOUT = 32
EPS = 1e-5


def param_shapes(degree: int = 2, in_dim: int = 2, hidden: int = HIDDEN, layers: int = LAYERS):
    """Ordered (name, shape) list of every trainable tensor."""
    shapes = []
    for l in range(layers):
        shapes.append((f"conv{l}.W", (in_dim if l == 0 else hidden, hidden)))
        shapes.append((f"conv{l}.b", (hidden,)))
        shapes.append((f"norm{l}.gamma", (hidden,)))
        shapes.append((f"norm{l}.beta", (hidden,)))
    for l in range(layers):
        shapes.append((f"readout{l}.W", (2 * hidden, READOUT)))
        shapes.append((f"readout{l}.b", (READOUT,)))
    jk = READOUT * layers
    shapes += [("ln.gamma", (jk,)), ("ln.beta", (jk,)),
               ("mlp0.W", (jk, 128)), ("mlp0.b", (128,)),
               ("mlp1.W", (128, 64)), ("mlp1.b", (64,)),
               ("mlp2.W", (64, 2 * degree + 1)), ("mlp2.b", (2 * degree + 1,))]
    return shapes


def param_count(degree: int = 2, hidden: int = HIDDEN) -> int:
    return int(sum(np.prod(s) for _, s in param_shapes(degree, hidden=hidden)))


def init_params(degree: int = 2, seed: int = 0, hidden: int = HIDDEN) -> dict:
    """Uniform(+-1/sqrt(fan_in)) weights, zero biases, unit/zero norm affines (FP64 numpy)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in param_shapes(degree, hidden=hidden):
        if name.endswith(".W"):
            bound = 1.0 / np.sqrt(shape[0])
            p[name] = rng.uniform(-bound, bound, size=shape)
        elif name.endswith("gamma"):
            p[name] = np.ones(shape)
        else:
            p[name] = np.zeros(shape)
    return p


class GraphBatch:
    """Block-diagonal batch of level graphs (Alg. 1, steps 3-6).

    Built from a list of CSR matrices (anything with rowptr/col/val or scipy CSR).
    """

    def __init__(self, mats):
        rows, cols, vals, feats, gid = [], [], [], [], []
        off = 0
        for g, A in enumerate(mats):
            if hasattr(A, "indptr"):
                rp, ci, va, n = A.indptr, A.indices, A.data, A.shape[0]
            else:
                rp, ci, va, n = A.rowptr, A.col, A.val, A.nrows
            rp = np.asarray(rp, np.int64)
            ci = np.asarray(ci, np.int64)
            va = np.asarray(va, np.float64)
            r = np.repeat(np.arange(n), np.diff(rp))
            isd = ci == r
            diag = np.zeros(n)
            diag[r[isd]] = va[isd]
            deg = np.bincount(r[~isd], minlength=n).astype(np.float64)
            # A_hat = off-diagonal part of A plus unit self-loops (Eq. 8)
            rows.append(np.concatenate([r[~isd], np.arange(n)]) + off)
            cols.append(np.concatenate([ci[~isd], np.arange(n)]) + off)
            vals.append(np.concatenate([va[~isd], np.ones(n)]))
            feats.append(np.stack([diag, deg], axis=1))
            gid.append(np.full(n, g))
            off += n
        self.n = off
        self.ngraphs = len(mats)
        idx = torch.tensor(np.stack([np.concatenate(rows), np.concatenate(cols)]))
        self.Ahat = torch.sparse_coo_tensor(idx, torch.tensor(np.concatenate(vals)), (off, off)).coalesce()
        self.x0 = torch.tensor(np.concatenate(feats))
        self.gid = torch.tensor(np.concatenate(gid))
        self.counts = torch.bincount(self.gid, minlength=self.ngraphs).to(torch.float64)


def _seg_mean(X, gid, G, counts):
    return torch.zeros(G, X.shape[1], dtype=X.dtype).index_add_(0, gid, X) / counts[:, None]


def _seg_max(X, gid, G):
    idx = gid[:, None].expand_as(X)
    return torch.full((G, X.shape[1]), -torch.inf, dtype=X.dtype).scatter_reduce(0, idx, X, "amax", include_self=False)


def forward(params: dict, batch: GraphBatch, degree: int = 2):
    """Coefficients [ngraphs, 2d+1] (torch FP64); ``params`` values may be tensors requiring grad."""
    P = {k: (v if torch.is_tensor(v) else torch.tensor(v)) for k, v in params.items()}
    G = batch.ngraphs
    X = batch.x0
    pooled = []
    for l in range(LAYERS):
        H = torch.sparse.mm(batch.Ahat, X)
        Y = H @ P[f"conv{l}.W"] + P[f"conv{l}.b"]
        mu = _seg_mean(Y, batch.gid, G, batch.counts)
        var = _seg_mean((Y - mu[batch.gid]) ** 2, batch.gid, G, batch.counts)
        Yn = (Y - mu[batch.gid]) / torch.sqrt(var[batch.gid] + EPS)
        X = torch.relu(Yn * P[f"norm{l}.gamma"] + P[f"norm{l}.beta"])
        pool = torch.cat([_seg_mean(X, batch.gid, G, batch.counts), _seg_max(X, batch.gid, G)], dim=1)
        pooled.append(pool @ P[f"readout{l}.W"] + P[f"readout{l}.b"])
    z = torch.cat(pooled, dim=1)
    m = z.mean(dim=1, keepdim=True)
    v = ((z - m) ** 2).mean(dim=1, keepdim=True)
    z = (z - m) / torch.sqrt(v + EPS) * P["ln.gamma"] + P["ln.beta"]
    z = torch.sigmoid(z)
    z = torch.relu(z @ P["mlp0.W"] + P["mlp0.b"])
    z = torch.relu(z @ P["mlp1.W"] + P["mlp1.b"])
    return z @ P["mlp2.W"] + P["mlp2.b"]


def forward_np(params: dict, mats, degree: int = 2) -> np.ndarray:
    with torch.no_grad():
        return forward(params, GraphBatch(mats), degree).numpy()


def gradient(params: dict, mats, dcoeffs: np.ndarray, degree: int = 2) -> dict:
    """d(sum(coeffs * dcoeffs))/d(params) by FP64 autograd: the vector-Jacobian product of the predictor."""
    T = {k: torch.tensor(v, requires_grad=True) for k, v in params.items()}
    out = forward(T, GraphBatch(mats), degree)
    (out * torch.tensor(dcoeffs)).sum().backward()
    return {k: t.grad.numpy() for k, t in T.items()}

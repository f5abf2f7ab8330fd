"""GCIN forward and backward against the FP64 oracle on graphs that span several reduction chunks.

The per-graph reductions of the network (InstanceNorm statistics, mean/max pooling and their
backward; Sec. 3.2, Eqs. 8-10) run in two stages on the GPU: per chunk of at most 256 tiles
of 64 nodes (16,384 nodes), then per graph over its chunks. The batch here holds a small
graph first (so the large ones start on a nonzero tile), a clustered P1 Delaunay mesh of
45,000 nodes with its whole RS hierarchy (fine level: 704 tiles = chunks of 256, 256 and 192;
first coarse level two chunks, the second partial), and a 200 x 200 structured grid (625 tiles:
256, 256, 113). Every output coefficient and every parameter gradient is compared with the
oracle at the tolerances of the single-chunk tests, for both hidden widths.
"""
import numpy as np
import pytest

import workloads as W
from oracle import amg
from oracle import gcin as OG

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_cache = {}
CHUNK_NODES = 256 * 64


def _mats():
    if "m" not in _cache:
        from paper_2606_19251_amd.solver import HostHierarchy

        small = W.grid5(20)
        big = W.delaunay_p1(W.gmm_points(45000, 11))
        grid = W.grid5(200)
        hb = HostHierarchy.build(big.rowptr, big.col, big.val, max_coarse=100)
        mats = [small] + [W.CSRMatrix(L.rowptr, L.col, L.val, L.n, L.n) for L in hb.levels] + [grid]
        sizes = [m.nrows for m in mats]
        print(f"[gpu] multichunk batch sizes {sizes}", flush=True)
        assert sum(1 for s in sizes if s > 2 * CHUNK_NODES) >= 2  # at least two graphs of >= 3 chunks
        _cache["m"] = mats
    return _cache["m"]


def _batch(hidden):
    from paper_2606_19251_amd.gcin import GraphBatch

    key = ("b", hidden)
    if key not in _cache:
        mats = _mats()
        dev = torch.device("cuda", 0)
        graphs = [tuple(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (m.rowptr, m.col, m.val))
                  for m in mats]
        _cache[key] = (GraphBatch(graphs, dev, hidden), graphs)
    return _cache[key][0]


def _params(seed, degree, hidden):
    from paper_2606_19251_amd import gcin as G

    p = OG.init_params(degree, seed, hidden=hidden)
    rng = np.random.default_rng(seed + 100)
    for l in range(4):
        p[f"norm{l}.beta"] = rng.uniform(-0.3, 0.6, hidden)
        p[f"norm{l}.gamma"] = rng.uniform(0.7, 1.3, hidden)
        p[f"conv{l}.b"] = rng.uniform(-0.1, 0.1, hidden)
    p["ln.gamma"] = rng.uniform(0.8, 1.2, 128)
    p["mlp2.b"] = np.zeros(2 * degree + 1)
    p["mlp2.W"] *= 3.0
    flat = G.pack(p, degree)
    return flat, G.unpack(flat, degree, hidden)


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("hidden,precision,tol", [(64, 0, 1e-4), (64, 1, 2e-2), (64, 2, 1e-3), (32, 0, 1e-4)])
@pytest.mark.parametrize("degree", [2, 3])
def test_forward_multichunk_matches_oracle(hidden, precision, tol, degree):
    flat, p64 = _params(21, degree, hidden)
    batch = _batch(hidden)
    out = batch.forward(torch.from_numpy(flat).cuda(), degree, precision).cpu().numpy()
    ref = OG.forward_np(p64, _mats(), degree)
    assert out.shape == ref.shape
    err = _rel(out, ref)
    print(f"[gpu] multichunk forward hidden {hidden} precision {precision} degree {degree}: {err:.2e}", flush=True)
    assert err <= tol, err
    # element by element, per graph: every coefficient of every graph within the bound
    assert np.all(np.abs(out - ref) <= tol * np.abs(ref).max())


@pytest.mark.parametrize("hidden,precision,tol,cos_min", [(64, 0, 2e-3, 0.99999), (64, 2, 5e-2, 0.999),
                                                          (32, 0, 2e-3, 0.99999)])
def test_backward_multichunk_matches_oracle(hidden, precision, tol, cos_min):
    from paper_2606_19251_amd import gcin as G

    flat, p64 = _params(22, 2, hidden)
    batch = _batch(hidden)
    mats = _mats()
    P = torch.from_numpy(flat).cuda()
    batch.forward(P, 2, precision)
    w = np.random.default_rng(23).standard_normal((len(mats), 5)).astype(np.float32)
    g = batch.backward(P, torch.from_numpy(w).cuda(), 2, precision).cpu().numpy()
    ref = OG.gradient(p64, mats, w.astype(np.float64))
    refflat = G.pack(ref).astype(np.float64)
    cos = g @ refflat / (np.linalg.norm(g) * np.linalg.norm(refflat))
    print(f"[gpu] multichunk backward hidden {hidden} precision {precision}: cosine {cos:.7f}", flush=True)
    assert cos >= cos_min, cos
    gd = G.unpack(g, 2, hidden)
    for name, r in ref.items():
        err = np.linalg.norm(gd[name] - r) / max(np.linalg.norm(r), 1e-3 * np.linalg.norm(refflat))
        assert err <= tol, (name, err)


def test_multichunk_graph_results_independent_of_batch():
    """The 45k-node mesh's coefficients are bitwise the same alone and inside the batch (the chunk
    boundaries are counted from each graph's first tile)."""
    from paper_2606_19251_amd import capi
    from paper_2606_19251_amd.gcin import GraphBatch

    flat, _ = _params(24, 2, 64)
    P = torch.from_numpy(flat).cuda()
    full = _batch(64).forward(P, 2, capi.GCIN_BF16).cpu().numpy()
    graphs = _cache[("b", 64)][1]
    alone = GraphBatch(graphs[1:2], torch.device("cuda", 0)).forward(P, 2, capi.GCIN_BF16).cpu().numpy()
    assert np.array_equal(full[1:2], alone)

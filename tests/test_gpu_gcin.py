"""GCIN predictor on the GPU against the FP64 oracle: forward, backward, Adam, training."""
import numpy as np
import pytest

import workloads as W
from oracle import amg
from oracle import gcin as OG

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_cache = {}


def _solvers():
    if "s" not in _cache:
        from paper_2606_19251_amd.solver import DeviceSolver, HostHierarchy

        out = []
        for seed, npts in [(1, 3000), (2, 5000), (3, 2100)]:
            A = W.delaunay_p1(W.gmm_points(npts, seed))
            hp = HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=40)
            ho = amg.setup(amg.to_scipy(A), max_coarse=40, singular=True)
            out.append((ho, DeviceSolver(hp, 0)))
            print(f"[gpu] gcin mesh seed={seed} levels={hp.nlevels}", flush=True)
        _cache["s"] = out
    return _cache["s"]


def _params(seed, degree=2):
    from paper_2606_19251_amd import gcin as G

    p = OG.init_params(degree, seed)
    rng = np.random.default_rng(seed + 100)
    for l in range(4):
        p[f"norm{l}.beta"] = rng.uniform(-0.3, 0.6, 64)
        p[f"norm{l}.gamma"] = rng.uniform(0.7, 1.3, 64)
        p[f"conv{l}.b"] = rng.uniform(-0.1, 0.1, 64)
    p["ln.gamma"] = rng.uniform(0.8, 1.2, 128)
    p["mlp2.b"] = np.zeros(2 * degree + 1)  # outputs then depend on the whole network, not a bias
    p["mlp2.W"] *= 3.0
    flat = G.pack(p, degree)
    return flat, G.unpack(flat, degree)  # the oracle sees the same FP32-rounded values


def _batch():
    from paper_2606_19251_amd.gcin import GraphBatch

    sol = _solvers()
    graphs, mats = [], []
    for ho, ds in sol:
        graphs += [ds.A[l] for l in range(ds.nlevels)]
        mats += [ho.levels[l].A for l in range(ho.nlevels)]
    return GraphBatch(graphs, torch.device("cuda", 0)), mats


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_tile_product_mfma_matches_fp32():
    """The 64 x 64 tile product on v_mfma_f32_16x16x32_bf16 (A split hi+lo) against FP64."""
    from paper_2606_19251_amd import capi

    rng = np.random.default_rng(0)
    A = (rng.standard_normal((64, 64)) + 30.0).astype(np.float32)  # uncentred, as aggregated features
    B = rng.standard_normal((64, 64)).astype(np.float32)
    D1 = torch.zeros(64, 64, device="cuda")
    D2 = torch.zeros(64, 64, device="cuda")
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()  # kept alive across the launch
    capi.gcin_tile_gemm_check(Ad.data_ptr(), Bd.data_ptr(), D1.data_ptr(), D2.data_ptr(),
                              torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ref = A.astype(np.float64) @ B.astype(np.float64)
    Bb = torch.from_numpy(B).to(torch.bfloat16).to(torch.float64).numpy()
    refb = A.astype(np.float64) @ Bb  # exact A, bf16-rounded B
    assert _rel(D1.cpu().numpy(), ref) <= 1e-6
    # the centred part (what InstanceNorm keeps) is accurate to the bf16 rounding of B only
    d2 = D2.cpu().numpy()
    assert _rel(d2 - d2.mean(0), refb - refb.mean(0)) <= 2e-4


@pytest.mark.parametrize("degree", [2, 3])
def test_forward_fp32_matches_oracle(degree):
    from paper_2606_19251_amd import capi

    flat, p64 = _params(1, degree)
    batch, mats = _batch()
    out = batch.forward(torch.from_numpy(flat).cuda(), degree, capi.GCIN_FP32).cpu().numpy()
    ref = OG.forward_np(p64, mats, degree)
    assert out.shape == ref.shape
    assert _rel(out, ref) <= 1e-4, _rel(out, ref)


def test_forward_bf16_matches_oracle():
    from paper_2606_19251_amd import capi

    flat, p64 = _params(2)
    batch, mats = _batch()
    out = batch.forward(torch.from_numpy(flat).cuda(), 2, capi.GCIN_BF16).cpu().numpy()
    ref = OG.forward_np(p64, mats)
    assert _rel(out, ref) <= 2e-2, _rel(out, ref)
    out32 = batch.forward(torch.from_numpy(flat).cuda(), 2, capi.GCIN_FP32).cpu().numpy()
    print(f"[gpu] forward rel err fp32 {_rel(out32, ref):.2e} bf16 {_rel(out, ref):.2e}", flush=True)


def _banded(n, half):
    """A symmetric M-matrix with 2 half + 1 entries per interior row: 256-row blocks of it hold more
    entries than the graph batch's entry-to-row map, so they are copied row by row."""
    import scipy.sparse as sp

    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    band = (np.abs(i - j) <= half) & (i != j)
    off = np.where(band, -(1.0 + 0.5 * ((i + j) % 7) / 7.0), 0.0)
    A = sp.csr_matrix(off + np.diag(-off.sum(axis=1) + 0.1))
    A.sort_indices()
    return A


@pytest.mark.parametrize("precision,tol", [(0, 1e-4), (1, 2e-2)])
def test_forward_with_row_by_row_copied_blocks_matches_oracle(precision, tol):
    """Graphs whose 256-row blocks exceed the batch copy's entry map (71 entries per row) next to
    ordinary mesh levels: the same coefficients as the oracle's forward."""
    from paper_2606_19251_amd.gcin import GraphBatch

    flat, p64 = _params(9)
    B = _banded(600, 35)
    assert min(B.indptr[256] - B.indptr[0], B.indptr[512] - B.indptr[256]) > 16384  # copied row by row
    ho, ds = _solvers()[2]
    graphs = [tuple(torch.from_numpy(a).cuda() for a in (B.indptr.astype(np.int32), B.indices.astype(np.int32),
                                                         B.data.astype(np.float64)))]
    graphs += [ds.A[l] for l in range(ds.nlevels)]
    mats = [B] + [ho.levels[l].A for l in range(ho.nlevels)]
    out = GraphBatch(graphs, torch.device("cuda", 0)).forward(torch.from_numpy(flat).cuda(), 2, precision)
    ref = OG.forward_np(p64, mats)
    err = _rel(out.cpu().numpy(), ref)
    print(f"[gpu] banded + mesh forward precision {precision}: {err:.2e}", flush=True)
    assert err <= tol, err


def test_forward_batch_independent_bitwise():
    from paper_2606_19251_amd import capi
    from paper_2606_19251_amd.gcin import GraphBatch

    flat, _ = _params(3)
    P = torch.from_numpy(flat).cuda()
    batch, _ = _batch()
    full = batch.forward(P, 2, capi.GCIN_BF16).cpu().numpy()
    ho, ds = _solvers()[1]
    first = _solvers()[0][1].nlevels
    alone = GraphBatch([ds.A[l] for l in range(ds.nlevels)], torch.device("cuda", 0)).forward(P, 2, capi.GCIN_BF16)
    assert np.array_equal(full[first:first + ds.nlevels], alone.cpu().numpy())


@pytest.mark.parametrize("precision,tol,cos_min", [(0, 2e-3, 0.99999), (2, 5e-2, 0.999)])
def test_backward_matches_oracle_autograd(precision, tol, cos_min):
    from paper_2606_19251_amd import gcin as G

    flat, p64 = _params(4)
    batch, mats = _batch()
    P = torch.from_numpy(flat).cuda()
    batch.forward(P, 2, precision)
    w = np.random.default_rng(8).standard_normal((len(mats), 5)).astype(np.float32)
    g = batch.backward(P, torch.from_numpy(w).cuda(), 2, precision).cpu().numpy()
    ref = OG.gradient(p64, mats, w.astype(np.float64))
    refflat = G.pack(ref).astype(np.float64)
    cos = g @ refflat / (np.linalg.norm(g) * np.linalg.norm(refflat))
    assert cos >= cos_min, cos
    gd = G.unpack(g)
    for name, r in ref.items():
        err = np.linalg.norm(gd[name] - r) / max(np.linalg.norm(r), 1e-3 * np.linalg.norm(refflat))
        assert err <= tol, (name, err)


def test_forward_bf16x3_matches_oracle():
    from paper_2606_19251_amd import capi

    flat, p64 = _params(5)
    batch, mats = _batch()
    out = batch.forward(torch.from_numpy(flat).cuda(), 2, capi.GCIN_BF16X3).cpu().numpy()
    ref = OG.forward_np(p64, mats)
    assert _rel(out, ref) <= 1e-3, _rel(out, ref)


def test_backward_bf16_products_match_fp32_products():
    """Plain-BF16 mode: the backward MFMA products against the FP32 backward of the same forward
    state (the BF16 forward's own rounding moves ReLU masks and arg-max choices, so its gradient is
    compared with the gradient of the network it evaluated)."""
    from paper_2606_19251_amd import capi

    flat, _ = _params(6)
    batch, mats = _batch()
    P = torch.from_numpy(flat).cuda()
    w = torch.from_numpy(np.random.default_rng(9).standard_normal((len(mats), 5)).astype(np.float32)).cuda()
    batch.forward(P, 2, capi.GCIN_BF16)
    g_bf = batch.backward(P, w, 2, capi.GCIN_BF16).cpu().numpy()
    g_32 = batch.backward(P, w, 2, capi.GCIN_FP32).cpu().numpy()
    cos = g_bf @ g_32 / (np.linalg.norm(g_bf) * np.linalg.norm(g_32))
    assert cos >= 0.999, cos
    assert np.linalg.norm(g_bf - g_32) <= 5e-2 * np.linalg.norm(g_32)


def test_adam_with_clipping_matches_torch():
    from paper_2606_19251_amd import capi

    rng = np.random.default_rng(0)
    n = 55045
    p0 = rng.standard_normal(n).astype(np.float32)
    grads = [rng.standard_normal(n).astype(np.float32) * s for s in (0.01, 0.5, 0.02)]
    # reference: torch's own Adam and clip_grad_norm_ on the CPU
    ref = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.Adam([ref], lr=1e-3)
    for g in grads:
        ref.grad = torch.from_numpy(g.copy())
        torch.nn.utils.clip_grad_norm_([ref], 1.0)
        opt.step()
    P = torch.from_numpy(p0.copy()).cuda()
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    scratch = torch.empty(capi.adam_scratch_bytes(), dtype=torch.uint8, device="cuda")
    gn = torch.zeros(1, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    for k, g in enumerate(grads):
        G = torch.from_numpy(g).cuda()
        capi.adam_step(P.data_ptr(), G.data_ptr(), m.data_ptr(), v.data_ptr(), n, 1e-3, 0.9, 0.999, 1e-8, k + 1, 1.0,
                       gn.data_ptr(), scratch.data_ptr(), st)
    got = P.cpu().numpy()
    want = ref.detach().numpy()
    assert np.abs(got - want).max() <= 1e-6 * max(1.0, np.abs(want).max()) + 2e-7
    assert abs(gn.item() - np.linalg.norm(grads[-1])) <= 1e-4 * np.linalg.norm(grads[-1])


def test_training_reduces_loss():
    """A few Adam steps of Alg. 1 on three clustered meshes lower the batch-mean one-cycle loss."""
    from paper_2606_19251_amd import gcin as G

    sol = _solvers()
    dev = torch.device("cuda", 0)
    rhs = []
    for ho, ds in sol:
        rhs.append(torch.from_numpy(W.rhs_uniform(ho.levels[0].A.shape[0], 5, zero_mean=True)).to(dev))
    pred = G.Predictor(G.init_flat(2, 0), dev, 2)
    tr = G.Trainer([ds for _, ds in sol], rhs, pred, lr=1e-3)
    tr.loss_and_grad()
    l0 = float(tr.losses.mean())
    for _ in range(30):
        tr.step()
    tr.loss_and_grad()
    l1 = float(tr.losses.mean())
    print(f"[gpu] loss {l0:.4f} -> {l1:.4f}", flush=True)
    assert np.isfinite(l1) and l1 < l0 - 0.02


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_inference_batch_bitwise_equal_and_smaller(precision):
    """An inference-only batch (no aggregates kept, two activation buffers in turn) gives bitwise the
    training batch's coefficients with a fraction of its workspace, and refuses a backward."""
    from paper_2606_19251_amd import capi
    from paper_2606_19251_amd.gcin import GraphBatch

    flat, _ = _params(7)
    P = torch.from_numpy(flat).cuda()
    train, _ = _batch()
    graphs = []
    for _, ds in _solvers():
        graphs += [ds.A[l] for l in range(ds.nlevels)]
    infer = GraphBatch(graphs, torch.device("cuda", 0), inference=True)
    a = train.forward(P, 2, precision).cpu().numpy()
    b = infer.forward(P, 2, precision).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert infer.ws_bytes < 0.45 * train.ws_bytes, (infer.ws_bytes, train.ws_bytes)
    with pytest.raises(capi.AmggError) as e:
        infer.backward(P, torch.zeros(len(graphs), 5, device="cuda"), 2, precision)
    assert e.value.code == capi.AMGG_ESTATE

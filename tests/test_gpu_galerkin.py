"""Device Galerkin product A_c = P^T (A P) (Sec. 2.2) against the oracle, bit for bit.

The oracle forms both sparse products row by row, accumulating each entry over the left
operand's row in ascending column order from 0.0, and drops exact zeros off the diagonal;
the device product must give the same pattern and the same FP64 bits. Cases: integer-valued
operands whose products cancel exactly (the zero-dropping path), interpolation operators of
the RS setup on real meshes, forced row chunking of the symbolic phase, dense hub rows and a
dense cluster, and whole hierarchies built with device products against host-built ones
(themselves bitwise equal to the oracle's on the CPU). Also: the allocator's failure is
reported and leaves nothing allocated.
"""
import os
import sys
import time

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import amg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))


def _bits(a):
    return np.ascontiguousarray(a, np.float64).view(np.uint64)


def _dev(S):
    S = sp.csr_matrix(S)
    S.sort_indices()
    return (torch.from_numpy(S.indptr.astype(np.int32)).cuda(), torch.from_numpy(S.indices.astype(np.int32)).cuda(),
            torch.from_numpy(S.data.astype(np.float64)).cuda())


def _device_galerkin(A, P, chunk=0, allocator=None):
    from paper_2606_19251_amd import capi

    rp, cl, vl = capi.amgg_galerkin_device(0, A.shape[0], P.shape[1], *_dev(A), *_dev(P), chunk_products=chunk,
                                           allocator=allocator)
    return rp.cpu().numpy(), cl.cpu().numpy(), vl.cpu().numpy()


def _assert_same(ref, got, what):
    rp, cl, vl = got
    assert np.array_equal(ref.indptr, rp), what
    assert np.array_equal(ref.indices, cl), what
    assert np.array_equal(_bits(ref.data), _bits(vl)), what


def _integer_operands(n, nc, seed):
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=6.0 / n, random_state=rng, data_rvs=lambda k: rng.integers(-2, 3, k).astype(float))
    A = sp.csr_matrix(M + M.T + sp.diags(np.full(n, 9.0)))
    rows = np.concatenate([np.arange(n), rng.integers(0, n, 2 * n)])
    cols = np.concatenate([rng.integers(0, nc, n), rng.integers(0, nc, 2 * n)])
    P = sp.csr_matrix((rng.choice([-1.0, 1.0, 2.0], rows.size), (rows, cols)), shape=(n, nc))
    P.sum_duplicates()
    return A, P


@pytest.mark.parametrize("seed", [0, 1])
def test_exact_cancellations_are_dropped(seed):
    A, P = _integer_operands(3000, 700, seed)
    ref = amg.galerkin(A, P)
    full = amg.spgemm_rowwise_vec(amg.transpose_exact(P), amg.spgemm_rowwise_vec(A, P))
    assert full.nnz > ref.nnz  # some entries cancel to exactly 0.0 and are dropped
    _assert_same(ref, _device_galerkin(A, P), seed)


def _rs_level(A, max_coarse=50):
    h = amg.setup(A, max_levels=2, max_coarse=max_coarse)
    return h.levels[0].A, h.levels[0].P


@pytest.mark.parametrize("kind", ["delaunay", "cmesh", "tet"])
@pytest.mark.parametrize("chunk", [0, 97, 5000])
def test_interpolation_operators_bitexact(kind, chunk):
    M = {"delaunay": lambda: W.delaunay_p1(W.gmm_points(12000, 5)),
         "cmesh": lambda: W.cmesh_fv(128, 64, "2412", 1e4),
         "tet": lambda: W.tet_fv_mesh(*W.kuhn_tets(14, 2))}[kind]()
    A, P = _rs_level(amg.to_scipy(M))
    _assert_same(amg.galerkin(A, P), _device_galerkin(A, P, chunk), (kind, chunk))


@pytest.mark.parametrize("kind", ["hub", "cluster", "isolated"])
def test_edge_case_hierarchies(kind):
    from test_gpu_edge_cases import make

    from paper_2606_19251_amd.solver import HostHierarchy

    A = make(kind)
    ho = amg.setup(amg.to_scipy(A), max_levels=10, max_coarse=100)
    hd = HostHierarchy.build(A.rowptr, A.col, A.val, max_levels=10, max_coarse=100, galerkin="device")
    assert hd.nlevels == ho.nlevels
    for l in range(1, ho.nlevels):
        L = hd.levels[l]
        _assert_same(ho.levels[l].A, (L.rowptr, L.col, L.val), (kind, l))


def _same_hierarchy(ha, hb):
    assert ha.nlevels == hb.nlevels and ha.singular == hb.singular
    for l, (La, Lb) in enumerate(zip(ha.levels, hb.levels)):
        assert np.array_equal(La.rowptr, Lb.rowptr) and np.array_equal(La.col, Lb.col), l
        assert np.array_equal(_bits(La.val), _bits(Lb.val)), l
        if La.p_rowptr is not None:
            assert np.array_equal(La.p_col, Lb.p_col) and np.array_equal(_bits(La.p_val), _bits(Lb.p_val)), l


def test_grid_hierarchy_with_chunks():
    from paper_2606_19251_amd.solver import HostHierarchy

    A = W.grid5(200)
    hh = HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=50)
    hd = HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=50, galerkin="device", chunk_products=20000)
    _same_hierarchy(hh, hd)


def test_full_size_delaunay_hierarchy():
    """1M-node Delaunay P1 Laplacian (the solve workload): every coarse matrix of the device
    build bitwise equal to the host build's; setup times reported."""
    from paper_2606_19251_amd.solver import HostHierarchy

    A = W.delaunay_p1(W.gmm_points(1_000_000, 0))
    t0 = time.perf_counter()
    hh = HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=500)
    t1 = time.perf_counter()
    hd = HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=500, galerkin="device")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"[gpu] delaunay1m setup: host Galerkin {t1 - t0:.2f} s, device Galerkin {t2 - t1:.2f} s, "
          f"levels {[L.n for L in hd.levels]}", flush=True)
    _same_hierarchy(hh, hd)


class _FailingAllocator:
    def __init__(self, after):
        from paper_2606_19251_amd import capi

        self.base = capi.TorchDeviceAllocator(torch, torch.device("cuda", 0))
        self.after = after
        self.calls = 0
        self.alloc = capi.ALLOC_FN(self._alloc)
        self.release = self.base.release
        self.live = self.base.live

    def _alloc(self, nbytes, user):
        self.calls += 1
        return None if self.calls > self.after else self.base._alloc(nbytes, user)

    def take(self, *a):
        return self.base.take(*a)


@pytest.mark.parametrize("after", [0, 3, 12, 25])
def test_allocation_failure_is_reported_and_releases_everything(after):
    from paper_2606_19251_amd import capi

    A, P = _rs_level(amg.to_scipy(W.grid5(60)))
    al = _FailingAllocator(after)
    with pytest.raises(capi.AmggError) as e:
        _device_galerkin(A, P, allocator=al)
    assert e.value.code == capi.AMGG_EWORKSPACE
    assert not al.live
    _assert_same(amg.galerkin(A, P), _device_galerkin(A, P), "after a failed call")


def test_rejects_bad_arguments():
    from paper_2606_19251_amd import capi

    A, P = _rs_level(amg.to_scipy(W.grid5(20)))
    a, p = _dev(A), _dev(P)
    al = capi.TorchDeviceAllocator(torch, torch.device("cuda", 0))
    # zero sizes, a negative chunk, and P's columns beyond a too small coarse size
    for n, nc, chunk in [(0, P.shape[1], 0), (A.shape[0], 0, 0), (A.shape[0], P.shape[1], -1),
                         (A.shape[0], P.shape[1] - 1, 0)]:
        with pytest.raises(capi.AmggError) as e:
            capi.amgg_galerkin_device(0, n, nc, *a, *p, chunk_products=chunk, allocator=al)
        assert e.value.code == capi.AMGG_EINVAL
    assert not al.live

"""Strength of connection and direct interpolation on the device (amgg_strength_device,
amgg_interp_device) against the oracle, bit for bit, and whole hierarchies whose strength,
interpolation and Galerkin products all run on the GPU (only the C/F split, a sequential greedy,
on the host) against the host setup.

Strength: one flag per stored entry, 1 where the oracle's S_i holds the entry (negative couplings
at least theta times the row's largest; positive couplings weak; rows without a positive largest
coupling empty). Interpolation: from the oracle's own C/F split, P's pattern and FP64 bits equal
to the oracle's direct interpolation (positive couplings lumped on the diagonal). Matrices: P1
Delaunay meshes (positive couplings on obtuse angles), an anisotropic C-mesh, Kuhn tetrahedra and
the hub / cluster / isolated edge cases, on the levels of their RS hierarchies.
"""
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import amg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))


def _bits(a):
    return np.ascontiguousarray(a, np.float64).view(np.uint64)


def _dev(S):
    return (torch.from_numpy(S.indptr.astype(np.int32)).cuda(), torch.from_numpy(S.indices.astype(np.int32)).cuda(),
            torch.from_numpy(S.data.astype(np.float64)).cuda())


def _oracle_flags(A, theta=0.25):
    S = amg.strength(A, theta)
    flags = np.zeros(A.nnz, np.uint8)
    for i in range(A.shape[0]):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        flags[A.indptr[i]:A.indptr[i + 1]] = np.isin(cols, S.indices[S.indptr[i]:S.indptr[i + 1]])
    return S, flags


def _matrix(kind):
    if kind == "delaunay":
        return W.delaunay_p1(W.gmm_points(12000, 5))
    if kind == "cmesh":
        return W.cmesh_fv(128, 64, "2412", 1e4)
    if kind == "tet":
        return W.tet_fv_mesh(*W.kuhn_tets(14, 2))
    from test_gpu_edge_cases import make

    return make(kind)


KINDS = ["delaunay", "cmesh", "tet", "hub", "cluster", "isolated"]


@pytest.mark.parametrize("kind", KINDS)
def test_strength_and_interpolation_bitexact_on_every_level(kind):
    from paper_2606_19251_amd import capi

    M = _matrix(kind)
    An, _, sing = amg.normalize(M, np.zeros(M.nrows))
    ho = amg.setup(An, singular=sing, max_levels=10, max_coarse=100)
    print(f"[gpu] device coarsening {kind}: levels {[L.A.shape[0] for L in ho.levels]}", flush=True)
    for l in range(ho.nlevels - 1):
        A = ho.levels[l].A
        n = A.shape[0]
        S, want = _oracle_flags(A)
        a = _dev(A)
        strong = torch.empty(max(A.nnz, 1), dtype=torch.uint8, device="cuda")
        capi.amgg_strength_device(0, n, *a, 0.25, strong)
        got = strong.cpu().numpy()[:A.nnz]
        assert np.array_equal(got, want), (kind, l)
        cf = (amg.cf_split(S) == amg.CPT).astype(np.int8)
        nc, (rp, cl, vl) = capi.amgg_interp_device(0, n, *a, strong, torch.from_numpy(cf).cuda())
        P = ho.levels[l].P
        assert nc == P.shape[1], (kind, l)
        assert np.array_equal(rp.cpu().numpy(), P.indptr), (kind, l)
        assert np.array_equal(cl.cpu().numpy(), P.indices), (kind, l)
        assert np.array_equal(_bits(vl.cpu().numpy()), _bits(P.data)), (kind, l)


def _same_hierarchy(ha, hb):
    assert ha.nlevels == hb.nlevels and ha.singular == hb.singular
    for l, (La, Lb) in enumerate(zip(ha.levels, hb.levels)):
        assert np.array_equal(La.rowptr, Lb.rowptr) and np.array_equal(La.col, Lb.col), l
        assert np.array_equal(_bits(La.val), _bits(Lb.val)), l
        assert np.array_equal(La.cf, Lb.cf), l
        if La.p_rowptr is not None:
            assert np.array_equal(La.p_rowptr, Lb.p_rowptr), l
            assert np.array_equal(La.p_col, Lb.p_col) and np.array_equal(_bits(La.p_val), _bits(Lb.p_val)), l


@pytest.mark.parametrize("kind", ["grid", "delaunay", "cmesh", "tet", "hub", "isolated"])
def test_device_coarsened_hierarchy_equals_host_setup(kind):
    from paper_2606_19251_amd.solver import HostHierarchy

    M = W.grid5(200) if kind == "grid" else _matrix(kind)
    hh = HostHierarchy.build(M.rowptr, M.col, M.val, max_coarse=50)
    tm = {}
    hd = HostHierarchy.build(M.rowptr, M.col, M.val, max_coarse=50, galerkin="device", coarsen="device", timings=tm)
    print(f"[gpu] {kind}: levels {[L.n for L in hd.levels]}, timings {tm}", flush=True)
    _same_hierarchy(hh, hd)


def test_full_size_delaunay_hierarchy_device_coarsening():
    """The 1M-node Delaunay P1 problem of the benchmark: every level of the device-coarsened build
    bitwise equal to the host build."""
    from paper_2606_19251_amd.solver import HostHierarchy

    A, _ = W.delaunay_p1_problem(1_000_000, 0)
    hh = HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=500)
    tm = {}
    hd = HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=500, galerkin="device", coarsen="device", timings=tm)
    print(f"[gpu] delaunay1m device coarsening: {tm}", flush=True)
    _same_hierarchy(hh, hd)


def test_rejects_bad_arguments():
    from paper_2606_19251_amd import capi

    A = amg.to_scipy(W.grid5(20))
    n = A.shape[0]
    a = _dev(A)
    strong = torch.empty(A.nnz, dtype=torch.uint8, device="cuda")
    for theta in (0.0, 1.0, -0.5):
        with pytest.raises(capi.AmggError) as e:
            capi.amgg_strength_device(0, n, *a, theta, strong)
        assert e.value.code == capi.AMGG_EINVAL
    unsorted = a[1].clone()
    unsorted[[0, 1]] = unsorted[[1, 0]]
    with pytest.raises(capi.AmggError) as e:
        capi.amgg_strength_device(0, n, a[0], unsorted, a[2], 0.25, strong)
    assert e.value.code == capi.AMGG_EINVAL
    capi.amgg_strength_device(0, n, *a, 0.25, strong)
    no_c = torch.zeros(n, dtype=torch.int8, device="cuda")
    with pytest.raises(capi.AmggError) as e:
        capi.amgg_interp_device(0, n, *a, strong, no_c)
    assert e.value.code == capi.AMGG_EINVAL


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


@pytest.mark.parametrize("after", [0, 1, 3, 5])
def test_interpolation_allocation_failure_releases_everything(after):
    from paper_2606_19251_amd import capi

    A = amg.to_scipy(W.grid5(40))
    n = A.shape[0]
    a = _dev(A)
    S, _ = _oracle_flags(A)
    strong = torch.empty(A.nnz, dtype=torch.uint8, device="cuda")
    capi.amgg_strength_device(0, n, *a, 0.25, strong)
    cf = torch.from_numpy((amg.cf_split(S) == amg.CPT).astype(np.int8)).cuda()
    al = _FailingAllocator(after)
    with pytest.raises(capi.AmggError) as e:
        capi.amgg_interp_device(0, n, *a, strong, cf, allocator=al)
    assert e.value.code == capi.AMGG_EWORKSPACE
    assert not al.live
    nc, _ = capi.amgg_interp_device(0, n, *a, strong, cf)
    assert nc == int(cf.sum().item())

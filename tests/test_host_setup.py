"""CPU tests of the product's host side: the library loads and exports its C ABI, the
C++ Ruge-Stueben setup agrees bit for bit with the oracle, argument errors are reported."""
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import amg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _capi():
    from paper_2606_19251_amd import capi
    return capi


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b((?:amgg|gcin|adam)_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    capi = _capi()
    lib = capi.lib()
    names = _declared_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"
        assert name in capi.SIGNATURES or name.startswith(("gcin_", "adam_")), f"{name} has no Python binding"


def _bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint64) if a.dtype == np.float64 else a


def _compare(A, **kw):
    from paper_2606_19251_amd.solver import HostHierarchy

    Ao = amg.to_scipy(A)
    sing = kw.pop("singular", False)
    ho = amg.setup(Ao, singular=sing, **kw)
    hp = HostHierarchy.build(A.rowptr, A.col, A.val, theta=0.25, max_levels=kw.get("max_levels", 10),
                             max_coarse=kw.get("max_coarse", 500))
    assert hp.nlevels == ho.nlevels
    assert hp.singular == sing
    for l in range(ho.nlevels):
        Lo, Lp = ho.levels[l], hp.levels[l]
        assert np.array_equal(Lo.A.indptr, Lp.rowptr)
        assert np.array_equal(Lo.A.indices, Lp.col)
        assert np.array_equal(_bits(Lo.A.data), _bits(Lp.val)), f"A_{l} values differ"
        if l + 1 < ho.nlevels:
            assert np.array_equal(Lo.state, Lp.cf.astype(np.int64)), f"C/F split of level {l} differs"
            assert Lo.P.shape[1] == Lp.p_ncols
            assert np.array_equal(Lo.P.indptr, Lp.p_rowptr)
            assert np.array_equal(Lo.P.indices, Lp.p_col)
            assert np.array_equal(_bits(Lo.P.data), _bits(Lp.p_val)), f"P_{l} values differ"
    return ho, hp


def test_rs_bitexact_grid64_three_levels():
    ho, hp = _compare(W.grid5(64), max_levels=3)
    assert [L.n for L in hp.levels][:2] == [4096, 2048]


def test_rs_bitexact_grid_full_depth():
    _compare(W.grid5(40), max_levels=10, max_coarse=10)


@pytest.mark.parametrize("npts,seed", [(2000, 0), (9000, 3)])
def test_rs_bitexact_delaunay(npts, seed):
    _compare(W.delaunay_p1(W.uniform_points(npts, seed)), singular=True, max_coarse=50)


@pytest.mark.parametrize("seed", [1, 2])
def test_rs_bitexact_gmm_meshes(seed):
    _compare(W.delaunay_p1(W.gmm_points(6000, seed)), singular=True, max_coarse=100)


def test_rs_setup_rejects_bad_pattern():
    capi = _capi()
    A = W.grid5(4)
    col = A.col.copy()
    col[[1, 2]] = col[[2, 1]]  # unsorted row
    with pytest.raises(capi.AmggError) as e:
        capi.amgg_rs_setup(A.rowptr, col, A.val, A.nrows, 0.25, 10, 5)
    assert e.value.code == capi.AMGG_EINVAL
    val = A.val.copy()
    val[A.col == np.repeat(np.arange(16), np.diff(A.rowptr))] *= -1  # negative diagonal
    with pytest.raises(capi.AmggError):
        capi.amgg_rs_setup(A.rowptr, A.col, val, A.nrows, 0.25, 10, 5)
    with pytest.raises(capi.AmggError):
        capi.amgg_rs_setup(A.rowptr, A.col, A.val, A.nrows, 1.5, 10, 5)


def test_create_rejects_bad_level_count():
    capi = _capi()
    with pytest.raises(capi.AmggError) as e:
        capi.amgg_create(0, 0)
    assert e.value.code == capi.AMGG_EINVAL
    with pytest.raises(capi.AmggError):
        capi.amgg_create(0, capi.AMGG_MAX_LEVELS + 1)


def test_one_level_hierarchy_when_small():
    from paper_2606_19251_amd.solver import HostHierarchy

    A = W.grid5(10)
    h = HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=500)
    assert h.nlevels == 1 and h.levels[0].p_rowptr is None


def test_rs_bitexact_airfoil_cmesh():
    _compare(W.cmesh_fv(96, 48, "4415", 1e4), max_coarse=60)


def test_rs_bitexact_kuhn_tetrahedra():
    _compare(W.tet_fv_mesh(*W.kuhn_tets(10, 1)), singular=True, max_coarse=60)


def _levels_equal(ha, hb):
    assert ha.nlevels == hb.nlevels and ha.singular == hb.singular
    for La, Lb in zip(ha.levels, hb.levels):
        assert np.array_equal(La.rowptr, Lb.rowptr) and np.array_equal(La.col, Lb.col)
        assert np.array_equal(_bits(La.val), _bits(Lb.val))
        assert np.array_equal(La.cf, Lb.cf)
        if La.p_rowptr is not None:
            assert np.array_equal(La.p_rowptr, Lb.p_rowptr) and np.array_equal(La.p_col, Lb.p_col)
            assert np.array_equal(_bits(La.p_val), _bits(Lb.p_val))


@pytest.mark.parametrize("source", ["host", "oracle"])
def test_stepwise_setup_equals_one_call_setup(source):
    """amgg_rs_begin / coarsen / galerkin (or push_level of the oracle's Galerkin products)
    gives the hierarchy of amgg_rs_setup bit for bit."""
    from paper_2606_19251_amd.solver import HostHierarchy

    capi = _capi()
    A = W.delaunay_p1(W.gmm_points(5000, 4))
    ref = HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=60)
    ho = amg.setup(amg.to_scipy(A), singular=True, max_coarse=60) if source == "oracle" else None
    h = capi.amgg_rs_begin(A.rowptr, A.col, A.val, A.nrows, 0.25, 10, 60)
    try:
        lvl = 0
        while capi.amgg_rs_coarsen(h):
            if source == "host":
                capi.amgg_rs_galerkin(h)
            else:
                Ac = ho.levels[lvl + 1].A
                capi.amgg_rs_push_level(h, Ac.shape[0], Ac.indptr, Ac.indices, Ac.data)
            lvl += 1
        assert not capi.amgg_rs_coarsen(h)  # stays stopped
        got = HostHierarchy.from_handle(h)
    finally:
        capi.amgg_rs_free(h)
    assert lvl == ref.nlevels - 1
    _levels_equal(ref, got)


def _oracle_strength_flags(A, theta=0.25):
    """One byte per stored entry of A (stored order): 1 where the oracle's S holds the entry."""
    S = amg.strength(A, theta)
    flags = np.zeros(A.nnz, np.uint8)
    for i in range(A.shape[0]):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        flags[A.indptr[i]:A.indptr[i + 1]] = np.isin(cols, S.indices[S.indptr[i]:S.indptr[i + 1]])
    return flags


@pytest.mark.parametrize("kind", ["delaunay", "cmesh"])
def test_split_from_strength_flags_equals_one_call_setup(kind):
    """amgg_rs_split from strength flags, amgg_rs_push_interp and amgg_rs_push_level, all fed
    from the oracle's strength, interpolation and Galerkin products, give the hierarchy of
    amgg_rs_setup bit for bit (the path of the device-built strength and interpolation)."""
    from paper_2606_19251_amd.solver import HostHierarchy

    capi = _capi()
    A = W.delaunay_p1(W.gmm_points(5000, 4)) if kind == "delaunay" else W.cmesh_fv(96, 48, "2412", 1e3)
    ref = HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=60)
    An, _, sing = amg.normalize(A, np.zeros(A.nrows))
    ho = amg.setup(An, singular=sing, max_coarse=60)
    h = capi.amgg_rs_begin(A.rowptr, A.col, A.val, A.nrows, 0.25, 10, 60)
    try:
        lvl = 0
        while capi.amgg_rs_split(h, None, None):
            L = ho.levels[lvl]
            cf = np.empty(L.A.shape[0], np.int8)
            if not capi.amgg_rs_split(h, _oracle_strength_flags(L.A), cf):
                break
            assert np.array_equal(cf, amg.cf_split(amg.strength(L.A, 0.25)) == amg.CPT)
            P = L.P
            capi.amgg_rs_push_interp(h, P.shape[1], P.indptr, P.indices, P.data)
            Ac = ho.levels[lvl + 1].A
            capi.amgg_rs_push_level(h, Ac.shape[0], Ac.indptr, Ac.indices, Ac.data)
            lvl += 1
        assert not capi.amgg_rs_split(h, None, None)  # stays stopped
        got = HostHierarchy.from_handle(h)
    finally:
        capi.amgg_rs_free(h)
    assert lvl == ref.nlevels - 1
    _levels_equal(ref, got)


def test_split_api_rejects_calls_out_of_sequence():
    capi = _capi()
    A = W.grid5(30)
    An = amg.to_scipy(A)
    h = capi.amgg_rs_begin(A.rowptr, A.col, A.val, A.nrows, 0.25, 10, 20)
    try:
        with pytest.raises(capi.AmggError) as e:  # no split yet
            capi.amgg_rs_push_interp(h, 1, np.zeros(A.nrows + 1, np.int32), np.zeros(0, np.int32), np.zeros(0))
        assert e.value.code == capi.AMGG_ESTATE
        assert capi.amgg_rs_split(h, None, None)
        cf = np.empty(A.nrows, np.int8)
        assert capi.amgg_rs_split(h, _oracle_strength_flags(An), cf)
        with pytest.raises(capi.AmggError) as e:  # the split level awaits its P
            capi.amgg_rs_coarsen(h)
        assert e.value.code == capi.AMGG_ESTATE
        S = amg.strength(An, 0.25)
        P = amg.direct_interpolation(An, S, amg.cf_split(S))
        assert np.array_equal(cf, amg.cf_split(S) == amg.CPT)
        with pytest.raises(capi.AmggError) as e:  # wrong column count
            capi.amgg_rs_push_interp(h, P.shape[1] + 1, P.indptr, P.indices, P.data)
        assert e.value.code == capi.AMGG_EINVAL
        bad = P.indices.copy()
        bad[0] = P.shape[1]
        with pytest.raises(capi.AmggError) as e:  # column out of range
            capi.amgg_rs_push_interp(h, P.shape[1], P.indptr, bad, P.data)
        assert e.value.code == capi.AMGG_EINVAL
        capi.amgg_rs_push_interp(h, P.shape[1], P.indptr, P.indices, P.data)
        with pytest.raises(capi.AmggError) as e:  # the coarse matrix is due
            capi.amgg_rs_split(h, None, None)
        assert e.value.code == capi.AMGG_ESTATE
        capi.amgg_rs_galerkin(h)
        assert capi.amgg_rs_info(h)[0] == 2
    finally:
        capi.amgg_rs_free(h)


def test_stepwise_setup_rejects_calls_out_of_sequence():
    capi = _capi()
    A = W.grid5(30)
    h = capi.amgg_rs_begin(A.rowptr, A.col, A.val, A.nrows, 0.25, 10, 20)
    try:
        with pytest.raises(capi.AmggError) as e:
            capi.amgg_rs_galerkin(h)  # nothing to coarsen yet
        assert e.value.code == capi.AMGG_ESTATE
        assert capi.amgg_rs_coarsen(h)
        with pytest.raises(capi.AmggError) as e:
            capi.amgg_rs_coarsen(h)  # the open level needs its coarse matrix first
        assert e.value.code == capi.AMGG_ESTATE
        _, _, nc, _ = capi.amgg_rs_level_size(h, 0)
        B = W.grid5(int(np.sqrt(nc)) + 1)
        with pytest.raises(capi.AmggError) as e:
            capi.amgg_rs_push_level(h, B.nrows, B.rowptr, B.col, B.val)  # wrong size
        assert e.value.code == capi.AMGG_EINVAL
        G = W.grid5(30)
        with pytest.raises(capi.AmggError) as e:
            capi.amgg_rs_push_level(h, G.nrows, G.rowptr, G.col, G.val)
        assert e.value.code == capi.AMGG_EINVAL
        capi.amgg_rs_galerkin(h)
        assert capi.amgg_rs_info(h)[0] == 2
    finally:
        capi.amgg_rs_free(h)


def test_block_diagonal_hierarchy_layout():
    """The batched hierarchy: super level l is the block diagonal of each problem's level
    min(l, L_p - 1); repeated coarsest levels get an identity P and no coefficient row."""
    import scipy.sparse as sp

    from paper_2606_19251_amd.solver import HostHierarchy, block_diagonal

    mats = [W.grid5(30), W.grid5(8), W.delaunay_p1(W.gmm_points(3000, 1))]
    hs = [HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=100) for A in mats]
    depths = [h.nlevels for h in hs]
    assert depths[1] == 1 and max(depths) >= 3
    bh, offsets, rows, sing = block_diagonal(hs)
    assert bh.nlevels == max(depths) and list(sing) == [int(h.singular) for h in hs]
    csr = lambda L: sp.csr_matrix((L.val, L.col, L.rowptr), shape=(L.n, L.n))
    first = np.cumsum([0] + depths)
    for l, L in enumerate(bh.levels):
        ref = sp.block_diag([csr(h.levels[min(l, h.nlevels - 1)]) for h in hs]).tocsr()
        assert (csr(L) != ref).nnz == 0
        assert list(offsets[l]) == list(np.cumsum([0] + [h.levels[min(l, h.nlevels - 1)].n for h in hs]))
        assert list(rows[l]) == [first[p] + l if l + 1 < h.nlevels else -1 for p, h in enumerate(hs)]
        if l + 1 < bh.nlevels:
            P = sp.csr_matrix((L.p_val, L.p_col, L.p_rowptr), shape=(L.n, L.p_ncols))
            parts = []
            for h in hs:
                if l + 1 < h.nlevels:
                    F = h.levels[l]
                    parts.append(sp.csr_matrix((F.p_val, F.p_col, F.p_rowptr), shape=(F.n, F.p_ncols)))
                else:
                    parts.append(sp.identity(h.levels[h.nlevels - 1].n, format="csr"))
            assert (P != sp.block_diag(parts).tocsr()).nnz == 0


def test_query_fill_setup_equals_handle_setup():
    """amgg_rs_setup_query / amgg_rs_setup_fill (the setup into caller-allocated host buffers)
    give the sizes and the arrays of the handle-based setup, bit for bit."""
    from paper_2606_19251_amd.solver import HostHierarchy

    capi = _capi()
    A = W.delaunay_p1(W.gmm_points(4000, 9))
    ref = HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=60)
    z = capi.amgg_rs_setup_query(A.rowptr, A.col, A.val, A.nrows, 0.25, 10, 60)
    assert z.nlevels == ref.nlevels and bool(z.singular) == ref.singular
    levels = []
    for l in range(z.nlevels):
        L = ref.levels[l]
        assert (z.n[l], z.nnz[l]) == (L.n, L.nnz)
        arrs = {"rowptr": np.empty(z.n[l] + 1, np.int32), "col": np.empty(z.nnz[l], np.int32),
                "val": np.empty(z.nnz[l], np.float64), "cf": np.empty(z.n[l], np.int8)}
        if l + 1 < z.nlevels:
            assert (z.p_ncols[l], z.p_nnz[l]) == (L.p_ncols, int(L.p_col.size))
            arrs.update(p_rowptr=np.empty(z.n[l] + 1, np.int32), p_col=np.empty(z.p_nnz[l], np.int32),
                        p_val=np.empty(z.p_nnz[l], np.float64))
        levels.append(arrs)
    capi.amgg_rs_setup_fill(A.rowptr, A.col, A.val, A.nrows, 0.25, 10, 60, levels)
    for l, arrs in enumerate(levels):
        L = ref.levels[l]
        assert np.array_equal(arrs["rowptr"], L.rowptr) and np.array_equal(arrs["col"], L.col)
        assert np.array_equal(_bits(arrs["val"]), _bits(L.val)) and np.array_equal(arrs["cf"], L.cf)
        if l + 1 < z.nlevels:
            assert np.array_equal(arrs["p_rowptr"], L.p_rowptr) and np.array_equal(arrs["p_col"], L.p_col)
            assert np.array_equal(_bits(arrs["p_val"]), _bits(L.p_val))
    levels[0]["col"] = None
    with pytest.raises(capi.AmggError) as e:
        capi.amgg_rs_setup_fill(A.rowptr, A.col, A.val, A.nrows, 0.25, 10, 60, levels)
    assert e.value.code == capi.AMGG_EINVAL

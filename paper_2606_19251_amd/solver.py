"""Plumbing around the C ABI: host hierarchy arrays, device memory held in torch tensors.

PyTorch is used here for device memory and streams only; every arithmetic step of the
setup and of the solve runs in libamggnn (host C++ setup, HIP kernels).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import capi


@dataclass
class HostLevel:
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    p_ncols: int = 0
    p_rowptr: np.ndarray | None = None
    p_col: np.ndarray | None = None
    p_val: np.ndarray | None = None
    cf: np.ndarray | None = None

    @property
    def nnz(self):
        return int(self.col.size)


@dataclass
class HostHierarchy:
    """Ruge-Stueben hierarchy computed by ``amgg_rs_setup`` and copied to numpy arrays."""

    levels: list = field(default_factory=list)
    singular: bool = False

    @classmethod
    def build(cls, rowptr, col, val, theta=0.25, max_levels=10, max_coarse=500, galerkin="host", device=0,
              chunk_products=0, timings=None, coarsen="host"):
        """RS hierarchy of a host CSR matrix. galerkin="host" forms every coarse matrix in the
        host setup; galerkin="device" forms them with amgg_galerkin_device on GPU `device`.
        With galerkin="device", coarsen="device" also forms the strength of connection and the
        interpolation on the GPU (amgg_strength_device, amgg_interp_device); the C/F split, a
        sequential greedy, stays on the host. The results are bitwise the same in every case.
        With galerkin="device", `timings` (a dict) receives the seconds spent in the host
        coarsening (all of it, or the split alone), the device strength and interpolation, the
        device products and the transfers between them."""
        rowptr = np.ascontiguousarray(rowptr, np.int32)
        n = rowptr.size - 1
        if coarsen not in ("host", "device") or (coarsen == "device" and galerkin != "device"):
            raise ValueError(f"coarsen must be 'host' or 'device' (the latter with galerkin='device'), not {coarsen!r}")
        if galerkin == "host":
            h = capi.amgg_rs_setup(rowptr, col, val, n, theta, max_levels, max_coarse)
        elif galerkin == "device":
            h = _rs_with_device_galerkin(rowptr, col, val, n, theta, max_levels, max_coarse, device, chunk_products,
                                         timings if timings is not None else {}, coarsen == "device")
        else:
            raise ValueError(f"galerkin must be 'host' or 'device', not {galerkin!r}")
        try:
            return cls.from_handle(h)
        finally:
            capi.amgg_rs_free(h)

    @classmethod
    def from_handle(cls, h):
        """Copy the levels held by an amgg_rs handle (which stays owned by the caller)."""
        nl, sing = capi.amgg_rs_info(h)
        out = cls([], bool(sing))
        for l in range(nl):
            n_l, nnz, pnc, pnnz = capi.amgg_rs_level_size(h, l)
            L = HostLevel(n_l, np.empty(n_l + 1, np.int32), np.empty(nnz, np.int32), np.empty(nnz, np.float64))
            L.cf = np.empty(n_l, np.int8)
            if l + 1 < nl:
                L.p_ncols = pnc
                L.p_rowptr = np.empty(n_l + 1, np.int32)
                L.p_col = np.empty(pnnz, np.int32)
                L.p_val = np.empty(pnnz, np.float64)
            capi.amgg_rs_copy_level(h, l, L.rowptr, L.col, L.val, L.p_rowptr, L.p_col, L.p_val, L.cf)
            out.levels.append(L)
        return out

    @property
    def nlevels(self):
        return len(self.levels)


def _rs_with_device_galerkin(rowptr, col, val, n, theta, max_levels, max_coarse, device, chunk_products, timings,
                             device_coarsen=False):
    """Stepwise RS setup whose Galerkin products (and, with device_coarsen, strength and
    interpolation) run on the GPU; returns the host handle."""
    import time

    import torch

    dev = torch.device("cuda", device)
    clock = time.perf_counter
    for k in ("coarsen_s", "galerkin_s", "transfer_s") + (("strength_s", "interp_s") if device_coarsen else ()):
        timings.setdefault(k, 0.0)
    h = capi.amgg_rs_begin(rowptr, col, val, n, theta, max_levels, max_coarse)
    try:
        t0 = clock()
        A = (torch.from_numpy(rowptr).to(dev), torch.from_numpy(np.ascontiguousarray(col, np.int32)).to(dev),
             torch.from_numpy(np.ascontiguousarray(val, np.float64)).to(dev))
        timings["transfer_s"] += clock() - t0
        lvl = 0
        while True:
            n_l = int(A[0].numel()) - 1
            if device_coarsen:
                if not capi.amgg_rs_split(h, None, None):
                    break
                t0 = clock()
                strong = torch.empty(max(int(A[1].numel()), 1), dtype=torch.uint8, device=dev)
                capi.amgg_strength_device(device, n_l, *A, theta, strong)
                torch.cuda.synchronize(dev)
                t1 = clock()
                flags = strong.cpu().numpy()
                cf = np.empty(n_l, np.int8)
                t2 = clock()
                more = capi.amgg_rs_split(h, flags, cf)
                t3 = clock()
                timings["strength_s"] += t1 - t0
                timings["transfer_s"] += t2 - t1
                timings["coarsen_s"] += t3 - t2
                if not more:
                    break
                cf_d = torch.from_numpy(cf).to(dev)
                t4 = clock()
                nc, P = capi.amgg_interp_device(device, n_l, *A, strong, cf_d)
                t5 = clock()
                capi.amgg_rs_push_interp(h, nc, *(a.cpu().numpy() for a in P))
                del strong, cf_d
                timings["interp_s"] += t5 - t4
                timings["transfer_s"] += (t4 - t3) + (clock() - t5)
            else:
                t0 = clock()
                more = capi.amgg_rs_coarsen(h)
                timings["coarsen_s"] += clock() - t0
                if not more:
                    break
                t0 = clock()
                _, _, nc, pnnz = capi.amgg_rs_level_size(h, lvl)
                prp, pcl, pvl = np.empty(n_l + 1, np.int32), np.empty(pnnz, np.int32), np.empty(pnnz, np.float64)
                capi.amgg_rs_copy_level(h, lvl, None, None, None, prp, pcl, pvl, None)
                P = tuple(torch.from_numpy(a).to(dev) for a in (prp, pcl, pvl))
                torch.cuda.synchronize(dev)
                timings["transfer_s"] += clock() - t0
            t1 = clock()
            A = capi.amgg_galerkin_device(device, n_l, nc, *A, *P, chunk_products=chunk_products)
            t2 = clock()
            capi.amgg_rs_push_level(h, nc, *(a.cpu().numpy() for a in A))
            timings["galerkin_s"] += t2 - t1
            timings["transfer_s"] += clock() - t2
            lvl += 1
        return h
    except BaseException:
        capi.amgg_rs_free(h)
        raise


def _stream_ptr(torch, device):
    return torch.cuda.current_stream(device).cuda_stream


class DeviceSolver:
    """A finalized solver context on one GPU; owns the device copies and the workspace."""

    def __init__(self, hier: HostHierarchy, device: int = 0, blocks=None):
        """blocks: for a block-diagonal hierarchy, (row offsets per level, coefficient rows per
        level, singular flag per block) as made by block_diagonal()."""
        import torch

        self.torch = torch
        self.hier = hier
        self.device = torch.device("cuda", device)
        self.nlevels = hier.nlevels
        self.n = hier.levels[0].n
        self.singular = bool(hier.singular)
        self.diag_levels = 0  # finest levels set in the diagonal form of Eq. 5 by set_coeffs_device
        self._keep = []
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(self.device)
        self.ctx = capi.amgg_create(device, self.nlevels)
        try:
            self.A = []
            for l, L in enumerate(hier.levels):
                rp, cl, vl = t(L.rowptr), t(L.col), t(L.val)
                self.A.append((rp, cl, vl))
                self._keep += [rp, cl, vl]
                capi.amgg_load_level(self.ctx, l, L.n, L.nnz, rp.data_ptr(), cl.data_ptr(), vl.data_ptr())
                if l + 1 < self.nlevels:
                    pr, pc, pv = t(L.p_rowptr), t(L.p_col), t(L.p_val)
                    self._keep += [pr, pc, pv]
                    capi.amgg_load_prolong(self.ctx, l, L.n, L.p_ncols, int(L.p_col.size), pr.data_ptr(),
                                           pc.data_ptr() if L.p_col.size else 0, pv.data_ptr() if L.p_col.size else 0)
            if blocks is not None:
                offsets, rows, sing = blocks
                for l in range(self.nlevels):
                    capi.amgg_set_level_blocks(self.ctx, l, offsets[l], rows[l],
                                               sing if l == self.nlevels - 1 else None)
            self.ws_bytes = capi.amgg_workspace_bytes(self.ctx)
            raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            off = (-raw.data_ptr()) % 256
            self.ws = raw[off:off + self.ws_bytes]
            self._raw = raw
            capi.amgg_finalize(self.ctx, int(hier.singular), self.ws.data_ptr(), self.ws_bytes, self.stream)
        except Exception:
            capi.amgg_destroy(self.ctx)
            self.ctx = None
            raise

    @property
    def stream(self):
        return _stream_ptr(self.torch, self.device)

    def set_fusion(self, enable: bool):
        capi.amgg_set_fusion(self.ctx, enable)

    def set_packed_columns(self, mode: int):
        """0: plain columns; 1: packed for matrices of >= 2^24 entries (default); 2: packed wherever built."""
        capi.amgg_set_packed_columns(self.ctx, mode)

    def close(self):
        if self.ctx:
            capi.amgg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- smoother
    def set_coeffs(self, coeffs, degree=2, levels=None):
        coeffs = np.asarray(coeffs, np.float64)
        if coeffs.ndim == 1:
            coeffs = np.tile(coeffs, (self.nlevels, 1))
        for l in (range(self.nlevels) if levels is None else levels):
            capi.amgg_set_smoother_coeffs(self.ctx, l, degree, coeffs[l], self.stream)

    def set_coeffs_device(self, coeffs_dev, degree, stream=None, diag_levels=None):
        """coeffs_dev: float32 CUDA tensor [nlevels, 2*degree+1]; queued on `stream` (a raw
        hipStream_t, default: the solver's stream). The `diag_levels` finest levels (default: the
        solver's diag_levels attribute, 0) take the diagonal form of Eq. 5 (f_o = 0)."""
        assert coeffs_dev.dtype == self.torch.float32 and coeffs_dev.is_contiguous()
        stride = coeffs_dev.shape[1] * 4
        st = self.stream if stream is None else stream
        k = self.diag_levels if diag_levels is None else diag_levels
        for l in range(self.nlevels):
            capi.amgg_set_smoother_coeffs_device_form(self.ctx, l, degree, coeffs_dev.data_ptr() + l * stride, l < k, st)

    def set_jacobi(self, omega=2.0 / 3.0):
        for l in range(self.nlevels):
            capi.amgg_set_smoother_jacobi(self.ctx, l, omega, self.stream)

    # ---------------------------------------------------------------- solve phase
    def vcycle(self, f, u, nu1=1, nu2=1, precision=64):
        capi.amgg_vcycle(self.ctx, nu1, nu2, precision, f.data_ptr(), u.data_ptr(), self.stream)
        return u

    def solve(self, b, x=None, outer=capi.AMGG_OUTER_FCG, precision=32, nu1=1, nu2=1, tol=1e-8, maxit=500,
              fallback=True, history_cap=0, div_factor=0.0, stag_ratio=0.0, stag_window=0, graphs=True):
        if x is None:
            x = self.torch.empty_like(b)
        o = capi.amgg_solve_opts(outer, precision, nu1, nu2, maxit, tol, int(fallback), div_factor, stag_ratio,
                                 stag_window, int(graphs))
        rc, info, hist = capi.amgg_solve(self.ctx, o, b.data_ptr(), x.data_ptr(), history_cap, self.stream)
        return x, rc, info, hist[: max(0, min(history_cap, info.iterations + 1))]

    def judge(self, b, coeffs_dev, degree, x=None, diag_levels=None, outer=capi.AMGG_OUTER_FCG, precision=32,
              nu1=1, nu2=1, tol=1e-8, iters=12, graphs=True):
        """amgg_judge_smoother: keeps the learned coefficients (float32 CUDA tensor [nlevels, 2d+1]) or
        omega-Jacobi, whichever predicts the shorter solve of b; returns the judge's record as a dict."""
        assert coeffs_dev.dtype == self.torch.float32 and coeffs_dev.is_contiguous()
        if x is None:
            x = self.torch.empty_like(b)
        k = self.diag_levels if diag_levels is None else diag_levels
        o = capi.amgg_solve_opts(outer, precision, nu1, nu2, iters, tol, 0, 0.0, 0.0, 0, int(graphs))
        j = capi.amgg_judge_smoother(self.ctx, o, iters, degree, coeffs_dev.data_ptr(), k, b.data_ptr(), x.data_ptr(),
                                     self.stream)
        pair = lambda a: [a[0], a[1]]
        return {"learned_wins": bool(j.learned_wins), "iterations": pair(j.iterations), "status": pair(j.status),
                "log10_relres": pair(j.log10_relres), "log10_rate": pair(j.log10_rate),
                "ms_per_iter": pair(j.ms_per_iter), "predicted_ms": pair(j.predicted_ms)}

    # ---------------------------------------------------------------- inspection
    def _ws_slice(self, ptr, count, dtype):
        torch = self.torch
        if not ptr:
            return None
        off = ptr - self.ws.data_ptr()
        itemsize = torch.empty((), dtype=dtype).element_size()
        return self.ws[off:off + count * itemsize].view(dtype)

    def level_view(self, lvl):
        torch = self.torch
        v = capi.amgg_level_view_get(self.ctx, lvl)
        s = self._ws_slice
        return {
            "r_rowptr": s(v.r_rowptr, v.n_coarse + 1, torch.int32) if v.r_rowptr else None,
            "r_col": s(v.r_col, v.p_nnz, torch.int32),
            "r_val": s(v.r_val, v.p_nnz, torch.float64),
            "a_val32": s(v.a_val32, v.nnz, torch.float32),
            "p_val32": s(v.p_val32, v.p_nnz, torch.float32),
            "r_val32": s(v.r_val32, v.p_nnz, torch.float32),
            "q_val": s(v.q_val, v.nnz, torch.float64),
            "q_val32": s(v.q_val32, v.nnz, torch.float32),
            "diag": s(v.diag, v.n, torch.float64),
            "scale": s(v.scale, 1, torch.float64),
            "coarse_inv": s(v.coarse_inv, v.n * v.n, torch.float64),
            "fused_rows": int(v.fused_rows),
            "pack_rows": [int(x) for x in v.pack_rows],  # A (and Q), P, R; 0 = plain columns
            "pack_far": [int(x) for x in v.pack_far],
            "stream_cap": [int(x) for x in v.stream_cap],  # LDS products per workgroup: A, P, R
        }


# ------------------------------------------------------------------------------------------
# Block-diagonal (batched) hierarchies
# ------------------------------------------------------------------------------------------
def block_diagonal(hiers):
    """One block-diagonal hierarchy holding several problems' hierarchies.

    Super level l holds, for each problem p (block p), its level min(l, L_p - 1): a problem
    with fewer levels repeats its coarsest matrix, with the identity as P and no smoother
    there, so that a V-cycle passes its residual down unchanged to the coarsest super level,
    whose block solve is the problem's own coarsest solve. Returns (HostHierarchy, offsets,
    coeff_rows, singular): per level the blocks' row offsets and coefficient rows, where the
    coefficient row of (p, l) is p's level-l graph in the order of all problems' levels
    (problem-major), or -1 for repeated and coarsest levels."""
    depth = max(h.nlevels for h in hiers)
    first = np.cumsum([0] + [h.nlevels for h in hiers])[:-1]
    levels, offsets, rows = [], [], []
    for l in range(depth):
        mats = [h.levels[min(l, h.nlevels - 1)] for h in hiers]
        off = np.cumsum([0] + [m.n for m in mats]).astype(np.int32)
        nnz = np.cumsum([0] + [m.nnz for m in mats])
        rowptr = np.concatenate([m.rowptr[:-1].astype(np.int64) + nnz[b] for b, m in enumerate(mats)] + [[nnz[-1]]])
        col = np.concatenate([m.col.astype(np.int64) + off[b] for b, m in enumerate(mats)])
        val = np.concatenate([m.val for m in mats])
        L = HostLevel(int(off[-1]), rowptr.astype(np.int32), col.astype(np.int32), val.astype(np.float64))
        if l + 1 < depth:
            cmats = [h.levels[min(l + 1, h.nlevels - 1)] for h in hiers]
            coff = np.cumsum([0] + [m.n for m in cmats])
            prp, pcl, pvl = [], [], []
            pnnz = 0
            for b, h in enumerate(hiers):
                if l + 1 < h.nlevels:
                    F = h.levels[l]
                    r, c, v = F.p_rowptr.astype(np.int64), F.p_col.astype(np.int64), F.p_val
                else:  # identity on the repeated coarsest level
                    k = mats[b].n
                    r, c, v = np.arange(k + 1, dtype=np.int64), np.arange(k, dtype=np.int64), np.ones(k)
                prp.append(r[:-1] + pnnz)
                pcl.append(c + coff[b])
                pvl.append(v)
                pnnz += int(r[-1])
            L.p_ncols = int(coff[-1])
            L.p_rowptr = np.concatenate(prp + [[pnnz]]).astype(np.int32)
            L.p_col = np.concatenate(pcl).astype(np.int32)
            L.p_val = np.concatenate(pvl).astype(np.float64)
        levels.append(L)
        offsets.append(off)
        rows.append(np.array([first[b] + l if l + 1 < h.nlevels else -1 for b, h in enumerate(hiers)], np.int32))
    sing = np.array([int(h.singular) for h in hiers], np.int32)
    return HostHierarchy(levels, False), offsets, rows, sing


class BatchSolver:
    """Several problems' hierarchies in one block-diagonal context on one GPU: one launch per
    level operation serves every problem of the batch."""

    def __init__(self, hiers, device: int = 0):
        self.hiers = list(hiers)
        bh, self.offsets, self.rows, self.sing = block_diagonal(self.hiers)
        self.ds = DeviceSolver(bh, device, blocks=(self.offsets, self.rows, self.sing))
        self.nblk = len(self.hiers)
        self.ngraphs = int(sum(h.nlevels for h in self.hiers))
        self.depth = bh.nlevels
        self.diag_levels = 0  # finest super levels set in the diagonal form of Eq. 5
        # problem owning each coefficient row (row = level graph, problem-major), for the chain rule
        owner = np.repeat(np.arange(self.nblk, dtype=np.int32), [h.nlevels for h in self.hiers])
        self.row_problem = self.ds.torch.from_numpy(owner).to(self.ds.device)

    @property
    def ctx(self):
        return self.ds.ctx

    def set_coeffs_device(self, coeffs_dev, degree, stream=None, diag_levels=None):
        """coeffs_dev: float32 CUDA tensor [ngraphs, 2*degree+1], one row per level graph of
        every problem (problem-major), as the batched GCIN forward returns them. Super level l
        holds level l of every problem deep enough, so the `diag_levels` finest super levels
        are each problem's finest levels (diagonal form of Eq. 5 there)."""
        assert coeffs_dev.dtype == self.ds.torch.float32 and coeffs_dev.is_contiguous()
        assert coeffs_dev.shape[0] == self.ngraphs
        st = self.ds.stream if stream is None else stream
        k = self.diag_levels if diag_levels is None else diag_levels
        for l in range(self.depth - 1):
            capi.amgg_set_smoother_coeffs_blocks_form(self.ctx, l, degree, coeffs_dev.data_ptr(), coeffs_dev.shape[1],
                                                      l < k, st)

    def loss_adjoint(self, f_cat, losses, dcoeffs, nu=(1, 1), precision=32, nvc=1, stream=None):
        """Per-problem losses [nblk] and coefficient gradients [ngraphs, 2*degree+1] (FP64)."""
        st = self.ds.stream if stream is None else stream
        capi.amgg_vcycle_loss_adjoint_blocks(self.ctx, nu[0], nu[1], precision, nvc, f_cat.data_ptr(), 0,
                                             losses.data_ptr(), dcoeffs.data_ptr(), self.ngraphs, st)

    def close(self):
        self.ds.close()

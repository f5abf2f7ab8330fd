"""Element-by-element check of the FP32 level operators of the cycle (the timed path).

Each operator's FP32 result is compared, row by row, with the same operator evaluated in FP64
on the FP32 operands the kernel sees (the correctly rounded FP32 copies of A, Q, R = P^T, P and
the FP32 input vectors). A sum of m rounded FP32 products and additions differs from its exact
value by at most gamma_m = m u / (1 - m u) times the sum of the magnitudes of its terms
(u = 2^-24, any summation order), which gives the per-row bound used here:
    |y_i - y_ref_i| <= (nnz_i + 4) u (|c_i| + sum_j |m_ij x_j|)
with c_i the row's additive term (f_i, y_i or x_i) and m_ij the operator's entries. A wrong
index, a dropped or doubled entry, or an FP16-sized rounding fails it on some row.
"""
import numpy as np
import scipy.sparse as sp

U32 = 2.0 ** -24


def _f32(a):
    return np.asarray(a, np.float32)


def _up(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _check(y, ref, bound, what):
    err = np.abs(y.astype(np.float64) - ref)
    worst = int(np.argmax(err / np.maximum(bound, 1e-300)))
    ok = np.all(err <= bound)
    assert ok, (what, worst, float(err[worst]), float(bound[worst]))
    return float(np.max(err / np.maximum(bound, 1e-300)))


def check_level(torch, capi, ds, A64, P64, Q64, lvl, seed):
    """A64: level matrix (scipy CSR, FP64), P64: prolongation (or None on the coarsest level),
    Q64: the smoother values set on the level (scipy CSR on A's pattern, FP64). Returns the
    largest error / bound ratio over the operators."""
    rng = np.random.default_rng(seed)
    n = A64.shape[0]
    A32 = sp.csr_matrix((_up(A64.data), A64.indices, A64.indptr), shape=A64.shape)
    Q32 = sp.csr_matrix((_up(Q64.data), Q64.indices, Q64.indptr), shape=Q64.shape)
    Aabs = abs(A32)
    Qabs = abs(Q32)
    nnz = np.diff(A64.indptr).astype(np.float64)
    x, f, y0 = (_f32(rng.standard_normal(n)) for _ in range(3))
    xu, fu, yu = _up(x), _up(f), _up(y0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()

    def run(op, xin, fin, yin, m):
        xd = dev(xin)
        fd = dev(fin) if fin is not None else xd
        yd = dev(yin) if yin is not None else torch.zeros(m, dtype=torch.float32, device="cuda")
        capi.amgg_level_apply(ds.ctx, lvl, op, 32, xd.data_ptr(), yd.data_ptr(), fd.data_ptr(), ds.stream)
        torch.cuda.synchronize()
        return yd.cpu().numpy()

    worst = 0.0
    # residual y = f - A x
    y = run(capi.AMGG_OP_RESIDUAL, x, f, None, n)
    worst = max(worst, _check(y, fu - A32 @ xu, (nnz + 4) * U32 * (np.abs(fu) + Aabs @ np.abs(xu)), "residual"))
    # smoothing correction y = y + Q x
    y = run(capi.AMGG_OP_SMOOTH, x, None, y0, n)
    worst = max(worst, _check(y, yu + Q32 @ xu, (nnz + 4) * U32 * (np.abs(yu) + Qabs @ np.abs(xu)), "smooth"))
    # one-pass diagonal step y = x + diag(Q) (f - A x)
    d = _up(Q64.diagonal())
    y = run(capi.AMGG_OP_JACOBI, x, f, None, n)
    ref = xu + d * (fu - A32 @ xu)
    bound = (nnz + 6) * U32 * (np.abs(xu) + np.abs(d) * (np.abs(fu) + Aabs @ np.abs(xu)))
    worst = max(worst, _check(y, ref, bound, "jacobi"))
    if P64 is not None:
        nc = P64.shape[1]
        P32 = sp.csr_matrix((_up(P64.data), P64.indices, P64.indptr), shape=P64.shape)
        R32 = P32.T.tocsr()
        pn = np.diff(P64.indptr).astype(np.float64)
        rn = np.diff(R32.indptr).astype(np.float64)
        y = run(capi.AMGG_OP_RESTRICT, x, None, None, nc)
        worst = max(worst, _check(y, R32 @ xu, (rn + 4) * U32 * (abs(R32) @ np.abs(xu)), "restrict"))
        xc = _f32(rng.standard_normal(nc))
        y = run(capi.AMGG_OP_PROLONG, xc, None, y0, n)
        worst = max(worst, _check(y, yu + P32 @ _up(xc), (pn + 4) * U32 * (np.abs(yu) + abs(P32) @ np.abs(_up(xc))),
                                  "prolong"))
    return worst

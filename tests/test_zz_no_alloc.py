"""adam_step_noalloc (the Adam step whose scratch is a static device array) against adam_step
(the same step with a caller-provided scratch buffer), through the C ABI: bitwise equal
parameters, moments and gradient norm on two calls in a row, the second with a smaller vector,
also after a call of the other entry point has left different values in the scratch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _run(capi, fn, p0, g, m0, v0, step, clip, use_scratch):
    P, G, M, V = (torch.from_numpy(a.copy()).cuda() for a in (p0, g, m0, v0))
    gn = torch.full((1,), np.nan, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    if use_scratch:
        scratch = torch.empty(capi.adam_scratch_bytes(), dtype=torch.uint8, device="cuda")
        fn(P.data_ptr(), G.data_ptr(), M.data_ptr(), V.data_ptr(), p0.size, 1e-3, 0.9, 0.999, 1e-8, step, clip,
           gn.data_ptr(), scratch.data_ptr(), st)
    else:
        fn(P.data_ptr(), G.data_ptr(), M.data_ptr(), V.data_ptr(), p0.size, 1e-3, 0.9, 0.999, 1e-8, step, clip,
           gn.data_ptr(), st)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (P, M, V, gn)]


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


@pytest.mark.parametrize("n1,n2", [(55045, 1000), (300000, 37)])
def test_noalloc_adam_matches_adam_step(n1, n2):
    from paper_2606_19251_amd import capi

    rng = np.random.default_rng(n1)
    for k, (n, scale, clip) in enumerate([(n1, 0.5, 1.0), (n2, 0.01, 1.0)]):
        p0 = rng.standard_normal(n).astype(np.float32)
        g = (rng.standard_normal(n) * scale).astype(np.float32)
        m0 = (rng.standard_normal(n) * 1e-2).astype(np.float32)
        v0 = (rng.random(n) * 1e-3).astype(np.float32)
        print(f"[gpu] noalloc adam call {k}: n={n}", flush=True)
        want = _run(capi, capi.adam_step, p0, g, m0, v0, k + 3, clip, True)
        got = _run(capi, capi.adam_step_noalloc, p0, g, m0, v0, k + 3, clip, False)
        for w, x in zip(want, got):
            assert np.array_equal(_bits(w), _bits(x)), (k, n)
        assert np.isfinite(got[3][0]) and abs(got[3][0] - np.linalg.norm(g.astype(np.float64))) <= 1e-4 * got[3][0]


def test_noalloc_adam_rejects_bad_arguments():
    from paper_2606_19251_amd import capi

    P = torch.zeros(8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    with pytest.raises(capi.AmggError) as e:
        capi.adam_step_noalloc(P.data_ptr(), P.data_ptr(), P.data_ptr(), P.data_ptr(), 0, 1e-3, 0.9, 0.999, 1e-8, 1,
                               1.0, 0, st)
    assert e.value.code == capi.AMGG_EINVAL
    with pytest.raises(capi.AmggError):
        capi.adam_step_noalloc(0, P.data_ptr(), P.data_ptr(), P.data_ptr(), 8, 1e-3, 0.9, 0.999, 1e-8, 1, 1.0, 0, st)

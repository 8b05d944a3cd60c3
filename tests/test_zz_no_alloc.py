"""GPU: the allocation-free V-cycle (p3mz_vcycle_noalloc) against the
context V-cycle (p3mz_vcycle) with the same mesh, precision and schedule, on
two calls in a row, the second on a smaller mesh (the fixed scratch array
keeps the first call's contents), in both precisions; and its argument
checks."""
import numpy as np
import pytest

from .gpu_util import GpuCtx, params_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no HIP device")
    return _t


def zero_mean_rhs(n, seed):
    r = np.random.default_rng(seed).standard_normal((n, n, n))
    return r - r.mean()


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_vcycle_equals_context_vcycle(torch, precision):
    from paper_2606_31379_amd import p3maze as P
    stream = torch.cuda.current_stream().cuda_stream
    for n, (nu1, nu2), seed in ((64, (2, 2), 1), (32, (1, 2), 2)):
        gp, _ = params_pair(20.0, 0.3, 8.0, n, 4, precision=precision, nu_pre=nu1, nu_post=nu2)
        g = GpuCtx(gp, np.array([1.0, -1.0]), torch)
        try:
            r = zero_mean_rhs(n, seed)
            e_ctx = g.vcycle(r)
            rr = torch.from_numpy(r).cuda()
            ee = torch.full_like(rr, float("nan"))
            P.p3mz_vcycle_noalloc(n, precision, nu1, nu2, rr.data_ptr(), ee.data_ptr(), stream)
            torch.cuda.synchronize()
            e_na = ee.cpu().numpy()
            assert np.all(np.isfinite(e_na))
            bar = 1e-10 if precision == 0 else 1e-5
            err = np.sqrt(((e_na - e_ctx) ** 2).sum() / (e_ctx ** 2).sum())
            assert err <= bar, (n, err)
            # same kernels, same arithmetic: bitwise equal in practice
            assert np.array_equal(e_na, e_ctx), (n, err)
        finally:
            g.close()


def test_noalloc_vcycle_rejects_bad_arguments(torch):
    from paper_2606_31379_amd import p3maze as P
    rr = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
    for args in ((128, 0, 2, 2), (12, 0, 2, 2), (4, 0, 2, 2), (16, 2, 2, 2), (16, 0, 0, 0), (16, 0, 17, 1)):
        with pytest.raises(P.P3MZError) as ei:
            P.p3mz_vcycle_noalloc(*args, rr.data_ptr(), rr.data_ptr(), None)
        assert ei.value.code == P.P3MZ_ERR_INVALID_ARG
    with pytest.raises(P.P3MZError):
        P.p3mz_vcycle_noalloc(16, 0, 2, 2, None, rr.data_ptr(), None)

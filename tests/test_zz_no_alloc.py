"""nfhmm_fit_device_noalloc (the fit that allocates nothing, its working memory a
fixed device area of the library) against nfhmm_fit_device on the same device
inputs: two calls in a row, the second with a smaller problem, so the second
runs over what the first left in the area.  Both entry points run the same
kernels on the same job in the same order, so every output is compared for
bitwise equality (stricter than the FP32 parity bounds)."""
import numpy as np
import pytest

from gen import make_problem, make_tiny

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_1206_6468_amd import nfhmm
    return nfhmm


@pytest.fixture(scope="module")
def ctx(L):
    c = L.Context(0)
    yield c
    c.close()


def _same(L, ctx, p, precision="fp32"):
    import torch
    ref = L.DeviceJob(p)
    L.fit_device(ctx, ref, precision)
    got = L.DeviceJob(p)
    L.fit_device_noalloc(ctx, got, precision)
    torch.cuda.synchronize()
    for k in ("alpha", "post", "sep", "elbo"):
        a, b = getattr(ref, k).cpu().numpy(), getattr(got, k).cpu().numpy()
        assert np.all(np.isfinite(b)), k
        assert np.array_equal(a, b), (k, float(np.max(np.abs(a.astype(np.float64) - b))))


def test_noalloc_two_calls_second_smaller(L, ctx):
    # the paper-typical job (S=2, N=40, K=10, F=513, T=1000), then a smaller one
    _same(L, ctx, dict(make_problem(1, 3), iters=4))
    _same(L, ctx, dict(make_problem(0, 4), iters=6))


def test_noalloc_warm_start_and_bf16(L, ctx):
    p = make_tiny(S=3, N=4, K=3, F=70, T=150, seed=12, quanta=900, iters=3)
    rng = np.random.default_rng(5)
    _same(L, ctx, dict(p, alpha_init=(1.0 + 10 * rng.random((p["T"], p["M"]))).astype(np.float32)))
    _same(L, ctx, dict(make_problem(0, 5), iters=3), "bf16")


def test_noalloc_rejects_a_job_over_its_area(L, ctx):
    # the long job (S=2, N=60, K=20, F=1025, T=4000) needs far more than the area
    p = make_problem(3, 0)
    j = L.DeviceJob(dict(p, iters=1))
    with pytest.raises(L.NfhmmError) as e:
        L.fit_device_noalloc(ctx, j)
    assert e.value.status == L.E_NOMEM and "working memory" in str(e.value)
    _same(L, ctx, dict(make_problem(0, 6), iters=2))

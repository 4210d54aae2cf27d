"""The serving loop (nfhmm_submit / poll / wait / cancel) on the GPU.

Jobs of different lengths and source counts are submitted while others are
resident; the context's device-memory budget is set so that admission has to
queue.  Each job's result must equal the same job run alone (nfhmm_fit, same
precision) -- bitwise, since every kernel computes a job's values from that
job's data only, in the same order, whatever else shares the launch.
"""
import time

import numpy as np
import pytest

from gen import make_problem, make_tiny

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_1206_6468_amd import nfhmm
    return nfhmm


def _mix():
    return [
        dict(make_problem(0, 20), iters=6),
        dict(make_tiny(S=3, N=4, K=3, F=70, T=150, seed=21, quanta=900), iters=5),
        dict(make_problem(0, 21), iters=3),
        dict(make_tiny(S=1, N=7, K=2, F=33, T=57, seed=22, quanta=500), iters=8),
        dict(make_tiny(S=2, N=5, K=4, F=129, T=300, seed=23, quanta=2000), iters=4),
        dict(make_problem(0, 22), iters=1),
    ]


def _same(a, b):
    for k in ("alpha", "post", "sep", "elbo"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_serving_results_equal_alone(L, precision):
    probs = _mix()
    alone_ctx = L.Context(0)
    alone = [L.fit(alone_ctx, p, precision) for p in probs]
    alone_ctx.close()
    fps = [L.footprint_bytes(p, precision) for p in probs]
    budget = sorted(fps)[-1] + sorted(fps)[-2]          # at most about two resident jobs
    ctx = L.Context(0, hbm_budget_bytes=budget, max_slots=3)
    try:
        subs = [L.submit(ctx, p, precision) for p in probs[:3]]
        # the rest arrive while the first ones are resident
        time.sleep(0.002)
        subs += [L.submit(ctx, p, precision) for p in probs[3:]]
        lat = []
        for s, a in zip(subs, alone):
            out, t = L.wait(ctx, s)
            lat.append(t)
            _same(out, a)
        assert all(t > 0 for t in lat)
    finally:
        ctx.close()


def test_serving_with_outputs_skipped(L):
    """Outputs left NULL are neither computed into nor copied back; the others equal
    those of the same job with every output requested."""
    probs = _mix()[:4]
    ctx = L.Context(0)
    try:
        full = [L.wait(ctx, L.submit(ctx, p, "bf16"))[0] for p in probs]
        for want in (("post", "sep", "elbo"), ("alpha",), ("sep",), ()):
            subs = [L.submit(ctx, p, "bf16", outputs=want) for p in probs]
            for s, f in zip(subs, full):
                out, _ = L.wait(ctx, s)
                assert set(out) == set(want)
                for k in want:
                    assert np.array_equal(out[k], f[k]), (want, k)
    finally:
        ctx.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_outputs_into_pinned_arrays(L, precision):
    """Output arrays in pinned host memory are written by a direct copy instead of
    through the pinned ring; the results are the same bit for bit, in serving and
    in the blocking host-array call."""
    probs = _mix()[:4]
    ctx = L.Context(0)
    try:
        ref = [L.fit(ctx, p, precision) for p in probs]
        pin = [L.fit_batch(ctx, [p], precision, pinned=True)[0] for p in probs]
        for a, b in zip(ref, pin):
            _same(a, b)
        subs = [L.submit(ctx, p, precision, pinned=True) for p in probs]
        for s, a in zip(subs, ref):
            _same(L.wait(ctx, s)[0], a)
        subs = [L.submit(ctx, p, precision, outputs=("sep", "elbo"), pinned=True) for p in probs]
        for s, a in zip(subs, ref):
            out, _ = L.wait(ctx, s)
            assert np.array_equal(out["sep"], a["sep"]) and np.array_equal(out["elbo"], a["elbo"])
    finally:
        ctx.close()


def _pinned_copy(x):
    import torch
    a = np.asarray(x, dtype=np.float32)
    t = torch.empty(a.shape, dtype=torch.float32, pin_memory=True)
    out = t.numpy()
    out[...] = a
    return out


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_inputs_from_pinned_arrays(L, precision):
    """Input arrays in pinned host memory are copied to the device directly, the
    rest through the pinned ring; a blocking host-array call gives the same bits
    whichever way each array went (all pinned, some pinned, a pinned warm start)."""
    probs = _mix()[:4]
    ctx = L.Context(0)
    try:
        ref = [L.fit(ctx, p, precision) for p in probs]
        for p, a in zip(probs, ref):
            allpin = dict(p, **{k: _pinned_copy(p[k]) for k in ("V", "W", "A", "pi")})
            _same(L.fit(ctx, allpin, precision), a)
            some = dict(p, V=_pinned_copy(p["V"]), pi=_pinned_copy(p["pi"]))
            _same(L.fit_batch(ctx, [some], precision, pinned=True)[0], a)
        warm = dict(probs[0], alpha_init=ref[0]["alpha"])
        want = L.fit(ctx, warm, precision)
        got = L.fit(ctx, dict(warm, alpha_init=_pinned_copy(ref[0]["alpha"]),
                              W=_pinned_copy(warm["W"])), precision)
        _same(got, want)
    finally:
        ctx.close()


def test_serving_poll_and_cancel(L):
    ctx = L.Context(0, max_slots=2)
    try:
        long_job = dict(make_problem(0, 30), iters=400)
        short = dict(make_problem(0, 31), iters=2)
        a = L.submit(ctx, long_job, "fp32")
        b = L.submit(ctx, short, "fp32")
        L.cancel(ctx, a)
        st, _, _ = L.wait_status(ctx, a)
        assert st == L.E_CANCELLED
        out, _ = L.wait(ctx, b)
        ref = L.fit(ctx, short, "fp32")
        _same(out, ref)
        c = L.submit(ctx, short, "fp32")
        while not L.poll(ctx, c):
            time.sleep(0.001)
        out, _ = L.wait(ctx, c)
        _same(out, ref)
    finally:
        ctx.close()


def test_serving_rejects_job_over_budget(L):
    p = make_problem(0, 32)
    ctx = L.Context(0, hbm_budget_bytes=L.footprint_bytes(p, "fp32") // 2)
    try:
        with pytest.raises(L.NfhmmError) as e:
            L.submit(ctx, p, "fp32")
        assert e.value.status == L.E_NOMEM
        bad = dict(p, V=p["V"].copy())
        bad["V"][0, 0] = -1.0
        with pytest.raises(L.NfhmmError) as e:
            L.submit(ctx, bad, "fp32")
        assert e.value.status == L.E_INVALID
    finally:
        ctx.close()


def test_host_fits_beside_serving(L):
    # host-array fits and the serving loop share the context's pinned copy ring
    # and its engine: fits made while submitted jobs are queued and resident must
    # still equal the same fits alone, and so must the served jobs
    probs = _mix()
    extra = [dict(make_problem(0, 30), iters=4), dict(make_tiny(S=2, N=6, K=3, F=90, T=200, seed=31,
                                                               quanta=1500), iters=5)]
    alone_ctx = L.Context(0)
    alone = [L.fit(alone_ctx, p, "fp32") for p in probs]
    alone_extra = L.fit_batch(alone_ctx, extra, "fp32")
    alone_ctx.close()
    fps = [L.footprint_bytes(p, "fp32") for p in probs]
    ctx = L.Context(0, hbm_budget_bytes=sorted(fps)[-1] + sorted(fps)[-2], max_slots=3)
    try:
        subs = [L.submit(ctx, p, "fp32") for p in probs]
        got_extra = [L.fit_batch(ctx, extra, "fp32") for _ in range(3)]   # while the jobs run
        for s, a in zip(subs, alone):
            out, _ = L.wait(ctx, s)
            _same(out, a)
        for ge in got_extra:
            for g, a in zip(ge, alone_extra):
                _same(g, a)
    finally:
        ctx.close()

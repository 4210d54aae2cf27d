"""EM learning of a source's N-HMM on the GPU (nfhmm_learn_nhmm and its batch form
through the C ABI) against the FP64 reference of oracle/nhmm_em_oracle.py (the steps derived
from the model of Section 2.1; the reference is pinned in tests/test_nhmm_em_pins.py).

Both start from the same float32 parameters and run the same number of
iterations; every learned parameter and the log-likelihood trace are compared
element by element.  The GPU keeps beta and theta in double between iterations
and keeps the chain's messages as float32 logarithms (A and pi too), each step a
log-sum-exp per lane, treating as zero what underflows a double (subnormals
still count), as the reference does; the differences are the chain's float32 rounding carried through the
updates.  Chains of T >= 98 frames take the time-parallel forward-backward when
the batch is small (one problem always is), the others and every chain of a batch
past 2^19 state-frames the sequential one: both are checked here.  Tolerances: dictionaries
|d beta| <= 1e-5 of their row's largest entry, theta |d| <= 1e-6, A |d| <= 2e-5,
pi |d| <= 1e-5, ln P(V) 1e-9 relative (measured at the paper's shapes: 6.4e-7,
9e-9, 2.2e-6, 0, 9e-11).
"""
import numpy as np
import pytest

from gen import make_nhmm_problem
from oracle import nhmm_em_oracle as EM

pytestmark = pytest.mark.gpu

TOL = dict(W=1e-5, theta=1e-6, A=2e-5, pi=1e-5, loglik=1e-9)


@pytest.fixture(scope="module")
def L():
    from paper_1206_6468_amd import nfhmm
    return nfhmm


@pytest.fixture(scope="module")
def ctx(L):
    c = L.Context(0)
    yield c
    c.close()


def _oracle(prob, iters):
    f64 = lambda k: np.asarray(prob[k], np.float64)  # noqa: E731
    V, beta, theta, A, pi = (f64(k) for k in ("V", "W", "theta", "A", "pi"))
    trace = []
    for _ in range(iters):
        beta, theta, A, pi, lnZ = EM.em_step(V, beta, theta, A, pi)
        trace.append(lnZ)
    return dict(W=beta, theta=theta, A=A, pi=pi, loglik=np.array(trace))


def _errs(g, r):
    rowmax = np.max(r["W"], axis=-1, keepdims=True)
    return dict(W=float(np.max(np.abs(g["W"] - r["W"]) / rowmax)),
                theta=float(np.max(np.abs(g["theta"] - r["theta"]))),
                A=float(np.max(np.abs(g["A"] - r["A"]))),
                pi=float(np.max(np.abs(g["pi"] - r["pi"]))),
                loglik=float(np.max(np.abs(g["loglik"] - r["loglik"]) / np.abs(r["loglik"]))))


def _fmt(e):
    return "  ".join(f"{k} {v:.2e}" for k, v in e.items())


@pytest.mark.parametrize("name,over", [
    ("small", dict(N=4, K=3, F=24, T=40, iters=8)),
    ("ragged", dict(N=7, K=5, F=70, T=131, iters=5)),
    ("one-state", dict(N=1, K=6, F=33, T=50, iters=5)),
    ("K-max", dict(N=3, K=32, F=65, T=66, iters=4)),
])
def test_em_matches_oracle(L, ctx, name, over):
    p = make_nhmm_problem(0, 1, **over)
    g = L.learn_nhmm(ctx, p)
    r = _oracle(p, p["iters"])
    e = _errs(g, r)
    print(f"\n{name} x{p['iters']}: {_fmt(e)}")
    for k, tol in TOL.items():
        assert e[k] <= tol, (k, e[k])


def test_em_paper_shape(L, ctx):
    """One speaker's model at the separation's shapes: N = 40 states of K = 10
    elements, F = 513 bins, T = 1000 frames; three iterations."""
    p = make_nhmm_problem(1, 0, iters=3)
    g = L.learn_nhmm(ctx, p)
    r = _oracle(p, 3)
    e = _errs(g, r)
    print(f"\npaper shape x3: {_fmt(e)}")
    for k, tol in TOL.items():
        assert e[k] <= tol, (k, e[k])


def test_em_far_tails_time_parallel(L, ctx):
    """A 200-frame, 10-state chain on which the FP64 reference drives dozens of
    transitions below the float32 range (42 entries of A between 0 and 1e-38 after
    the first iteration, 2 after the eighth; some with subnormal counts, one of
    which comes back to e^-506), the values a later iteration can bring back: the
    GPU keeps them as the reference does, alone (the time-parallel forward-backward)
    and in a batch past 2^19 state-frames (the sequential one)."""
    p = make_nhmm_problem(1, 5, N=10, K=4, F=40, T=200, iters=8)
    r = _oracle(p, 8)
    big = [make_nhmm_problem(1, 60 + i, K=4, F=64, iters=1) for i in range(14)]
    for tag, g in (("time-parallel", L.learn_nhmm(ctx, p)), ("sequential", L.learn_nhmm_batch(ctx, [p] + big)[0])):
        e = _errs(g, r)
        print(f"\nfar tails x8 {tag}: {_fmt(e)}")
        for k, tol in TOL.items():
            assert e[k] <= tol, (tag, k, e[k])


def test_em_sequential_sweeps_past_the_line(L, ctx):
    """Fourteen 1000-frame, 40-state problems (5.6e5 state-frames, past 2^19) take
    the sequential forward-backward in a batch; alone, each takes the time-parallel
    one.  Both match the FP64 reference, and each other, to the parity bar."""
    probs = [make_nhmm_problem(1, 40 + i, K=4, F=64, iters=2) for i in range(14)]
    assert sum(p["N"] * p["T"] for p in probs) > 1 << 19
    batch = L.learn_nhmm_batch(ctx, probs)
    for i in (0, 13):
        alone = L.learn_nhmm(ctx, probs[i])
        r = _oracle(probs[i], 2)
        for tag, g in (("sequential", batch[i]), ("time-parallel", alone)):
            e = _errs(g, r)
            print(f"\nproblem {i} {tag} x2: {_fmt(e)}")
            for k, tol in TOL.items():
                assert e[k] <= tol, (tag, k, e[k])
        e = _errs(batch[i], alone)
        for k, tol in TOL.items():
            assert e[k] <= tol, ("sequential vs time-parallel", k, e[k])


def test_em_likelihood_never_decreases(L, ctx):
    p = make_nhmm_problem(1, 1, N=20, K=8, T=400, iters=25)
    g = L.learn_nhmm(ctx, p)
    tr = g["loglik"]
    print(f"\nln P(V): {tr[0]:.6e} -> {tr[-1]:.6e}")
    assert np.all(np.isfinite(tr))
    assert np.all(np.diff(tr) >= -1e-9 * np.abs(tr[1:]))
    assert tr[-1] > tr[0]
    np.testing.assert_allclose(g["W"].sum(-1), 1.0, atol=2e-6)
    np.testing.assert_allclose(g["theta"].sum(-1), 1.0, atol=2e-6)
    np.testing.assert_allclose(g["A"].sum(-1), 1.0, atol=2e-6)


def test_em_device_path_equals_host_path(L, ctx):
    import torch
    p = make_nhmm_problem(0, 2, N=6, K=4, F=50, T=90, iters=4)
    h = L.learn_nhmm(ctx, p)
    j = L.DeviceNhmm(p)
    L.learn_nhmm_device(ctx, j)
    torch.cuda.synchronize()
    for k, t in (("W", j.W_out), ("theta", j.theta_out), ("A", j.A_out), ("pi", j.pi_out), ("loglik", j.loglik)):
        assert np.array_equal(h[k], t.cpu().numpy()), k


def test_em_rejects_invalid_starts(L, ctx):
    p = make_nhmm_problem(0, 3, N=3, K=2, F=16, T=20, iters=2)
    bad_theta = dict(p, theta=p["theta"].copy())
    bad_theta["theta"][4, 1] = [1.0, 0.0]
    W = p["W"].astype(np.float64).copy()
    W[1, :, 5] = 0.0
    W /= W.sum(-1, keepdims=True)
    V = p["V"].copy()
    V[:, 5] = np.maximum(V[:, 5], 1.0)
    bad_cover = dict(p, W=W.astype(np.float32), V=V)
    for bad, needle in ((bad_theta, "theta"), (bad_cover, "bin 5")):
        with pytest.raises(L.NfhmmError) as e:
            L.learn_nhmm(ctx, bad)
        assert e.value.status == L.E_INVALID and needle in str(e.value)
    assert np.all(np.isfinite(L.learn_nhmm(ctx, p)["loglik"]))


def test_em_batch_equals_alone(L, ctx):
    """A batch of problems that differ in every size and in their iteration counts
    (states 1 to 40, so the chain's register tile spans all four widths; K from 3
    to 32; T = 131 and 300 on the time-parallel forward-backward, the rest on the
    sequential one): each problem's learned parameters and trace equal learning it alone,
    bit for bit, and one problem of the batch matches the FP64 reference."""
    probs = [make_nhmm_problem(0, 11, N=4, K=3, F=24, T=40, iters=8),
             make_nhmm_problem(1, 12, N=40, K=10, T=300, iters=3),
             make_nhmm_problem(0, 13, N=7, K=32, F=70, T=131, iters=5),
             make_nhmm_problem(0, 14, N=1, K=6, F=33, T=50, iters=4),
             make_nhmm_problem(0, 15, N=20, K=5, F=129, T=77, iters=6)]
    batch = L.learn_nhmm_batch(ctx, probs)
    for i, (p, b) in enumerate(zip(probs, batch)):
        a = L.learn_nhmm(ctx, p)
        for k in ("W", "theta", "A", "pi", "loglik"):
            assert np.array_equal(a[k], b[k]), (i, k)
    e = _errs(batch[2], _oracle(probs[2], probs[2]["iters"]))
    print(f"\nbatch problem 2 x{probs[2]['iters']}: {_fmt(e)}")
    for k, tol in TOL.items():
        assert e[k] <= tol, (k, e[k])


def test_em_batch_rejects_a_bad_problem(L, ctx):
    probs = [make_nhmm_problem(0, 16, N=3, K=2, F=16, T=20, iters=2) for _ in range(3)]
    bad = dict(probs[2], theta=probs[2]["theta"].copy())
    bad["theta"][4, 1] = [1.0, 0.0]
    with pytest.raises(L.NfhmmError) as e:
        L.learn_nhmm_batch(ctx, probs[:2] + [bad])
    assert e.value.status == L.E_INVALID and "problem 2" in str(e.value)
    assert all(np.all(np.isfinite(r["loglik"])) for r in L.learn_nhmm_batch(ctx, probs))

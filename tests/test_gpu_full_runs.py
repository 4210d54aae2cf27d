"""Whole runs of the loop (Section 3.2: Eqs. 6-8 and the forward-backward,
iterated) on the GPU against the FP64 oracle, and edge cases of the inputs.

* the paper-typical job (S=2, N=40, K=10, F=513, T=1000) over its 50
  iterations from the default start, in FP32 and with BF16 contraction
  operands; the BF16 run is also compared with the FP32 GPU run, which measures
  the drift the BF16 operands cause over a whole fit;
* a batch whose 24 jobs all end in different rounds (every job that finishes
  makes the engine build new work lists), each job bitwise equal to the same job
  fitted alone;
* a device-path batch in which one job has counts in a bin that no dictionary
  element explains (its bound is minus infinity): that job reports
  NFHMM_E_NONFINITE and the other jobs of the batch are untouched;
* zeros in pi, and a bin that every element leaves at zero with no counts there.

Tolerances of a whole fit.  One step from a given alpha-hat is held to the FP32
contract (1e-5; tests/test_gpu_parity.py).  Over a whole fit the fixed-point map
of Section 3.2 amplifies the per-iteration rounding of the contractions: fed
relative noise eps in c at every iteration, the FP64 oracle's own alpha-hat moves
by about 22 eps after the 50 iterations of the paper-typical job (eps = 1e-6:
2.3e-5; d-hat by 2e-10, V* by 1.5e-6).  The float32 contractions carry about 1e-6
per iteration, so a whole FP32 fit is held to alpha-hat 3e-5 rel, d-hat 3e-5 abs,
V* 1e-5 of max(V, 1) and the bound 1e-6 rel.  With bfloat16 operands (unit
roundoff 2^-8) the same amplification gives a few 1e-2 in alpha-hat: a whole BF16
fit is held to alpha-hat 1.5e-1 rel, d-hat 5e-2 abs, V* 2e-2 and the bound 1e-3
rel (one BF16 step: alpha-hat 2e-2).
"""
import numpy as np
import pytest

from gen import make_problem, make_tiny
from oracle import nfhmm_oracle as O

pytestmark = pytest.mark.gpu

TOL_A, TOL_SEP, TOL_L, TOL_D_FULL = 1e-5, 1e-5, 1e-6, 3e-5
TOL_A_FULL = 3e-5
BF16_TOL = dict(alpha=1.5e-1, post=5e-2, sep=2e-2, elbo=1e-3)


@pytest.fixture(scope="module")
def L():
    from paper_1206_6468_amd import nfhmm
    return nfhmm


@pytest.fixture(scope="module")
def ctx(L):
    c = L.Context(0)
    yield c
    c.close()


def _errs(g, ref, V):
    Vd = np.maximum(np.asarray(V, np.float64)[None], 1.0)
    return dict(alpha=float(np.max(np.abs(g["alpha"] - ref["alpha"]) / ref["alpha"])),
                post=float(np.max(np.abs(g["post"] - ref["post"]))),
                sep=float(np.max(np.abs(g["sep"] - ref["sep"]) / Vd)),
                elbo=float(np.max(np.abs(g["elbo"] - ref["elbo"]) / np.abs(ref["elbo"]))))


def _fmt(e):
    return "  ".join(f"{k} {v:.2e}" for k, v in e.items())


# ------------------------------------------------------------------ paper-typical job, whole fit
@pytest.fixture(scope="module")
def cfg1_run(L, ctx):
    p = make_problem(1, 0)
    ref = O.fit_problem(p)
    g32 = L.fit(ctx, p, "fp32")
    g16 = L.fit(ctx, p, "bf16")
    return p, ref, g32, g16


def test_cfg1_whole_fit_fp32(cfg1_run):
    p, ref, g32, _ = cfg1_run
    e = _errs(g32, ref, p["V"])
    print(f"\ncfg1 x{p['iters']} fp32 vs oracle: {_fmt(e)}")
    assert e["alpha"] < TOL_A_FULL and e["post"] < TOL_D_FULL and e["sep"] < TOL_SEP and e["elbo"] < TOL_L
    tr = g32["elbo"]
    assert np.all(np.diff(tr) >= -2e-7 * np.abs(tr[1:]))


def test_cfg1_whole_fit_bf16(cfg1_run):
    p, ref, g32, g16 = cfg1_run
    e = _errs(g16, ref, p["V"])
    print(f"\ncfg1 x{p['iters']} bf16 vs oracle: {_fmt(e)}")
    f = _errs(g16, dict(g32, alpha=g32["alpha"].astype(np.float64), elbo=g32["elbo"]), p["V"])
    print(f"cfg1 x{p['iters']} bf16 vs fp32 GPU: {_fmt(f)}")
    for k, tol in BF16_TOL.items():
        assert e[k] < tol, (k, e[k])
        assert f[k] < tol, (k, f[k])


# ------------------------------------------------------------------ many finishing rounds in one batch
def test_batch_of_jobs_ending_in_different_rounds(L, ctx):
    rng = np.random.default_rng(2406)
    iters = rng.permutation(np.arange(1, 25))
    probs = [dict(make_tiny(S=2, N=3, K=3, F=37, T=40 + 3 * i, seed=100 + i, quanta=300), iters=int(it))
             for i, it in enumerate(iters)]
    batch = L.fit_batch(ctx, probs)
    for i, p in enumerate(probs):
        alone = L.fit(ctx, p)
        for k in ("alpha", "post", "sep", "elbo"):
            assert np.array_equal(alone[k], batch[i][k]), (i, k)


# ------------------------------------------------------------------ a job whose bound is -inf
def _unexplained_bin(p, l):
    """Every element leaves bin l at zero (rows renormalised), V keeps its counts there."""
    W = p["W"].astype(np.float64).copy()
    W[..., l] = 0.0
    W /= W.sum(-1, keepdims=True)
    V = p["V"].copy()
    V[:, l] = np.maximum(V[:, l], 3.0)
    return dict(p, W=W.astype(np.float32), V=V)


def test_device_batch_nonfinite_job_is_isolated(L, ctx):
    import torch
    good = [make_problem(0, 20), make_problem(0, 21)]
    bad = _unexplained_bin(make_problem(0, 22), 5)
    st, _ = L.validate(bad)
    assert st == L.E_INVALID          # the host check names it; the device path does not run that check
    solo = []
    for p in good:
        j = L.DeviceJob(p)
        L.fit_device(ctx, j)
        solo.append(j)
    jobs = [L.DeviceJob(good[0]), L.DeviceJob(bad), L.DeviceJob(good[1])]
    with pytest.raises(L.NfhmmError) as e:
        L.fit_batch_device(ctx, jobs)
    assert e.value.status == L.E_NONFINITE
    torch.cuda.synchronize()
    assert not np.all(np.isfinite(jobs[1].elbo.cpu().numpy()))
    for a, b in zip(solo, (jobs[0], jobs[2])):
        for k in ("alpha", "post", "sep", "elbo"):
            assert torch.equal(getattr(a, k), getattr(b, k)), k
    # the context keeps working
    g = L.fit(ctx, dict(good[0], iters=2))
    assert np.all(np.isfinite(g["elbo"]))


# ------------------------------------------------------------------ zeros in pi, silent bins
def test_chain_posterior_with_zeros_in_pi(L, ctx):
    rng = np.random.default_rng(77)
    N, T = 24, 500
    A = rng.random((N, N)) + 0.05
    A /= A.sum(1, keepdims=True)
    pi = np.zeros(N)
    pi[[2, 9, 17]] = [0.5, 0.3, 0.2]
    logev = rng.normal(scale=3.0, size=(T, N)).astype(np.float32)
    post, lnZ = L.chain_posterior(ctx, logev, A.astype(np.float32), pi.astype(np.float32))
    d, z = O.forward_backward(logev.astype(np.float64), A.astype(np.float32).astype(np.float64),
                              pi.astype(np.float32).astype(np.float64))
    assert np.all(post[0][pi == 0] == 0.0)
    assert np.max(np.abs(post - d)) < 1e-5
    assert abs(lnZ - z) <= 1e-6 * abs(z) + 1e-4


def test_fit_with_zeros_in_pi(L, ctx):
    p = make_tiny(S=2, N=5, K=4, F=50, T=80, seed=31, quanta=1000)
    pi = np.array([[0.0, 0.6, 0.0, 0.4, 0.0], [0.25, 0.0, 0.75, 0.0, 0.0]], np.float32)
    p = dict(p, pi=pi, iters=6)
    g = L.fit(ctx, p)
    ref = O.fit_problem(p)
    e = _errs(g, ref, p["V"])
    print(f"\nzeros in pi x6: {_fmt(e)}")
    assert e["alpha"] < TOL_A and e["post"] < TOL_D_FULL and e["sep"] < TOL_SEP and e["elbo"] < TOL_L


def test_fit_with_a_bin_no_element_covers(L, ctx):
    """Bins 7 (inside the contraction tiles) and 128 (the tail bin of F = 129) are
    zero in every element and carry no counts: R and V* are 0 there."""
    p = make_problem(0, 23)
    W = p["W"].astype(np.float64).copy()
    W[..., [7, 128]] = 0.0
    W /= W.sum(-1, keepdims=True)
    V = p["V"].copy()
    V[:, [7, 128]] = 0.0
    p = dict(p, W=W.astype(np.float32), V=V, iters=8)
    assert L.validate(p)[0] == L.OK
    g = L.fit(ctx, p)
    ref = O.fit_problem(p)
    e = _errs(g, ref, p["V"])
    print(f"\nuncovered bins x8: {_fmt(e)}")
    assert np.all(g["sep"][:, :, [7, 128]] == 0.0)
    assert e["alpha"] < TOL_A and e["post"] < TOL_D_FULL and e["sep"] < TOL_SEP and e["elbo"] < TOL_L

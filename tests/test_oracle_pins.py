"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check compares the oracle with something other than itself: brute-force
enumeration, an exact integral on tiny inputs, closed forms, textbook special
cases (LDA) or exact invariants.  CPU only.
"""
import numpy as np
import pytest
from scipy.special import digamma

import brute
from gen import make_problem, make_tiny
from oracle import nfhmm_oracle as O


def _rand_chain(rng, N, sparse=True):
    A = rng.random((N, N)) + 0.05
    if sparse and N > 2:
        A[rng.random((N, N)) < 0.35] = 0.0
        A[np.arange(N), np.arange(N)] = 0.5
    A /= A.sum(1, keepdims=True)
    pi = rng.random(N) + 0.1
    if N > 2:
        pi[0] = 0.0
    pi /= pi.sum()
    return A, pi


# ------------------------------------------------------------------ P1
@pytest.mark.parametrize("N,T,seed", [(1, 4, 0), (2, 7, 1), (3, 6, 2), (4, 5, 3), (5, 7, 4), (5, 1, 5)])
def test_P1_forward_backward_vs_enumeration(N, T, seed):
    rng = np.random.default_rng(seed)
    A, pi = _rand_chain(rng, N)
    logev = rng.normal(scale=3.0, size=(T, N))
    d, lnZ = O.forward_backward(logev, A, pi)
    db, lnZb = brute.fb_brute(logev, A, pi)
    assert abs(lnZ - lnZb) < 1e-12 * max(1.0, abs(lnZb))
    np.testing.assert_allclose(d, db, atol=1e-12, rtol=0)


def test_P1_forward_backward_handles_unreachable_states():
    A = np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.0, 0.0, 1.0]])
    pi = np.array([1.0, 0.0, 0.0])
    logev = np.random.default_rng(7).normal(size=(5, 3))
    d, lnZ = O.forward_backward(logev, A, pi)
    db, lnZb = brute.fb_brute(logev, A, pi)
    np.testing.assert_allclose(d, db, atol=1e-12)
    assert abs(lnZ - lnZb) < 1e-12
    assert d[0, 1] == 0.0 and d[0, 2] == 0.0


# ------------------------------------------------------------------ P2
@pytest.mark.parametrize("S,N,T", [(2, 5, 20), (3, 4, 10), (2, 3, 6)])
def test_P2_product_chain_factorises(S, N, T):
    """The N^S joint chain with summed evidence has marginals equal to the
    product of per-source marginals and ln Z equal to the sum (the factored
    q(D) of Section 3.2 is exact given the evidence)."""
    rng = np.random.default_rng(S * 100 + N)
    As, pis = zip(*[_rand_chain(rng, N) for _ in range(S)])
    evs = [rng.normal(scale=2.0, size=(T, N)) for _ in range(S)]
    ds, lnZs = zip(*[O.forward_backward(e, a, p) for e, a, p in zip(evs, As, pis)])
    Aj, pij = brute.product_chain(list(As), list(pis))
    evj = evs[0]
    for e in evs[1:]:
        evj = (evj[:, :, None] + e[:, None, :]).reshape(T, -1)
    if N ** (S * T) <= 200_000:
        dj, lnZj = brute.fb_brute(evj, Aj, pij)
    else:
        dj, lnZj = O.forward_backward(evj, Aj, pij)
    assert abs(lnZj - sum(lnZs)) < 1e-10 * max(1.0, abs(lnZj))
    prod = ds[0]
    for d in ds[1:]:
        prod = (prod[:, :, None] * d[:, None, :]).reshape(T, -1)
    np.testing.assert_allclose(dj, prod, atol=1e-12)


# ------------------------------------------------------------------ P3
def test_P3_explicit_responsibilities():
    p = make_tiny(S=2, N=3, K=2, F=7, T=9, seed=3)
    V, beta, A, pi = O.paper_arrays(p)
    rng = np.random.default_rng(0)
    alpha = 1.0 + rng.gamma(2.0, 3.0, size=(p["T"], p["M"]))
    E = O.expected_log_theta(alpha)
    # the digamma terms themselves
    np.testing.assert_allclose(E, digamma(alpha) - digamma(alpha.sum(1))[:, None], rtol=0, atol=0)
    c, Lam = O.expected_counts(V, beta, E)
    z = brute.zhat_explicit(E, beta)                 # T x F x M
    np.testing.assert_allclose(z.sum(2), 1.0, atol=1e-13)
    c_exp = np.einsum("lt,tlk->tk", V, z)
    np.testing.assert_allclose(c, c_exp, rtol=1e-12, atol=1e-12)
    # kappa of Eq. 7 (log normaliser over k at fixed t, l) equals ln Lambda
    lz = np.log(beta)[None] + digamma(alpha)[:, None, :] - digamma(alpha.sum(1))[:, None, None]
    kappa = np.log(np.exp(lz).sum(2))               # T x F
    np.testing.assert_allclose(np.log(Lam).T, kappa, rtol=1e-12)


# ------------------------------------------------------------------ P4
@pytest.mark.parametrize("seed,gamma", [(0, 1.0), (1, 1.0), (2, 0.5), (3, 2.0)])
def test_P4_closed_form_elbo_equals_direct(seed, gamma):
    S, N, K, F, T = 2, 2, 2, 5, 4
    p = make_tiny(S=S, N=N, K=K, F=F, T=T, seed=seed, quanta=12)
    V, beta, A, pi = O.paper_arrays(p)
    rng = np.random.default_rng(seed)
    B = O.mask_B(S, N, K)
    alpha = 1.0 + rng.gamma(1.5, 2.0, size=(T, S * N * K))     # arbitrary q(theta)
    E_z = rng.normal(scale=1.0, size=(T, S * N * K))           # arbitrary q(Z)
    phi = rng.normal(scale=2.0, size=(S, T, N))                # arbitrary q(D)
    c, Lam = O.expected_counts(V, beta, E_z)
    d = np.empty((S, T, N)); lnZ = np.empty(S)
    for s in range(S):
        d[s], lnZ[s] = O.forward_backward(gamma * phi[s], A[s], pi[s])
    Lc = O.elbo(alpha=alpha, E_z=E_z, Lam=Lam, c=c, d=d, phi=phi, lnZ=lnZ, V=V, B=B,
                gamma=gamma, S=S, N=N, K=K)
    Ld = brute.elbo_direct(alpha, E_z, phi, V, beta, A, pi, gamma, S, N, K)
    assert abs(Lc - Ld) <= 1e-10 * abs(Ld), (Lc, Ld)


# ------------------------------------------------------------------ P5
def _direct_at(alpha, E_z, phi, p, gamma=1.0):
    V, beta, A, pi = O.paper_arrays(p)
    return brute.elbo_direct(alpha, E_z, phi, V, beta, A, pi, gamma, p["S"], p["N"], p["K"])


def test_P5_block_optimality():
    """At each block's fixed point (Eqs. 6, 7, 8) moving that block away lowers
    the directly evaluated bound; the finite-difference gradient in alpha
    vanishes at the Eq. 6 point."""
    p = make_tiny(S=2, N=2, K=2, F=5, T=4, seed=11, quanta=15)
    S, N, K = p["S"], p["N"], p["K"]
    V, beta, A, pi = O.paper_arrays(p)
    B = O.mask_B(S, N, K)
    out = O.fit(V, beta, A, pi, S, N, K, iters=3, keep=True)
    h = out["history"][-1]
    alpha_prev = out["history"][-2]["alpha"]
    # q(theta) block: Eq. 6 point given (E_z = h.E, phi = h.phi)
    a6, Ez, ph = h["alpha"], h["E"], h["phi"]
    base = _direct_at(a6, Ez, ph, p)
    rng = np.random.default_rng(5)
    for _ in range(3):
        jit = a6 * np.exp(rng.normal(scale=0.05, size=a6.shape))
        assert _direct_at(jit, Ez, ph, p) < base
    eps = 1e-5
    for (t, k) in [(0, 0), (1, 3), (3, 7), (2, 5)]:
        ap = a6.copy(); ap[t, k] += eps
        am = a6.copy(); am[t, k] -= eps
        g = (_direct_at(ap, Ez, ph, p) - _direct_at(am, Ez, ph, p)) / (2 * eps)
        assert abs(g) < 1e-6 * max(1.0, abs(base)), g
    # q(Z) and q(D) blocks: Eqs. 7 and 8 are optimal given q(theta) = Dir(alpha_prev)
    E7 = O.expected_log_theta(alpha_prev)
    phi8 = O.state_evidence(E7, B)
    base2 = _direct_at(alpha_prev, E7, phi8, p)
    for _ in range(3):
        assert _direct_at(alpha_prev, E7 + rng.normal(scale=0.1, size=E7.shape), phi8, p) < base2
        assert _direct_at(alpha_prev, E7, phi8 + rng.normal(scale=0.3, size=phi8.shape), p) < base2


# ------------------------------------------------------------------ P6
def _half_step_elbos(p, iters):
    S, N, K = p["S"], p["N"], p["K"]
    g = p.get("gamma", 1.0)
    V, beta, A, pi = O.paper_arrays(p)
    B = O.mask_B(S, N, K)

    def L(alpha, E_z, phi):
        c, Lam = O.expected_counts(V, beta, E_z)
        d = np.empty((S, alpha.shape[0], N)); lnZ = np.empty(S)
        for s in range(S):
            d[s], lnZ[s] = O.forward_backward(g * phi[s], A[s], pi[s])
        return O.elbo(alpha=alpha, E_z=E_z, Lam=Lam, c=c, d=d, phi=phi, lnZ=lnZ, V=V, B=B,
                      gamma=g, S=S, N=N, K=K)

    out = O.fit(V, beta, A, pi, S, N, K, iters=iters, keep=True)
    seq = []
    hist = out["history"]
    for i in range(1, len(hist)):
        a_prev, Ez_prev, phi_prev = hist[i - 1]["alpha"], hist[i - 1]["E"], hist[i - 1]["phi"]
        seq.append(L(a_prev, Ez_prev, phi_prev))          # end of previous iteration
        seq.append(L(a_prev, hist[i]["E"], phi_prev))     # after the q(Z) update (Eq. 7)
        seq.append(L(a_prev, hist[i]["E"], hist[i]["phi"]))  # after q(D) (Eq. 8 + FB)
        seq.append(hist[i]["elbo"])                        # after q(theta) (Eq. 6)
    return np.array(seq), out["elbo"]


@pytest.mark.parametrize("which", ["tiny", "cfg0"])
def test_P6_elbo_non_decreasing(which):
    p = make_tiny(S=2, N=3, K=3, F=11, T=15, seed=4, quanta=40) if which == "tiny" else make_problem(0, 0)
    seq, trace = _half_step_elbos(p, iters=6 if which == "cfg0" else 12)
    assert np.all(np.diff(seq) >= -1e-12 * np.abs(seq[1:])), np.diff(seq)
    assert np.all(np.diff(trace) >= -1e-12 * np.abs(trace[1:]))


@pytest.mark.slow
def test_P6_elbo_non_decreasing_cfg1():
    p = make_problem(1, 0)
    out = O.fit_problem(p, iters=4)
    tr = out["elbo"]
    assert np.all(np.diff(tr) >= -1e-12 * np.abs(tr[1:]))


# ------------------------------------------------------------------ P7
def test_P7_elbo_below_exact_log_evidence():
    """With a few quanta per frame the evidence ln P(f) of the N^S model is
    computable exactly (theta and Z integrated, joint states summed); the
    bound must not exceed it."""
    p = make_tiny(S=2, N=5, K=2, F=8, T=20, seed=21, small_quanta=(1, 3), trans="dense", diag=0.6)
    S, N, K = p["S"], p["N"], p["K"]
    V, beta, A, pi = O.paper_arrays(p)
    out = O.fit(V, beta, A, pi, S, N, K, iters=30)
    lnP, marg = brute.log_evidence_exact(V, beta, A, pi, 1.0, S, N, K)
    gap = lnP - out["elbo"][-1]
    assert gap >= -1e-10 * abs(lnP), gap
    tv = 0.5 * np.abs(out["post"] - marg).sum(-1).max()
    print(f"P7: lnP={lnP:.6f} ELBO={out['elbo'][-1]:.6f} gap={gap:.4e} max TV(d, exact)={tv:.3f}")
    assert np.all(np.isfinite(out["elbo"]))


# ------------------------------------------------------------------ P8
@pytest.mark.parametrize("which", ["tiny", "cfg0"])
def test_P8_invariants(which):
    p = make_tiny(S=3, N=3, K=2, F=9, T=12, seed=8) if which == "tiny" else make_problem(0, 1)
    S, N, K, g = p["S"], p["N"], p["K"], 1.0
    V, beta, A, pi = O.paper_arrays(p)
    out = O.fit(V, beta, A, pi, S, N, K, iters=5, keep=True)
    v = V.sum(0)
    for h in out["history"]:
        np.testing.assert_allclose(h["d"].sum(-1), 1.0, atol=1e-9)
        np.testing.assert_allclose(h["c"].sum(1), v, rtol=1e-12)
        np.testing.assert_allclose(h["alpha"].sum(1), v + g * S * K + S * N * K, rtol=1e-12)
        assert h["alpha"].min() >= 1.0
    sep = out["sep"]
    assert sep.min() >= 0.0
    np.testing.assert_allclose(sep.sum(0), V, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------ P9
def test_P9_gamma_zero_gives_prior_marginals():
    p = make_tiny(S=2, N=4, K=2, F=6, T=8, seed=9)
    S, N, K = p["S"], p["N"], p["K"]
    V, beta, A, pi = O.paper_arrays(p)
    A = A / A.sum(-1, keepdims=True)      # exactly stochastic in float64
    pi = pi / pi.sum(-1, keepdims=True)
    out = O.fit(V, beta, A, pi, S, N, K, iters=3, gamma=0.0)
    for s in range(S):
        m = pi[s].copy()
        for t in range(p["T"]):
            np.testing.assert_allclose(out["post"][s, t], m, atol=1e-12)
            m = m @ A[s]
    # with gamma = 0 the chains do not feed Eq. 6: alpha = c + 1 with c from alpha
    out_b = O.fit(V, beta, A * 0 + 1.0 / N, pi, S, N, K, iters=3, gamma=0.0)
    np.testing.assert_allclose(out["alpha"], out_b["alpha"], rtol=1e-13)


def test_P9_single_state_is_lda_estep():
    """N = 1: every element is always available, d-hat = 1, and Eqs. 6-7 are
    the variational E-step of LDA with fixed topics and prior 1 + gamma."""
    p = make_tiny(S=2, N=1, K=3, F=6, T=4, seed=10, quanta=25)
    S, N, K = p["S"], p["N"], p["K"]
    g = 1.0
    V, beta, A, pi = O.paper_arrays(p)
    M = S * N * K
    v = V.sum(0)
    g0 = np.tile(1.0 + g + (v / M)[:, None], (1, 1)) * np.ones((p["T"], M))
    out = O.fit(V, beta, A, pi, S, N, K, iters=7, gamma=g, alpha_init=g0)
    np.testing.assert_allclose(out["post"], 1.0, atol=1e-14)
    for t in range(p["T"]):
        words = brute.quanta_of(V[:, t:t + 1])[0]
        gt = brute.lda_estep(words, beta, np.full(M, 1.0 + g), g0[t], iters=7)
        np.testing.assert_allclose(out["alpha"][t], gt, rtol=1e-11)


def test_P9_single_frame_softmax():
    p = make_tiny(S=2, N=4, K=2, F=6, T=1, seed=12)
    S, N, K = p["S"], p["N"], p["K"]
    V, beta, A, pi = O.paper_arrays(p)
    B = O.mask_B(S, N, K)
    out = O.fit(V, beta, A, pi, S, N, K, iters=2, keep=True)
    h = out["history"][-1]
    for s in range(S):
        z = np.log(pi[s]) + h["phi"][s, 0]
        sm = np.exp(z - z.max()); sm /= sm.sum()
        np.testing.assert_allclose(h["d"][s, 0], sm, atol=1e-14)
    assert B.shape == (S, N, S * N * K)


def test_P9_single_source_separation_is_identity():
    p = make_tiny(S=1, N=3, K=2, F=6, T=7, seed=13)
    V, beta, A, pi = O.paper_arrays(p)
    out = O.fit(V, beta, A, pi, 1, 3, 2, iters=3)
    np.testing.assert_allclose(out["sep"][0], V, rtol=1e-14)


def test_P9_evidence_shift_invariance():
    rng = np.random.default_rng(14)
    A, pi = _rand_chain(rng, 4)
    ev = rng.normal(size=(9, 4))
    shift = rng.normal(size=(9, 1)) * 10
    d1, z1 = O.forward_backward(ev, A, pi)
    d2, z2 = O.forward_backward(ev + shift, A, pi)
    np.testing.assert_allclose(d1, d2, atol=1e-13)
    assert abs((z2 - z1) - shift.sum()) < 1e-10


# ------------------------------------------------------------------ P11
def test_P11_source_swap_symmetry():
    p = make_tiny(S=2, N=3, K=2, F=8, T=10, seed=15)
    S, N, K = p["S"], p["N"], p["K"]
    q = dict(p)
    q["W"] = p["W"][::-1].copy(); q["A"] = p["A"][::-1].copy(); q["pi"] = p["pi"][::-1].copy()
    a = O.fit_problem(p, iters=6)
    b = O.fit_problem(q, iters=6)
    M1 = N * K
    perm = np.concatenate([np.arange(M1, 2 * M1), np.arange(M1)])
    np.testing.assert_allclose(b["alpha"], a["alpha"][:, perm], rtol=1e-12)
    np.testing.assert_allclose(b["post"], a["post"][::-1], atol=1e-12)
    np.testing.assert_allclose(b["sep"], a["sep"][::-1], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(b["elbo"], a["elbo"], rtol=1e-12)


# ------------------------------------------------------------------ P12 (report only)
def test_P12_recovery_report():
    p = make_problem(0, 2)
    out = O.fit_problem(p)
    acc = float((out["post"].argmax(-1) == p["states"]).mean())
    print(f"P12: config-0 argmax state recovery {acc:.3f}")
    assert acc > 0.5


# ------------------------------------------------------------------ P13 (the default start, reading R1)
def check_default_start(init_alpha):
    """Reading R1 (Eq. 6 with z-hat proportional to beta and d-hat = 1/N) against two
    things it fixes: (a) sum_k alpha0[t, k] = v_t + gamma S K + M, since the counts
    of a frame sum to v_t and each source's N state weights 1/N cover K elements
    each; (b) alpha0 - 1 - gamma/N equals sum_l V[l, t] z[t, l, k] with Eq. 7's
    responsibilities written out element by element at equal expected log-weights
    (brute.zhat_explicit at E = 0)."""
    for seed, (S, N, K), gamma in ((0, (2, 3, 2), 1.0), (1, (3, 4, 1), 0.5), (2, (2, 5, 3), 2.5)):
        p = make_tiny(S=S, N=N, K=K, F=7, T=6, seed=40 + seed, quanta=60)
        V, beta, A, pi = O.paper_arrays(p)
        M = S * N * K
        a0 = init_alpha(V, beta, O.mask_B(S, N, K), gamma, N)
        assert a0.shape == (p["T"], M)
        np.testing.assert_allclose(a0.sum(1), V.sum(0) + gamma * S * K + M, rtol=1e-12)
        z = brute.zhat_explicit(np.zeros((p["T"], M)), beta)            # T x F x M
        np.testing.assert_allclose(a0 - 1.0 - gamma / N, np.einsum("lt,tlk->tk", V, z), rtol=1e-12, atol=1e-12)


def test_P13_default_start():
    check_default_start(O.init_alpha)


# ------------------------------------------------------------------ P14 (Section 4, worked examples)
def _golden_separation_cases():
    import json
    import os
    from fractions import Fraction
    with open(os.path.join(os.path.dirname(__file__), "golden", "separation_mask.json")) as f:
        d = json.load(f)
    fr = lambda a: np.array([[float(Fraction(x)) for x in row] for row in a])  # noqa: E731
    for c in d["cases"]:
        Vstar = np.stack([fr(s) for s in c["Vstar"]])                       # S x T x F
        yield c, fr(c["beta"]).T, fr(c["alpha"]), fr(c["V"]).T, Vstar


def check_separation_golden(separate):
    """Section 4's split on hand-derived cases (tests/golden/separation_mask.json):
    the right block of elements per source, the posterior-mean weights of reading
    R6, and the zero cases of reading R7."""
    for c, beta, alpha, V, Vstar in _golden_separation_cases():
        out = separate(alpha, beta, V, c["S"], c["N"], c["K"])             # S x F x T
        np.testing.assert_allclose(np.transpose(out, (0, 2, 1)), Vstar, rtol=1e-14, atol=1e-14,
                                   err_msg=c["name"])


def test_P14_separation_worked_examples():
    check_separation_golden(O.separate)

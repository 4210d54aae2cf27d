"""Pins of the FP64 EM reference for one source's N-HMM (oracle/nhmm_em_oracle.py),
on the CPU: each checks it against something other than itself."""
import itertools

import numpy as np
import pytest

from oracle import nhmm_em_oracle as EM


def _model(rng, N, K, F, T, total=200):
    beta = rng.dirichlet(np.full(F, 0.5), size=(N, K))
    theta = rng.dirichlet(np.ones(K), size=(T, N))
    A = rng.dirichlet(np.ones(N), size=N)
    pi = rng.dirichlet(np.ones(N))
    V = rng.multinomial(total, np.full(F, 1.0 / F), size=T).astype(float)
    return V, beta, theta, A, pi


def test_chain_posteriors_match_enumeration():
    # gamma, the pairwise marginals and ln Z against a sum over all N^T paths
    rng = np.random.default_rng(1)
    N, T = 3, 5
    ll = rng.normal(size=(T, N)) * 3.0
    A = rng.dirichlet(np.ones(N), size=N)
    A[0, 2] = 0.0
    A[0] /= A[0].sum()
    pi = rng.dirichlet(np.ones(N))
    Z = 0.0
    g = np.zeros((T, N))
    xi = np.zeros((N, N))
    for path in itertools.product(range(N), repeat=T):
        w = pi[path[0]] * np.exp(ll[0, path[0]])
        for t in range(1, T):
            w *= A[path[t - 1], path[t]] * np.exp(ll[t, path[t]])
        Z += w
        for t in range(T):
            g[t, path[t]] += w
        for t in range(1, T):
            xi[path[t - 1], path[t]] += w
    gamma, xis, lnZ = EM.chain_posteriors(ll, A, pi)
    assert abs(lnZ - np.log(Z)) < 1e-12
    assert np.max(np.abs(gamma - g / Z)) < 1e-12
    assert np.max(np.abs(xis - xi / Z)) < 1e-12


def test_frame_loglik_is_the_multinomial_log_likelihood():
    # sum_f V ln P_t(f|d) against the quanta drawn one by one: the log of the
    # product of the per-quantum probabilities sum_z theta beta
    rng = np.random.default_rng(2)
    N, K, F, T = 2, 3, 5, 4
    V, beta, theta, A, pi = _model(rng, N, K, F, T, total=7)
    ll = EM.frame_loglik(V, beta, theta)
    for t in range(T):
        for d in range(N):
            lp = 0.0
            for f in range(F):
                for _ in range(int(V[t, f])):
                    lp += np.log(sum(theta[t, d, z] * beta[d, z, f] for z in range(K)))
            assert abs(ll[t, d] - lp) < 1e-10


def test_em_never_lowers_the_likelihood():
    rng = np.random.default_rng(3)
    V, beta, theta, A, pi = _model(rng, 4, 3, 12, 30)
    prev = -np.inf
    for _ in range(25):
        beta, theta, A, pi, lnZ = EM.em_step(V, beta, theta, A, pi)
        assert lnZ >= prev - 1e-9
        prev = lnZ
    assert EM.log_likelihood(V, beta, theta, A, pi) >= prev - 1e-9
    # the parameters stay distributions
    assert np.allclose(beta.sum(-1), 1.0) and np.allclose(theta.sum(-1), 1.0)
    assert np.allclose(A.sum(1), 1.0) and abs(pi.sum() - 1.0) < 1e-12


def test_one_state_is_kl_nmf():
    # with a single state the chain is certain and EM is PLCA, i.e. the
    # multiplicative KL-NMF updates (Lee and Seung) on W = beta^T [F][K] and
    # H[k][t] = v_t theta_t(k), with W's columns renormalised
    rng = np.random.default_rng(4)
    K, F, T = 3, 9, 15
    V, beta, theta, A, pi = _model(rng, 1, K, F, T)
    b1, th1, _, _, _ = EM.em_step(V, beta, theta, np.ones((1, 1)), np.ones(1))
    W = beta[0].T                                  # [F][K]
    v = V.sum(1)
    H = (theta[:, 0, :] * v[:, None]).T            # [K][T]
    X = V.T                                        # [F][T]
    WH = W @ H
    Wn = W * ((X / WH) @ H.T) / H.sum(1)[None, :]
    Hn = H * (W.T @ (X / WH)) / W.sum(0)[:, None]
    Wn = Wn / Wn.sum(0, keepdims=True)
    Hn = Hn / Hn.sum(0, keepdims=True)
    assert np.max(np.abs(b1[0] - Wn.T)) < 1e-12
    assert np.max(np.abs(th1[:, 0, :] - Hn.T)) < 1e-12


def test_transitions_follow_the_pairwise_counts():
    # with evidence that pins the states exactly, one EM step gives the empirical
    # transition frequencies of that path and pi at its first state
    N, K, F = 3, 1, 3
    path = [0, 0, 1, 2, 2, 2, 0, 1, 1, 2]
    T = len(path)
    beta = np.eye(N)[:, None, :]                   # state d emits only bin d
    theta = np.ones((T, N, K))
    V = np.zeros((T, F))
    for t, d in enumerate(path):
        V[t, d] = 5.0
    A = np.full((N, N), 1.0 / N)
    pi = np.full(N, 1.0 / N)
    _, _, A1, pi1, _ = EM.em_step(V, beta, theta, A, pi)
    C = np.zeros((N, N))
    for a, b in zip(path[:-1], path[1:]):
        C[a, b] += 1
    assert np.max(np.abs(A1 - C / C.sum(1, keepdims=True))) < 1e-12
    assert pi1[path[0]] == pytest.approx(1.0, abs=1e-12)


def test_dictionary_and_weight_updates_are_expected_counts_by_enumeration():
    # one EM step's beta and theta against the expected counts built by brute
    # force: state marginals from all N^T paths, and each quantum's element
    # posterior from Bayes' rule, P(z | f, d) = theta_t(d, z) beta(d, z, f) /
    # sum_z' theta_t(d, z') beta(d, z', f)
    rng = np.random.default_rng(5)
    N, K, F, T = 2, 2, 4, 4
    V, beta, theta, A, pi = _model(rng, N, K, F, T, total=6)
    b1, th1, _, _, _ = EM.em_step(V, beta, theta, A, pi)
    # state marginals by enumeration, with the quanta's likelihood written out
    def frame_p(t, d):
        p = 1.0
        for f in range(F):
            pf = sum(theta[t, d, z] * beta[d, z, f] for z in range(K))
            p *= pf ** V[t, f]
        return p
    g = np.zeros((T, N))
    for path in itertools.product(range(N), repeat=T):
        w = pi[path[0]] * frame_p(0, path[0])
        for t in range(1, T):
            w *= A[path[t - 1], path[t]] * frame_p(t, path[t])
        for t in range(T):
            g[t, path[t]] += w
    g /= g.sum(1, keepdims=True)
    cb = np.zeros((N, K, F))
    ct = np.zeros((T, N, K))
    for t in range(T):
        for d in range(N):
            for f in range(F):
                den = sum(theta[t, d, z] * beta[d, z, f] for z in range(K))
                for z in range(K):
                    q = theta[t, d, z] * beta[d, z, f] / den
                    cb[d, z, f] += g[t, d] * V[t, f] * q
                    ct[t, d, z] += V[t, f] * q
    assert np.max(np.abs(b1 - cb / cb.sum(-1, keepdims=True))) < 1e-12
    assert np.max(np.abs(th1 - ct / ct.sum(-1, keepdims=True))) < 1e-12

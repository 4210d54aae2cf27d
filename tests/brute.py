"""Brute-force and textbook checkers that pin the FP64 oracle.

Each routine is written from a definition in the paper (or a textbook it
cites), independently of ``oracle.nfhmm_oracle``: nothing here imports it.
They are only usable on tiny problems.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.special import digamma, gammaln, logsumexp
from scipy.stats import dirichlet


def owner(S, N, K):
    """(source, state) owning each element; B of Section 2.2 as index arrays."""
    pairs = [(s, n) for s in range(S) for n in range(N) for _ in range(K)]
    return np.array([p[0] for p in pairs]), np.array([p[1] for p in pairs])


def all_sequences(N, T):
    return np.array(list(itertools.product(range(N), repeat=T)), dtype=np.int64)


def chain_log_prob(seqs, A, pi):
    """ln P(D) of every sequence under a Markov chain (row-stochastic A)."""
    with np.errstate(divide="ignore"):
        lp = np.log(pi[seqs[:, 0]])
        for t in range(1, seqs.shape[1]):
            lp = lp + np.log(A[seqs[:, t - 1], seqs[:, t]])
    return lp


def fb_brute(logev, A, pi):
    """Marginals and ln Z of the chain posterior by enumerating all N^T paths."""
    T, N = logev.shape
    seqs = all_sequences(N, T)
    lp = chain_log_prob(seqs, A, pi) + logev[np.arange(T)[None, :], seqs].sum(1)
    lnZ = logsumexp(lp)
    p = np.exp(lp - lnZ)
    d = np.zeros((T, N))
    for t in range(T):
        np.add.at(d[t], seqs[:, t], p)
    return d, float(lnZ)


def product_chain(A_list, pi_list):
    """The joint chain over N^S configurations of independent sources."""
    A, pi = A_list[0], pi_list[0]
    for As, ps in zip(A_list[1:], pi_list[1:]):
        A, pi = np.kron(A, As), np.kron(pi, ps)
    return A, pi


def zhat_explicit(E_q, beta):
    """Eq. 7 written out: ln z[t,l,k] = ln beta[l,k] + E_q[t,k] - kappa[t,l],
    normalised over k for every (t, l)."""
    with np.errstate(divide="ignore"):
        lz = np.log(beta)[None, :, :] + E_q[:, None, :]          # T x F x M
    lz = lz - logsumexp(lz, axis=2, keepdims=True)
    return np.exp(lz)


def elbo_direct(alpha, E_q, phi, V, beta, A, pi, gamma, S, N, K):
    """The evidence lower bound evaluated term by term from the model of
    Section 2.2 and the factorised posterior of Section 3.2.

    q(theta_t) = Dir(alpha[t]); q(Z) from Eq. 7 with log-weights E_q;
    q(D^(s)) proportional to P(D^(s)) exp(gamma sum_t phi[s,t,D_t]),
    enumerated over all N^T paths.  Needs tiny N and T."""
    T, M = alpha.shape
    src, st = owner(S, N, K)
    Ebar = digamma(alpha) - digamma(alpha.sum(1, keepdims=True))
    total = 0.0
    seqs = all_sequences(N, T)
    d = np.zeros((S, T, N))
    for s in range(S):
        lprior = chain_log_prob(seqs, A[s], pi[s])
        lq = lprior + gamma * phi[s][np.arange(T)[None, :], seqs].sum(1)
        ok = np.isfinite(lq)
        lq = lq - logsumexp(lq[ok])
        q = np.where(ok, np.exp(lq), 0.0)
        total += float(np.sum(q[ok] * lprior[ok]))        # E ln P(D)
        total += float(-np.sum(q[ok] * lq[ok]))           # H[q(D)]
        for t in range(T):
            np.add.at(d[s, t], seqs[:, t], q)
    # E ln P(theta | D): enumerate joint states with product weights
    for t in range(T):
        for joint in itertools.product(range(N), repeat=S):
            wgt = np.prod([d[s, t, joint[s]] for s in range(S)])
            if wgt == 0.0:
                continue
            a = np.ones(M)
            for s in range(S):
                a[(src == s) & (st == joint[s])] += gamma
            lp = gammaln(a.sum()) - gammaln(a).sum() + np.sum((a - 1.0) * Ebar[t])
            total += wgt * lp
    # Z and f terms with the explicit responsibilities
    z = zhat_explicit(E_q, beta)                                  # T x F x M
    Vt = V.T                                                      # T x F
    with np.errstate(divide="ignore", invalid="ignore"):
        inner = Ebar[:, None, :] + np.log(beta)[None] - np.log(z)
        term = np.where(z > 0, Vt[:, :, None] * z * inner, 0.0)
    total += float(term.sum())
    for t in range(T):
        total += float(dirichlet(alpha[t]).entropy())              # H[q(theta_t)]
    return total


def quanta_of(V):
    """Frequencies of the quanta of each frame (one entry per quantum)."""
    F, T = V.shape
    return [np.repeat(np.arange(F), V[:, t].astype(np.int64)) for t in range(T)]


def _joint_alpha(joint, S, N, K, gamma):
    src, st = owner(S, N, K)
    a = np.ones(S * N * K)
    for s in range(S):
        a[(src == s) & (st == joint[s])] += gamma
    return a


def exact_frame_loglik(fs, beta, gamma, S, N, K):
    """ln P(f_t | joint state) for every frame and joint state, integrating
    theta and Z exactly: the sum over all z in [M]^v of prod_v beta[f_v, z_v]
    times the Dirichlet moment E[prod_k theta_k^{n_k(z)}] =
    Gamma(a0)/Gamma(a0+v) prod_k Gamma(a_k+n_k)/Gamma(a_k).  Returns T x N^S."""
    F, M = beta.shape
    joints = list(itertools.product(range(N), repeat=S))
    alphas = np.stack([_joint_alpha(j, S, N, K, gamma) for j in joints])   # J x M
    cache = {}
    out = np.zeros((len(fs), len(joints)))
    for t, f in enumerate(fs):
        v = len(f)
        if v == 0:
            continue
        if v not in cache:
            zs = np.array(list(itertools.product(range(M), repeat=v)))
            cnt = np.zeros((zs.shape[0], M))
            for j in range(v):
                np.add.at(cnt, (np.arange(zs.shape[0]), zs[:, j]), 1.0)
            a0 = alphas.sum(1)                                              # J
            mom = (gammaln(a0)[:, None] - gammaln(a0 + v)[:, None]
                   + np.sum(gammaln(alphas[:, None, :] + cnt[None]) - gammaln(alphas)[:, None, :], axis=2))
            cache[v] = (zs, np.exp(mom))                                    # J x nz
        zs, emom = cache[v]
        bprod = np.prod(beta[np.asarray(f)[None, :], zs], axis=1)          # nz
        out[t] = np.log(emom @ bprod)
    return out


def log_evidence_exact(V, beta, A, pi, gamma, S, N, K):
    """ln P(f) of the whole mixture: exact frame likelihoods on the N^S joint
    chain, summed over joint paths by the forward recursion.  Also returns the
    exact posterior marginals of each source's state."""
    Aj, pij = product_chain(list(A), list(pi))
    ll = exact_frame_loglik(quanta_of(V), beta, gamma, S, N, K)           # T x N^S
    T = ll.shape[0]
    with np.errstate(divide="ignore"):
        lA = np.log(Aj)
        la = np.empty_like(ll)
        lb = np.zeros_like(ll)
        la[0] = np.log(pij) + ll[0]
    for t in range(1, T):
        la[t] = ll[t] + logsumexp(la[t - 1][:, None] + lA, axis=0)
    for t in range(T - 2, -1, -1):
        lb[t] = logsumexp(lA + (ll[t + 1] + lb[t + 1])[None, :], axis=1)
    lnP = float(logsumexp(la[-1]))
    post = np.exp(la + lb - lnP).reshape((T,) + (N,) * S)
    marg = np.stack([post.sum(axis=tuple(1 + x for x in range(S) if x != s)) for s in range(S)])
    return lnP, marg


def lda_estep(words, beta, prior, gamma0, iters):
    """Variational E-step of latent Dirichlet allocation for one document with
    fixed topics (Blei, Ng & Jordan 2003): per word, phi_n ∝ beta[w_n] exp(psi(g));
    then g = prior + sum_n phi_n.  Word by word, no grouping by frequency."""
    g = np.array(gamma0, float)
    for _ in range(iters):
        acc = np.zeros_like(g)
        eg = np.exp(digamma(g))
        for wn in words:
            ph = beta[wn] * eg
            acc += ph / ph.sum()
        g = prior + acc
    return g

"""FP64 reference of learning one source's N-HMM by EM (TEST INFRASTRUCTURE ONLY:
imported by tests/, never by the product path).

Section 2.1 defines the model: states D_t follow a Markov chain (transitions rho,
initial pi); each of the v_t quanta of frame t draws an element Z ~ theta_t(D_t)
and a frequency F ~ beta(D_t, Z).  It states that EM finds the maximum-likelihood
beta and rho (with theta_t as per-frame nuisance parameters) but gives no steps.
The steps here are derived from that model (a reading, listed with the others):

  E-step   P_t(f | d) = sum_z theta_t(d, z) beta(d, z, f)
           ll[t, d]   = sum_f V[t, f] ln P_t(f | d)   (the multinomial constant dropped)
           gamma, xi  = state marginals and pairwise marginals of the chain with
                        evidence exp(ll)
  M-step   with q(z | t, d, f) = theta_t(d, z) beta(d, z, f) / P_t(f | d):
           beta(d, z, f)  ~ sum_t gamma_t(d) V[t, f] q(z | t, d, f)   (normalised over f)
           theta_t(d, z)  ~ sum_f V[t, f] q(z | t, d, f)             (over z; gamma_t(d)
                                                                       is a common factor)
           rho(i, j) ~ sum_t xi_t(i, j)  (over j),  pi ~ gamma_0.

Shapes: V [T][F] counts, beta [N][K][F], theta [T][N][K], A [N][N] row-stochastic
(A[i][j] = P(D_t = j | D_{t-1} = i)), pi [N].  The likelihood ln P(V) (up to the
multinomial constant) is the chain's ln Z; EM never lowers it.
"""
from __future__ import annotations

import numpy as np


def _lse(x, axis):
    m = np.max(x, axis=axis, keepdims=True)
    m = np.where(np.isfinite(m), m, 0.0)
    with np.errstate(divide="ignore"):
        return np.squeeze(m, axis=axis) + np.log(np.sum(np.exp(x - m), axis=axis))


def _log(x):
    with np.errstate(divide="ignore"):
        return np.log(x)


def frame_probs(beta, theta):
    """P_t(f | d) [T][N][F]."""
    return np.einsum("tnk,nkf->tnf", theta, beta)


def frame_loglik(V, beta, theta):
    """ll[t, d] = sum_f V[t, f] ln P_t(f | d); terms with V = 0 contribute 0."""
    P = frame_probs(beta, theta)
    Vb = np.asarray(V, float)[:, None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        terms = np.where(Vb > 0, Vb * _log(P), 0.0)
    return terms.sum(-1)


def chain_posteriors(ll, A, pi):
    """Log-space forward-backward: (gamma [T][N], xi_sum [N][N], lnZ), xi_sum[i, j] =
    sum_t P(D_{t-1} = i, D_t = j | V)."""
    T, N = ll.shape
    lnA, lnpi = _log(np.asarray(A, float)), _log(np.asarray(pi, float))
    la = np.empty((T, N))
    lb = np.zeros((T, N))
    la[0] = lnpi + ll[0]
    for t in range(1, T):
        la[t] = ll[t] + _lse(la[t - 1][:, None] + lnA, axis=0)
    for t in range(T - 2, -1, -1):
        lb[t] = _lse(lnA + (ll[t + 1] + lb[t + 1])[None, :], axis=1)
    lnZ = float(_lse(la[T - 1], axis=0))
    gamma = np.exp(la + lb - lnZ)
    xi = np.zeros((N, N))
    for t in range(1, T):
        xi += np.exp(la[t - 1][:, None] + lnA + (ll[t] + lb[t])[None, :] - lnZ)
    return gamma, xi, lnZ


def em_step(V, beta, theta, A, pi):
    """One EM iteration; returns (beta, theta, A, pi, lnZ of the parameters given)."""
    V = np.asarray(V, float)
    ll = frame_loglik(V, beta, theta)
    gamma, xi, lnZ = chain_posteriors(ll, A, pi)
    P = frame_probs(beta, theta)
    with np.errstate(divide="ignore", invalid="ignore"):
        R = np.where(V[:, None, :] > 0, V[:, None, :] / P, 0.0)          # [T][N][F]
    nb = beta * np.einsum("tn,tnk,tnf->nkf", gamma, theta, R)
    nt = theta * np.einsum("nkf,tnf->tnk", beta, R)
    # rows that received no expected counts keep their previous values
    beta_new = _normalise(nb, beta, -1)
    theta_new = _normalise(nt, theta, -1)
    A_new = _normalise(xi, np.asarray(A, float), 1)
    pi_new = gamma[0] / gamma[0].sum()
    return beta_new, theta_new, A_new, pi_new, lnZ


def _normalise(x, old, axis):
    s = x.sum(axis, keepdims=True)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(s > 0, x / np.where(s > 0, s, 1.0), old)


def log_likelihood(V, beta, theta, A, pi):
    """ln P(V) up to the multinomial constant: the chain's ln Z."""
    return chain_posteriors(frame_loglik(V, beta, theta), A, pi)[2]

"""FP64 CPU oracle of variational inference in the Bayesian N-FHMM.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the
HIP library is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never calls it
and shares no code with it.

It follows Mysore & Sahani, "Variational Inference in Non-negative Factorial
Hidden Markov Models for Efficient Audio Source Separation":

* model: Section 2.2 (per-source Markov chains D^(s), Dirichlet prior on the
  mixture weights theta_t with parameters alpha_k(D_t) = 1 + gamma * sum_s
  sum_n delta B_snk, quanta Z ~ theta_t, frequencies F ~ beta(Z));
* factorised posterior: Section 3.2 (q(theta_t), q(Z_tv), q(D^(s)));
* updates: Eq. 6 (Dirichlet posterior alpha-hat), Eq. 7 (responsibilities
  z-hat), Eq. 8 (surrogate state log-likelihood phi-hat), forward-backward
  per source for the state marginals d-hat;
* separation: Section 4 (reconstruction from the estimated weights and the
  ratio mask).

Notation is the paper's: V[l,t] mixture spectrogram (F x T), beta[l,k]
dictionary elements (F x M, columns sum to one), alpha[t,k] = alpha-hat,
d[s,t,n] = d-hat, phi[s,t,n] = phi-hat.  Element k belongs to source s and
state n through the layout k = (s*N + n)*K + j, which is the mask B of
Section 2.2 (B[s,n,k] = 1 iff k lies in block (s, n)).

Readings taken where the paper is silent or ambiguous (each is also listed in
the design notes):

R1  initialisation: alpha-hat^(0) by Eq. 6 with z-hat proportional to beta
    (all expected log-weights equal, so w = 1) and d-hat = 1/N.
R2  one iteration = [Eq. 7 and Eq. 8 + forward-backward, both from the same
    alpha-hat] then Eq. 6, then the ELBO; alpha-hat is the only carried state.
R3  the chain evidence is gamma * phi-hat (the mean-field derivation gives the
    factor gamma, which Eq. 8 leaves out; the two agree for gamma = 1).
R4  transitions are passed row-stochastic, A[i,j] = P(D_t = j | D_{t-1} = i),
    the transpose of the paper's column convention for rho.
R6  reconstruction uses E[theta_tk] = alpha-hat_tk / sum_k alpha-hat_tk.
R7  R = V / Lambda is 0 where V = 0; V* = 0 where V = 0; V* = V / S where the
    reconstructions of all sources are 0 but V > 0.
R8  zero entries of A and pi are allowed (minus infinity in log space).
R9  every dictionary has the same K elements and no element is shared, so
    sum_k alpha_k(D) = M + gamma*S*K for every joint state.
R10 a fixed number of iterations; no convergence test.
R11 the "reconstruction cross entropy" diagnostic is
    -sum V ln P / sum V with P[:,t] = beta E[theta_t] (diagnostic only).
"""
from __future__ import annotations

import numpy as np
from scipy.special import digamma, gammaln

__all__ = [
    "element_layout", "mask_B", "expected_log_theta", "state_evidence",
    "lse", "forward_backward", "expected_counts", "dirichlet_update",
    "dirichlet_const", "elbo", "separate", "init_alpha", "one_iteration",
    "fit", "fit_problem", "paper_arrays", "reconstruction_cross_entropy",
]


# ---------------------------------------------------------------- layout / mask
def element_layout(S: int, N: int, K: int):
    """Source and state owning each element k = (s*N + n)*K + j."""
    k = np.arange(S * N * K)
    return k // (N * K), (k // K) % N


def mask_B(S: int, N: int, K: int) -> np.ndarray:
    """B[s, n, k] = 1 iff element k is available when source s is in state n
    (Section 2.2, the mask inside alpha_k(D))."""
    src, st = element_layout(S, N, K)
    B = np.zeros((S, N, S * N * K))
    B[src, st, np.arange(S * N * K)] = 1.0
    return B


# ---------------------------------------------------------------- Eq. 7 / Eq. 8
def expected_log_theta(alpha: np.ndarray) -> np.ndarray:
    """E_q[ln theta_tk] = psi(alpha_tk) - psi(sum_k alpha_tk): the digamma terms
    shared by Eq. 7 and Eq. 8.  alpha: [T, M]."""
    return digamma(alpha) - digamma(alpha.sum(axis=1, keepdims=True))


def state_evidence(E: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Eq. 8: phi[s,t,n] = sum_k B[s,n,k] * E[t,k]."""
    return np.einsum("snk,tk->stn", B, E)


# ---------------------------------------------------------------- forward-backward
def lse(x: np.ndarray, axis: int) -> np.ndarray:
    """log-sum-exp that returns -inf for an all -inf slice and never forms
    (-inf) - (-inf)."""
    m = np.max(x, axis=axis, keepdims=True)
    finite = np.isfinite(m)
    safe_m = np.where(finite, m, 0.0)
    with np.errstate(divide="ignore"):
        s = np.log(np.sum(np.exp(x - safe_m), axis=axis, keepdims=True))
    out = np.where(finite, safe_m + s, -np.inf)
    return np.squeeze(out, axis=axis)


def _log(x):
    with np.errstate(divide="ignore"):
        return np.log(x)


def forward_backward(logev: np.ndarray, A: np.ndarray, pi: np.ndarray):
    """Log-space forward-backward for one chain (the step after Eq. 8; the
    recursion is the standard one the paper cites from Rabiner 1989).

    logev[t, n] = log evidence of state n at frame t (here gamma * phi-hat),
    A[i, j] = P(D_t = j | D_{t-1} = i), pi[n] = P(D_0 = n).
    Returns (d[t, n] marginals, lnZ)."""
    T, N = logev.shape
    lnA, lnpi = _log(np.asarray(A, float)), _log(np.asarray(pi, float))
    la = np.empty((T, N))
    lb = np.zeros((T, N))
    la[0] = lnpi + logev[0]
    for t in range(1, T):
        la[t] = logev[t] + lse(la[t - 1][:, None] + lnA, axis=0)
    for t in range(T - 2, -1, -1):
        lb[t] = lse(lnA + (logev[t + 1] + lb[t + 1])[None, :], axis=1)
    lnZ = float(lse(la[T - 1], axis=0))
    with np.errstate(invalid="ignore"):
        d = np.exp(la + lb - lnZ)
    d = np.where(np.isfinite(la) & np.isfinite(lb), d, 0.0)
    return d, lnZ


# ---------------------------------------------------------------- Eq. 6 / Eq. 7
def expected_counts(V: np.ndarray, beta: np.ndarray, E: np.ndarray):
    """sum_l V[l,t] z[t,l,k] with z from Eq. 7.

    Eq. 7 gives z[t,l,k] = beta[l,k] w[t,k] / Lambda[l,t] with w = exp(E) and
    the log-normaliser kappa = ln Lambda[l,t] = ln sum_k beta[l,k] w[t,k] (the
    -psi(alpha_0) term is common to all k and cancels).  The sum over l then
    is c[t,k] = w[t,k] * sum_l beta[l,k] V[l,t] / Lambda[l,t].
    Returns (c[T, M], Lambda[F, T])."""
    w = np.exp(E)
    Lam = beta @ w.T
    with np.errstate(divide="ignore", invalid="ignore"):
        R = np.where(V > 0, V / Lam, 0.0)
    c = w * (beta.T @ R).T
    return c, Lam


def dirichlet_update(c: np.ndarray, d: np.ndarray, B: np.ndarray, gamma: float):
    """Eq. 6: alpha[t,k] = c[t,k] + gamma * sum_s sum_n d[s,t,n] B[s,n,k] + 1."""
    return c + gamma * np.einsum("stn,snk->tk", d, B) + 1.0


# ---------------------------------------------------------------- ELBO
def dirichlet_const(S: int, N: int, K: int, gamma: float) -> float:
    """ln Gamma(sum_k alpha_k(D)) - sum_k ln Gamma(alpha_k(D)), identical for
    every joint state under R9: M elements at 1, S*K of them raised to 1+gamma."""
    M = S * N * K
    return float(gammaln(M + gamma * S * K) - S * K * gammaln(1.0 + gamma))


def elbo(*, alpha, E_z, Lam, c, d, phi, lnZ, V, B, gamma, S, N, K) -> float:
    """Evidence lower bound of the factorised posterior of Section 3.2 for an
    arbitrary triple: q(theta_t) = Dir(alpha[t]); q(Z) given by Eq. 7 with the
    expected log-weights E_z (so ln w = E_z, counts c, normaliser Lambda); q(D^(s))
    the chain posterior with evidence gamma*phi[s] (marginals d[s], log
    normaliser lnZ[s]).  Expanded in closed form from the model of
    Section 2.2:

      L = sum_s [lnZ_s - gamma sum d*phi]                      (E ln P(D) + H[q(D)])
        + sum (c + gamma B'd - (alpha - 1)) * Ebar            (Ebar = E_q(theta) ln theta)
        - sum c * E_z + sum V ln Lambda                         (Z and f terms, H[q(Z)])
        + sum_t [sum_k lnG(alpha) - lnG(alpha_0)] + T * C       (prior const, H[q(theta)])
    """
    T = alpha.shape[0]
    Ebar = expected_log_theta(alpha)
    chain = float(np.sum(lnZ) - gamma * np.sum(d * phi))
    prior_k = c + gamma * np.einsum("stn,snk->tk", d, B) - (alpha - 1.0)
    lin = float(np.sum(prior_k * Ebar))
    with np.errstate(divide="ignore", invalid="ignore"):
        vlog = np.where(V > 0, V * np.log(Lam), 0.0)
    zf = float(-np.sum(c * E_z) + np.sum(vlog))
    ent = float(np.sum(gammaln(alpha)) - np.sum(gammaln(alpha.sum(axis=1))))
    return chain + lin + zf + ent + T * dirichlet_const(S, N, K, gamma)


# ---------------------------------------------------------------- Section 4
def separate(alpha: np.ndarray, beta: np.ndarray, V: np.ndarray, S: int, N: int, K: int):
    """Section 4: Vhat^(s) = beta_s E[theta]_s, V*^(s) = V Vhat^(s) / sum_s' Vhat^(s').
    Returns Vstar[s, l, t] (paper orientation)."""
    F, T = V.shape
    theta = alpha / alpha.sum(axis=1, keepdims=True)
    src, _ = element_layout(S, N, K)
    Vhat = np.stack([beta[:, src == s] @ theta[:, src == s].T for s in range(S)])
    tot = Vhat.sum(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        Vs = np.where(tot > 0, V[None] * Vhat / tot[None], V[None] / S)
    return np.where(V[None] > 0, Vs, 0.0)


def reconstruction_cross_entropy(alpha, beta, V):
    """Diagnostic of the Fig. 9 kind (reading R11); not pinned."""
    theta = alpha / alpha.sum(axis=1, keepdims=True)
    P = beta @ theta.T
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(V > 0, V * np.log(P), 0.0)
    return float(-t.sum() / V.sum())


# ---------------------------------------------------------------- the loop
def init_alpha(V, beta, B, gamma, N):
    """Reading R1: Eq. 6 with w = 1 (z-hat proportional to beta) and d-hat = 1/N."""
    T = V.shape[1]
    c, _ = expected_counts(V, beta, np.zeros((T, beta.shape[1])))
    S = B.shape[0]
    d = np.full((S, T, N), 1.0 / N)
    return dirichlet_update(c, d, B, gamma)


def one_iteration(alpha, V, beta, A, pi, B, gamma, S, N, K):
    """One pass of R2.  Returns every intermediate, for one-step parity."""
    E = expected_log_theta(alpha)                     # Eq. 7/8 digamma terms
    phi = state_evidence(E, B)                        # Eq. 8
    T = alpha.shape[0]
    d = np.empty((S, T, N))
    lnZ = np.empty(S)
    for s in range(S):                                # forward-backward per source
        d[s], lnZ[s] = forward_backward(gamma * phi[s], A[s], pi[s])
    c, Lam = expected_counts(V, beta, E)              # Eq. 7 inside Eq. 6
    alpha_new = dirichlet_update(c, d, B, gamma)      # Eq. 6
    L = elbo(alpha=alpha_new, E_z=E, Lam=Lam, c=c, d=d, phi=phi, lnZ=lnZ, V=V, B=B,
             gamma=gamma, S=S, N=N, K=K)
    return dict(E=E, w=np.exp(E), phi=phi, d=d, lnZ=lnZ, c=c, Lam=Lam,
                alpha=alpha_new, elbo=L)


def paper_arrays(prob: dict):
    """ABI layouts -> paper orientation, in float64."""
    S, N, K, F, T = (int(prob[k]) for k in ("S", "N", "K", "F", "T"))
    V = np.asarray(prob["V"], np.float64).reshape(T, F).T               # F x T
    beta = np.asarray(prob["W"], np.float64).reshape(S * N * K, F).T    # F x M
    A = np.asarray(prob["A"], np.float64).reshape(S, N, N)
    pi = np.asarray(prob["pi"], np.float64).reshape(S, N)
    return V, beta, A, pi


def fit(V, beta, A, pi, S, N, K, iters, gamma=1.0, alpha_init=None, keep=False):
    """Run R1 + `iters` iterations of R2 + the separation of Section 4.

    Returns dict(alpha[T,M], post[S,T,N], sep[S,F,T], elbo[iters])."""
    B = mask_B(S, N, K)
    alpha = init_alpha(V, beta, B, gamma, N) if alpha_init is None else np.array(alpha_init, float)
    trace, hist = [], []
    d = np.full((S, alpha.shape[0], N), 1.0 / N)
    for _ in range(int(iters)):
        r = one_iteration(alpha, V, beta, A, pi, B, gamma, S, N, K)
        alpha, d = r["alpha"], r["d"]
        trace.append(r["elbo"])
        if keep:
            hist.append(r)
    out = dict(alpha=alpha, post=d, sep=separate(alpha, beta, V, S, N, K),
               elbo=np.array(trace))
    if keep:
        out["history"] = hist
    return out


def fit_problem(prob: dict, iters=None, gamma=None, alpha_init=None, keep=False):
    """fit() on a problem dict in the ABI layouts; outputs in ABI layouts:
    alpha [T][M], post [S][T][N], sep [S][T][F], elbo [iters]."""
    S, N, K = (int(prob[k]) for k in ("S", "N", "K"))
    V, beta, A, pi = paper_arrays(prob)
    out = fit(V, beta, A, pi, S, N, K, prob["iters"] if iters is None else iters,
              prob.get("gamma", 1.0) if gamma is None else gamma, alpha_init, keep)
    out["sep"] = np.ascontiguousarray(np.transpose(out["sep"], (0, 2, 1)))
    return out

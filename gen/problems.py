"""Seeded synthetic N-FHMM separation problems.

Every array is drawn from ``numpy.random.default_rng(SeedSequence([12066468,
cfg_id, job_id]))`` so that the FP64 oracle and the HIP path see identical
inputs.  Nothing here performs inference; the only arithmetic is sampling
from the generative process of the Bayesian N-FHMM (Section 2.2: per-source
Markov states, Dirichlet mixture weights, quanta drawn from the selected
elements) with the source-model shapes of the experiments (Section 5:
1024-point STFT gives F = 513 bins; N-HMMs with N dictionaries of K
elements each).  TIMIT speech and trained N-HMMs are not available, so
these draws stand in for them.

Array layouts (the C ABI's):
    V   [T][F]      float32 counts of quanta, V >= 0
    W   [S][N][K][F] float32; W[s,n,j,:] is one normalised dictionary element
    A   [S][N][N]   float32 row-stochastic, A[s,i,j] = P(D_t = j | D_{t-1} = i)
    pi  [S][N]      float32 initial-state probabilities (uniform)
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 12066468

# workload id -> defaults.  0: the small case the FP64 oracle runs in seconds;
# 1: the paper-typical job (1024-point STFT, 40 states of 10 elements, 1000
# frames); 2: the same with three sources; 3: the long precision-form job
# (2048-point STFT, 60 states of 20 elements, 4000 frames); 4: the serving mix,
# which draws S and T per job.  The id also seeds every draw.
CONFIGS = {
    0: dict(S=2, N=5, K=8, F=129, T=100, iters=20, dict_conc=0.5, trans="dense",
            diag=0.8, weights="bayes", loud=False, quanta=10_000),
    1: dict(S=2, N=40, K=10, F=513, T=1000, iters=50, dict_conc=0.3, trans="sparse",
            diag=0.9, weights="active", loud=True, quanta=10_000),
    2: dict(S=3, N=40, K=10, F=513, T=1000, iters=50, dict_conc=0.3, trans="sparse",
            diag=0.9, weights="active", loud=True, quanta=10_000),
    3: dict(S=2, N=60, K=20, F=1025, T=4000, iters=100, dict_conc=0.3, trans="sparse",
            diag=0.9, weights="active", loud=True, quanta=10_000),
    4: dict(S=None, N=40, K=10, F=513, T=None, iters=50, dict_conc=0.3, trans="sparse",
            diag=0.9, weights="active", loud=True, quanta=10_000),
}


def _rng(cfg_id: int, job_id: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_BASE, int(cfg_id), int(job_id)]))


def _normalise_f32(x: np.ndarray, axis: int = -1) -> np.ndarray:
    """Normalise in float64, then store as float32."""
    x = np.asarray(x, dtype=np.float64)
    return (x / x.sum(axis=axis, keepdims=True)).astype(np.float32)


def _dictionaries(rng, S, N, K, F, conc):
    g = rng.gamma(conc, size=(S, N, K, F))
    # a column of all-zero draws is astronomically unlikely; guard anyway
    g[g.sum(-1) == 0.0] = 1.0
    return _normalise_f32(g, axis=-1)


def _transitions(rng, S, N, kind, diag):
    A = np.zeros((S, N, N), dtype=np.float64)
    for s in range(S):
        for i in range(N):
            if N == 1:
                A[s, i, i] = 1.0
                continue
            others = np.array([j for j in range(N) if j != i])
            if kind == "dense":
                A[s, i, others] = (1.0 - diag) * rng.dirichlet(np.ones(N - 1))
            else:  # diagonal plus a sparse remainder on a few distinct states
                r = min(3, N - 1)
                pick = rng.choice(others, size=r, replace=False)
                A[s, i, pick] = (1.0 - diag) * rng.dirichlet(np.ones(r))
            A[s, i, i] = diag
    return _normalise_f32(A, axis=-1)


def _markov_states(rng, A, pi, T):
    S, N, _ = A.shape
    D = np.zeros((S, T), dtype=np.int64)
    A64 = A.astype(np.float64)
    A64 /= A64.sum(-1, keepdims=True)
    p0 = pi.astype(np.float64)
    p0 /= p0.sum(-1, keepdims=True)
    for s in range(S):
        D[s, 0] = rng.choice(N, p=p0[s])
        u = rng.random(T)
        cdf = np.cumsum(A64[s], axis=-1)
        for t in range(1, T):
            D[s, t] = min(int(np.searchsorted(cdf[D[s, t - 1]], u[t], side="right")), N - 1)
    return D


def problem_dims(S, N, K):
    return dict(M=S * N * K)


def _sample(rng, S, N, K, F, T, *, dict_conc, trans, diag, weights, loud, quanta,
            gamma=1.0, small_quanta=None):
    W = _dictionaries(rng, S, N, K, F, dict_conc)
    A = _transitions(rng, S, N, trans, diag)
    pi = np.full((S, N), 1.0 / N, dtype=np.float32)
    D = _markov_states(rng, A, pi, T)
    M = S * N * K
    # active[t, k] = 1 iff element k belongs to the dictionary a source is in at t
    active = np.zeros((T, M), dtype=bool)
    for s in range(S):
        base = (s * N + D[s]) * K  # [T]
        for j in range(K):
            active[np.arange(T), base + j] = True
    if weights == "bayes":   # theta_t ~ Dir(1 + gamma * active), the model's own prior
        conc = 1.0 + gamma * active
        g = rng.gamma(conc)
        theta = g / g.sum(-1, keepdims=True)
    else:                    # Dir(1) over the active elements only, zero elsewhere
        g = np.where(active, rng.gamma(1.0, size=(T, M)), 0.0)
        theta = g / g.sum(-1, keepdims=True)
    if small_quanta is not None:
        lo, hi = small_quanta
        v = rng.integers(lo, hi + 1, size=T)
    elif loud:
        v = np.maximum(1, np.round(quanta * np.exp(rng.standard_normal(T)))).astype(np.int64)
    else:
        v = np.full(T, quanta, dtype=np.int64)
    Wfm = W.reshape(M, F).astype(np.float64).T          # F x M
    p = theta @ Wfm.T                                    # T x F, rows sum to 1
    p = np.clip(p, 0.0, None)
    p /= p.sum(-1, keepdims=True)
    V = rng.multinomial(v, p).astype(np.float32)         # T x F
    return dict(V=V, W=W, A=A, pi=pi, states=D, v=v.astype(np.int64))


def make_problem(cfg_id: int, job_id: int = 0, **over) -> dict:
    """One seeded problem of a named workload (0..4).  ``over`` overrides dims."""
    cfg = dict(CONFIGS[int(cfg_id)])
    rng = _rng(cfg_id, job_id)
    if cfg["S"] is None:
        cfg["S"] = int(rng.integers(2, 4))
    if cfg["T"] is None:
        cfg["T"] = int(rng.integers(200, 4001))
    cfg.update(over)
    S, N, K, F, T = (int(cfg[k]) for k in ("S", "N", "K", "F", "T"))
    out = _sample(rng, S, N, K, F, T, dict_conc=cfg["dict_conc"], trans=cfg["trans"],
                  diag=cfg["diag"], weights=cfg["weights"], loud=cfg["loud"],
                  quanta=cfg["quanta"])
    out.update(cfg=int(cfg_id), job=int(job_id), S=S, N=N, K=K, F=F, T=T,
               M=S * N * K, iters=int(cfg["iters"]), gamma=1.0)
    return out


def make_tiny(S=2, N=3, K=2, F=7, T=9, seed=0, *, trans="dense", diag=0.7,
              dict_conc=0.7, weights="bayes", quanta=50, small_quanta=None,
              iters=5) -> dict:
    """A small problem with explicit dims, for pins and edge-case parity."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 99, int(seed), S, N, K, F, T]))
    out = _sample(rng, S, N, K, F, T, dict_conc=dict_conc, trans=trans, diag=diag,
                  weights=weights, loud=False, quanta=quanta, small_quanta=small_quanta)
    out.update(cfg=-1, job=int(seed), S=S, N=N, K=K, F=F, T=T, M=S * N * K,
               iters=int(iters), gamma=1.0)
    return out


def make_nhmm_problem(cfg_id: int, job_id: int = 0, **over) -> dict:
    """Learning one source's N-HMM (Section 2.1): the spectrogram of that source
    alone, drawn from the generative process with the source-model shapes of a
    named workload (one source), and a start for the parameters -- dictionaries
    drawn afresh from Dirichlet(1), uniform per-frame weights, transitions with 1/2
    on the diagonal and the rest uniform, uniform initial states.  ``over``
    overrides dims or sets ``iters``."""
    cfg = dict(CONFIGS[int(cfg_id)])
    cfg.update(S=1, T=cfg["T"] or 1000)
    cfg.update(over)
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 77, int(cfg_id), int(job_id)]))
    N, K, F, T = (int(cfg[k]) for k in ("N", "K", "F", "T"))
    src = _sample(rng, 1, N, K, F, T, dict_conc=cfg["dict_conc"], trans=cfg["trans"], diag=cfg["diag"],
                  weights=cfg["weights"], loud=cfg["loud"], quanta=cfg["quanta"])
    W0 = _normalise_f32(rng.gamma(1.0, size=(N, K, F)) + 1e-3, axis=-1)
    theta0 = np.full((T, N, K), 1.0 / K, dtype=np.float32)
    A0 = np.full((N, N), 0.5 / max(N - 1, 1))
    A0[np.arange(N), np.arange(N)] = 0.5 if N > 1 else 1.0
    return dict(V=src["V"], W=W0, theta=theta0, A=_normalise_f32(A0, axis=-1),
                pi=np.full(N, 1.0 / N, dtype=np.float32), N=N, K=K, F=F, T=T,
                iters=int(cfg.get("iters", 20)), W_true=src["W"][0], A_true=src["A"][0], states=src["states"][0])

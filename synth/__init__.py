"""Seeded synthetic inputs with the shapes of the paper's logistic-regression
workloads.

The paper (Sec. 3.1.1, Sec. 3.2, Sec. 4.1, Sec. 4.2) measures on generated
data of its own that it does not publish: tall N x K design matrices with a
binary response.  This module draws stand-ins for those inputs, and for the
five measured workload shapes (small plain, big plain, storage-precision,
hierarchical groups, serving), from fixed seeds so that every consumer (the
oracle tests, the GPU parity tests and the benchmark) sees the same numbers.

It holds none of the log-posterior or gradient arithmetic.  The response is
drawn from the logistic model through its latent-variable form,
y_n = 1[x_n . beta_true + e_n > 0] with e_n ~ Logistic(0, 1), which has
P(y_n = 1) = 1 / (1 + exp(-x_n . beta_true)) without evaluating any term of the
likelihood.

Large matrices are generated in row chunks, each chunk from its own child of
one ``numpy.random.SeedSequence``, so the values do not depend on the number of
worker threads.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 20131006
CHUNK_ROWS = 1 << 16

# Stream names spawned from each workload's SeedSequence, in a fixed order.
_STREAMS = ("X", "beta_true", "y", "trajectory", "mh_prop", "mh_unif",
            "groups", "arrivals", "extra")


def seed_seq(workload_index: int) -> np.random.SeedSequence:
    return np.random.SeedSequence(ROOT_SEED + int(workload_index))


def streams(ss: np.random.SeedSequence) -> dict:
    kids = ss.spawn(len(_STREAMS))
    return dict(zip(_STREAMS, kids))


def _rng(ss: np.random.SeedSequence) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(ss))


def _n_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def design_matrix(N: int, K: int, ss: np.random.SeedSequence,
                  dtype=np.float32, n_binary: int = 0, p_binary: float = 0.3,
                  out: np.ndarray | None = None) -> np.ndarray:
    """N x K row-major matrix: the first K - n_binary columns N(0, 1), the last
    n_binary columns Bernoulli(p_binary) in {0, 1}."""
    dtype = np.dtype(dtype)
    assert dtype in (np.float32, np.float64)
    assert 0 <= n_binary <= K
    X = np.empty((N, K), dtype) if out is None else out
    nchunks = max(1, -(-N // CHUNK_ROWS))
    kids = ss.spawn(nchunks)
    kc = K - n_binary

    def fill(c: int) -> None:
        a, b = c * CHUNK_ROWS, min(N, (c + 1) * CHUNK_ROWS)
        if a >= b:
            return
        g = _rng(kids[c])
        if kc:
            X[a:b, :kc] = g.standard_normal((b - a, kc), dtype=dtype)
        if n_binary:
            X[a:b, kc:] = (g.random((b - a, n_binary)) < p_binary).astype(dtype)

    if nchunks == 1:
        fill(0)
    else:
        with ThreadPoolExecutor(_n_threads()) as ex:
            list(ex.map(fill, range(nchunks)))
    return X


def true_coefficients(K: int, ss: np.random.SeedSequence) -> np.ndarray:
    """beta_true ~ N(0, 1/K) per component (variance 1/K)."""
    return _rng(ss).standard_normal(K) / math.sqrt(K)


def logistic_labels(X: np.ndarray, beta_true: np.ndarray,
                    ss: np.random.SeedSequence) -> np.ndarray:
    """y_n ~ Bernoulli(sigmoid(x_n . beta_true)) drawn as the sign of
    x_n . beta_true + Logistic(0, 1) noise; linear predictor in float64 on the
    stored values of X."""
    N = X.shape[0]
    y = np.empty(N, np.uint8)
    nchunks = max(1, -(-N // CHUNK_ROWS))
    kids = ss.spawn(nchunks)
    bt = np.asarray(beta_true, np.float64)

    def fill(c: int) -> None:
        a, b = c * CHUNK_ROWS, min(N, (c + 1) * CHUNK_ROWS)
        if a >= b:
            return
        eta = X[a:b].astype(np.float64) @ bt
        eps = _rng(kids[c]).logistic(0.0, 1.0, b - a)
        y[a:b] = (eta + eps > 0.0)

    if nchunks == 1:
        fill(0)
    else:
        with ThreadPoolExecutor(_n_threads()) as ex:
            list(ex.map(fill, range(nchunks)))
    return y


def poisson_counts(X: np.ndarray, beta_true: np.ndarray, ss: np.random.SeedSequence,
                   cap: int = 255) -> np.ndarray:
    """y_n ~ Poisson(exp(x_n . beta_true)) truncated at cap (stored as bytes);
    linear predictor in float64 on the stored values of X, drawn in row
    chunks with their own child seeds."""
    N = X.shape[0]
    y = np.empty(N, np.uint8)
    nchunks = max(1, -(-N // CHUNK_ROWS))
    kids = ss.spawn(nchunks)
    bt = np.asarray(beta_true, np.float64)

    def fill(c: int) -> None:
        a, b = c * CHUNK_ROWS, min(N, (c + 1) * CHUNK_ROWS)
        if a >= b:
            return
        rate = np.exp(X[a:b].astype(np.float64) @ bt)
        y[a:b] = np.minimum(_rng(kids[c]).poisson(rate), cap)

    if nchunks == 1:
        fill(0)
    else:
        with ThreadPoolExecutor(_n_threads()) as ex:
            list(ex.map(fill, range(nchunks)))
    return y


def random_walk(start_mean: np.ndarray, n: int, ss: np.random.SeedSequence,
                start_sd: float = 0.1, step_sd: float = 0.01) -> np.ndarray:
    """beta_0 ~ N(start_mean, start_sd^2 I), beta_{t+1} = beta_t + N(0, step_sd^2 I);
    returns an (n, K) float64 array."""
    g = _rng(ss)
    K = len(start_mean)
    b0 = np.asarray(start_mean, np.float64) + start_sd * g.standard_normal(K)
    steps = step_sd * g.standard_normal((max(n - 1, 0), K))
    traj = np.empty((n, K))
    if n:
        traj[0] = b0
        if n > 1:
            traj[1:] = b0 + np.cumsum(steps, axis=0)
    return traj


def scattered(center: np.ndarray, n: int, sd: float,
              ss: np.random.SeedSequence) -> np.ndarray:
    """n independent draws N(center, sd^2 I): an (n, K) float64 array."""
    g = _rng(ss)
    c = np.asarray(center, np.float64)
    return c + sd * g.standard_normal((n, len(c)))


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

@dataclass
class Plain:
    """One logistic-regression data set with an evaluation schedule."""
    X: np.ndarray              # N x K, float32 or float64, row-major
    y: np.ndarray              # N, uint8 in {0, 1}
    beta_true: np.ndarray      # K, float64
    betas: np.ndarray          # (n_evals, K) float64 evaluation points
    prec: float                # prior precision 1 / sigma^2
    name: str = ""
    meta: dict = field(default_factory=dict)


def plain_small(n_evals: int = 100) -> Plain:
    """Small plain workload: N=10,000, K=20, X float64 ~ N(0, 1),
    beta_true ~ N(0, 1/K), prior sd 10; beta ~ N(beta_true, 0.1^2 I) at n_evals
    points followed by beta = 0."""
    s = streams(seed_seq(0))
    N, K = 10_000, 20
    X = design_matrix(N, K, s["X"], np.float64)
    bt = true_coefficients(K, s["beta_true"])
    y = logistic_labels(X, bt, s["y"])
    betas = np.vstack([scattered(bt, n_evals, 0.1, s["trajectory"]),
                       np.zeros((1, K))])
    return Plain(X, y, bt, betas, 1.0 / 100.0, "plain_small_n10000_k20_f64")


def plain_big(N: int = 4_000_000, K: int = 256, n_evals: int = 1000,
              dtype=np.float32, workload_index: int = 1) -> Plain:
    """Big plain workload: X ~ N(0, 1) with the last round(0.1 K) columns
    Bernoulli(0.3), beta_true ~ N(0, 1/K), prior sd 10, a random-walk beta
    trajectory (start N(beta_true, 0.1^2 I), step N(0, 0.01^2 I))."""
    s = streams(seed_seq(workload_index))
    nb = int(round(0.1 * K))
    X = design_matrix(N, K, s["X"], dtype, n_binary=nb, p_binary=0.3)
    bt = true_coefficients(K, s["beta_true"])
    y = logistic_labels(X, bt, s["y"])
    betas = random_walk(bt, n_evals, s["trajectory"])
    return Plain(X, y, bt, betas, 1.0 / 100.0,
                 f"plain_big_n{N}_k{K}_{np.dtype(dtype).name}",
                 {"n_binary": nb})


def plain_poisson(N: int = 4_000_000, K: int = 256, n_evals: int = 1000,
                  dtype=np.float32) -> Plain:
    """Poisson regression on the big plain shape: X as plain_big (last
    round(0.1 K) columns Bernoulli(0.3)), beta_true ~ N(0, 1/(4K)) so that
    the rates exp(x . beta_true) stay moderate, y ~ Poisson(rate) as bytes,
    prior sd 10, the same random-walk trajectory recipe."""
    s = streams(seed_seq(5))
    nb = int(round(0.1 * K))
    X = design_matrix(N, K, s["X"], dtype, n_binary=nb, p_binary=0.3)
    bt = 0.5 * true_coefficients(K, s["beta_true"])
    y = poisson_counts(X, bt, s["y"])
    betas = random_walk(bt, n_evals, s["trajectory"])
    return Plain(X, y, bt, betas, 1.0 / 100.0,
                 f"plain_poisson_n{N}_k{K}_{np.dtype(dtype).name}", {"n_binary": nb})


def precision_big(N: int = 8_000_000, K: int = 512, n_evals: int = 1000) -> Plain:
    """Storage-precision workload: the big generator at N=8M, K=512 with an
    FP32 reference X (quantised copies are made from it)."""
    return plain_big(N, K, n_evals, np.float32, workload_index=2)


def mh_chain_inputs(K: int, n_steps: int, N: int, workload_index: int = 2):
    """Random-walk Metropolis inputs: proposal increments N(0, s^2 I) with
    s = 2.38/sqrt(K) / sqrt(0.2 N), and log-uniforms for the accept test."""
    s = streams(seed_seq(workload_index))
    sd = 2.38 / math.sqrt(K) / math.sqrt(0.2 * N)
    inc = sd * _rng(s["mh_prop"]).standard_normal((n_steps, K))
    logu = np.log(_rng(s["mh_unif"]).random(n_steps))
    return inc, logu, sd


@dataclass
class Groups:
    """Hierarchical workload: G groups stacked row-wise."""
    X: np.ndarray              # sum(N_g) x K float32
    y: np.ndarray              # sum(N_g) uint8
    offsets: np.ndarray        # G + 1 int64 row offsets
    mu: np.ndarray             # K float64 shared prior mean
    betas: np.ndarray          # (G, K) float64 starting group coefficients
    prec: float                # prior precision 1 / 0.5^2
    steps: np.ndarray | None = None   # (n_steps, G, K) increments, lazily drawn
    name: str = ""


def group_sizes(G: int, ss: np.random.SeedSequence) -> np.ndarray:
    """N_g = clip(round(LogNormal(ln 500, 1.2)), 20, 50,000)."""
    g = _rng(ss)
    return np.clip(np.round(g.lognormal(math.log(500.0), 1.2, G)),
                   20, 50_000).astype(np.int64)


def hierarchical(G: int = 2000, K: int = 32, sizes: np.ndarray | None = None) -> Groups:
    """Hierarchical logistic regression: mu ~ N(0, 1/K), beta_g ~ N(mu, 0.5^2 I),
    X ~ N(0, 1) float32, y per group from its beta_g."""
    s = streams(seed_seq(3))
    if sizes is None:
        sizes = group_sizes(G, s["groups"])
    sizes = np.asarray(sizes, np.int64)
    G = len(sizes)
    off = np.zeros(G + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    X = design_matrix(int(off[-1]), K, s["X"], np.float32)
    mu = true_coefficients(K, s["beta_true"])
    gk = s["extra"].spawn(2)
    betas = mu + 0.5 * _rng(gk[0]).standard_normal((G, K))
    y = np.empty(int(off[-1]), np.uint8)
    ykids = s["y"].spawn(G)
    for g in range(G):
        a, b = off[g], off[g + 1]
        eta = X[a:b].astype(np.float64) @ betas[g]
        y[a:b] = eta + _rng(ykids[g]).logistic(0.0, 1.0, b - a) > 0.0
    return Groups(X, y, off, mu, betas, 1.0 / 0.25, name=f"hier_g{G}_k{K}_f32")


def hierarchical_steps(G: int, K: int, n_steps: int) -> np.ndarray:
    """Per-step random-walk increments N(0, 0.01^2 I) for every group."""
    s = streams(seed_seq(3))
    gk = s["extra"].spawn(2)
    return 0.01 * _rng(gk[1]).standard_normal((n_steps, G, K))


@dataclass
class ServingSpec:
    N: np.ndarray        # per-dataset row counts
    K: np.ndarray        # per-dataset column counts
    dtype: list          # "bf16" or "f32" per dataset


def serving_specs(n_datasets: int = 64) -> ServingSpec:
    """N log-uniform on [1e3, 2e6], K uniform on {8, 32, 128, 512}, storage
    BF16 or FP32 50/50."""
    s = streams(seed_seq(4))
    g = _rng(s["groups"])
    N = np.exp(g.uniform(math.log(1e3), math.log(2e6), n_datasets)).astype(np.int64)
    K = g.choice(np.array([8, 32, 128, 512]), n_datasets)
    dt = ["bf16" if b else "f32" for b in (g.random(n_datasets) < 0.5)]
    return ServingSpec(N, K, dt)


def serving_dataset(i: int, spec: ServingSpec):
    """Data set i of the serving workload: float32 X ~ N(0, 1), beta_true,
    y; the caller quantises to BF16 when spec.dtype[i] says so."""
    s = streams(seed_seq(4))
    kids = s["X"].spawn(len(spec.N))
    k2 = kids[i].spawn(3)
    N, K = int(spec.N[i]), int(spec.K[i])
    X = design_matrix(N, K, k2[0], np.float32)
    bt = true_coefficients(K, k2[1])
    y = logistic_labels(X, bt, k2[2])
    return X, y, bt


def poisson_arrivals(rate: float, n: int, n_chains: int, seed_offset: int = 0):
    """Open-loop Poisson arrivals: n exponential gaps at the given rate (s) and
    a uniformly random chain index for each request."""
    s = streams(seed_seq(4))
    g = _rng(s["arrivals"].spawn(seed_offset + 1)[seed_offset])
    t = np.cumsum(g.exponential(1.0 / rate, n))
    chain = g.integers(0, n_chains, n)
    return t, chain

"""Seeded inputs of the GPU parity sweeps (pure numpy).  The GPU tests and
the CPU negative controls draw the same cases from here, so a control
perturbs exactly the data a sweep evaluates."""
from __future__ import annotations

import math

import numpy as np

# plain FP32 sweep: K covers every lanes-per-row / chunks-per-lane instance
# (16-byte chunks of 4 columns: 1, 2, 4, ..., 64 lanes and 2 or 4 chunks)
F32_K = [4, 8, 16, 32, 64, 128, 256, 512, 1024]
F32_N = [0, 1, 63, 64, 65, 1000, 40_003]
F64_K = [2, 4, 8, 16, 32, 64, 128, 256, 512]
F64_N = [0, 1, 65, 9_001]
BF16_K = [8, 16, 32, 64, 128, 256, 512, 1024, 2048]
FP8_K = [16, 32, 64, 128, 256, 512, 1024, 2048, 4096]
CODES_N = [1, 65, 20_011]
RAGGED_K = [1, 3, 5, 10, 50, 255, 1021]
RAGGED_N = [1, 257, 30_011]
POISSON_K = [4, 13, 64, 256, 1000]
POISSON_N = [1, 777, 40_009]
MULTI_K = [8, 32, 128, 512]
MULTI_NB = [1, 3, 8, 11]
MX_K = [20, 65, 72, 100, 128, 200, 257, 260, 512]
MX_NB = [2, 4, 7]
GROUP_SIZES = [0, 1, 63, 64, 65, 127, 128, 129, 1000, 1025, 5000, 20, 0, 3, 2049, 700]


def plain(N, K, seed, dtype=np.float32, nbin=0):
    """X ~ N(0,1) (last nbin columns Bernoulli(0.3)), y from the logistic model
    at beta_true ~ N(0, 1/K), evaluation point beta_true + N(0, 0.1^2 I)."""
    g = np.random.default_rng(seed)
    X = g.standard_normal((N, K)).astype(dtype)
    if nbin:
        X[:, K - nbin:] = (g.random((N, nbin)) < 0.3)
    beta = g.standard_normal(K) / math.sqrt(K)
    y = (g.random(N) < 1.0 / (1.0 + np.exp(-(X.astype(np.float64) @ beta)))).astype(np.uint8)
    return X, y, beta + 0.1 * g.standard_normal(K)


def plain_f32_case(N, K):
    return plain(N, K, 1000 * K + N % 997)


def plain_f64_case(N, K):
    return plain(N, K, 7 * K + N, np.float64)


def precision_matrix(N, K, seed):
    """FP32 X with 10 % binary columns and a few special values (an exact 0,
    a value below every FP8 step after scaling, a small negative one)."""
    g = np.random.default_rng(seed)
    X = g.standard_normal((N, K)).astype(np.float32)
    X[:, -max(1, K // 10):] = (g.random((N, max(1, K // 10))) < 0.3)
    X[0, 0] = 0.0
    if N > 3 and K > 2:
        X[1, 1] = 1e-30
        X[2, 2] = -7.25e-3
    return X


def codes_case(N, K, kind):
    """(X float32, y, beta) of the BF16 / FP8 sweeps on stored codes."""
    if kind == "bf16":
        X = precision_matrix(N, K, 10 + K)
        g_ = np.random.default_rng(K + N)
    else:
        X = precision_matrix(N, K, 20 + K)
        g_ = np.random.default_rng(K * 3 + N)
    beta = g_.standard_normal(K) / math.sqrt(K)
    y = (g_.random(N) < 0.5).astype(np.uint8)
    return X, y, beta


def ragged_case(N, K):
    g_ = np.random.default_rng(K * 7 + N)
    X = g_.standard_normal((N, K)).astype(np.float32)
    y = (g_.random(N) < 0.5).astype(np.uint8)
    beta = g_.standard_normal(K) / math.sqrt(K)
    return X, y, beta


def serving_data(N, K, seed, dtype=np.float32):
    """X, y and beta_true of the several-beta and server tests."""
    g = np.random.default_rng(seed)
    X = g.standard_normal((N, K)).astype(dtype)
    bt = g.standard_normal(K) / math.sqrt(K)
    y = (g.random(N) < 1.0 / (1.0 + np.exp(-(X.astype(np.float64) @ bt)))).astype(np.uint8)
    return X, y, bt


def betas_near(bt, n, seed):
    return bt + 0.1 * np.random.default_rng(seed).standard_normal((n, len(bt)))


def poisson(N, K, seed, dtype=np.float32):
    """Counts y ~ Poisson(exp(x beta_true)) (capped at 255), beta_true ~
    N(0, 0.25/K); evaluation point beta_true + N(0, 0.05^2 I)."""
    g = np.random.default_rng(seed)
    X = g.standard_normal((N, K)).astype(dtype)
    bt = 0.5 * g.standard_normal(K) / math.sqrt(K)
    y = np.minimum(g.poisson(np.exp(X.astype(np.float64) @ bt)), 255).astype(np.uint8)
    return X, y, bt + 0.05 * g.standard_normal(K)


def groups(sizes, K, seed, dtype=np.float32):
    """Stacked groups of the given sizes: (X, y, offsets, betas G x K)."""
    g = np.random.default_rng(seed)
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    X = g.standard_normal((int(off[-1]), K)).astype(dtype)
    B = g.standard_normal((len(sizes), K)) / math.sqrt(K)
    y = (g.random(int(off[-1])) < 0.5).astype(np.uint8)
    return X, y, off, B

"""FP64 CPU oracle for the logistic-regression log-posterior and gradient.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg use this package; the GPU library never imports,
links or calls it, and the two share no code.  The arithmetic lives in
``glm_oracle.c`` (plain C, IEEE double, ascending-row compensated sums); this
module builds it with gcc and marshals numpy arrays into it.

Every function follows the plain definition of the quantity (Sec. 3.1.1
eq-loglike-binlogit for the likelihood, Sec. 4.2 eq-grad-compact for the
gradient, a Gaussian prior N(m, prec^-1 I)):

    f(beta) = sum_n [y_n u_n - softplus(u_n)] - prec/2 |beta - m|^2
    g(beta) = X^t (y - sigmoid(u)) - prec (beta - m),    u = X beta.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "glm_oracle.c")
LIB = os.path.join(HERE, "libglm_oracle.so")

F64, F32, BF16, FP8 = 0, 1, 2, 3
FAMILIES = {"logistic": 0, "poisson": 1}
_DT = {np.dtype(np.float64): F64, np.dtype(np.float32): F32}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off",
                               "-std=c11", "-Wall", "-shared", "-fPIC", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        P, I64, I, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.orc_logpost_grad.argtypes = [P, I, I64, P, P, I64, I, P, D, P, I, P]
        L.orc_logpost_grad_multi.argtypes = [P, I, I64, P, P, I64, I, P, I, D, P, I, P]
        L.orc_linpred.argtypes = [P, I, I64, P, I64, I, P, P]
        L.orc_hessian.argtypes = [P, I, I64, P, I64, I, P, D, I, P]
        L.orc_logpost_grad_groups.argtypes = [P, I, I64, P, P, P, I, I, P, D, P, I, I, P]
        L.orc_quantize_bf16.argtypes = [P, I64, I, I64, P, I64]
        L.orc_fp8_col_scales.argtypes = [P, I64, I, I64, P]
        L.orc_quantize_fp8.argtypes = [P, I64, I, I64, P, P, I64]
        L.orc_bf16_to_double.argtypes = [ctypes.c_uint16]
        L.orc_bf16_to_double.restype = D
        L.orc_fp8_to_double.argtypes = [ctypes.c_uint8]
        L.orc_fp8_to_double.restype = D
        L.orc_softplus.argtypes = [D]
        L.orc_softplus.restype = D
        L.orc_sigmoid.argtypes = [D]
        L.orc_sigmoid.restype = D
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _xinfo(X, dtype):
    """Returns (dtype code, ldx, row-major array) for a 2-D X; integer arrays
    are raw codes whose format is named by dtype ('bf16' or 'fp8')."""
    X = np.asarray(X)
    assert X.ndim == 2
    if dtype is None:
        code = _DT[X.dtype]
    else:
        code = {"f64": F64, "f32": F32, "bf16": BF16, "fp8": FP8}[dtype]
    want = {F64: np.float64, F32: np.float32, BF16: np.uint16, FP8: np.uint8}[code]
    assert X.dtype == want, (X.dtype, want)
    if X.shape[0] == 0:
        return code, X.shape[1], X
    if X.strides[1] != X.itemsize or X.strides[0] % X.itemsize or X.strides[0] < X.strides[1] * X.shape[1]:
        X = np.ascontiguousarray(X)
    return code, X.strides[0] // X.itemsize, X


def logpost_grad(X, y, beta, prec, mean=None, dtype=None, scale=None, family="logistic"):
    """f and g at one beta.  X: float64/float32 array, or uint16 (dtype='bf16')
    / uint8 (dtype='fp8' with FP32 column scales) codes; family 'logistic'
    (y in {0, 1}) or 'poisson' (y counts).  Returns (f, g)."""
    code, ldx, X = _xinfo(X, dtype)
    N, K = X.shape
    y = np.ascontiguousarray(y, np.uint8)
    assert y.shape == (N,)
    beta = np.ascontiguousarray(beta, np.float64)
    mean = None if mean is None else np.ascontiguousarray(mean, np.float64)
    scale = None if scale is None else np.ascontiguousarray(scale, np.float32)
    out = np.empty(1 + K)
    rc = lib().orc_logpost_grad(_p(X), code, ldx, _p(scale), _p(y), N, K, _p(beta),
                                float(prec), _p(mean), FAMILIES[family], _p(out))
    if rc:
        raise ValueError("oracle rejected its arguments")
    return out[0], out[1:].copy()


def row_blocks(N: int, parts: int):
    """[a, b) row ranges splitting N rows into at most `parts` blocks."""
    b = np.linspace(0, N, max(1, parts) + 1).astype(np.int64)
    return [(int(b[i]), int(b[i + 1])) for i in range(len(b) - 1) if b[i + 1] > b[i]]


def logpost_grad_blocks(X, y, beta, prec, mean=None, threads=None, dtype=None, scale=None,
                        family="logistic", pool=None):
    """logpost_grad over row blocks in host threads (the C code releases the
    interpreter lock).  Each block is evaluated with the prior left out, the
    block values are added in block order with math.fsum (per component of
    g too) and the prior is added once: the likelihood is a sum over rows, so
    this is the same quantity (row-split additivity, pinned by the oracle
    tests).  Returns (f, g)."""
    X = np.asarray(X)
    N, K = X.shape
    threads = threads or max(1, min(16, os.cpu_count() or 1))
    blocks = row_blocks(N, 4 * threads)

    def one(ab):
        a, b = ab
        return logpost_grad(X[a:b], y[a:b], beta, 0.0, None, dtype, scale, family)

    if pool is None:
        with ThreadPoolExecutor(threads) as ex:
            parts = list(ex.map(one, blocks))
    else:
        parts = list(pool.map(one, blocks))
    beta = np.asarray(beta, np.float64)
    d = beta - (0.0 if mean is None else np.asarray(mean, np.float64))
    f = math.fsum([p[0] for p in parts]) - 0.5 * prec * math.fsum(d * d)
    G = np.array([p[1] for p in parts]).reshape(len(parts), K)
    g = np.array([math.fsum(G[:, k]) for k in range(K)]) - prec * d
    return f, g


def linpred(X, beta, dtype=None, scale=None):
    """u = X beta in FP64 (k order) for every row."""
    code, ldx, X = _xinfo(X, dtype)
    N, K = X.shape
    beta = np.ascontiguousarray(beta, np.float64)
    scale = None if scale is None else np.ascontiguousarray(scale, np.float32)
    u = np.empty(N)
    if lib().orc_linpred(_p(X), code, ldx, _p(scale), N, K, _p(beta), _p(u)):
        raise ValueError("oracle rejected its arguments")
    return u


def hessian(X, beta, prec, dtype=None, scale=None, family="logistic"):
    """H = -X^t W X - prec I at beta (K x K, FP64)."""
    code, ldx, X = _xinfo(X, dtype)
    N, K = X.shape
    beta = np.ascontiguousarray(beta, np.float64)
    scale = None if scale is None else np.ascontiguousarray(scale, np.float32)
    H = np.empty((K, K))
    if lib().orc_hessian(_p(X), code, ldx, _p(scale), N, K, _p(beta), float(prec),
                         FAMILIES[family], _p(H)):
        raise ValueError("oracle rejected its arguments")
    return H


def logpost_grad_multi(X, y, betas, prec, means=None, dtype=None, scale=None, family="logistic"):
    """Several betas (b x K) on one data set; returns a b x (1 + K) array."""
    code, ldx, X = _xinfo(X, dtype)
    N, K = X.shape
    y = np.ascontiguousarray(y, np.uint8)
    betas = np.ascontiguousarray(betas, np.float64).reshape(-1, K)
    means = None if means is None else np.ascontiguousarray(means, np.float64).reshape(-1, K)
    scale = None if scale is None else np.ascontiguousarray(scale, np.float32)
    out = np.empty((betas.shape[0], 1 + K))
    rc = lib().orc_logpost_grad_multi(_p(X), code, ldx, _p(scale), _p(y), N, K, _p(betas),
                                      betas.shape[0], float(prec), _p(means), FAMILIES[family],
                                      _p(out))
    if rc:
        raise ValueError("oracle rejected its arguments")
    return out


def logpost_grad_groups(X, y, offsets, betas, prec, mean=None, dtype=None, scale=None,
                        family="logistic"):
    """Hierarchical groups stacked row-wise; returns a G x (1 + K) array."""
    code, ldx, X = _xinfo(X, dtype)
    K = X.shape[1]
    y = np.ascontiguousarray(y, np.uint8)
    offsets = np.ascontiguousarray(offsets, np.int64)
    G = len(offsets) - 1
    betas = np.ascontiguousarray(betas, np.float64).reshape(G, K)
    per_group = 0
    if mean is not None:
        mean = np.ascontiguousarray(mean, np.float64)
        per_group = int(mean.ndim == 2)
    scale = None if scale is None else np.ascontiguousarray(scale, np.float32)
    out = np.empty((G, 1 + K))
    rc = lib().orc_logpost_grad_groups(_p(X), code, ldx, _p(scale), _p(y), _p(offsets), G, K,
                                       _p(betas), float(prec), _p(mean), per_group,
                                       FAMILIES[family], _p(out))
    if rc:
        raise ValueError("oracle rejected its arguments")
    return out


def quantize_bf16(X):
    X = np.ascontiguousarray(X, np.float32)
    N, K = X.shape
    Q = np.empty((N, K), np.uint16)
    assert lib().orc_quantize_bf16(_p(X), N, K, K, _p(Q), K) == 0
    return Q


def fp8_col_scales(X):
    X = np.ascontiguousarray(X, np.float32)
    N, K = X.shape
    s = np.empty(K, np.float32)
    assert lib().orc_fp8_col_scales(_p(X), N, K, K, _p(s)) == 0
    return s


def quantize_fp8(X, scale=None):
    """Returns (codes uint8 N x K, scales float32 K)."""
    X = np.ascontiguousarray(X, np.float32)
    N, K = X.shape
    s = fp8_col_scales(X) if scale is None else np.ascontiguousarray(scale, np.float32)
    Q = np.empty((N, K), np.uint8)
    assert lib().orc_quantize_fp8(_p(X), N, K, K, _p(s), _p(Q), K) == 0
    return Q, s


def decode_bf16(Q):
    """BF16 codes -> float64 values (exact)."""
    Q = np.asarray(Q, np.uint16)
    return (Q.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def decode_fp8(Q, scale=None):
    """FP8 E4M3FN codes -> float64 values (times the column scales if given)."""
    L = lib()
    table = np.array([L.orc_fp8_to_double(i) for i in range(256)])
    v = table[np.asarray(Q, np.uint8)]
    return v if scale is None else v * np.asarray(scale, np.float32).astype(np.float64)


def softplus(u: float) -> float:
    return lib().orc_softplus(float(u))


def sigmoid(u: float) -> float:
    return lib().orc_sigmoid(float(u))

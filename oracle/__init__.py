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
        U64p = ctypes.POINTER(ctypes.c_uint64)
        L.orc_philox4x64_10.argtypes = [U64p, U64p, U64p]
        L.orc_u01.argtypes = [ctypes.c_uint64]
        L.orc_u01.restype = D
        L.orc_polar_pair.argtypes = [ctypes.c_uint64] * 5 + [ctypes.POINTER(D)]
        L.orc_polar_pair.restype = I
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


# ---------------------------------------------------------------- random numbers
#
# Counter-based Philox4x64-10 (Salmon et al., SC'11) and the streams the
# library's on-device generator defines on it (purposes: 1 uniforms, 2
# normals, 16 HMC momenta, 17 HMC accept uniforms; key = (seed, chain)).

RNG_UNIFORM, RNG_NORMAL, RNG_HMC_MOMENTUM, RNG_HMC_ACCEPT = 1, 2, 16, 17


def philox(ctr, key):
    """The Philox4x64-10 block of a four-word counter under a two-word key."""
    c = (ctypes.c_uint64 * 4)(*[int(v) & (2**64 - 1) for v in ctr])
    k = (ctypes.c_uint64 * 2)(*[int(v) & (2**64 - 1) for v in key])
    o = (ctypes.c_uint64 * 4)()
    lib().orc_philox4x64_10(c, k, o)
    return np.array(list(o), np.uint64)


def u01(w) -> float:
    """Uniform in (0, 1) from a 64-bit word (top 52 bits plus one half, times
    2^-52)."""
    return lib().orc_u01(int(w))


def rng_uniforms(seed, chain, stream, offset, n, purpose=RNG_UNIFORM):
    """Uniforms offset .. offset + n - 1 of a stream: value i is word i mod 4
    of the block at counter (i / 4, 0, purpose, stream)."""
    out = np.empty(n)
    blk, cache = None, None
    for j in range(n):
        i = offset + j
        if i // 4 != blk:
            blk = i // 4
            cache = philox((blk, 0, purpose, stream), (seed, chain))
        out[j] = u01(cache[i % 4])
    return out


def polar_pair(seed, chain, purpose, stream, p):
    """Normals 2p and 2p + 1 of a stream (Marsaglia's polar method) and the
    attempts it took."""
    z = (ctypes.c_double * 2)()
    a = lib().orc_polar_pair(int(seed), int(chain), int(purpose), int(stream), int(p), z)
    return z[0], z[1], a


def rng_normals(seed, chain, stream, offset, n, purpose=RNG_NORMAL):
    """Standard normals offset .. offset + n - 1 of a stream (value i is
    component i mod 2 of pair i / 2)."""
    out = np.empty(n)
    for j in range(n):
        i = offset + j
        out[j] = polar_pair(seed, chain, purpose, stream, i // 2)[i % 2]
    return out


# ---------------------------------------------------------------- HMC
#
# Hamiltonian Monte Carlo, named in Sec. 4.2 among the samplers that use the
# gradient.  The algorithm is the standard one (R. M. Neal, "MCMC using
# Hamiltonian dynamics", Handbook of MCMC, 2011): momenta p ~ N(0, I), the
# leapfrog integrator with step eps for n_leap steps on H = -f(beta) + p.p/2,
# then a Metropolis correction accepting iff log U < H(start) - H(end).  The
# random numbers come from the library's streams above: iteration t draws its
# K momenta from purpose RNG_HMC_MOMENTUM, stream t (normal k of the
# iteration), and its accept uniform as word 0 of the block at counter
# (0, 0, RNG_HMC_ACCEPT, t).


def hmc_momenta(seed, chain, t, K):
    return rng_normals(seed, chain, t, 0, K, purpose=RNG_HMC_MOMENTUM)


def hmc_log_u(seed, chain, t) -> float:
    return math.log(u01(philox((0, 0, RNG_HMC_ACCEPT, t), (seed, chain))[0]))


def leapfrog(grad_f, beta, g, p, eps, n_leap):
    """n_leap leapfrog steps from (beta, p) with g = grad f(beta): half a
    momentum step, then alternating full position and momentum steps, and a
    closing half momentum step.  grad_f(b) returns (f, g).  Returns (beta, p,
    f, g) at the end."""
    p = p + 0.5 * eps * g
    f = None
    for l in range(n_leap):
        beta = beta + eps * p
        f, g = grad_f(beta)
        if l < n_leap - 1:
            p = p + eps * g
    p = p + 0.5 * eps * g
    return beta, p, f, g


def hmc_chain(X, y, beta0, prec, n_iter, n_leap, eps, seed, chain, mean=None, follow=None,
              iter0=0, **kw):
    """n_iter HMC iterations (t = iter0 .. iter0 + n_iter - 1) from beta0 with
    the oracle's f and g.  follow:
    optional sequence of accept decisions to take instead of the oracle's own
    (for replaying a chain whose decisions were taken elsewhere).  Returns a
    dict with the final beta, f, g, the decisions, the oracle's log U and
    H(start) - H(end) of every iteration and the f trace."""
    def fg(b):
        return logpost_grad(X, y, b, prec, mean, **kw)

    beta = np.asarray(beta0, np.float64).copy()
    f, g = fg(beta)
    K = beta.size
    acc = np.zeros(n_iter, np.uint8)
    dH = np.zeros(n_iter)
    logu = np.zeros(n_iter)
    trace = np.zeros(n_iter)
    for j in range(n_iter):
        t = iter0 + j
        p0 = hmc_momenta(seed, chain, t, K)
        b1, p1, f1, g1 = leapfrog(fg, beta, g, p0, eps, n_leap)
        dH[j] = (f1 - 0.5 * float(p1 @ p1)) - (f - 0.5 * float(p0 @ p0))
        logu[j] = hmc_log_u(seed, chain, t)
        a = logu[j] < dH[j] if follow is None else bool(follow[j])
        acc[j] = a
        if a:
            beta, f, g = b1, f1, g1
        trace[j] = f
    return {"beta": beta, "f": f, "g": g, "accepted": acc, "dH": dH, "logu": logu,
            "f_trace": trace}

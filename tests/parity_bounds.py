"""Error bounds of the GPU kernels' arithmetic, and the checker that holds a
GPU result to them.  Pure numpy: the CPU negative-control tests apply the same
checker to oracle results on perturbed data.

Summation structure the bounds are built from.  A row of K stored values is
read as 16-byte chunks of VE = 16 / size values; NC = ceil(K / VE) chunks
are spread over LPR = min(64, pow2ceil(NC)) lanes, CPL = 1 chunk per lane up
to 64 chunks, else pow2ceil(NC / 64).

  u_n  vector ALU kernels, every storage type: each stored value is exact
       in FP64; each lane adds its CPL * VE products into an FP64 FMA chain,
       then log2(LPR) butterfly additions in FP64 combine the lanes.  A
       product therefore meets at most m = CPL * VE + log2(LPR) + 1 roundings
       of unit 2^-53: |du_n| <= gamma_m A_n with A_n = sum_k |x_nk beta_k|
       (the bound adds K more, for the oracle's own dot product).  FP8: the
       column scale is folded into beta in FP64 (one rounding of beta).
       BF16 several-beta passes on the matrix cores: beta in four BF16 pieces,
       each accumulated in FP32 over LPR / 4 instructions of 32 exact products;
       the bound takes every one of the 32 + LPR / 4 additions as a rounding
       and the unit as 2^-23 (no assumption on how an instruction rounds
       inside).
  t_n, r_n   FP64 per-row map; r is rounded to FP32 for the products.
  g    FP32 products r_n x_nk summed over at most R = 16 rows, then FP64.
  f    FP64 from each row's t_n; every cross-lane, cross-wave and cross-block
       sum is FP64.

Error of beta's representation (the FP8 fold: 2^-53 |beta|; four BF16
pieces: 2^-31 |beta|): it is the same for every row, so its effect enters
at its worst case.

Two bounds are checked for every f and every g_k, and the result must meet
the smaller one:
  * worst case (rigorous): every rounding at its largest magnitude;
  * probabilistic: rounding errors are independent random variables of mean
    zero (the model of Higham & Mary, "A new approach to probabilistic
    rounding error analysis", SIAM J. Sci. Comput. 41(5), 2019).  The error of
    a sum over rows is then a sum of independent, bounded, mean-zero terms,
    and Hoeffding's inequality bounds it by LAMBDA * sqrt(sum of the squared
    per-term bounds), failing with probability at most 2 exp(-LAMBDA^2 / 2)
    (2.5e-14 for LAMBDA = 8).  The FP32 partial gradient sums are terms of
    their own: by Cauchy-Schwarz their squared bounds add up to at most
    R (R-1)^2 2^-48 sum_n (r_n x_nk)^2 whatever rows they group.
Terms that are the same for every row (the split of beta), one-signed (the
second-order term of the per-row map) or FP64 (sums, per-row functions, the
oracle's own rounding, the prior) enter both bounds at their worst case.

At beta = 0 every u_n is exactly 0, so t_n = -log 2, r_n = y_n - 1/2 and every
product is exact: the bounds reduce to the FP32 partial sums of g and the FP64
terms, which is why each sweep also checks beta = 0 (a dropped, repeated or
relabelled row then shows at once).
"""
from __future__ import annotations

import math

import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53
LAMBDA = 8.0
R_MAX = 16                     # rows of one FP32 gradient partial
ES = {"f64": 8, "f32": 4, "bf16": 2, "fp8": 1}


def _pow2ceil(v: int) -> int:
    p = 1
    while p < v:
        p <<= 1
    return p


def layout(K: int, storage: str):
    """(VE, NC, LPR, CPL) of a row of K values in the given storage."""
    ve = 16 // ES[storage]
    nc = max(1, -(-K // ve))
    lpr = min(64, _pow2ceil(nc))
    cpl = 1 if nc <= 64 else _pow2ceil(-(-nc // 64))
    return ve, nc, lpr, cpl


def _gamma(m: int, unit: float) -> float:
    return m * unit / (1.0 - m * unit)


def u_model(K: int, storage: str, form: str = "any"):
    """(gamma, piece factor, beta split residual) of the linear predictor.

    form: 'valu' (vector ALU kernels), 'mx' (matrix-core several-beta kernel,
    BF16 rows of 9 to 64 chunks) or 'any' (the larger of the two where the
    library may pick either)."""
    ve, nc, lpr, cpl = layout(K, storage)
    valu = (_gamma(cpl * ve + int(math.log2(lpr)) + 1 + K, U64), 1.0,
            U64 if storage == "fp8" else 0.0)
    if storage == "f64":
        return valu
    mx_ok = storage == "bf16" and 9 <= nc <= 64
    mx = (_gamma(32 + lpr // 4 + 1, 2.0 ** -23), 1.0 + 2.0 ** -7, 2.0 ** -31)
    if form == "mx":
        assert mx_ok, "the matrix-core form covers BF16 rows of 9 to 64 chunks"
        return mx
    if form == "any" and mx_ok:
        return tuple(max(a, b) for a, b in zip(valu, mx))
    return valu


def error_bounds(Xd, y, beta, prec=0.0, mean=None, storage="f32", family="logistic",
                 form="any"):
    """Worst-case and probabilistic bounds on |f_gpu - f_oracle| and on every
    |g_gpu,k - g_oracle,k|, for decoded X (float64) and the given beta."""
    Xd = np.asarray(Xd, np.float64)
    N, K = Xd.shape
    beta = np.asarray(beta, np.float64)
    m = np.zeros(K) if mean is None else np.asarray(mean, np.float64)
    yv = np.asarray(y).astype(np.float64)
    f64 = storage == "f64"
    gam, piece, split = u_model(K, storage, form)
    aX = np.abs(Xd)
    X2 = Xd * Xd
    u = Xd @ beta
    A = aX @ np.abs(beta)
    du_rand = gam * piece * A + 2 * U64 * np.abs(u)            # per row, random
    du_sys = aX @ (split * np.abs(beta))                        # same split for every row
    du = du_rand + du_sys
    if family == "poisson":
        mu = np.exp(u)
        r = yv - mu
        slope = mu * np.exp(du)                                 # |dr/du| on the interval
        curv = slope                                            # |d2r/du2|, |d2t/du2|
        tmag = np.abs(yv * u) + mu
    else:
        sig = 0.5 * (1.0 + np.tanh(0.5 * u))
        r = yv - sig
        slope = np.full(N, 0.25)
        curv = np.full(N, 0.1)                                  # |sigma''| <= 0.0963
        tmag = np.abs(yv * u) + np.logaddexp(0.0, u)
    ar = np.abs(r)
    gl = Xd.T @ r                                               # likelihood gradient
    sum_arx = aX.T @ ar                                         # sum_n |r_n x_nk|

    # ---- f
    b_f = ar * du_rand                                          # per-row random terms
    f_sys = np.sum(split * piece * np.abs(beta) * (np.abs(gl) + N * U64 * sum_arx))
    f_2nd = np.sum(curv * du * du) / 2
    f_fp64 = ((N / 8 + 512) * U64 + 16 * U64) * np.sum(tmag)   # FP64 sums, per-row functions
    f_orc = np.sum(ar * K * U64 * A) + 4 * U64 * np.sum(tmag)
    d = beta - m
    f_pri = (K + 4) * U64 * 0.5 * prec * np.dot(d, d)
    f_det = f_sys + f_2nd + f_fp64 + f_orc + f_pri
    f_worst = np.sum(b_f) + f_det
    f_prob = f_worst if f64 else LAMBDA * math.sqrt(np.sum(b_f * b_f)) + f_det

    # ---- g: per-row terms |x_nk| c_n, sums over rows as products with |X|, X^2
    if f64:
        g_worst = aX.T @ (slope * du) + (N + 64) * U64 * sum_arx
        g_prob = None
    else:
        c = slope * du_rand + 2 * U32 * ar                      # + r rounding, product rounding
        part = R_MAX * (R_MAX - 1) ** 2 * U32 * U32 * (X2.T @ (ar * ar))
        g_worst = aX.T @ c + (R_MAX - 1) * U32 * sum_arx
        g_prob = LAMBDA * np.sqrt(X2.T @ (c * c) + part)
    g_det = (aX.T @ (slope * du_sys + curv * du * du / 2 + slope * K * U64 * A)
             + ((N / 8 + 512) * U64 + 4 * U64) * sum_arx        # FP64 sums, oracle sums
             + 4 * U64 * np.abs(gl) + 4 * U64 * prec * np.abs(d))
    g_worst = g_worst + g_det
    g_prob = g_worst if g_prob is None else g_prob + g_det
    return {"f_worst": float(f_worst), "f_prob": float(f_prob),
            "g_worst": g_worst, "g_prob": g_prob}


def oracle_ref(oracle, X_oracle, y, beta, prec, mean=None, oracle_kw=None):
    return oracle.logpost_grad(X_oracle, y, beta, prec, mean, **(oracle_kw or {}))


def check(got_f, got_g, Xd, y, beta, prec, mean=None, storage="f32", family="logistic",
          form="any", ref=None, oracle=None, X_oracle=None, oracle_kw=None, bounds=None):
    """Asserts |got - ref| within the smaller of the two bounds for f and for
    every g_k; ref = (f, g) of the oracle (computed here when not given).
    bounds: the result of error_bounds for the same arguments, when already
    computed.  Returns a dict with the relative errors and the worst bound
    usage."""
    if ref is None:
        okw = dict(oracle_kw or {})
        okw.setdefault("family", family)
        ref = oracle_ref(oracle, Xd if X_oracle is None else X_oracle, y, beta, prec, mean, okw)
    f, g = ref
    got_g = np.asarray(got_g, np.float64)
    assert np.isfinite(got_f) and np.all(np.isfinite(got_g)), "non-finite result"
    b = bounds or error_bounds(Xd, y, beta, prec, mean, storage, family, form)
    bf = min(b["f_worst"], b["f_prob"])
    bg = np.minimum(b["g_worst"], b["g_prob"])
    ef = abs(got_f - f)
    eg = np.abs(got_g - g)
    assert ef <= bf, f"|df| = {ef:.3e} > bound {bf:.3e} (f = {f!r}, got {got_f!r})"
    bad = np.nonzero(eg > bg)[0]
    assert bad.size == 0, f"g[{bad[:5]}] errors {eg[bad[:5]]} > bounds {bg[bad[:5]]}"
    return {"f_rel": ef / max(abs(f), 1e-300),
            "g_rel": float(np.linalg.norm(got_g - g) / max(np.linalg.norm(g), 1e-300)),
            "f_use": ef / bf if bf > 0 else 0.0,
            "g_use": float(np.max(eg / np.maximum(bg, 1e-300))) if len(eg) else 0.0}

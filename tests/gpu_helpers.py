"""Shared helpers of the GPU parity tests: device evaluation through the C
interface, and error bounds derived from the kernels' arithmetic.

Derived bounds (first order, worst case).  For storage in FP32, BF16 or FP8
the kernels form u_n as an FP32 sum of K products with the FP64 beta split
into two FP32 parts, so |du_n| <= gamma * A_n with A_n = sum_k |x_nk beta_k|
and gamma = (K + 2) 2^-24.  The per-row terms are then evaluated in FP64, so
|dt_n| <= |r_n| |du_n| and |dr_n| <= |du_n| / 4 + 2^-24 |r_n| (r is rounded to
FP32 for the products).  Gradient products and their partial sums over at
most 16 rows are FP32 (relative error <= 18 * 2^-24), then FP64.  Hence

    |df|   <= gamma sum_n |r_n| A_n
    |dg_k| <= sum_n |x_nk| (gamma A_n / 4 + 20 * 2^-24 |r_n|)

plus FP64 rounding, which the bounds cover with a 1e-12 relative margin.
For FP64 storage gamma = (K + 2) 2^-53 and the accumulation terms use 2^-53
per row of the longest per-lane chain.  For the Poisson model r = y - exp(u),
so |dr| <= exp(u) |du| + 2^-24 |r| takes the place of the 1/4 above.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_1310_1537_amd import glm

DEV = torch.device("cuda:0")


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


class Ctx:
    def __init__(self):
        self.h = glm.glm_create(0)

    def close(self):
        if self.h:
            glm.glm_destroy(self.h)
            self.h = None


def eval_gpu(ctx: int, X: torch.Tensor, y: torch.Tensor, beta: np.ndarray, prec: float,
             mean: np.ndarray | None = None, dtype=None, scale=None, stream=None, ds=None,
             family: int = 0):
    """f, g on the GPU through glm_logpost_grad (registers a data set unless
    ds is given)."""
    own = ds is None
    if own:
        ds = glm.glm_dataset_register(ctx, glm.make_desc(X, y, dtype=dtype, col_scale=scale,
                                                         family=family))
    K = X.shape[1]
    b = to_dev(np.asarray(beta, np.float64))
    m = None if mean is None else to_dev(np.asarray(mean, np.float64))
    out = torch.full((1 + K,), float("nan"), dtype=torch.float64, device=DEV)
    glm.glm_logpost_grad(ctx, ds, b, glm.make_prior(prec, m), out, stream)
    torch.cuda.synchronize()
    if own:
        glm.glm_dataset_unregister(ctx, ds)
    o = out.cpu().numpy()
    return o[0], o[1:].copy()


def bounds(Xd: np.ndarray, y: np.ndarray, beta: np.ndarray, f_ref: float, g_ref: np.ndarray,
           storage: str = "f32", family: str = "logistic"):
    """(bound on |df|, per-component bound on |dg|) for the given decoded X.
    The residual's sensitivity |dr/du| is 1/4 for the logistic model and
    exp(u) for the Poisson one."""
    K = Xd.shape[1]
    eps = 2.0 ** -53 if storage == "f64" else 2.0 ** -24
    gamma = (K + 2) * eps
    u = Xd @ beta
    yv = y.astype(np.float64)
    if family == "poisson":
        mu = np.exp(u)
        r, slope, tmag = yv - mu, mu, np.abs(yv * u) + mu
    else:
        r, slope, tmag = yv - 0.5 * (1.0 + np.tanh(0.5 * u)), 0.25, np.abs(u) + 1
    A = np.abs(Xd) @ np.abs(beta)
    acc = (np.abs(r) * 20 * eps) if storage != "f64" else (np.abs(r) * (len(y) + 20) * eps)
    bf = gamma * np.sum(np.abs(r) * A) + 1e-12 * abs(f_ref) + 1e-12 * np.sum(tmag)
    if storage == "f64":
        bf += (len(y) + 64) * eps * np.sum(tmag)
    bg = (np.abs(Xd).T @ (gamma * A * slope + acc) + 1e-12 * (np.abs(Xd).T @ np.abs(r))
          + 1e-12 * np.abs(g_ref))
    return bf, bg


def check_against_oracle(got_f, got_g, Xd, y, beta, prec, mean=None, storage="f32",
                         X_for_oracle=None, oracle_kw=None):
    """Compares a GPU result with the oracle within the derived bounds;
    returns (f rel err, g rel-norm err)."""
    oracle_kw = oracle_kw or {}
    Xo = Xd if X_for_oracle is None else X_for_oracle
    f, g = oracle.logpost_grad(Xo, y, beta, prec, mean, **oracle_kw)
    bf, bg = bounds(Xd, y, beta, f, g, storage, oracle_kw.get("family", "logistic"))
    ef = abs(got_f - f)
    eg = np.abs(got_g - g)
    assert np.isfinite(got_f) and np.all(np.isfinite(got_g))
    assert ef <= bf, f"|df| = {ef:.3e} > bound {bf:.3e} (f = {f!r}, got {got_f!r})"
    bad = np.nonzero(eg > bg)[0]
    assert bad.size == 0, f"g[{bad[:5]}] errors {eg[bad[:5]]} > bounds {bg[bad[:5]]}"
    return ef / max(abs(f), 1e-300), np.linalg.norm(got_g - g) / max(np.linalg.norm(g), 1e-300)

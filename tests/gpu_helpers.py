"""Shared helpers of the GPU parity tests: device evaluation through the C
interface, and the parity check against the oracle.

The check (tests/parity_bounds.py) holds every f and every g_k to bounds
derived from the kernels' own summation structure, worst case and
probabilistic, whichever is smaller.  Sweeps also evaluate beta = 0, where u
is exact and a single dropped, repeated or relabelled row is outside the
bound at every size (the CPU negative controls check that).
"""
from __future__ import annotations

import numpy as np
import torch

import oracle
import parity_bounds as pb
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


def check_against_oracle(got_f, got_g, Xd, y, beta, prec, mean=None, storage="f32",
                         X_for_oracle=None, oracle_kw=None, form="any", ref=None):
    """Compares a GPU result with the oracle within the derived bounds;
    returns a dict with the relative errors (f_rel, g_rel norm-wise) and the
    fraction of the bound used (f_use, g_use)."""
    okw = dict(oracle_kw or {})
    family = okw.get("family", "logistic")
    return pb.check(got_f, got_g, Xd, y, beta, prec, mean, storage, family, form, ref=ref,
                    oracle=oracle, X_oracle=X_for_oracle, oracle_kw=okw)


def sweep_point(ctx, X, y, Xd, y_host, beta, prec, mean=None, storage="f32", dtype=None,
                scale=None, X_for_oracle=None, oracle_kw=None, family=0):
    """One sweep point: the GPU result at beta and at beta = 0, each checked
    against the oracle.  X, y: device arrays; Xd: the decoded X (float64)."""
    ds = glm.glm_dataset_register(ctx, glm.make_desc(X, y, dtype=dtype, col_scale=scale,
                                                     family=family))
    try:
        res = []
        for b in (np.asarray(beta, np.float64), np.zeros(len(beta))):
            f, g = eval_gpu(ctx, X, y, b, prec, mean, ds=ds)
            res.append(check_against_oracle(f, g, Xd, y_host, b, prec, mean, storage,
                                            X_for_oracle, oracle_kw))
        return res
    finally:
        glm.glm_dataset_unregister(ctx, ds)


def check_rows(got, Xd, y, betas, prec, means=None, storage="f32", X_for_oracle=None,
               oracle_kw=None, form="any"):
    """Several results (rows of got: f, g) against the oracle at betas."""
    out = []
    for b in range(len(betas)):
        m = None if means is None else means[b]
        out.append(check_against_oracle(got[b, 0], got[b, 1:], Xd, y, betas[b], prec, m, storage,
                                        X_for_oracle, oracle_kw, form))
    return out

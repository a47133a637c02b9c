"""Random-walk Metropolis accept decisions taken with the GPU library's f,
checked against the decisions the oracle's f gives (shadow mode), for one X
stored as FP32, BF16 and FP8-E4M3 (per-column scales).

TEST INFRASTRUCTURE: imports the oracle.  Used by tests/test_gpu_mh.py and
runnable on its own for the full-size storage-precision workload:

    python tests/mh_check.py --n 8000000 --k 512 --steps 20000 --audit 0.0025 \
        --out mh_full.json

The sampler (Sec. 2.2 describes the MH step inside Gibbs; Sec. 3.1.1 gives the
logistic model) proposes beta' = beta + e, e ~ N(0, s^2 I), and accepts iff
log U < f(beta') - f(beta).  Proposal increments and log U come from the
seeded generators, so the GPU side and the oracle side see the same
(beta, beta', U) at every step.

Certification.  Evaluating the oracle at every step of a 20,000-step chain on
an 8M x 512 X is too slow, so a step is taken as settled by the GPU alone when
|log U - (f'_gpu - f_gpu)| > tau (|f'_gpu| + |f_gpu|): if each GPU f is within
the stated relative tolerance tau of the oracle's, the oracle's difference is
on the same side of log U.  Every other step, and a random audit fraction of
all steps, is re-evaluated on the oracle; the audited steps also check that
each GPU f met tau.  The chain follows the FP32 oracle decision (settled or
re-evaluated); BF16 and FP8 are evaluated at the same points, and their
decisions are compared with their own oracle (the oracle on the same stored
codes: kernel check) and with the FP32 chain's decision (storage effect,
reported only).

A mismatch between a GPU decision and its oracle's is acceptable only when
both differences are within the tolerance band of each other (then log U lies
between two results that are both correct to tau); every mismatch is reported
with that flag.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)

import oracle  # noqa: E402
import synth  # noqa: E402

TAU = 1e-9   # stated relative tolerance of f for FP32 products with FP64 sums


def n_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def row_blocks(N: int, parts: int):
    b = np.linspace(0, N, parts + 1).astype(np.int64)
    return [(int(b[i]), int(b[i + 1])) for i in range(parts) if b[i + 1] > b[i]]


class RowOracle:
    """The oracle's f over row blocks in threads.  Each block is evaluated
    with the prior left out, the block values are added with math.fsum and
    the prior is added once: the likelihood is a sum over rows, so this is
    the same quantity (the oracle tests pin the row-split additivity)."""

    def __init__(self, X, y, pool, dtype=None, scale=None):
        self.X, self.y, self.pool = X, y, pool
        self.kw = {"dtype": dtype, "scale": scale}
        self.blocks = row_blocks(X.shape[0], 4 * n_threads())
        self.calls = 0

    def f(self, beta, prec):
        self.calls += 1

        def one(ab):
            a, b = ab
            return oracle.logpost_grad(self.X[a:b], self.y[a:b], beta, 0.0, None, **self.kw)[0]

        parts = list(self.pool.map(one, self.blocks))
        return math.fsum(parts) - 0.5 * prec * math.fsum(np.asarray(beta) ** 2)


def quantize_rows(pool, X, kind, scale=None):
    """The oracle's encoders applied to row blocks in threads (elementwise,
    so the codes equal a single call's)."""
    N, K = X.shape
    Q = np.empty((N, K), np.uint16 if kind == "bf16" else np.uint8)

    def one(ab):
        a, b = ab
        if kind == "bf16":
            Q[a:b] = oracle.quantize_bf16(X[a:b])
        else:
            Q[a:b] = oracle.quantize_fp8(X[a:b], scale)[0]

    list(pool.map(one, row_blocks(N, 4 * n_threads())))
    return Q


class Formats:
    """One X of the storage-precision generator in three stored forms, both
    on the GPU (registered data sets) and for the oracle."""

    NAMES = ("fp32", "bf16", "fp8")

    def __init__(self, N: int, K: int, pool, log=print):
        import torch

        from paper_1310_1537_amd import glm
        t0 = time.perf_counter()
        w = synth.plain_big(N, K, 1000, np.float32, workload_index=2)
        log(f"[mh] generated N={N} K={K} in {time.perf_counter() - t0:.1f} s")
        t0 = time.perf_counter()
        Qb = quantize_rows(pool, w.X, "bf16")
        s8 = oracle.fp8_col_scales(w.X)
        Q8 = quantize_rows(pool, w.X, "fp8", s8)
        log(f"[mh] oracle encoders in {time.perf_counter() - t0:.1f} s")
        self.w, self.Qb, self.Q8, self.s8 = w, Qb, Q8, s8
        self.glm, self.torch = glm, torch
        dev = torch.device("cuda:0")
        self.ctx = glm.glm_create(0)
        self.dev_arrays = [torch.from_numpy(a).to(dev) for a in (w.X, Qb, Q8, s8, w.y)]
        Xd, Qbd, Q8d, s8d, yd = self.dev_arrays
        self.ds = [
            glm.glm_dataset_register(self.ctx, glm.make_desc(Xd, yd)),
            glm.glm_dataset_register(self.ctx, glm.make_desc(Qbd, yd, dtype=glm.GLM_BF16)),
            glm.glm_dataset_register(self.ctx, glm.make_desc(Q8d, yd, dtype=glm.GLM_FP8_E4M3,
                                                             col_scale=s8d)),
        ]
        self.oracles = [RowOracle(w.X, w.y, pool),
                        RowOracle(Qb, w.y, pool, dtype="bf16"),
                        RowOracle(Q8, w.y, pool, dtype="fp8", scale=s8)]
        self.prec = w.prec
        self.prior = glm.make_prior(w.prec)

    def eval_gpu(self, beta):
        """f of every stored form at beta (one host call each)."""
        return [self.glm.glm_logpost_grad_host(self.ctx, d, beta, self.prior) for d in self.ds]

    def close(self):
        for d in self.ds:
            self.glm.glm_dataset_unregister(self.ctx, d)
        self.glm.glm_destroy(self.ctx)
        self.dev_arrays = None


def shadow_chain(fm: Formats, inc, logu, audit_frac: float, seed: int, tau: float = TAU,
                 log=print, progress_every: int = 1000):
    """Runs the chain from beta_true; returns a report dict."""
    n = len(logu)
    F = len(fm.NAMES)
    audit = np.random.default_rng(seed).random(n) < audit_frac
    beta = fm.w.beta_true.copy()
    fg = fm.eval_gpu(beta)
    fo = [None] * F                       # oracle f at the current state, when known
    st = [{"certified": 0, "oracle_checked": 0, "audited": 0, "mismatches": [],
           "max_rel_err_checked": 0.0, "tolerance_violations": 0,
           "min_abs_margin": math.inf} for _ in range(F)]
    storage = [0] * F
    accepts = 0
    t0 = time.perf_counter()
    for t in range(n):
        bp = beta + inc[t]
        fgp = fm.eval_gpu(bp)
        dec = [False] * F
        gpu_dec = [False] * F
        fop = [None] * F
        for i in range(F):
            d_gpu = fgp[i] - fg[i]
            margin = logu[t] - d_gpu
            gpu_dec[i] = bool(logu[t] < d_gpu)
            band = tau * (abs(fgp[i]) + abs(fg[i]))
            s = st[i]
            s["min_abs_margin"] = min(s["min_abs_margin"], abs(margin))
            certified = abs(margin) > band
            if certified:
                s["certified"] += 1
            if certified and not audit[t]:
                dec[i] = gpu_dec[i]
                continue
            if audit[t]:
                s["audited"] += 1
            s["oracle_checked"] += 1
            if fo[i] is None:
                fo[i] = fm.oracles[i].f(beta, fm.prec)
            fop[i] = fm.oracles[i].f(bp, fm.prec)
            d_or = fop[i] - fo[i]
            dec[i] = bool(logu[t] < d_or)
            e = max(abs(fgp[i] - fop[i]) / abs(fop[i]), abs(fg[i] - fo[i]) / abs(fo[i]))
            s["max_rel_err_checked"] = max(s["max_rel_err_checked"], e)
            if e > tau:
                s["tolerance_violations"] += 1
            if dec[i] != gpu_dec[i]:
                s["mismatches"].append({
                    "step": t, "logu": float(logu[t]), "df_gpu": d_gpu, "df_oracle": d_or,
                    "within_band": bool(abs(d_gpu - d_or) <= band)})
        acc = dec[0]
        for i in range(1, F):
            storage[i] += int(gpu_dec[i] != acc)
        if acc:
            accepts += 1
            beta = bp
            fg = fgp
            fo = fop
        if progress_every and (t + 1) % progress_every == 0:
            log(f"[mh] step {t + 1}/{n} accept {accepts / (t + 1):.3f} "
                f"oracle calls {sum(o.calls for o in fm.oracles)} "
                f"{time.perf_counter() - t0:.0f} s")
    rep = {"steps": n, "accept_rate": accepts / max(n, 1), "tau": tau, "audit_frac": audit_frac,
           "formats": {}}
    for i, name in enumerate(fm.NAMES):
        s = dict(st[i])
        s["n_mismatches"] = len(s["mismatches"])
        s["unexplained_mismatches"] = sum(not m["within_band"] for m in s["mismatches"])
        s["uncertified"] = n - s["certified"]
        if i:
            s["decisions_differing_from_fp32_chain"] = storage[i]
        rep["formats"][name] = s
    rep["seconds"] = time.perf_counter() - t0
    return rep


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=8_000_000)
    ap.add_argument("--k", type=int, default=512)
    ap.add_argument("--steps", type=int, default=20_000)
    ap.add_argument("--audit", type=float, default=0.01)
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    with ThreadPoolExecutor(n_threads()) as pool:
        fm = Formats(a.n, a.k, pool, log)
        inc, logu, sd = synth.mh_chain_inputs(a.k, a.steps, a.n)
        log(f"[mh] proposal sd {sd:.3e}, {a.steps} steps, audit {a.audit}")
        rep = shadow_chain(fm, inc, logu, a.audit, seed=20131006, log=log)
        rep.update({"N": a.n, "K": a.k, "proposal_sd": sd, "oracle_threads": n_threads()})
        fm.close()
    txt = json.dumps(rep, indent=1, default=float)
    print(txt, flush=True)
    if a.out:
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        with open(a.out, "w") as fh:
            fh.write(txt + "\n")
    bad = sum(f["unexplained_mismatches"] + f["tolerance_violations"]
              for f in rep["formats"].values())
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main())

"""CPU checks of the shadow-chain checker used by the storage-precision MH
test: with an exact stand-in for the GPU it reports no mismatch; planted
errors (on the CPU, in the stand-in) are caught."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth
from mh_check import RowOracle, quantize_rows, shadow_chain

N, K, STEPS = 3000, 8, 300


class Stand:
    NAMES = ("fp32", "bf16", "fp8")

    def __init__(self, pool, bias=None):
        w = synth.plain_big(N, K, 1, np.float32, workload_index=2)
        Qb = quantize_rows(pool, w.X, "bf16")
        s8 = oracle.fp8_col_scales(w.X)
        Q8 = quantize_rows(pool, w.X, "fp8", s8)
        self.w, self.prec = w, w.prec
        self.oracles = [RowOracle(w.X, w.y, pool), RowOracle(Qb, w.y, pool, dtype="bf16"),
                        RowOracle(Q8, w.y, pool, dtype="fp8", scale=s8)]
        self.ref = [RowOracle(w.X, w.y, pool), RowOracle(Qb, w.y, pool, dtype="bf16"),
                    RowOracle(Q8, w.y, pool, dtype="fp8", scale=s8)]
        self.bias = bias or (lambda i, beta, f: f)

    def eval_gpu(self, beta):
        return [self.bias(i, beta, o.f(beta, self.prec)) for i, o in enumerate(self.ref)]


@pytest.fixture(scope="module")
def pool():
    with ThreadPoolExecutor(4) as p:
        yield p


def test_row_oracle_equals_single_call(pool):
    w = synth.plain_big(N, K, 1, np.float32, workload_index=2)
    f1 = RowOracle(w.X, w.y, pool).f(w.betas[0], w.prec)
    f0, _ = oracle.logpost_grad(w.X, w.y, w.betas[0], w.prec)
    assert abs(f1 - f0) <= 1e-13 * abs(f0)


def test_quantize_rows_equals_single_call(pool):
    w = synth.plain_big(N, K, 1, np.float32, workload_index=2)
    assert np.array_equal(quantize_rows(pool, w.X, "bf16"), oracle.quantize_bf16(w.X))
    q, s = oracle.quantize_fp8(w.X)
    assert np.array_equal(quantize_rows(pool, w.X, "fp8", s), q)


def test_exact_stand_in_has_no_mismatch(pool):
    st = Stand(pool)
    inc, logu, _ = synth.mh_chain_inputs(K, STEPS, N)
    rep = shadow_chain(st, inc, logu, 0.2, seed=1, progress_every=0)
    assert 0.05 < rep["accept_rate"] < 0.8
    for f in rep["formats"].values():
        assert f["n_mismatches"] == 0 and f["tolerance_violations"] == 0
        assert f["audited"] > 20


def test_planted_tolerance_violation_is_caught(pool):
    st = Stand(pool, bias=lambda i, b, f: f * (1 + 1e-7) if i == 1 else f)
    inc, logu, _ = synth.mh_chain_inputs(K, STEPS, N)
    rep = shadow_chain(st, inc, logu, 0.2, seed=1, progress_every=0)
    assert rep["formats"]["bf16"]["tolerance_violations"] > 0
    assert rep["formats"]["fp32"]["tolerance_violations"] == 0


def test_planted_decision_flip_is_caught(pool):
    """The FP8 stand-in adds 0.7 to f on every other evaluation, so the
    difference of f at about half of the steps is off by 0.7 and decisions
    near the threshold flip; with every step audited they are all caught
    (and so is the tolerance breach behind them)."""
    calls = [0]

    def bias(i, b, f):
        if i == 2:
            calls[0] += 1
            return f + 0.7 * (calls[0] % 2)
        return f

    st = Stand(pool, bias=bias)
    inc, logu, _ = synth.mh_chain_inputs(K, STEPS, N)
    rep = shadow_chain(st, inc, logu, 1.0, seed=1, progress_every=0)
    f8 = rep["formats"]["fp8"]
    assert f8["n_mismatches"] > 0 and f8["unexplained_mismatches"] == f8["n_mismatches"]
    assert f8["tolerance_violations"] > 0
    assert rep["formats"]["fp32"]["n_mismatches"] == 0

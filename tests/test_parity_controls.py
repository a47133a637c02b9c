"""CPU controls of the GPU parity checker (tests/parity_bounds.py).

Negative controls: the checker must reject the oracle's own result on data
with one row dropped, one row repeated, or one response flipped (the last
row, which the kernels handle in their ragged tail), at every (N, K, storage)
the GPU sweeps evaluate, both at the sweep's beta and at beta = 0.

Positive control: a numpy emulation of the kernels' arithmetic (the FP64
product chains per lane, the butterfly additions, r rounded to FP32, FP32
gradient partials over 16 rows, FP64 beyond) must stay within the bounds,
which shows that they are not tighter than the arithmetic they describe.
"""
import math

import numpy as np
import pytest

import oracle
import parity_bounds as pb
import sweeps

PERTURBATIONS = ("drop", "repeat", "flip")


def _perturb(X, y, kind):
    if kind == "drop":
        return X[:-1], y[:-1]
    if kind == "repeat":
        return np.concatenate([X, X[-1:]]), np.concatenate([y, y[-1:]])
    y2 = y.copy()
    y2[-1] = 1 - y2[-1] if y2.max(initial=0) <= 1 else y2[-1] + 1
    return X, y2


def _rejected(Xo, y, beta, prec, storage, Xd=None, mean=None, family="logistic", kw=None,
              form="any"):
    """For each perturbation and both legs (beta, 0): True when the checker
    rejects the oracle result of the perturbed data as a result for y, X."""
    kw = dict(kw or {})
    kw["family"] = family
    Xd = np.asarray(Xo, np.float64) if Xd is None else Xd
    out = {}
    for leg, b in (("beta", beta), ("zero", np.zeros_like(beta))):
        ref = oracle.logpost_grad(Xo, y, b, prec, mean, **kw)
        bd = pb.error_bounds(Xd, y, b, prec, mean, storage, family, form)
        pb.check(*ref, Xd, y, b, prec, mean, storage, family, form, ref=ref, bounds=bd)
        for kind in PERTURBATIONS:
            Xp, yp = _perturb(Xo, y, kind)
            got = oracle.logpost_grad(Xp, yp, b, prec, mean, **kw)
            try:
                pb.check(*got, Xd, y, b, prec, mean, storage, family, form, ref=ref, bounds=bd)
                out[(leg, kind)] = False
            except AssertionError:
                out[(leg, kind)] = True
    return out


def _assert_all_rejected(res, case, beta_leg=True):
    """Every perturbation is rejected by the sweep (the beta and the beta = 0
    legs together); with beta_leg, by the beta leg on its own as well."""
    missed = [kind for kind in PERTURBATIONS
              if not (res[("beta", kind)] or res[("zero", kind)])]
    if beta_leg:
        missed += [("beta", kind) for kind in PERTURBATIONS if not res[("beta", kind)]]
    assert not missed, (case, missed)


def test_layout_follows_the_kernel_plan():
    # (VE, NC, LPR, CPL): 16-byte chunks, lanes per row, chunks per lane
    assert pb.layout(256, "f32") == (4, 64, 64, 1)
    assert pb.layout(1024, "f32") == (4, 256, 64, 4)
    assert pb.layout(512, "f32") == (4, 128, 64, 2)
    assert pb.layout(20, "f64") == (2, 10, 16, 1)
    assert pb.layout(32, "f32") == (4, 8, 8, 1)
    assert pb.layout(512, "bf16") == (8, 64, 64, 1)
    assert pb.layout(4096, "fp8") == (16, 256, 64, 4)
    assert pb.layout(1, "f32") == (4, 1, 1, 1)


@pytest.mark.parametrize("K", sweeps.F32_K)
def test_negative_controls_plain_f32(K):
    for N in sweeps.F32_N:
        if N == 0:
            continue
        X, y, beta = sweeps.plain_f32_case(N, K)
        _assert_all_rejected(_rejected(X, y, beta, 0.01, "f32"), (N, K))


@pytest.mark.parametrize("K", sweeps.F64_K)
def test_negative_controls_plain_f64(K):
    for N in sweeps.F64_N:
        if N == 0:
            continue
        X, y, beta = sweeps.plain_f64_case(N, K)
        res = _rejected(X, y, beta, 0.5, "f64", mean=np.full(K, 0.05))
        _assert_all_rejected(res, (N, K))


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_negative_controls_stored_codes(kind):
    for K in (sweeps.BF16_K if kind == "bf16" else sweeps.FP8_K):
        for N in sweeps.CODES_N:
            X, y, beta = sweeps.codes_case(N, K, kind)
            if kind == "bf16":
                Q = oracle.quantize_bf16(X)
                res = _rejected(Q, y, beta, 0.01, "bf16", Xd=oracle.decode_bf16(Q),
                                kw={"dtype": "bf16"})
            else:
                Q, s = oracle.quantize_fp8(X)
                res = _rejected(Q, y, beta, 0.01, "fp8", Xd=oracle.decode_fp8(Q, s),
                                kw={"dtype": "fp8", "scale": s})
            _assert_all_rejected(res, (kind, N, K))


def test_negative_controls_ragged_k():
    for K in sweeps.RAGGED_K:
        for N in sweeps.RAGGED_N:
            X, y, beta = sweeps.ragged_case(N, K)
            _assert_all_rejected(_rejected(X, y, beta, 0.01, "f32"), (N, K))


def test_negative_controls_poisson():
    for K in sweeps.POISSON_K:
        for N in sweeps.POISSON_N:
            X, y, beta = sweeps.poisson(N, K, K + N)
            res = _rejected(X, y, beta, 0.01, "f32", family="poisson")
            _assert_all_rejected(res, (N, K))


def test_negative_controls_several_beta():
    for K in sweeps.MULTI_K:
        for nb in sweeps.MULTI_NB:
            X, y, bt = sweeps.serving_data(20_011, K, K + nb)
            B = sweeps.betas_near(bt, nb, 7)
            _assert_all_rejected(_rejected(X, y, B[-1], 0.01, "f32"), (K, nb))
    for K in sweeps.MX_K:
        for nb in sweeps.MX_NB:
            X, y, bt = sweeps.serving_data(10_007, K, 100 + K + nb)
            Q = oracle.quantize_bf16(X)
            B = sweeps.betas_near(bt, nb, K + 3 * nb)
            res = _rejected(Q, y, B[0], 0.01, "bf16", Xd=oracle.decode_bf16(Q),
                            kw={"dtype": "bf16"})
            # the matrix-core form's bound counts every product of an
            # instruction as a rounding: the beta = 0 leg (exact u) is the
            # one that sees a single row there
            _assert_all_rejected(res, (K, nb), beta_leg=pb.u_model(K, "bf16")[2] < 2.0 ** -40)


def test_negative_controls_groups():
    """Each group of the ragged-group sweep, perturbed alone."""
    X, y, off, B = sweeps.groups(sweeps.GROUP_SIZES, 32, 1)
    mu = np.linspace(-0.3, 0.3, 32)
    for g in range(len(sweeps.GROUP_SIZES)):
        a, b = off[g], off[g + 1]
        if b == a:
            continue
        res = _rejected(X[a:b], y[a:b], B[g], 4.0, "f32", mean=mu)
        _assert_all_rejected(res, g)


# ------------------------------------------------------------ positive control

def _emulate(Xv, y, beta, prec, storage="f32", scale=None):
    """The kernels' arithmetic in numpy: Xv holds the float32 values the
    kernel multiplies (FP8: the unscaled codes, with the scales folded into
    beta and applied to g at the end)."""
    N, K = Xv.shape
    ve, nc, lpr, cpl = pb.layout(K, storage)
    W = lpr * cpl * ve
    Xp = np.zeros((N, W), np.float32)
    Xp[:, :K] = Xv
    bp = np.zeros(W)
    bp[:K] = beta if scale is None else beta * scale.astype(np.float64)
    Xr = Xp.reshape(N, cpl, lpr, ve)     # column (cl + i LPR) VE + e of lane cl, chunk i
    br = bp.reshape(cpl, lpr, ve)
    acc = np.zeros((N, lpr))
    for i in range(cpl):
        for e in range(ve):   # FP64 products and sums (two roundings where the kernel's FMA has one)
            acc = acc + Xr[:, i, :, e].astype(np.float64) * br[i, :, e]
    w = lpr
    while w > 1:              # butterfly additions in FP64
        w //= 2
        acc = acc[:, :w] + acc[:, w:2 * w]
    u = acc[:, 0]
    yv = y.astype(np.float64)
    e = np.exp(-np.abs(u))
    t = yv * u - (np.maximum(u, 0.0) + np.log1p(e))
    r32 = (yv - np.where(u >= 0, 1.0 / (1.0 + e), e / (1.0 + e))).astype(np.float32)
    nparts = -(-N // 16)
    P = np.zeros((nparts * 16, K), np.float32)
    P[:N] = r32[:, None] * Xv
    P = P.reshape(nparts, 16, K)
    s = np.zeros((nparts, K), np.float32)
    for j in range(16):           # FP32 partials over 16 rows
        s = s + P[:, j, :]
    g = s.astype(np.float64).sum(axis=0)
    if scale is not None:
        g = g * scale.astype(np.float64)
    return math.fsum(t) - 0.5 * prec * float(np.dot(beta, beta)), g - prec * beta


@pytest.mark.parametrize("N,K,nbin", [(40_003, 256, 0), (40_003, 1024, 0), (200_000, 256, 26),
                                      (65, 1024, 0), (1_000, 8, 0)])
def test_emulated_arithmetic_within_bounds(N, K, nbin):
    X, y, beta = sweeps.plain(N, K, 5 + K, nbin=nbin)
    for b in (beta, np.zeros(K)):
        f, g = _emulate(X, y, b, 0.01)
        r = pb.check(f, g, X.astype(np.float64), y, b, 0.01, oracle=oracle, X_oracle=X)
        assert r["f_use"] < 0.5 and r["g_use"] < 0.5, r


def test_emulated_stored_codes_within_bounds():
    X, y, beta = sweeps.codes_case(20_011, 2048, "bf16")
    Q = oracle.quantize_bf16(X)
    f, g = _emulate(oracle.decode_bf16(Q).astype(np.float32), y, beta, 0.01, "bf16")
    pb.check(f, g, oracle.decode_bf16(Q), y, beta, 0.01, storage="bf16", form="valu",
             oracle=oracle, X_oracle=Q, oracle_kw={"dtype": "bf16"})
    X, y, beta = sweeps.codes_case(20_011, 4096, "fp8")
    Q, s = oracle.quantize_fp8(X)
    f, g = _emulate(oracle.decode_fp8(Q).astype(np.float32), y, beta, 0.01, "fp8", scale=s)
    pb.check(f, g, oracle.decode_fp8(Q, s), y, beta, 0.01, storage="fp8", oracle=oracle,
             X_oracle=Q, oracle_kw={"dtype": "fp8", "scale": s})


def test_old_worst_case_bound_missed_a_dropped_row():
    """The bound the sweeps used before, (K + 2) 2^-24 sum_n |r_n| A_n, passes
    a result with the last row dropped at K = 1024, N = 40,003; the new
    checker rejects it."""
    X, y, beta = sweeps.plain_f32_case(40_003, 1024)
    Xd = X.astype(np.float64)
    f, g = oracle.logpost_grad(X, y, beta, 0.01)
    fd, gd = oracle.logpost_grad(X[:-1], y[:-1], beta, 0.01)
    u = Xd @ beta
    r = y - 0.5 * (1 + np.tanh(0.5 * u))
    old = (1024 + 2) * 2.0 ** -24 * np.sum(np.abs(r) * (np.abs(Xd) @ np.abs(beta)))
    assert abs(fd - f) < old
    with pytest.raises(AssertionError):
        pb.check(fd, gd, Xd, y, beta, 0.01, ref=(f, g))

"""Pins for the FP64 oracle: each test checks it against something other than
itself -- a closed form, an invariant of the model, an independent library
routine, a complex-step derivative, or a 40-digit brute force.  The
combination is chosen so that a dropped term, a wrong sign, a wrong index or a
transposed operand anywhere in the oracle fails at least one of them.

The paper prints no worked numeric value of f or g, so no test compares with
a number from the paper; the model and its derivatives come from Sec. 3.1.1
(eq-loglike-binlogit) and Sec. 4.2 (eq-grad-expanded, eq-grad-compact).
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle
import synth

LN2 = math.log(2.0)


def _data(N, K, seed, dtype=np.float64, scale=1.0):
    g = np.random.default_rng(seed)
    X = (scale * g.standard_normal((N, K))).astype(dtype)
    y = (g.random(N) < 0.4).astype(np.uint8)
    beta = g.standard_normal(K) / math.sqrt(K)
    return X, y, beta


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# ---------------------------------------------------------------- closed forms

def test_f_at_zero_is_minus_n_ln2():
    """u = 0 for every row: each row contributes y*0 - ln 2, the prior is 0."""
    w = synth.plain_small(n_evals=1)
    f, _ = oracle.logpost_grad(w.X, w.y, np.zeros(20), w.prec)
    assert _rel(f, -10_000 * LN2) < 1e-15
    assert f == pytest.approx(-6931.471805599453, rel=1e-15)


def test_g_at_zero_is_xt_y_minus_half():
    """sigma(0) = 1/2, so g(0) = X^t (y - 1/2); the products x (y - 1/2) are exact
    in double and fsum rounds their sum once."""
    X, y, _ = _data(3000, 9, 1)
    _, g = oracle.logpost_grad(X, y, np.zeros(9), 0.25)
    for k in range(9):
        exact = math.fsum(X[:, k] * (y - 0.5))
        assert abs(g[k] - exact) <= 1e-15 * math.fsum(np.abs(X[:, k]))


def test_prior_only_when_no_rows():
    K = 6
    beta = np.linspace(-1, 2, K)
    m = np.linspace(0.5, -0.5, K)
    lam = 3.5
    f, g = oracle.logpost_grad(np.zeros((0, K)), np.zeros(0, np.uint8), beta, lam, m)
    d = beta - m
    assert _rel(f, -0.5 * lam * math.fsum(d * d)) < 1e-15
    np.testing.assert_allclose(g, -lam * d, rtol=1e-15)


def test_prior_mean_and_precision_enter_with_the_right_sign():
    """At beta = 0 with mean m: the prior adds -lam/2 |m|^2 to f(0) = -N ln 2 and
    +lam m to g(0) = X^t (y - 1/2)."""
    X, y, _ = _data(500, 4, 2)
    m = np.array([0.3, -0.2, 1.0, 0.0])
    lam = 2.0
    f, g = oracle.logpost_grad(X, y, np.zeros(4), lam, m)
    assert _rel(f, -500 * LN2 - 0.5 * lam * math.fsum(m * m)) < 1e-14
    for k in range(4):
        assert abs(g[k] - (math.fsum(X[:, k] * (y - 0.5)) + lam * m[k])) < 1e-12


def test_single_constant_column_closed_form():
    """K = 1 and x_n = c for every row: f = beta c S - N softplus(beta c)
    - lam beta^2 / 2 and g = c S - N c sigmoid(beta c) - lam beta, S = sum y."""
    N, c, beta, lam = 777, 0.37, 1.9, 0.5
    y = (np.random.default_rng(3).random(N) < 0.6).astype(np.uint8)
    S = int(y.sum())
    X = np.full((N, 1), c)
    f, g = oracle.logpost_grad(X, y, np.array([beta]), lam)
    z = beta * c
    sp = math.log1p(math.exp(z))
    sig = 1.0 / (1.0 + math.exp(-z))
    assert _rel(f, beta * c * S - N * sp - 0.5 * lam * beta * beta) < 1e-13
    assert _rel(g[0], c * S - N * c * sig - lam * beta) < 1e-12


def test_extreme_linear_predictor_stays_finite():
    """|u| ~ 1e3: softplus(u) -> u for u >> 0 and -> exp(u) for u << 0."""
    X = np.array([[1000.0], [1000.0], [-1000.0], [-1000.0]])
    y = np.array([1, 0, 1, 0], np.uint8)
    f, g = oracle.logpost_grad(X, y, np.array([1.0]), 0.0)
    # rows: y=1,u=1000 -> 0 ; y=0,u=1000 -> -1000 ; y=1,u=-1000 -> -1000 ; y=0,u=-1000 -> 0
    assert f == -2000.0
    # r: 0, -1, 1, 0 -> g = 0*1000 - 1000 + 1*(-1000) + 0 = -2000
    assert g[0] == -2000.0
    assert oracle.softplus(800.0) == 800.0
    assert oracle.softplus(-800.0) == pytest.approx(math.exp(-800.0), rel=1e-15)


# -------------------------------------------------------------- invariants

def test_response_linearity():
    """f(y=1) - f(y=0) = sum_n u_n = beta . (column sums of X), and
    g(y=1) - g(y=0) = column sums of X, whatever beta is."""
    X, _, beta = _data(2000, 7, 4)
    N = X.shape[0]
    f1, g1 = oracle.logpost_grad(X, np.ones(N, np.uint8), beta, 0.3)
    f0, g0 = oracle.logpost_grad(X, np.zeros(N, np.uint8), beta, 0.3)
    colsum = np.array([math.fsum(X[:, k]) for k in range(7)])
    su = math.fsum(colsum * beta)
    scale = math.fsum(np.abs(X @ beta)) + N
    assert abs((f1 - f0) - su) < 1e-13 * scale
    np.testing.assert_allclose(g1 - g0, colsum, rtol=0, atol=1e-12 * N)


def test_flip_symmetry():
    """(x_n, y_n) -> (-x_n, 1 - y_n) leaves every row's term unchanged."""
    X, y, beta = _data(1500, 5, 5)
    f, g = oracle.logpost_grad(X, y, beta, 0.1)
    ff, gf = oracle.logpost_grad(-X, (1 - y).astype(np.uint8), beta, 0.1)
    assert _rel(ff, f) < 1e-13
    np.testing.assert_allclose(gf, g, rtol=1e-12, atol=1e-10)


def test_row_permutation_and_split_additivity():
    """Exchangeable rows (Sec. 2.3): the sum does not depend on row order, and
    splitting the rows adds the likelihood parts (prior counted once)."""
    X, y, beta = _data(2500, 6, 6)
    m = np.full(6, 0.1)
    lam = 0.7
    f, g = oracle.logpost_grad(X, y, beta, lam, m)
    p = np.random.default_rng(7).permutation(len(y))
    fp, gp = oracle.logpost_grad(X[p], y[p], beta, lam, m)
    assert _rel(fp, f) < 1e-14
    np.testing.assert_allclose(gp, g, rtol=1e-12, atol=1e-11)
    fa, ga = oracle.logpost_grad(X[:900], y[:900], beta, 0.0)
    fb, gb = oracle.logpost_grad(X[900:], y[900:], beta, lam, m)
    assert _rel(fa + fb, f) < 1e-14
    np.testing.assert_allclose(ga + gb, g, rtol=1e-12, atol=1e-11)


def test_concavity_of_the_log_posterior():
    """The logistic log-likelihood is concave: (g(b1) - g(b2)) . (b1 - b2) < 0."""
    X, y, _ = _data(800, 5, 8)
    rng = np.random.default_rng(9)
    for _ in range(10):
        b1, b2 = rng.standard_normal(5), rng.standard_normal(5)
        _, g1 = oracle.logpost_grad(X, y, b1, 0.01)
        _, g2 = oracle.logpost_grad(X, y, b2, 0.01)
        assert (g1 - g2) @ (b1 - b2) < 0


# ------------------------------------------------------ derivative pins

def _f_complex(X, y, beta_c, lam, m):
    """log-posterior on complex beta (an independent, differentiable form)."""
    u = X @ beta_c
    d = beta_c - m
    return np.sum(y * u - np.log(1.0 + np.exp(u))) - 0.5 * lam * np.sum(d * d)


def test_gradient_matches_complex_step_derivative():
    """Im f(beta + i h e_k) / h with h = 1e-30 is the exact derivative up to
    rounding; it exercises f only, not the analytic gradient code."""
    X, y, beta = _data(300, 6, 10)
    m = np.linspace(-0.2, 0.2, 6)
    lam = 1.3
    _, g = oracle.logpost_grad(X, y, beta, lam, m)
    h = 1e-30
    for k in range(6):
        bc = beta.astype(np.complex128)
        bc[k] += 1j * h
        dk = _f_complex(X, y, bc, lam, m).imag / h
        assert abs(g[k] - dk) < 1e-12 * max(1.0, abs(dk))


def test_gradient_matches_central_differences():
    X, y, beta = _data(400, 4, 11)
    f0, g = oracle.logpost_grad(X, y, beta, 0.2)
    for k in range(4):
        e = np.zeros(4)
        e[k] = 1e-5
        fp, _ = oracle.logpost_grad(X, y, beta + e, 0.2)
        fm, _ = oracle.logpost_grad(X, y, beta - e, 0.2)
        assert abs((fp - fm) / 2e-5 - g[k]) < 1e-6 * max(1.0, abs(g[k]))


# ------------------------------------------------------- library pins

def test_matches_torch_bce_with_logits_and_autograd():
    """The logistic log-likelihood is minus the summed binary cross-entropy on
    logits u; torch's CPU float64 routine and its autograd give f and g."""
    torch = pytest.importorskip("torch")
    X, y, beta = _data(4000, 12, 12)
    m = np.full(12, -0.05)
    lam = 0.01
    f, g = oracle.logpost_grad(X, y, beta, lam, m)
    Xt = torch.from_numpy(X)
    b = torch.tensor(beta, requires_grad=True)
    u = Xt @ b
    d = b - torch.from_numpy(m)
    ft = -torch.nn.functional.binary_cross_entropy_with_logits(
        u, torch.from_numpy(y.astype(np.float64)), reduction="sum") - 0.5 * lam * (d * d).sum()
    ft.backward()
    assert _rel(f, ft.item()) < 1e-13
    np.testing.assert_allclose(g, b.grad.numpy(), rtol=1e-11, atol=1e-10)


def test_gradient_vanishes_at_sklearn_map_estimate():
    """scikit-learn's L2 logistic regression (no intercept) minimises
    C sum(log-loss) + |w|^2 / 2, i.e. maximises the log-posterior with prior
    precision 1/C; the oracle's gradient must vanish there.  The prior is made
    strong so that a wrong sign or scale of its term would be visible."""
    sk = pytest.importorskip("sklearn.linear_model")
    X, y, _ = _data(300, 5, 13)
    lam = 20.0
    clf = sk.LogisticRegression(C=1.0 / lam, fit_intercept=False, tol=1e-12,
                                max_iter=10_000, solver="newton-cg")
    clf.fit(X, y)
    bhat = clf.coef_.ravel()
    _, g = oracle.logpost_grad(X, y, bhat, lam)
    assert np.linalg.norm(g) < 1e-6 * lam * np.linalg.norm(bhat)
    _, gwrong = oracle.logpost_grad(X, y, bhat, 2 * lam)
    assert np.linalg.norm(gwrong) > 0.5 * lam * np.linalg.norm(bhat)


# ------------------------------------------------------ 40-digit brute force

def test_matches_40_digit_brute_force():
    getcontext().prec = 40
    X, y, beta = _data(40, 6, 14)
    m = np.linspace(-0.3, 0.3, 6)
    lam = 0.9
    f, g = oracle.logpost_grad(X, y, beta, lam, m)
    D = Decimal
    one = D(1)
    fs = D(0)
    gs = [D(0)] * 6
    for n in range(40):
        u = sum(D(float(X[n, k])) * D(float(beta[k])) for k in range(6))
        e = u.exp()
        fs += D(int(y[n])) * u - (one + e).ln()
        r = D(int(y[n])) - e / (one + e)
        gs = [gs[k] + r * D(float(X[n, k])) for k in range(6)]
    dd = [D(float(beta[k])) - D(float(m[k])) for k in range(6)]
    fs -= D(lam) / 2 * sum(d * d for d in dd)
    gs = [gs[k] - D(lam) * dd[k] for k in range(6)]
    assert _rel(f, float(fs)) < 1e-15
    for k in range(6):
        assert abs(g[k] - float(gs[k])) < 1e-15 * max(1.0, abs(float(gs[k])))


# ----------------------------------------------- storage formats (decoders)

def test_fp8_decoder_matches_torch_for_all_codes():
    torch = pytest.importorskip("torch")
    codes = np.arange(256, dtype=np.uint8)
    mine = oracle.decode_fp8(codes)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(np.isnan(mine), np.isnan(ref))
    ok = ~np.isnan(ref)
    np.testing.assert_array_equal(mine[ok], ref[ok])
    assert np.nanmax(mine) == 448.0 and mine[1] == 2.0 ** -9


def test_bf16_encoder_matches_torch():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(15)
    v = np.concatenate([
        g.standard_normal(20000).astype(np.float32),
        (g.standard_normal(2000) * 1e-39).astype(np.float32),       # subnormals
        np.array([0.0, -0.0, 1.0, 3.0e38, -3.0e38, 1e-45], np.float32),
        # exact ties: low 16 bits 0x8000 with odd and even kept parts
        np.array([0x3F808000, 0x3F818000, 0x3F800001, 0x3F80FFFF],
                 np.uint32).view(np.float32),
    ]).reshape(-1, 1)
    mine = oracle.quantize_bf16(v).ravel()
    ref = torch.from_numpy(v.ravel()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(mine, ref)


def test_fp8_encoder_matches_torch():
    """Encoding x / s_k: torch's float8_e4m3fn cast rounds to nearest even but
    returns NaN beyond +-464, so the torch side clamps to +-448 first."""
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(16)
    v = np.concatenate([
        (g.standard_normal(50000) * 60).astype(np.float32),
        (g.standard_normal(5000) * 0.01).astype(np.float32),          # subnormal codes
        np.array([0.0, -0.0, 448.0, 463.9, 464.0, 465.0, 1e9, -1e9,
                  2.0 ** -10, 3 * 2.0 ** -10, 2.0 ** -6, 1.0625, 1.1875], np.float32),
    ])
    s = np.ones(1, np.float32)
    mine, _ = oracle.quantize_fp8(v.reshape(-1, 1), s)
    ref = torch.from_numpy(np.clip(v, -448, 448)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(mine.ravel(), ref)


def test_fp8_column_scales_and_binary_columns():
    X = np.array([[1.0, -3.0, 0.0], [0.0, 2.0, 0.0], [1.0, 0.5, 0.0]], np.float32)
    Q, s = oracle.quantize_fp8(X)
    assert s[0] == np.float32(1.0) / np.float32(448.0)
    assert s[1] == np.float32(3.0) / np.float32(448.0)
    assert s[2] == 1.0                                  # all-zero column
    assert Q[0, 0] == 0x7E and Q[1, 0] == 0 and Q[1, 2] == 0
    assert Q[0, 1] == 0xFE                              # -448
    deq = oracle.decode_fp8(Q, s)
    assert abs(deq[0, 0] - 1.0) < 1e-6 and abs(deq[0, 1] + 3.0) < 1e-6


def test_stored_formats_feed_the_same_arithmetic():
    """The oracle on codes equals the oracle on their float64 decodings, bit for
    bit (the conversion is exact and the arithmetic identical)."""
    X32, y, beta = _data(700, 9, 17, np.float32)
    fa, ga = oracle.logpost_grad(X32, y, beta, 0.01)
    fb, gb = oracle.logpost_grad(X32.astype(np.float64), y, beta, 0.01)
    assert fa == fb and np.array_equal(ga, gb)
    Qb = oracle.quantize_bf16(X32)
    fa, ga = oracle.logpost_grad(Qb, y, beta, 0.01, dtype="bf16")
    fb, gb = oracle.logpost_grad(oracle.decode_bf16(Qb), y, beta, 0.01)
    assert fa == fb and np.array_equal(ga, gb)
    Q8, s = oracle.quantize_fp8(X32)
    fa, ga = oracle.logpost_grad(Q8, y, beta, 0.01, dtype="fp8", scale=s)
    fb, gb = oracle.logpost_grad(oracle.decode_fp8(Q8, s), y, beta, 0.01)
    assert fa == fb and np.array_equal(ga, gb)


# -------------------------------------------------- composite entry points

def test_groups_and_multi_equal_plain_calls():
    X, y, _ = _data(1000, 5, 18)
    off = np.array([0, 0, 13, 400, 1000])
    rng = np.random.default_rng(19)
    B = rng.standard_normal((4, 5))
    mu = rng.standard_normal(5)
    out = oracle.logpost_grad_groups(X, y, off, B, 4.0, mu)
    for gidx in range(4):
        a, b = off[gidx], off[gidx + 1]
        f, g = oracle.logpost_grad(X[a:b], y[a:b], B[gidx], 4.0, mu)
        assert out[gidx, 0] == f and np.array_equal(out[gidx, 1:], g)
    outm = oracle.logpost_grad_multi(X, y, B, 0.01)
    for i in range(4):
        f, g = oracle.logpost_grad(X, y, B[i], 0.01)
        assert outm[i, 0] == f and np.array_equal(outm[i, 1:], g)


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_groups_and_multi_on_codes_equal_plain_calls_on_decoded_slices(kind):
    """The grouped and several-beta drivers on BF16 / FP8 codes (their own
    byte strides and, for FP8, the column scales) give, bit for bit, the
    plain function on the FP64-decoded rows of each group; the decoders are
    pinned against torch's casts above.  Per-group prior means and the
    Poisson family included."""
    X32, y, _ = _data(1500, 24, 30, np.float32)
    off = np.array([0, 1, 1, 300, 777, 1500])
    G = len(off) - 1
    rng = np.random.default_rng(31)
    B = 0.2 * rng.standard_normal((G, 24))
    M = rng.standard_normal((G, 24))
    if kind == "bf16":
        Q, s = oracle.quantize_bf16(X32), None
        Xd = oracle.decode_bf16(Q)
    else:
        Q, s = oracle.quantize_fp8(X32)
        Xd = oracle.decode_fp8(Q, s)
    yp = np.minimum(rng.poisson(1.5, len(y)), 255).astype(np.uint8)
    for yy, fam in ((y, "logistic"), (yp, "poisson")):
        out = oracle.logpost_grad_groups(Q, yy, off, B, 2.0, M, dtype=kind, scale=s, family=fam)
        for gi in range(G):
            a, b = off[gi], off[gi + 1]
            f, g = oracle.logpost_grad(Xd[a:b], yy[a:b], B[gi], 2.0, M[gi], family=fam)
            assert out[gi, 0] == f and np.array_equal(out[gi, 1:], g), (kind, fam, gi)
        outm = oracle.logpost_grad_multi(Q, yy, B, 0.5, M, dtype=kind, scale=s, family=fam)
        for i in range(G):
            f, g = oracle.logpost_grad(Xd, yy, B[i], 0.5, M[i], family=fam)
            assert outm[i, 0] == f and np.array_equal(outm[i, 1:], g), (kind, fam, i)


def test_rejects_invalid_arguments():
    X, y, beta = _data(10, 3, 20)
    with pytest.raises(ValueError):
        bad = y.copy()
        bad[3] = 2
        oracle.logpost_grad(X, bad, beta, 0.1)


def test_numpy_sequence_of_maps_cross_check():
    """An independent float64 NumPy evaluation in the paper's sequence-of-maps
    shape (Sec. 4.2): X beta, the elementwise map, then X^t g_f."""
    w = synth.plain_small(n_evals=5)
    for beta in w.betas:
        f, g = oracle.logpost_grad(w.X, w.y, beta, w.prec)
        u = w.X @ beta
        fl = np.sum(w.y * u - np.logaddexp(0.0, u)) - 0.5 * w.prec * beta @ beta
        gl = w.X.T @ (w.y - 0.5 * (1.0 + np.tanh(0.5 * u))) - w.prec * beta
        assert _rel(f, fl) < 1e-12
        np.testing.assert_allclose(g, gl, rtol=1e-10, atol=1e-9)


def test_golden_record_of_small_workload():
    """tests/golden/plain_small.json: the closed-form f(0) = -N ln 2 and the
    oracle's own values at three seeded points (written by make_golden.py)."""
    import json
    import os
    rec = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "plain_small.json")))
    assert rec["f_at_zero_closed_form"] == -10_000 * LN2
    w = synth.plain_small(n_evals=3)
    for p, beta in zip(rec["points"], w.betas):
        assert np.array_equal(np.array(p["beta"]), beta)
        f, g = oracle.logpost_grad(w.X, w.y, beta, w.prec)
        assert f == p["f"] and np.array_equal(g, np.array(p["g"]))


# ------------------------------------------------------------ linear predictor

def test_linpred_exact_on_dyadic_inputs():
    """Small integers times dyadic coefficients: every product and partial sum
    is exact in FP64, so u must equal the rational result exactly."""
    from fractions import Fraction
    g = np.random.default_rng(21)
    X = g.integers(-50, 51, (300, 9)).astype(np.float64)
    beta = g.integers(-1000, 1001, 9) / 256.0
    u = oracle.linpred(X, beta)
    for n in range(300):
        want = sum(Fraction(int(X[n, k])) * Fraction(beta[k]) for k in range(9))
        assert Fraction(u[n]) == want


def test_linpred_is_what_the_log_posterior_uses():
    """sum_n u_n = f(y=1) - f(y=0) (response linearity of the likelihood), and
    for stored BF16 / FP8 codes u equals u of the decoded values."""
    X, _, beta = _data(1500, 12, 22)
    N = X.shape[0]
    u = oracle.linpred(X, beta)
    f1, _ = oracle.logpost_grad(X, np.ones(N, np.uint8), beta, 0.0)
    f0, _ = oracle.logpost_grad(X, np.zeros(N, np.uint8), beta, 0.0)
    assert abs(math.fsum(u) - (f1 - f0)) < 1e-13 * (math.fsum(np.abs(u)) + N)
    X32 = X.astype(np.float32)
    Qb = oracle.quantize_bf16(X32)
    np.testing.assert_array_equal(oracle.linpred(Qb, beta, dtype="bf16"),
                                  oracle.linpred(oracle.decode_bf16(Qb), beta))
    Q8, s8 = oracle.quantize_fp8(X32)
    np.testing.assert_array_equal(oracle.linpred(Q8, beta, dtype="fp8", scale=s8),
                                  oracle.linpred(oracle.decode_fp8(Q8, s8), beta))


# --------------------------------------------------------- Poisson family

def _pdata(N, K, seed):
    g = np.random.default_rng(seed)
    X = g.standard_normal((N, K))
    beta = 0.5 * g.standard_normal(K) / math.sqrt(K)
    y = np.minimum(g.poisson(np.exp(X @ beta)), 255).astype(np.uint8)
    return X, y, beta


def test_poisson_closed_forms_at_zero():
    """beta = 0: every row has u = 0, t = -exp(0) = -1 and r = y - 1, so
    f(0) = -N and g(0) = X^t (y - 1) exactly."""
    X, y, _ = _pdata(3000, 7, 30)
    f, g = oracle.logpost_grad(X, y, np.zeros(7), 0.4, family="poisson")
    assert f == -3000.0
    want = [math.fsum(X[:, k] * (y.astype(np.float64) - 1.0)) for k in range(7)]
    np.testing.assert_allclose(g, want, rtol=0, atol=1e-12 * 3000)


def test_poisson_response_linearity():
    """f(y) - f(y') = sum_n (y_n - y'_n) u_n and g(y) - g(y') = X^t (y - y'),
    whatever beta is: the counts enter linearly."""
    X, y, beta = _pdata(2000, 6, 31)
    y2 = np.random.default_rng(32).integers(0, 40, 2000).astype(np.uint8)
    f1, g1 = oracle.logpost_grad(X, y, beta, 0.1, family="poisson")
    f2, g2 = oracle.logpost_grad(X, y2, beta, 0.1, family="poisson")
    dy = y.astype(np.float64) - y2
    u = oracle.linpred(X, beta)
    assert abs((f1 - f2) - math.fsum(dy * u)) < 1e-12 * (math.fsum(np.abs(dy * u)) + 1)
    want = [math.fsum(X[:, k] * dy) for k in range(6)]
    np.testing.assert_allclose(g1 - g2, want, rtol=0, atol=1e-10 * 2000)


def test_poisson_matches_torch_nll_and_autograd():
    """torch's PoissonNLLLoss on log-rates (without the Stirling term) is
    sum exp(u) - y u, minus the log-likelihood up to the left-out constant."""
    torch = pytest.importorskip("torch")
    X, y, beta = _pdata(5000, 10, 33)
    m = np.full(10, 0.03)
    lam = 0.5
    f, g = oracle.logpost_grad(X, y, beta, lam, m, family="poisson")
    b = torch.tensor(beta, requires_grad=True)
    u = torch.from_numpy(X) @ b
    d = b - torch.from_numpy(m)
    loss = torch.nn.PoissonNLLLoss(log_input=True, full=False, reduction="sum")(
        u, torch.from_numpy(y.astype(np.float64)))
    ft = -loss - 0.5 * lam * (d * d).sum()
    ft.backward()
    assert _rel(f, ft.item()) < 1e-12
    np.testing.assert_allclose(g, b.grad.numpy(), rtol=1e-10, atol=1e-9)


def test_poisson_gradient_vanishes_at_sklearn_map_estimate():
    """scikit-learn's PoissonRegressor (no intercept) minimises
    mean half-deviance + alpha/2 |w|^2, whose stationary point is that of the
    Poisson log-posterior with prior precision N alpha."""
    sk = pytest.importorskip("sklearn.linear_model")
    X, y, _ = _pdata(400, 5, 34)
    alpha = 0.05
    reg = sk.PoissonRegressor(alpha=alpha, fit_intercept=False, tol=1e-12, max_iter=10_000)
    reg.fit(X, y)
    w = reg.coef_.ravel()
    lam = 400 * alpha
    _, g = oracle.logpost_grad(X, y, w, lam, family="poisson")
    assert np.linalg.norm(g) < 1e-5 * lam * np.linalg.norm(w)
    _, gwrong = oracle.logpost_grad(X, y, w, 2 * lam, family="poisson")
    assert np.linalg.norm(gwrong) > 0.5 * lam * np.linalg.norm(w)


def test_poisson_complex_step_and_40_digit_brute_force():
    X, y, beta = _pdata(30, 5, 35)
    m = np.linspace(-0.1, 0.1, 5)
    lam = 0.7
    f, g = oracle.logpost_grad(X, y, beta, lam, m, family="poisson")
    h = 1e-30
    for k in range(5):
        bc = beta.astype(np.complex128)
        bc[k] += 1j * h
        uc = X @ bc
        dd = bc - m
        fc = np.sum(y * uc - np.exp(uc)) - 0.5 * lam * np.sum(dd * dd)
        assert abs(g[k] - fc.imag / h) < 1e-12 * max(1.0, abs(g[k]))
    getcontext().prec = 40
    D = Decimal
    fs = D(0)
    gs = [D(0)] * 5
    for n in range(30):
        u = sum(D(float(X[n, k])) * D(float(beta[k])) for k in range(5))
        mu = u.exp()
        fs += D(int(y[n])) * u - mu
        gs = [gs[k] + (D(int(y[n])) - mu) * D(float(X[n, k])) for k in range(5)]
    dd = [D(float(beta[k])) - D(float(m[k])) for k in range(5)]
    fs -= D(lam) / 2 * sum(d * d for d in dd)
    gs = [gs[k] - D(lam) * dd[k] for k in range(5)]
    assert _rel(f, float(fs)) < 1e-15
    for k in range(5):
        assert abs(g[k] - float(gs[k])) < 1e-14 * max(1.0, abs(float(gs[k])))


def test_poisson_rejects_nothing_the_logistic_model_rejects_for_counts():
    """Counts above 1 are invalid for the logistic model and valid for the
    Poisson one."""
    X, y, beta = _pdata(50, 3, 36)
    y[0] = 7
    with pytest.raises(ValueError):
        oracle.logpost_grad(X, y, beta, 0.1)
    f, _ = oracle.logpost_grad(X, y, beta, 0.1, family="poisson")
    assert np.isfinite(f)


# ------------------------------------------------------------------ Hessian

@pytest.mark.parametrize("family", ["logistic", "poisson"])
def test_hessian_matches_torch_autograd(family):
    """torch.autograd.functional.hessian of torch's own loss (BCE on logits or
    Poisson NLL on log-rates) plus the Gaussian prior."""
    torch = pytest.importorskip("torch")
    if family == "logistic":
        X, y, beta = _data(1500, 7, 40)
    else:
        X, y, beta = _pdata(1500, 7, 40)
    m = np.linspace(-0.1, 0.1, 7)
    lam = 0.8
    H = oracle.hessian(X, beta, lam, family=family)
    Xt = torch.from_numpy(X)
    yt = torch.from_numpy(y.astype(np.float64))
    mt = torch.from_numpy(m)

    def f(b):
        u = Xt @ b
        if family == "logistic":
            ll = -torch.nn.functional.binary_cross_entropy_with_logits(u, yt, reduction="sum")
        else:
            ll = -torch.nn.PoissonNLLLoss(log_input=True, full=False, reduction="sum")(u, yt)
        d = b - mt
        return ll - 0.5 * lam * (d * d).sum()

    Ht = torch.autograd.functional.hessian(f, torch.tensor(beta)).numpy()
    np.testing.assert_allclose(H, Ht, rtol=1e-11, atol=1e-11 * np.abs(Ht).max())


def test_hessian_is_the_derivative_of_the_gradient():
    X, y, beta = _data(800, 5, 41)
    H = oracle.hessian(X, beta, 0.3)
    h = 1e-5
    for k in range(5):
        e = np.zeros(5)
        e[k] = h
        _, gp = oracle.logpost_grad(X, y, beta + e, 0.3)
        _, gm = oracle.logpost_grad(X, y, beta - e, 0.3)
        np.testing.assert_allclose((gp - gm) / (2 * h), H[:, k], rtol=1e-6, atol=1e-6)


def test_hessian_at_zero_and_its_structure():
    """beta = 0 (logistic): every weight is 1/4 exactly, so H = -X^t X / 4 -
    lam I, exact on integer-valued X; H is symmetric (to the rounding of
    w x_i x_j in either order) and H + lam I is negative semi-definite."""
    g = np.random.default_rng(42)
    X = g.integers(-9, 10, (400, 6)).astype(np.float64)
    H = oracle.hessian(X, np.zeros(6), 2.0)
    want = -(X.T @ X) / 4.0 - 2.0 * np.eye(6)
    np.testing.assert_array_equal(H, want)
    X2, _, b2 = _data(300, 8, 43)
    H2 = oracle.hessian(X2, b2, 0.5)
    np.testing.assert_allclose(H2, H2.T, rtol=1e-14, atol=1e-14 * np.abs(H2).max())
    assert np.linalg.eigvalsh(H2 + 0.5 * np.eye(8)).max() <= 1e-12

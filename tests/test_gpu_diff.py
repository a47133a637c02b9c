"""GPU parity of the differential-update calls (glm_transpose, glm_linpred,
glm_diff_logpost, glm_diff_commit) against the oracle: f(beta + delta e_k)
is the plain log-posterior at the moved point."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402

if torch.cuda.is_available():
    from gpu_helpers import DEV, Ctx, to_dev  # noqa: E402
    from paper_1310_1537_amd import glm  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


def _data(N, K, seed):
    g = np.random.default_rng(seed)
    X = g.standard_normal((N, K)).astype(np.float32)
    beta = g.standard_normal(K) / math.sqrt(K)
    y = (g.random(N) < 1.0 / (1.0 + np.exp(-(X.astype(np.float64) @ beta)))).astype(np.uint8)
    return X, y, beta


def _stored(X, kind):
    """(stored array for the GPU and the oracle, decoded FP64 values, oracle kwargs, scales)."""
    if kind == "f64":
        X64 = X.astype(np.float64)
        return X64, X64, {}, None
    if kind == "f32":
        return X, X.astype(np.float64), {}, None
    if kind == "bf16":
        Q = oracle.quantize_bf16(X)
        return Q, oracle.decode_bf16(Q), {"dtype": "bf16"}, None
    Q, s = oracle.quantize_fp8(X)
    return Q, oracle.decode_fp8(Q, s), {"dtype": "fp8", "scale": s}, s


class Cols:
    """A row-major data set on the GPU, its column-major copy and column set."""

    def __init__(self, ctx, S, y, scale=None, pad=0):
        self.ctx = ctx
        N, K = S.shape
        self.Xd = to_dev(S)
        self.yd = to_dev(y)
        self.sd = None if scale is None else to_dev(scale)
        dt = {np.dtype(np.float64): glm.GLM_F64, np.dtype(np.float32): glm.GLM_F32,
              np.dtype(np.uint16): glm.GLM_BF16, np.dtype(np.uint8): glm.GLM_FP8_E4M3}[S.dtype]
        ld = N + pad
        self.Xt = torch.empty((K, ld), dtype=self.Xd.dtype, device=DEV)
        glm.glm_transpose(ctx, glm.make_desc(self.Xd, self.yd, dtype=dt, col_scale=self.sd),
                          self.Xt, ld)
        self.cs = glm.glm_colset_register(
            ctx, glm.make_colset_desc(self.Xt, self.yd, N=N, dtype=dt, col_scale=self.sd))

    def close(self):
        glm.glm_colset_unregister(self.ctx, self.cs)


def _fbound(Xd, y, beta, f):
    """FP64 path: the GPU's u differs from the oracle's by a few ulps of
    sum_k |x_k beta_k| per row; everything else is FP64 summation."""
    A = np.abs(Xd) @ np.abs(beta)
    K = Xd.shape[1]
    return (2 * K + 4) * 2.0 ** -53 * np.sum(A) + 1e-13 * (abs(f) + len(y))


@pytest.mark.parametrize("kind", ["f64", "f32", "bf16", "fp8"])
@pytest.mark.parametrize("shape", [(1, 1), (63, 65), (1000, 7), (4099, 130)])
def test_transpose_is_bitwise(ctx, kind, shape):
    X, y, _ = _data(*shape, 1)
    S, _, _, s = _stored(X, kind)
    c = Cols(ctx, S, y, s, pad=3)
    torch.cuda.synchronize()
    got = c.Xt.cpu().numpy()[:, :shape[0]]
    np.testing.assert_array_equal(got, S.T)
    c.close()


@pytest.mark.parametrize("kind", ["f64", "f32", "bf16", "fp8"])
def test_linpred_against_oracle(ctx, kind):
    X, y, beta = _data(30_011, 37, 2)
    S, Xd, kw, s = _stored(X, kind)
    c = Cols(ctx, S, y, s)
    u = torch.empty(30_011, dtype=torch.float64, device=DEV)
    glm.glm_linpred(ctx, c.cs, to_dev(beta), u)
    torch.cuda.synchronize()
    want = oracle.linpred(S, beta, **kw)
    A = np.abs(Xd) @ np.abs(beta)
    assert np.all(np.abs(u.cpu().numpy() - want) <= (2 * 37 + 2) * 2.0 ** -53 * A)
    c.close()


@pytest.mark.parametrize("kind", ["f64", "f32", "bf16", "fp8"])
@pytest.mark.parametrize("nd", [1, 5, 16, 21])
def test_diff_logpost_against_oracle(ctx, kind, nd):
    N, K = 20_011, 24
    X, y, beta = _data(N, K, 3)
    S, Xd, kw, s = _stored(X, kind)
    c = Cols(ctx, S, y, s)
    mean = np.linspace(-0.2, 0.2, K)
    md = to_dev(mean)
    bd = to_dev(beta)
    u = torch.empty(N, dtype=torch.float64, device=DEV)
    glm.glm_linpred(ctx, c.cs, bd, u)
    deltas = np.linspace(-0.7, 0.9, nd)
    dd = to_dev(deltas)
    out = torch.full((nd,), float("nan"), dtype=torch.float64, device=DEV)
    for k in (0, 11, K - 1):
        glm.glm_diff_logpost(ctx, c.cs, u, bd, k, dd, nd, glm.make_prior(0.5, md), out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        for j in range(nd):
            b2 = beta.copy()
            b2[k] += deltas[j]
            f, _ = oracle.logpost_grad(S, y, b2, 0.5, mean, **kw)
            assert abs(got[j] - f) <= _fbound(Xd, y, b2, f), (k, j, got[j], f)
    c.close()


def test_sweep_with_commits_tracks_the_oracle(ctx):
    """A Gibbs-style sweep: for every coordinate evaluate three step sizes,
    commit one of them; the committed u and beta match the oracle's u at the
    final beta, and each committed step's f is reproduced bit for bit by a
    zero step evaluated after the commit."""
    N, K = 50_000, 16
    X, y, beta0 = _data(N, K, 4)
    c = Cols(ctx, X, y)
    bd = to_dev(beta0)
    u = torch.empty(N, dtype=torch.float64, device=DEV)
    glm.glm_linpred(ctx, c.cs, bd, u)
    prior = glm.make_prior(0.01)
    steps = np.random.default_rng(5).normal(0.0, 0.05, (2 * K, 3))
    out = torch.empty(3, dtype=torch.float64, device=DEV)
    out0 = torch.empty(1, dtype=torch.float64, device=DEV)
    zero = to_dev(np.zeros(1))
    beta = beta0.copy()
    for t in range(2 * K):
        k = t % K
        dd = to_dev(steps[t])
        glm.glm_diff_logpost(ctx, c.cs, u, bd, k, dd, 3, prior, out)
        torch.cuda.synchronize()
        f3 = out.cpu().numpy().copy()
        pick = int(np.argmax(f3))
        glm.glm_diff_commit(ctx, c.cs, u, bd, k, dd[pick:pick + 1])
        beta[k] += steps[t, pick]
        glm.glm_diff_logpost(ctx, c.cs, u, bd, k, zero, 1, prior, out0)
        torch.cuda.synchronize()
        assert out0.cpu().numpy()[0] == f3[pick]
    np.testing.assert_array_equal(bd.cpu().numpy(), beta)
    want = oracle.linpred(X, beta)
    A = np.abs(X.astype(np.float64)) @ np.abs(beta)
    assert np.all(np.abs(u.cpu().numpy() - want) <= (K + 4 * K) * 2.0 ** -53 * (A + np.abs(want)))
    f_or, _ = oracle.logpost_grad(X, y, beta, 0.01)
    glm.glm_diff_logpost(ctx, c.cs, u, bd, 0, zero, 1, prior, out0)
    torch.cuda.synchronize()
    assert abs(out0.cpu().numpy()[0] - f_or) <= 1e-12 * abs(f_or)
    c.close()


def test_empty_data_and_errors(ctx):
    K = 5
    Xt = torch.empty((K, 0), dtype=torch.float32, device=DEV)
    yd = torch.empty(0, dtype=torch.uint8, device=DEV)
    cs = glm.glm_colset_register(ctx, glm.make_colset_desc(Xt, yd, N=0))
    beta = np.array([0.5, -1.0, 2.0, 0.0, 0.25])
    bd = to_dev(beta)
    dd = to_dev(np.array([0.0, 1.0]))
    out = torch.empty(2, dtype=torch.float64, device=DEV)
    glm.glm_diff_logpost(ctx, cs, None, bd, 2, dd, 2, glm.make_prior(2.0), out)
    torch.cuda.synchronize()
    for j, d in enumerate((0.0, 1.0)):
        b2 = beta.copy()
        b2[2] += d
        assert out.cpu().numpy()[j] == pytest.approx(-1.0 * np.sum(b2 ** 2), rel=1e-15)
    for bad in (-1, K):
        with pytest.raises(glm.GlmError) as e:
            glm.glm_diff_logpost(ctx, cs, None, bd, bad, dd, 2, glm.make_prior(2.0), out)
        assert e.value.status == glm.GLM_EINVAL
    with pytest.raises(glm.GlmError) as e:
        glm.glm_diff_logpost(ctx, cs, None, bd, 0, dd, 0, glm.make_prior(2.0), out)
    assert e.value.status == glm.GLM_EINVAL
    glm.glm_colset_unregister(ctx, cs)
    with pytest.raises(glm.GlmError) as e:
        glm.glm_linpred(ctx, cs, bd, out)
    assert e.value.status == glm.GLM_ENOTFOUND


def test_probe_diff_map(ctx):
    """The per-row map probe runs for both families and rejects bad arguments."""
    for fam in (glm.GLM_LOGISTIC, glm.GLM_POISSON):
        us = glm.glm_probe_diff_map(ctx, 1_000_000, fam, 3)
        assert 0.0 < us < 1e5
    assert glm.glm_probe_diff_map(ctx, 0, 0, 2) > 0.0
    for bad in ((-1, 0, 2), (100, 7, 2), (100, 0, 0)):
        with pytest.raises(glm.GlmError):
            glm.glm_probe_diff_map(ctx, *bad)

"""GPU parity of the fused Hessian (glm_logpost_grad_hess) against the oracle's
H = -X^t W X - prec I, with per-entry bounds derived from the arithmetic:
the row weights come from u, whose error is that of the fused kernel
(FP32 products for FP32/BF16/FP8 storage), and the sums over rows are FP64."""
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402

if torch.cuda.is_available():
    from gpu_helpers import DEV, Ctx, eval_gpu, to_dev  # noqa: E402
    from paper_1310_1537_amd import glm  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


def _hess_gpu(ctx, Xd, yd, beta, prec, family=0, dtype=None, scale=None, mean=None):
    K = Xd.shape[1]
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xd, yd, dtype=dtype, col_scale=scale,
                                                     family=family))
    out = torch.full((K + 1,), float("nan"), dtype=torch.float64, device=DEV)
    H = torch.full((K, K), float("nan"), dtype=torch.float64, device=DEV)
    md = None if mean is None else to_dev(mean)
    glm.glm_logpost_grad_hess(ctx, ds, to_dev(beta), glm.make_prior(prec, md), out, H)
    torch.cuda.synchronize()
    glm.glm_dataset_unregister(ctx, ds)
    return out.cpu().numpy(), H.cpu().numpy()


def _bound(Xd, beta, storage="f32", family="logistic"):
    """Per-entry bound: sum_n |x_ni x_nj| (|w'_n| |du_n| + (N + 64) 2^-53 w_n)."""
    N, K = Xd.shape
    eps = 2.0 ** -53 if storage == "f64" else 2.0 ** -24
    u = Xd @ beta
    A = np.abs(Xd) @ np.abs(beta)
    if family == "poisson":
        w = np.exp(u)
        dw = w
    else:
        s = 0.5 * (1.0 + np.tanh(0.5 * u))
        w = s * (1 - s)
        dw = w * np.abs(1 - 2 * s)
    c = dw * (K + 2) * eps * A * 1.01 + (N + 64) * 2.0 ** -53 * w + 1e-300
    Ax = np.abs(Xd)
    return (Ax * c[:, None]).T @ Ax + 1e-13 * (Ax * w[:, None]).T @ Ax


def _check(Hg, Ho, bound):
    err = np.abs(Hg - Ho)
    bad = np.argwhere(err > bound)
    assert bad.size == 0, (bad[:4], err[tuple(bad[0])], bound[tuple(bad[0])])
    np.testing.assert_array_equal(Hg, Hg.T)


@pytest.mark.parametrize("K", [1, 5, 16, 64, 65, 130, 256])
@pytest.mark.parametrize("N", [1, 100, 20_011])
def test_f32_shapes(ctx, K, N):
    g = np.random.default_rng(K * 31 + N)
    X = g.standard_normal((N, K)).astype(np.float32)
    beta = g.standard_normal(K) / math.sqrt(K)
    y = (g.random(N) < 0.5).astype(np.uint8)
    Xd, yd = glm.aligned_rows(to_dev(X)), to_dev(y)
    out, H = _hess_gpu(ctx, Xd, yd, beta, 0.7)
    X64 = X.astype(np.float64)
    Ho = oracle.hessian(X, beta, 0.7)
    _check(H, Ho, _bound(X64, beta))
    # f and g are those of the plain call, bit for bit
    f, gg = eval_gpu(ctx, Xd, yd, beta, 0.7)
    assert out[0] == f and np.array_equal(out[1:], gg)


@pytest.mark.parametrize("K", [5, 130, 260])
def test_f32_nan_row_padding(ctx, K):
    """FP32 rows whose padding past column K (up to a leading dimension 12
    columns wider) holds NaN: the padding may reach the staged tile, but only
    entries past K could see it, and those are not in H."""
    g = np.random.default_rng(K + 5)
    N = 20_011
    X = g.standard_normal((N, K)).astype(np.float32)
    beta = g.standard_normal(K) / math.sqrt(K)
    y = (g.random(N) < 0.5).astype(np.uint8)
    ld = (K + 3) // 4 * 4 + 12
    buf = torch.full((N, ld), float("nan"), dtype=torch.float32, device=DEV)
    buf[:, :K] = to_dev(X)
    Xd, yd = buf[:, :K], to_dev(y)
    out, H = _hess_gpu(ctx, Xd, yd, beta, 0.7)
    assert np.isfinite(H).all() and np.isfinite(out).all()
    _check(H, oracle.hessian(X, beta, 0.7), _bound(X.astype(np.float64), beta))


@pytest.mark.parametrize("kind", ["f64", "bf16", "fp8", "poisson"])
def test_other_storage_and_poisson(ctx, kind):
    g = np.random.default_rng(7)
    N, K = 9_001, 40
    X = g.standard_normal((N, K)).astype(np.float32)
    beta = 0.5 * g.standard_normal(K) / math.sqrt(K)
    y = (g.random(N) < 0.5).astype(np.uint8)
    if kind == "f64":
        X64 = X.astype(np.float64)
        _, H = _hess_gpu(ctx, to_dev(X64), to_dev(y), beta, 0.1)
        _check(H, oracle.hessian(X64, beta, 0.1), _bound(X64, beta, "f64"))
    elif kind == "bf16":
        Q = oracle.quantize_bf16(X)
        _, H = _hess_gpu(ctx, to_dev(Q), to_dev(y), beta, 0.1, dtype=glm.GLM_BF16)
        _check(H, oracle.hessian(Q, beta, 0.1, dtype="bf16"), _bound(oracle.decode_bf16(Q), beta))
    elif kind == "fp8":
        Q, s = oracle.quantize_fp8(X)
        _, H = _hess_gpu(ctx, glm.aligned_rows(to_dev(Q)), to_dev(y), beta, 0.1,
                         dtype=glm.GLM_FP8_E4M3, scale=to_dev(s))
        _check(H, oracle.hessian(Q, beta, 0.1, dtype="fp8", scale=s),
               _bound(oracle.decode_fp8(Q, s), beta))
    else:
        yp = np.minimum(g.poisson(np.exp(X.astype(np.float64) @ beta)), 255).astype(np.uint8)
        _, H = _hess_gpu(ctx, to_dev(X), to_dev(yp), beta, 0.1, family=glm.GLM_POISSON)
        _check(H, oracle.hessian(X, beta, 0.1, family="poisson"),
               _bound(X.astype(np.float64), beta, family="poisson"))


def test_empty_data_gives_the_prior(ctx):
    K = 70
    Xd = torch.empty((0, 72), dtype=torch.float32, device=DEV)[:, :K]
    yd = torch.empty(0, dtype=torch.uint8, device=DEV)
    _, H = _hess_gpu(ctx, Xd, yd, np.ones(K), 3.0)
    np.testing.assert_array_equal(H, -3.0 * np.eye(K))


def test_repeated_calls_bitwise_and_mid_size(ctx):
    """N = 200,000, K = 256 FP32 (the big generator's shape at a smaller N):
    within the bound of the oracle (evaluated over row blocks in threads and
    summed, the Hessian being a sum over rows), and bitwise equal on repeat."""
    w = synth.plain_big(200_000, 256, 1)
    b = w.betas[0]
    Xd, yd = to_dev(w.X), to_dev(w.y)
    _, H1 = _hess_gpu(ctx, Xd, yd, b, w.prec)
    _, H2 = _hess_gpu(ctx, Xd, yd, b, w.prec)
    np.testing.assert_array_equal(H1, H2)
    edges = np.linspace(0, 200_000, 33).astype(int)
    with ThreadPoolExecutor(16) as ex:
        parts = list(ex.map(lambda i: oracle.hessian(w.X[edges[i]:edges[i + 1]], b, 0.0),
                            range(32)))
    Ho = np.sum(parts, axis=0) - w.prec * np.eye(256)
    _check(H1, Ho, _bound(w.X.astype(np.float64), b) + 64 * 2.0 ** -53 * np.abs(Ho))


def test_mfma_probe(ctx):
    tf = glm.glm_probe_mfma_f64(ctx, 200)
    assert 1.0 < tf < 200.0
    with pytest.raises(glm.GlmError) as e:
        glm.glm_probe_mfma_f64(ctx, 0)
    assert e.value.status == glm.GLM_EINVAL

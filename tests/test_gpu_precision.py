"""GPU parity of the storage-precision forms: the BF16 and FP8 E4M3FN
encoders (bit-exact against the oracle's encoders) and the fused kernel on
BF16 / FP8 storage (against the oracle on the same stored codes)."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import sweeps  # noqa: E402

if torch.cuda.is_available():
    from gpu_helpers import DEV, Ctx, eval_gpu, sweep_point, to_dev  # noqa: E402
    from paper_1310_1537_amd import glm  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


_matrix = sweeps.precision_matrix


def test_bf16_encoder_bit_exact(ctx):
    X = _matrix(3001, 96, 1)
    X[5, :8] = np.array([0x3F808000, 0x3F818000, 0x3F800001, 0x3F80FFFF, 0x7F7FFFFF,
                         0x00000001, 0x80000000, 0x3F7FFFFF], np.uint32).view(np.float32)
    Xd = to_dev(X)
    Q = torch.empty((3001, 96), dtype=torch.uint16, device=DEV)
    glm.glm_quantize_bf16(ctx, Xd, Q)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Q.cpu().numpy(), oracle.quantize_bf16(X))


@pytest.mark.parametrize("shape", [(1, 1), (1000, 7), (4099, 512)])
def test_fp8_scales_and_encoder_bit_exact(ctx, shape):
    N, K = shape
    X = _matrix(N, K, 2) * np.float32(3.5)
    if K > 3:
        X[:, 3] = 0.0                         # all-zero column -> scale 1
    Xd = to_dev(X)
    s = torch.empty(K, dtype=torch.float32, device=DEV)
    glm.glm_fp8_col_scales(ctx, Xd, s)
    Q = torch.empty((N, K), dtype=torch.uint8, device=DEV)
    glm.glm_quantize_fp8(ctx, Xd, s, Q)
    torch.cuda.synchronize()
    Qo, so = oracle.quantize_fp8(X)
    np.testing.assert_array_equal(s.cpu().numpy(), so)
    np.testing.assert_array_equal(Q.cpu().numpy(), Qo)


def test_fp8_encoder_special_values(ctx):
    v = np.array([0.0, -0.0, 448.0, 463.9, 464.0, 465.0, 1e9, -1e9, 2.0 ** -10,
                  3 * 2.0 ** -10, 2.0 ** -6, 1.0625, 1.1875, 2.0 ** -9 * 0.5,
                  2.0 ** -9 * 1.5, 2.0 ** -9 * 2.5, 7 * 2.0 ** -9 * 1.0001], np.float32)
    X = v.reshape(-1, 1)
    s = to_dev(np.ones(1, np.float32))
    Q = torch.empty((len(v), 1), dtype=torch.uint8, device=DEV)
    glm.glm_quantize_fp8(ctx, to_dev(X), s, Q)
    torch.cuda.synchronize()
    Qo, _ = oracle.quantize_fp8(X, np.ones(1, np.float32))
    np.testing.assert_array_equal(Q.cpu().numpy(), Qo)


def test_fp8_decode_every_code_through_the_kernel(ctx):
    """One row holding every finite code, beta = 0, y = 1, flat prior:
    g_k = (1 - 1/2) x_k s_k exactly, so g reveals the kernel's decoding."""
    codes = np.arange(256, dtype=np.uint8)
    codes[codes == 0x7F] = 0
    codes[codes == 0xFF] = 0
    Q = codes.reshape(1, 256)
    s = np.random.default_rng(3).uniform(0.5, 2.0, 256).astype(np.float32)
    y = np.ones(1, np.uint8)
    f, g = eval_gpu(ctx, to_dev(Q), to_dev(y), np.zeros(256), 0.0, dtype=glm.GLM_FP8_E4M3,
                    scale=to_dev(s))
    want = 0.5 * oracle.decode_fp8(Q, s).ravel()
    np.testing.assert_array_equal(g, want)
    assert f == -math.log(2.0)


@pytest.mark.parametrize("K", sweeps.BF16_K)
@pytest.mark.parametrize("N", sweeps.CODES_N)
def test_bf16_kernel_against_oracle_on_codes(ctx, K, N):
    X, y, beta = sweeps.codes_case(N, K, "bf16")
    Qo = oracle.quantize_bf16(X)
    sweep_point(ctx, to_dev(Qo), to_dev(y), oracle.decode_bf16(Qo), y, beta, 0.01,
                storage="bf16", dtype=glm.GLM_BF16, X_for_oracle=Qo, oracle_kw={"dtype": "bf16"})


@pytest.mark.parametrize("K", sweeps.FP8_K)
@pytest.mark.parametrize("N", sweeps.CODES_N)
def test_fp8_kernel_against_oracle_on_codes(ctx, K, N):
    X, y, beta = sweeps.codes_case(N, K, "fp8")
    Qo, so = oracle.quantize_fp8(X)
    sweep_point(ctx, to_dev(Qo), to_dev(y), oracle.decode_fp8(Qo, so), y, beta, 0.01,
                storage="fp8", dtype=glm.GLM_FP8_E4M3, scale=to_dev(so), X_for_oracle=Qo,
                oracle_kw={"dtype": "fp8", "scale": so})

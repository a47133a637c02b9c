"""The allocation-free plain call (glm_logpost_grad_noalloc) through the C
interface: bitwise equal to glm_logpost_grad on the same data set and beta,
and within the oracle's bound, on two calls in a row (the second on a smaller
data set, which reuses the static scratch the first one left behind); a
launch whose partials do not fit the static scratch is refused on the host."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import sweeps  # noqa: E402
import synth  # noqa: E402

if torch.cuda.is_available():
    from gpu_helpers import DEV, Ctx, check_against_oracle, to_dev  # noqa: E402
    from paper_1310_1537_amd import glm  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


def _both(ctx, ds, K, beta, prec):
    """(noalloc result, glm_logpost_grad result) at beta on the torch stream."""
    b = to_dev(np.asarray(beta, np.float64))
    pr = glm.make_prior(prec)
    o1 = torch.full((1 + K,), float("nan"), dtype=torch.float64, device=DEV)
    o2 = torch.full((1 + K,), float("nan"), dtype=torch.float64, device=DEV)
    s = torch.cuda.current_stream().cuda_stream
    glm.glm_logpost_grad_noalloc(ctx, ds, b, pr, o1, s)
    glm.glm_logpost_grad(ctx, ds, b, pr, o2, s)
    torch.cuda.synchronize()
    return o1.cpu().numpy(), o2.cpu().numpy()


def test_noalloc_matches_plain_call_twice_second_smaller(ctx):
    # first call: 200,003 x 256 FP32 rows (every compute unit's block, two
    # merge levels, a ragged last batch)
    X, y, beta = sweeps.plain_f32_case(200_003, 256)
    Xt, yt = to_dev(X), to_dev(y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xt, yt))
    print("noalloc: N=200003 K=256 f32", flush=True)
    a, b = _both(ctx, ds, 256, beta, 0.01)
    assert np.array_equal(a, b), "noalloc result differs from glm_logpost_grad"
    check_against_oracle(a[0], a[1:], X.astype(np.float64), y, beta, 0.01)
    glm.glm_dataset_unregister(ctx, ds)
    # second call: the small FP64 workload (10,000 x 20, fewer blocks, one
    # merge level) over the partials the first call left
    w = synth.plain_small(n_evals=3)
    Xs, ys = to_dev(w.X), to_dev(w.y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xs, ys))
    print("noalloc: N=10000 K=20 f64", flush=True)
    for beta in w.betas:
        a, b = _both(ctx, ds, 20, beta, w.prec)
        assert np.array_equal(a, b)
        r = check_against_oracle(a[0], a[1:], w.X, w.y, beta, w.prec, storage="f64")
        assert r["f_rel"] < 1e-12 and r["g_rel"] < 1e-10, r
    glm.glm_dataset_unregister(ctx, ds)


def test_noalloc_refuses_partials_beyond_the_static_scratch(ctx):
    # BF16 rows of 2,048 columns over enough rows for a block per compute
    # unit need 8 (nblocks + ngroups)(1 + K) > 4 MiB: refused before launch
    K, N = 2048, 8192
    Xq = torch.zeros((N, K), dtype=torch.bfloat16, device=DEV)
    yq = torch.zeros(N, dtype=torch.uint8, device=DEV)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xq, yq, dtype=glm.GLM_BF16))
    out = torch.zeros(1 + K, dtype=torch.float64, device=DEV)
    beta = torch.zeros(K, dtype=torch.float64, device=DEV)
    with pytest.raises(glm.GlmError) as ei:
        glm.glm_logpost_grad_noalloc(ctx, ds, beta, glm.make_prior(0.01), out)
    assert ei.value.status == glm.GLM_EINVAL
    assert "static scratch" in str(ei.value)
    glm.glm_dataset_unregister(ctx, ds)

"""GPU parity of the batched hierarchical-model evaluation
(glm_logpost_grad_batched) against the FP64 oracle's per-group results."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import parity_bounds as pb  # noqa: E402
import sweeps  # noqa: E402
import synth  # noqa: E402

if torch.cuda.is_available():
    from gpu_helpers import DEV, Ctx, check_against_oracle, eval_gpu, to_dev  # noqa: E402
    from paper_1310_1537_amd import glm  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


_groups = sweeps.groups


def _run(ctx, X, y, off, B, prec, mean=None, per_group=False, tune=False, dtype=None, scale=None,
         repeat=1, zero_leg=False):
    """Batched results (repeat calls); with zero_leg, one more call at
    beta = 0 for every group is appended."""
    Xd, yd = to_dev(X), to_dev(y)
    desc = glm.make_desc(Xd, yd, dtype=dtype, col_scale=scale)
    gs = glm.glm_groupset_create(ctx, desc, off, tune=tune)
    G, K = B.shape
    md = None if mean is None else to_dev(mean)
    out = torch.full((G, K + 1), float("nan"), dtype=torch.float64, device=DEV)
    res = []
    for Bc in [B] * repeat + ([np.zeros_like(B)] if zero_leg else []):
        glm.glm_logpost_grad_batched(ctx, gs, to_dev(Bc), glm.make_prior(prec, md, per_group), out)
        torch.cuda.synchronize()
        res.append(out.cpu().numpy().copy())
    info = glm.glm_groupset_query(gs)
    glm.glm_groupset_destroy(gs)
    return res, info


def _check_groups(got, Xd64, y, off, B, prec, mean=None, storage="f32", X_oracle=None, okw=None):
    okw = okw or {}
    Xo = Xd64 if X_oracle is None else X_oracle
    ref = oracle.logpost_grad_groups(Xo, y, off, B, prec, mean, **okw)
    for g in range(len(off) - 1):
        a, b = off[g], off[g + 1]
        mg = None if mean is None else (mean[g] if mean.ndim == 2 else mean)
        pb.check(got[g, 0], got[g, 1:], Xd64[a:b], y[a:b], B[g], prec, mg, storage,
                 okw.get("family", "logistic"), ref=(ref[g, 0], ref[g, 1:]))


def _check_both(res, Xd64, y, off, B, prec, **kw):
    """res = [at B, at 0] from _run(..., zero_leg=True)."""
    _check_groups(res[0], Xd64, y, off, B, prec, **kw)
    _check_groups(res[1], Xd64, y, off, np.zeros_like(B), prec, **kw)


SIZES = [0, 1, 63, 64, 65, 127, 128, 129, 1000, 1025, 5000, 20, 0, 3, 2049, 700]


@pytest.mark.parametrize("tune", [False, True])
def test_ragged_groups_f32(ctx, tune):
    X, y, off, B = _groups(SIZES, 32, 1)
    mu = np.linspace(-0.3, 0.3, 32)
    res, info = _run(ctx, X, y, off, B, 4.0, mean=mu, tune=tune, zero_leg=True)
    assert info["items"] >= len(SIZES)
    _check_both(res, X.astype(np.float64), y, off, B, 4.0, mean=mu)


def test_split_groups_are_merged(ctx):
    """Default tile length is 8 batches (1024 rows at K=32): the 5000- and
    2049-row groups are split and merged in-kernel."""
    X, y, off, B = _groups(SIZES, 32, 2)
    res, info = _run(ctx, X, y, off, B, 0.5, zero_leg=True)
    assert info["split_tiles"] >= 2
    _check_both(res, X.astype(np.float64), y, off, B, 0.5)


def test_per_group_prior_mean(ctx):
    X, y, off, B = _groups(SIZES, 24, 3)
    M = np.random.default_rng(4).standard_normal((len(SIZES), 24))
    (got,), _ = _run(ctx, X, y, off, B, 2.0, mean=M, per_group=True)
    _check_groups(got, X.astype(np.float64), y, off, B, 2.0, mean=M)


@pytest.mark.parametrize("K", [4, 8, 16, 64, 128, 256])
def test_widths_and_f64(ctx, K):
    X, y, off, B = _groups([50, 0, 3000, 700, 1], K, 5 + K)
    res, _ = _run(ctx, X, y, off, B, 0.1, zero_leg=True)
    _check_both(res, X.astype(np.float64), y, off, B, 0.1)
    X64 = X.astype(np.float64)
    res64, _ = _run(ctx, X64, y, off, B, 0.1, zero_leg=True)
    _check_both(res64, X64, y, off, B, 0.1, storage="f64")


def test_bf16_and_fp8_groups(ctx):
    X, y, off, B = _groups(SIZES, 64, 6)
    Qb = oracle.quantize_bf16(X)
    res, _ = _run(ctx, Qb, y, off, B, 1.0, dtype=glm.GLM_BF16, zero_leg=True)
    _check_both(res, oracle.decode_bf16(Qb), y, off, B, 1.0, storage="bf16", X_oracle=Qb,
                okw={"dtype": "bf16"})
    Q8, s = oracle.quantize_fp8(X)
    res, _ = _run(ctx, Q8, y, off, B, 1.0, dtype=glm.GLM_FP8_E4M3, scale=to_dev(s), zero_leg=True)
    _check_both(res, oracle.decode_fp8(Q8, s), y, off, B, 1.0, storage="fp8", X_oracle=Q8,
                okw={"dtype": "fp8", "scale": s})


def test_repeated_calls_are_bitwise_identical(ctx):
    X, y, off, B = _groups(SIZES, 32, 7)
    res, _ = _run(ctx, X, y, off, B, 4.0, repeat=3)
    assert np.array_equal(res[0], res[1]) and np.array_equal(res[0], res[2])


def test_group_result_matches_plain_call(ctx):
    """Each group's batched result equals a plain call on that group's rows
    within twice the derived bound (both are FP32-product paths that sum in
    different orders)."""
    X, y, off, B = _groups(SIZES, 32, 8)
    (got,), _ = _run(ctx, X, y, off, B, 4.0)
    for g in (2, 10, 14):
        a, b = off[g], off[g + 1]
        f, gg = eval_gpu(ctx, to_dev(X[a:b]), to_dev(y[a:b]), B[g], 4.0)
        bd = pb.error_bounds(X[a:b].astype(np.float64), y[a:b], B[g], 4.0)
        assert abs(f - got[g, 0]) <= 2 * min(bd["f_worst"], bd["f_prob"])
        assert np.all(np.abs(gg - got[g, 1:]) <= 2 * np.minimum(bd["g_worst"], bd["g_prob"]))
        check_against_oracle(f, gg, X[a:b].astype(np.float64), y[a:b], B[g], 4.0)


def test_invalid_offsets(ctx):
    X, y, off, B = _groups([10, 20], 8, 9)
    Xd, yd = to_dev(X), to_dev(y)
    for bad in ([0, 20, 10], [1, 10, 30], [0, 10, 29]):
        with pytest.raises(glm.GlmError) as e:
            glm.glm_groupset_create(ctx, glm.make_desc(Xd, yd), bad)
        assert e.value.status == glm.GLM_EINVAL


def test_hierarchical_workload_full_size(ctx):
    """2,000 groups, sizes round(LogNormal(ln 500, 1.2)) clipped to
    [20, 50,000], K = 32, FP32; autotuned schedule; every group within its
    derived bound of the oracle."""
    w = synth.hierarchical()
    res, info = _run(ctx, w.X, w.y, w.offsets, w.betas, w.prec, mean=w.mu, tune=True,
                     zero_leg=True)
    print("hierarchical schedule:", info, flush=True)
    _check_both(res, w.X.astype(np.float64), w.y, w.offsets, w.betas, w.prec, mean=w.mu)


@pytest.mark.parametrize("K", [3, 13, 37])
def test_ragged_k_groups(ctx, K):
    """Group rows whose K is not a whole number of 16-byte chunks, padding
    NaN: split and whole groups both ignore the padding."""
    X, y, off, B = _groups(SIZES, K, 40 + K)
    step = 4
    ld = (K + step - 1) // step * step + step
    buf = np.full((X.shape[0], ld), np.nan, np.float32)
    buf[:, :K] = X
    Xd = torch.from_numpy(buf).to(DEV)[:, :K]
    yd = to_dev(y)
    gs = glm.glm_groupset_create(ctx, glm.make_desc(Xd, yd), off, tune=False)
    out = torch.full((len(SIZES), K + 1), float("nan"), dtype=torch.float64, device=DEV)
    glm.glm_logpost_grad_batched(ctx, gs, to_dev(B), glm.make_prior(1.0), out)
    torch.cuda.synchronize()
    glm.glm_groupset_destroy(gs)
    _check_groups(out.cpu().numpy(), X.astype(np.float64), y, off, B, 1.0)

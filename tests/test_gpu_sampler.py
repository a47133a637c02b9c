"""The on-device random-walk Metropolis loop (glm_mh_run) against the oracle:
the chain is replayed on the CPU with the same increments and log-uniforms,
every decision the oracle settles beyond the tolerance band must match, and
the recorded f trace and final state must agree with the oracle."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402

if torch.cuda.is_available():
    from gpu_helpers import DEV, Ctx, to_dev  # noqa: E402
    from paper_1310_1537_amd import glm  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


def _run(ctx, ds, beta0, incs, logu, prec, n=None, stream=None):
    n = len(logu) if n is None else n
    K = len(beta0)
    b = to_dev(beta0)
    fg = torch.empty(K + 1, dtype=torch.float64, device=DEV)
    acc = torch.zeros(max(n, 1), dtype=torch.uint8, device=DEV)
    tr = torch.zeros(max(n, 1), dtype=torch.float64, device=DEV)
    inc_d, lu_d = to_dev(incs), to_dev(logu)     # alive until the chain has run
    glm.glm_mh_run(ctx, ds, b, fg, inc_d, lu_d, n, glm.make_prior(prec), acc, tr, stream)
    torch.cuda.synchronize()
    return b.cpu().numpy(), fg.cpu().numpy(), acc.cpu().numpy()[:n], tr.cpu().numpy()[:n]


def _replay(X, y, beta0, incs, logu, prec, acc_gpu, trace_gpu, tol, okw=None):
    """Replays the chain with the oracle, following the GPU's decisions;
    returns (final beta, number of oracle-settled steps, accept count)."""
    okw = okw or {}
    beta = beta0.copy()
    f_cur, _ = oracle.logpost_grad(X, y, beta, prec, **okw)
    settled = 0
    for t in range(len(logu)):
        bp = beta + incs[t]
        fp, _ = oracle.logpost_grad(X, y, bp, prec, **okw)
        d = fp - f_cur
        band = tol * (abs(fp) + abs(f_cur))
        if abs(logu[t] - d) > band:
            settled += 1
            assert bool(acc_gpu[t]) == bool(logu[t] < d), (t, logu[t], d)
        if acc_gpu[t]:
            beta, f_cur = bp, fp
        assert abs(trace_gpu[t] - f_cur) <= tol * abs(f_cur), (t, trace_gpu[t], f_cur)
    return beta, settled, int(acc_gpu.sum())


def test_small_fp64_chain_matches_the_oracle(ctx):
    w = synth.plain_small(1)
    N, K = w.X.shape
    incs, logu, _ = synth.mh_chain_inputs(K, 2000, N, workload_index=0)
    Xd, yd = to_dev(w.X), to_dev(w.y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xd, yd))
    b, fg, acc, tr = _run(ctx, ds, w.beta_true, incs, logu, w.prec)
    beta, settled, n_acc = _replay(w.X, w.y, w.beta_true, incs, logu, w.prec, acc, tr, 1e-12)
    assert 0.1 < n_acc / 2000 < 0.6 and settled > 1990
    np.testing.assert_array_equal(b, beta)
    fo, go = oracle.logpost_grad(w.X, w.y, beta, w.prec)
    assert abs(fg[0] - fo) <= 1e-12 * abs(fo)
    assert np.linalg.norm(fg[1:] - go) <= 1e-10 * np.linalg.norm(go)
    glm.glm_dataset_unregister(ctx, ds)


def test_fp32_chain_matches_the_oracle(ctx):
    w = synth.plain_big(200_000, 64, 1)
    N, K = w.X.shape
    incs, logu, _ = synth.mh_chain_inputs(K, 400, N, workload_index=1)
    Xd, yd = to_dev(w.X), to_dev(w.y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xd, yd))
    b, fg, acc, tr = _run(ctx, ds, w.beta_true, incs, logu, w.prec)
    beta, settled, n_acc = _replay(w.X, w.y, w.beta_true, incs, logu, w.prec, acc, tr, 1e-9)
    assert 0.05 < n_acc / 400 < 0.7 and settled > 380
    np.testing.assert_array_equal(b, beta)
    glm.glm_dataset_unregister(ctx, ds)


def test_split_run_equals_one_run_bitwise(ctx):
    w = synth.plain_small(1)
    N, K = w.X.shape
    incs, logu, _ = synth.mh_chain_inputs(K, 500, N, workload_index=0)
    Xd, yd = to_dev(w.X), to_dev(w.y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xd, yd))
    b1, fg1, acc1, tr1 = _run(ctx, ds, w.beta_true, incs, logu, w.prec)
    bh, _, acch, trh = _run(ctx, ds, w.beta_true, incs[:300], logu[:300], w.prec)
    b2, fg2, acc2, tr2 = _run(ctx, ds, bh, incs[300:], logu[300:], w.prec)
    np.testing.assert_array_equal(b1, b2)
    np.testing.assert_array_equal(fg1, fg2)
    np.testing.assert_array_equal(acc1, np.concatenate([acch, acc2]))
    np.testing.assert_array_equal(tr1, np.concatenate([trh, tr2]))
    # on another stream, the same chain
    s = torch.cuda.Stream()
    b3, fg3, acc3, _ = _run(ctx, ds, w.beta_true, incs, logu, w.prec, stream=s)
    np.testing.assert_array_equal(b1, b3)
    np.testing.assert_array_equal(acc1, acc3)
    glm.glm_dataset_unregister(ctx, ds)


def test_zero_steps_and_poisson_chain(ctx):
    g = np.random.default_rng(3)
    N, K = 30_000, 16
    X = g.standard_normal((N, K))
    bt = 0.5 * g.standard_normal(K) / math.sqrt(K)
    y = np.minimum(g.poisson(np.exp(X @ bt)), 255).astype(np.uint8)
    Xd, yd = to_dev(X), to_dev(y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xd, yd, family=glm.GLM_POISSON))
    b, fg, _, _ = _run(ctx, ds, bt, np.zeros((0, K)), np.zeros(0), 0.5, n=0)
    fo, _ = oracle.logpost_grad(X, y, bt, 0.5, family="poisson")
    assert abs(fg[0] - fo) <= 1e-12 * abs(fo)
    sd = 2.38 / math.sqrt(K) / math.sqrt(N)
    incs = sd * g.standard_normal((300, K))
    logu = np.log(g.random(300))
    b, fg, acc, tr = _run(ctx, ds, bt, incs, logu, 0.5)
    beta, settled, n_acc = _replay(X, y, bt, incs, logu, 0.5, acc, tr, 1e-12,
                                   {"family": "poisson"})
    assert n_acc > 10 and settled > 290
    np.testing.assert_array_equal(b, beta)
    glm.glm_dataset_unregister(ctx, ds)


def test_bad_arguments(ctx):
    w = synth.plain_small(1)
    Xd, yd = to_dev(w.X), to_dev(w.y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xd, yd))
    b = to_dev(w.beta_true)
    fg = torch.empty(21, dtype=torch.float64, device=DEV)
    with pytest.raises(glm.GlmError) as e:
        glm.glm_mh_run(ctx, ds, b, fg, None, None, 5, glm.make_prior(0.01))
    assert e.value.status == glm.GLM_EINVAL
    with pytest.raises(glm.GlmError) as e:
        glm.glm_mh_run(ctx, 12345, b, fg, None, None, 0, glm.make_prior(0.01))
    assert e.value.status == glm.GLM_ENOTFOUND
    glm.glm_dataset_unregister(ctx, ds)

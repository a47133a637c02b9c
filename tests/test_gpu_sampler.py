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


# ------------------------------------------------------------ device generator

def _fill(ctx, kind, seed, chain, stream_id, offset, n, scale=1.0):
    out = torch.full((max(n, 1),), float("nan"), dtype=torch.float64, device=DEV)
    glm.glm_rng_fill(ctx, kind, seed, chain, stream_id, offset, n, out, scale)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:n]


@pytest.mark.parametrize("offset,n", [(0, 4), (3, 1), (6, 10_001), (2 ** 40 + 1, 37)])
def test_rng_uniforms_bitwise_and_log_uniforms(ctx, offset, n):
    """Uniforms equal the oracle's stream bit for bit; log-uniforms are the
    library's log of the same values (within 4 ulps of the C library's)."""
    got = _fill(ctx, glm.GLM_RNG_UNIFORM, 77, 5, 12, offset, n)
    ref = oracle.rng_uniforms(77, 5, 12, offset, n)
    np.testing.assert_array_equal(got, ref)
    lg = _fill(ctx, glm.GLM_RNG_LOG_UNIFORM, 77, 5, 12, offset, n)
    lr = np.log(ref)
    assert np.all(np.abs(lg - lr) <= 4 * np.spacing(np.abs(lr)))


@pytest.mark.parametrize("offset,n", [(0, 2), (1, 1), (5, 20_001)])
def test_rng_normals_match_the_oracle(ctx, offset, n):
    """Same attempts (u, v and s are exact, equal bits on both sides), so
    the normals differ only by the two logarithms' last bits."""
    got = _fill(ctx, glm.GLM_RNG_NORMAL, 3, 9, 4, offset, n, scale=0.5)
    ref = 0.5 * oracle.rng_normals(3, 9, 4, offset, n)
    assert np.all(np.abs(got - ref) <= 8 * np.spacing(np.abs(ref)) + 1e-300)


def test_rng_fills_join_and_reject_bad_arguments(ctx):
    a = _fill(ctx, glm.GLM_RNG_NORMAL, 1, 2, 3, 0, 1001)
    b = np.concatenate([_fill(ctx, glm.GLM_RNG_NORMAL, 1, 2, 3, 0, 500),
                        _fill(ctx, glm.GLM_RNG_NORMAL, 1, 2, 3, 500, 501)])
    np.testing.assert_array_equal(a, b)
    out = torch.zeros(4, dtype=torch.float64, device=DEV)
    for kind, n in ((9, 4), (glm.GLM_RNG_UNIFORM, -1)):
        with pytest.raises(glm.GlmError) as e:
            glm.glm_rng_fill(ctx, kind, 0, 0, 0, 0, n, out)
        assert e.value.status == glm.GLM_EINVAL


def test_metropolis_with_device_drawn_inputs(ctx):
    """Increments and log-uniforms drawn on the device (glm_rng_fill) drive
    glm_mh_run; the oracle replays the chain with its own draws of the same
    streams: every decision it settles agrees, the states agree to rounding."""
    w = synth.plain_small(1)
    N, K = w.X.shape
    n = 600
    sd = 2.38 / math.sqrt(K) / math.sqrt(0.2 * N)
    incs = torch.empty(n * K, dtype=torch.float64, device=DEV)
    logu = torch.empty(n, dtype=torch.float64, device=DEV)
    glm.glm_rng_fill(ctx, glm.GLM_RNG_NORMAL, 2024, 1, 0, 0, n * K, incs, sd)
    glm.glm_rng_fill(ctx, glm.GLM_RNG_LOG_UNIFORM, 2024, 1, 1, 0, n, logu)
    Xd, yd = to_dev(w.X), to_dev(w.y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xd, yd))
    b = to_dev(w.beta_true)
    fg = torch.empty(K + 1, dtype=torch.float64, device=DEV)
    acc = torch.zeros(n, dtype=torch.uint8, device=DEV)
    tr = torch.zeros(n, dtype=torch.float64, device=DEV)
    glm.glm_mh_run(ctx, ds, b, fg, incs, logu, n, glm.make_prior(w.prec), acc, tr)
    torch.cuda.synchronize()
    acc = acc.cpu().numpy()
    inc_o = sd * oracle.rng_normals(2024, 1, 0, 0, n * K).reshape(n, K)
    lu_o = np.log(oracle.rng_uniforms(2024, 1, 1, 0, n))
    beta = w.beta_true.copy()
    f_cur, _ = oracle.logpost_grad(w.X, w.y, beta, w.prec)
    settled = 0
    for t in range(n):
        bp = beta + inc_o[t]
        fp, _ = oracle.logpost_grad(w.X, w.y, bp, w.prec)
        d = fp - f_cur
        if abs(lu_o[t] - d) > 1e-10 * (abs(fp) + abs(f_cur)):
            settled += 1
            assert bool(acc[t]) == bool(lu_o[t] < d), t
        if acc[t]:
            beta, f_cur = bp, fp
    assert settled > n - 5 and 0.1 < acc.mean() < 0.6
    np.testing.assert_allclose(b.cpu().numpy(), beta, rtol=1e-12, atol=1e-14)
    glm.glm_dataset_unregister(ctx, ds)


# ------------------------------------------------------------ HMC

def _hmc(ctx, ds, beta0, n_iter, n_leap, eps, seed, chain, prec, iter0=0):
    K = len(beta0)
    b = to_dev(beta0)
    fg = torch.empty(K + 1, dtype=torch.float64, device=DEV)
    acc = torch.zeros(max(n_iter, 1), dtype=torch.uint8, device=DEV)
    tr = torch.zeros(max(n_iter, 1), dtype=torch.float64, device=DEV)
    glm.glm_hmc_run(ctx, ds, b, fg, n_iter, n_leap, eps, seed, chain, glm.make_prior(prec), acc,
                    tr, iter0=iter0)
    torch.cuda.synchronize()
    return (b.cpu().numpy(), fg.cpu().numpy(), acc.cpu().numpy()[:n_iter],
            tr.cpu().numpy()[:n_iter])


def _hmc_replay(X, y, beta0, prec, n_iter, n_leap, eps, seed, chain, acc, tol, iter0=0):
    """The oracle's HMC chain following the GPU's decisions; every decision
    the oracle settles outside the band must agree."""
    r = oracle.hmc_chain(X, y, beta0, prec, n_iter, n_leap, eps, seed, chain, follow=acc,
                         iter0=iter0)
    settled = 0
    for t in range(n_iter):
        if abs(r["logu"][t] - r["dH"][t]) > tol:
            settled += 1
            assert bool(acc[t]) == bool(r["logu"][t] < r["dH"][t]), (t, r["logu"][t], r["dH"][t])
    return r, settled


def test_hmc_small_fp64_chain_matches_the_oracle(ctx):
    w = synth.plain_small(1)
    Xd, yd = to_dev(w.X), to_dev(w.y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xd, yd))
    n_iter, L, eps = 60, 5, 0.01
    b, fg, acc, tr = _hmc(ctx, ds, w.beta_true, n_iter, L, eps, 7, 1, w.prec)
    r, settled = _hmc_replay(w.X, w.y, w.beta_true, w.prec, n_iter, L, eps, 7, 1, acc, 1e-9)
    assert settled >= n_iter - 2 and 0.5 < acc.mean() <= 1.0 and 0 < acc.sum() < n_iter
    np.testing.assert_allclose(b, r["beta"], rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(tr, r["f_trace"], rtol=1e-12)
    assert abs(fg[0] - r["f"]) <= 1e-12 * abs(r["f"])
    np.testing.assert_allclose(fg[1:], r["g"], rtol=1e-8, atol=1e-9)
    glm.glm_dataset_unregister(ctx, ds)


def test_hmc_fp32_chain_matches_the_oracle(ctx):
    w = synth.plain_big(200_000, 64, 1)
    Xd, yd = to_dev(w.X), to_dev(w.y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xd, yd))
    n_iter, L, eps = 12, 6, 0.002
    b, fg, acc, tr = _hmc(ctx, ds, w.beta_true, n_iter, L, eps, 11, 4, w.prec)
    r, settled = _hmc_replay(w.X, w.y, w.beta_true, w.prec, n_iter, L, eps, 11, 4, acc, 1e-6)
    assert settled >= n_iter - 1 and acc.sum() > 0
    np.testing.assert_allclose(b, r["beta"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(tr, r["f_trace"], rtol=1e-11)
    glm.glm_dataset_unregister(ctx, ds)


def test_hmc_split_run_and_streams(ctx):
    """A chain run in two pieces (iter0 = 25 for the second) is the same
    chain, bit for bit; on another stream too; n_iter = 0 evaluates the
    start only; bad arguments are refused."""
    w = synth.plain_small(1)
    Xd, yd = to_dev(w.X), to_dev(w.y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xd, yd))
    b1, fg1, acc1, tr1 = _hmc(ctx, ds, w.beta_true, 40, 3, 0.012, 5, 2, w.prec)
    bh, _, acch, trh = _hmc(ctx, ds, w.beta_true, 25, 3, 0.012, 5, 2, w.prec)
    b2, fg2, acc2, tr2 = _hmc(ctx, ds, bh, 15, 3, 0.012, 5, 2, w.prec, iter0=25)
    np.testing.assert_array_equal(b1, b2)
    np.testing.assert_array_equal(fg1, fg2)
    np.testing.assert_array_equal(acc1, np.concatenate([acch, acc2]))
    np.testing.assert_array_equal(tr1, np.concatenate([trh, tr2]))
    b0, fg0, _, _ = _hmc(ctx, ds, w.beta_true, 0, 3, 0.012, 5, 2, w.prec)
    np.testing.assert_array_equal(b0, w.beta_true)
    fo, _ = oracle.logpost_grad(w.X, w.y, w.beta_true, w.prec)
    assert abs(fg0[0] - fo) <= 1e-12 * abs(fo)
    bt = to_dev(w.beta_true)
    fgt = torch.empty(21, dtype=torch.float64, device=DEV)
    for n_leap, eps in ((0, 0.01), (3, 0.0), (3, -1.0)):
        with pytest.raises(glm.GlmError) as e:
            glm.glm_hmc_run(ctx, ds, bt, fgt, 5, n_leap, eps, 1, 1, glm.make_prior(w.prec))
        assert e.value.status == glm.GLM_EINVAL
    glm.glm_dataset_unregister(ctx, ds)

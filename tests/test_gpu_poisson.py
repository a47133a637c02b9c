"""GPU parity of the Poisson response family (log link; only the per-row map
differs from the logistic model) on every entry point that evaluates f and
g: plain, several-beta, batched groups, differential update and the server."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import parity_bounds as pb  # noqa: E402
import sweeps  # noqa: E402
import synth  # noqa: E402

if torch.cuda.is_available():
    from gpu_helpers import (DEV, Ctx, check_against_oracle, eval_gpu, sweep_point,  # noqa: E402
                             to_dev)
    from paper_1310_1537_amd import glm  # noqa: E402

POI = {"family": "poisson"}


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


_data = sweeps.poisson


@pytest.mark.parametrize("K", sweeps.POISSON_K)
@pytest.mark.parametrize("N", sweeps.POISSON_N)
def test_plain_f32(ctx, K, N):
    X, y, beta = _data(N, K, K + N)
    Xd, yd = to_dev(X), to_dev(y)
    if (K * 4) % 16:
        Xd = glm.aligned_rows(Xd)
    sweep_point(ctx, Xd, yd, X.astype(np.float64), y, beta, 0.01, oracle_kw=POI,
                family=glm.GLM_POISSON)


@pytest.mark.parametrize("kind", ["f64", "bf16", "fp8"])
def test_plain_other_storage(ctx, kind):
    X, y, beta = _data(20_011, 96, 3)
    m = np.linspace(-0.1, 0.1, 96)
    yd = to_dev(y)
    if kind == "f64":
        X64 = X.astype(np.float64)
        f, g = eval_gpu(ctx, to_dev(X64), yd, beta, 0.5, m, family=glm.GLM_POISSON)
        check_against_oracle(f, g, X64, y, beta, 0.5, m, storage="f64", oracle_kw=POI)
    elif kind == "bf16":
        Q = oracle.quantize_bf16(X)
        f, g = eval_gpu(ctx, to_dev(Q), yd, beta, 0.5, m, dtype=glm.GLM_BF16,
                        family=glm.GLM_POISSON)
        check_against_oracle(f, g, oracle.decode_bf16(Q), y, beta, 0.5, m, storage="bf16",
                             X_for_oracle=Q, oracle_kw={"dtype": "bf16", **POI})
    else:
        Q, s = oracle.quantize_fp8(X)
        f, g = eval_gpu(ctx, to_dev(Q), yd, beta, 0.5, m, dtype=glm.GLM_FP8_E4M3,
                        scale=to_dev(s), family=glm.GLM_POISSON)
        check_against_oracle(f, g, oracle.decode_fp8(Q, s), y, beta, 0.5, m, storage="fp8",
                             X_for_oracle=Q, oracle_kw={"dtype": "fp8", "scale": s, **POI})


def test_closed_form_at_zero(ctx):
    """beta = 0 gives f = -N exactly (every row contributes -exp(0))."""
    X, y, _ = _data(12_345, 32, 4)
    f, g = eval_gpu(ctx, to_dev(X), to_dev(y), np.zeros(32), 0.0, family=glm.GLM_POISSON)
    assert f == -12_345.0
    # g = X^t (y - 1): only the FP32 products and partial sums round
    check_against_oracle(f, g, X.astype(np.float64), y, np.zeros(32), 0.0, oracle_kw=POI)


def test_multi(ctx):
    X, y, beta = _data(30_011, 40, 5)
    Xd, yd = to_dev(X), to_dev(y)
    Xa = glm.aligned_rows(Xd)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xa, yd, family=glm.GLM_POISSON))
    B = beta + 0.02 * np.random.default_rng(6).standard_normal((7, 40))
    out = torch.empty((7, 41), dtype=torch.float64, device=DEV)
    glm.glm_logpost_grad_multi(ctx, ds, to_dev(B), 7, glm.make_prior(0.01), out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    for b in range(7):
        check_against_oracle(o[b, 0], o[b, 1:], X.astype(np.float64), y, B[b], 0.01,
                             oracle_kw=POI)
    glm.glm_dataset_unregister(ctx, ds)


def test_batched_groups(ctx):
    sizes = [0, 5, 64, 700, 3000, 129, 2049, 1]
    K = 16
    g = np.random.default_rng(7)
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    X = g.standard_normal((int(off[-1]), K)).astype(np.float32)
    B = 0.3 * g.standard_normal((len(sizes), K)) / math.sqrt(K)
    y = np.empty(int(off[-1]), np.uint8)
    for i in range(len(sizes)):
        a, b = off[i], off[i + 1]
        y[a:b] = np.minimum(g.poisson(np.exp(X[a:b].astype(np.float64) @ B[i])), 255)
    Xd, yd = to_dev(X), to_dev(y)
    gs = glm.glm_groupset_create(ctx, glm.make_desc(Xd, yd, family=glm.GLM_POISSON), off,
                                 tune=False)
    out = torch.empty((len(sizes), K + 1), dtype=torch.float64, device=DEV)
    glm.glm_logpost_grad_batched(ctx, gs, to_dev(B), glm.make_prior(4.0), out)
    torch.cuda.synchronize()
    glm.glm_groupset_destroy(gs)
    got = out.cpu().numpy()
    ref = oracle.logpost_grad_groups(X, y, off, B, 4.0, family="poisson")
    X64 = X.astype(np.float64)
    for i in range(len(sizes)):
        a, b = off[i], off[i + 1]
        pb.check(got[i, 0], got[i, 1:], X64[a:b], y[a:b], B[i], 4.0, None, "f32", "poisson",
                 ref=(ref[i, 0], ref[i, 1:]))


def test_differential_update(ctx):
    N, K = 25_000, 12
    X, y, beta = _data(N, K, 8)
    Xd, yd = to_dev(X), to_dev(y)
    Xt = torch.empty((K, N), dtype=torch.float32, device=DEV)
    glm.glm_transpose(ctx, glm.make_desc(glm.aligned_rows(Xd), yd), Xt, N)
    cs = glm.glm_colset_register(ctx, glm.make_colset_desc(Xt, yd, family=glm.GLM_POISSON))
    bd = to_dev(beta)
    u = torch.empty(N, dtype=torch.float64, device=DEV)
    glm.glm_linpred(ctx, cs, bd, u)
    deltas = np.array([-0.2, 0.0, 0.15])
    out = torch.empty(3, dtype=torch.float64, device=DEV)
    glm.glm_diff_logpost(ctx, cs, u, bd, 5, to_dev(deltas), 3, glm.make_prior(0.01), out)
    torch.cuda.synchronize()
    for j, d in enumerate(deltas):
        b2 = beta.copy()
        b2[5] += d
        f, _ = oracle.logpost_grad(X, y, b2, 0.01, family="poisson")
        A = np.abs(X.astype(np.float64)) @ np.abs(b2)
        bound = (2 * K + 4) * 2.0 ** -53 * np.sum(A * (1 + y + np.exp(X.astype(np.float64) @ b2)))
        assert abs(out.cpu().numpy()[j] - f) <= bound + 1e-13 * abs(f)
    glm.glm_colset_unregister(ctx, cs)


def test_server_mixes_families(ctx):
    """Logistic and Poisson data sets served side by side; every result
    matches its own model's oracle."""
    Xp, yp, bp = _data(20_000, 32, 9)
    gl = np.random.default_rng(10)
    Xl = gl.standard_normal((15_000, 32)).astype(np.float32)
    yl = (gl.random(15_000) < 0.5).astype(np.uint8)
    srv = glm.glm_server_create(ctx, 1 << 32, 8, 2, 4, 1 << 16)
    dp = glm.glm_server_add_dataset(srv, glm.make_host_desc(Xp, yp, family=glm.GLM_POISSON))
    dl = glm.glm_server_add_dataset(srv, glm.make_host_desc(Xl, yl))
    rng = np.random.default_rng(11)
    reqs = []
    for i in range(40):
        poisson = i % 2 == 0
        beta = (bp if poisson else np.zeros(32)) + 0.05 * rng.standard_normal(32)
        reqs.append((poisson, beta, glm.glm_server_submit(srv, dp if poisson else dl, beta, 0.01)))
    for poisson, beta, t in reqs:
        g = np.empty(32)
        f = glm.glm_server_wait(srv, t, g)
        if poisson:
            check_against_oracle(f, g, Xp.astype(np.float64), yp, beta, 0.01, oracle_kw=POI)
        else:
            check_against_oracle(f, g, Xl.astype(np.float64), yl, beta, 0.01)
    glm.glm_server_destroy(srv)


def test_poisson_workload_full_size(ctx):
    """N = 4,000,000, K = 256 Poisson workload at its first trajectory point,
    within the derived bound of the oracle and f <= 1e-9, g <= 1e-7
    relative."""
    w = synth.plain_poisson(n_evals=1)
    f, g = eval_gpu(ctx, to_dev(w.X), to_dev(w.y), w.betas[0], w.prec, family=glm.GLM_POISSON)
    fo, go = oracle.logpost_grad_blocks(w.X, w.y, w.betas[0], w.prec, family="poisson")
    assert abs(f - fo) <= 1e-9 * abs(fo)
    assert np.linalg.norm(g - go) <= 1e-7 * np.linalg.norm(go)

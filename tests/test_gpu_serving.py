"""GPU tests of the several-beta pass (glm_logpost_grad_multi) and of the
request server (continuous batching over resident data sets)."""
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import sweeps  # noqa: E402

if torch.cuda.is_available():
    from gpu_helpers import DEV, Ctx, check_against_oracle, to_dev  # noqa: E402
    from paper_1310_1537_amd import glm  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


_data = sweeps.serving_data
_betas = sweeps.betas_near


def _check(f, g, Xd, y, beta, prec, mean=None, storage="f32", Xo=None, okw=None):
    check_against_oracle(f, g, Xd, y, beta, prec, mean, storage, X_for_oracle=Xo,
                         oracle_kw=okw)


def _multi(ctx, ds, B, K, prec=0.01, M=None):
    nb = len(B)
    out = torch.full((nb, K + 1), float("nan"), dtype=torch.float64, device=DEV)
    glm.glm_logpost_grad_multi(ctx, ds, to_dev(B), nb,
                               glm.make_prior(prec, None if M is None else to_dev(M)), out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("K", sweeps.MULTI_K)
@pytest.mark.parametrize("nb", sweeps.MULTI_NB)
def test_multi_against_oracle(ctx, K, nb):
    """Every vector of the passes against the oracle, at its beta and (a
    second call) at beta = 0 in every slot."""
    X, y, bt = _data(20_011, K, K + nb)
    B = _betas(bt, nb, 7)
    Xd, yd = to_dev(X), to_dev(y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xd, yd))
    for Bc in (B, np.zeros_like(B)):
        o = _multi(ctx, ds, Bc, K)
        for b in range(nb):
            _check(o[b, 0], o[b, 1:], X.astype(np.float64), y, Bc[b], 0.01)
    glm.glm_dataset_unregister(ctx, ds)


def test_multi_per_vector_means_and_bf16(ctx):
    X, y, bt = _data(9_000, 64, 3)
    Q = oracle.quantize_bf16(X)
    B = _betas(bt, 5, 8)
    M = np.random.default_rng(9).standard_normal((5, 64))
    Qd, yd = to_dev(Q), to_dev(y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Qd, yd, dtype=glm.GLM_BF16))
    out = torch.empty((5, 65), dtype=torch.float64, device=DEV)
    glm.glm_logpost_grad_multi(ctx, ds, to_dev(B), 5, glm.make_prior(2.0, to_dev(M)), out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    for b in range(5):
        _check(o[b, 0], o[b, 1:], oracle.decode_bf16(Q), y, B[b], 2.0, M[b], storage="bf16", Xo=Q,
               okw={"dtype": "bf16"})
    glm.glm_dataset_unregister(ctx, ds)


@pytest.mark.parametrize("K", [8, 16, 24, 32])
@pytest.mark.parametrize("nb", [3, 4, 11])
def test_multi_bf16_short_rows(ctx, K, nb):
    """BF16 rows of at most 32 columns (one chunk on at most four lanes, the
    instances with four row slots; at K = 24 the fourth lane holds no column)
    against the oracle on the codes, at beta and at beta = 0."""
    X, y, bt = _data(20_011, K, 3 * K + nb)
    Q = oracle.quantize_bf16(X)
    B = _betas(bt, nb, 9)
    Qd, yd = to_dev(Q), to_dev(y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Qd, yd, dtype=glm.GLM_BF16))
    for Bc in (B, np.zeros_like(B)):
        o = _multi(ctx, ds, Bc, K)
        for b in range(nb):
            _check(o[b, 0], o[b, 1:], oracle.decode_bf16(Q), y, Bc[b], 0.01, storage="bf16", Xo=Q,
                   okw={"dtype": "bf16"})
    glm.glm_dataset_unregister(ctx, ds)


@pytest.mark.parametrize("K,dt", [(200, np.float64), (256, np.float64), (300, np.float64),
                                  (512, np.float64), (600, np.float32), (1024, np.float32)])
@pytest.mark.parametrize("nb", [2, 3, 4, 8])
def test_multi_wide_rows(ctx, K, dt, nb):
    """Rows of 2 to 4 chunks per lane (FP64 rows of 129 to 512 columns, FP32
    rows of 513 to 1024), the instances with 4 row slots, against the oracle
    at beta and at beta = 0."""
    X, y, bt = _data(9_001, K, 5 * K + nb, dt)
    B = _betas(bt, nb, 11)
    Xd, yd = to_dev(X), to_dev(y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xd, yd))
    storage = "f64" if dt == np.float64 else "f32"
    for Bc in (B, np.zeros_like(B)):
        o = _multi(ctx, ds, Bc, K)
        for b in range(nb):
            _check(o[b, 0], o[b, 1:], X.astype(np.float64), y, Bc[b], 0.01, storage=storage)
    glm.glm_dataset_unregister(ctx, ds)


def test_multi_result_independent_of_companions(ctx):
    """Slot 0 of a pass gives the same bits whatever the other slots hold."""
    X, y, bt = _data(30_000, 128, 4)
    B = _betas(bt, 8, 10)
    Xd, yd = to_dev(X), to_dev(y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xd, yd))
    out8 = torch.empty((8, 129), dtype=torch.float64, device=DEV)
    glm.glm_logpost_grad_multi(ctx, ds, to_dev(B), 8, glm.make_prior(0.01), out8)
    B2 = B.copy()
    B2[1:] = _betas(bt, 7, 11)
    out8b = torch.empty((8, 129), dtype=torch.float64, device=DEV)
    glm.glm_logpost_grad_multi(ctx, ds, to_dev(B2), 8, glm.make_prior(0.01), out8b)
    torch.cuda.synchronize()
    assert np.array_equal(out8.cpu().numpy()[0], out8b.cpu().numpy()[0])
    glm.glm_dataset_unregister(ctx, ds)


# ------------------------------------------------------------------ server

def _server(ctx, budget=1 << 34, nbmax=8, slots=8, streams=4, qcap=1 << 20, max_sets=0):
    return glm.glm_server_create(ctx, budget, nbmax, streams, slots, qcap, max_sets)


def test_server_results_match_oracle(ctx):
    sets = [_data(5_000, 8, 20), _data(12_345, 32, 21), _data(3_000, 128, 22, np.float64)]
    srv = _server(ctx)
    ids = [glm.glm_server_add_dataset(srv, glm.make_host_desc(X, y)) for X, y, _ in sets]
    reqs = []
    rng = np.random.default_rng(23)
    for i in range(120):
        d = int(rng.integers(0, 3))
        beta = sets[d][2] + 0.1 * rng.standard_normal(sets[d][0].shape[1])
        reqs.append((d, beta, glm.glm_server_submit(srv, ids[d], beta, 0.01)))
    for d, beta, t in reqs:
        X, y, _ = sets[d]
        g = np.empty(X.shape[1])
        f = glm.glm_server_wait(srv, t, g)
        _check(f, g, X.astype(np.float64), y, beta, 0.01,
               storage="f64" if X.dtype == np.float64 else "f32")
    st = glm.glm_server_stats(srv)
    assert st["completed"] == 120 and st["failed"] == 0
    assert st["betas_in_passes"] == 120 and st["passes"] <= 120
    glm.glm_server_destroy(srv)


def test_server_alone_equals_in_mix_bitwise(ctx):
    """A request's result is the same bits alone in its pass and packed with
    seven other chains' requests (the slot position may differ too)."""
    X, y, bt = _data(1_000_000, 128, 30)
    srv = _server(ctx, slots=1, streams=1)   # one slot: later requests queue up
    ds = glm.glm_server_add_dataset(srv, glm.make_host_desc(X, y))
    B = _betas(bt, 16, 31)
    alone = []
    for b in range(8):
        t = glm.glm_server_submit(srv, ds, B[b], 0.01)
        g = np.empty(128)
        f = glm.glm_server_wait(srv, t, g)
        alone.append((f, g))
    # keep the single slot busy with a pass, queue 8+ requests behind it
    ts = [glm.glm_server_submit(srv, ds, B[8 + b], 0.01) for b in range(8)]
    ts = [glm.glm_server_submit(srv, ds, B[(7 - b)], 0.01) for b in range(8)] + ts
    mixed = {}
    for k, t in enumerate(ts[:8]):
        g = np.empty(128)
        f = glm.glm_server_wait(srv, t, g)
        mixed[7 - k] = (f, g)
    for t in ts[8:]:
        glm.glm_server_wait(srv, t)
    st = glm.glm_server_stats(srv)
    assert sum(st["pass_width_hist"][2:]) >= 1, st["pass_width_hist"]   # some packing happened
    for b in range(8):
        assert mixed[b][0] == alone[b][0]
        assert np.array_equal(mixed[b][1], alone[b][1])
    glm.glm_server_destroy(srv)


def test_server_admission_and_eviction(ctx):
    """Budget for one data set at a time: alternating requests force
    evictions; results stay exact."""
    a = _data(40_000, 32, 40)
    b = _data(40_000, 32, 41)
    one = 40_000 * 32 * 4 + 40_000
    srv = _server(ctx, budget=int(1.5 * one), slots=1, streams=1)
    ia = glm.glm_server_add_dataset(srv, glm.make_host_desc(a[0], a[1]))
    ib = glm.glm_server_add_dataset(srv, glm.make_host_desc(b[0], b[1]))
    for r in range(4):
        for (X, y, bt), i in ((a, ia), (b, ib)):
            beta = bt + 0.01 * r
            g = np.empty(32)
            f = glm.glm_server_wait(srv, glm.glm_server_submit(srv, i, beta, 0.01), g)
            _check(f, g, X.astype(np.float64), y, beta, 0.01)
    st = glm.glm_server_stats(srv)
    assert st["evictions"] >= 6 and st["admissions"] >= 7
    assert st["resident_datasets"] == 1
    glm.glm_server_destroy(srv)


def _serve_all(srv, ids, sets, reqs):
    """Submits every (data set index, beta) at once, then waits for each;
    returns [(f, g)]."""
    ts = [glm.glm_server_submit(srv, ids[d], b, 0.01) for d, b in reqs]
    out = []
    for (d, _), t in zip(reqs, ts):
        g = np.empty(sets[d][0].shape[1])
        out.append((glm.glm_server_wait(srv, t, g), g))
    return out


def test_server_churn_under_a_binding_budget(ctx):
    """Four host-sourced data sets, a budget that holds one and a half of
    them, 96 requests queued at once in random order: admissions and
    evictions churn while passes run; every result equals (bitwise) the one
    a server with room for all four gives, and is within the oracle bound.
    Afterwards the server holds at most the budget (resident plus evicted
    allocations kept for reuse)."""
    sets = [_data(60_000 + 1000 * i, 32, 70 + i) for i in range(4)]
    one = max(X.shape[0] * (32 * 4 + 1) for X, _, _ in sets)
    rng = np.random.default_rng(75)
    reqs = []
    for _ in range(96):
        d = int(rng.integers(0, 4))
        reqs.append((d, sets[d][2] + 0.05 * rng.standard_normal(32)))
    results = {}
    for budget in (int(1.5 * one), 1 << 34):
        srv = _server(ctx, budget=budget, slots=2, streams=2)
        ids = [glm.glm_server_add_dataset(srv, glm.make_host_desc(X, y)) for X, y, _ in sets]
        results[budget] = _serve_all(srv, ids, sets, reqs)
        st = glm.glm_server_stats(srv)
        assert st["completed"] == 96 and st["failed"] == 0
        if budget < 1 << 34:
            # every set was admitted, and holding one and a half of four forces
            # at least three evictions
            assert st["evictions"] >= 3 and st["admissions"] >= 4, st
            assert st["resident_bytes"] + st["cached_bytes"] <= budget, st
            assert st["bytes_admitted"] >= 4 * 60_000 * 129
        glm.glm_server_destroy(srv)
    small, big = results[int(1.5 * one)], results[1 << 34]
    for (d, beta), (f1, g1), (f2, g2) in zip(reqs, small, big):
        assert f1 == f2 and np.array_equal(g1, g2)
    for k in range(0, 96, 12):
        d, beta = reqs[k]
        X, y, _ = sets[d]
        _check(small[k][0], small[k][1], X.astype(np.float64), y, beta, 0.01)


def test_server_pinned_and_pageable_sources_agree(ctx):
    """A data set given in pinned host memory is copied directly, a pageable
    one through the staging buffers (two chunks of 32 MiB and a tail here):
    same results, bitwise."""
    X, y, bt = _data(300_000, 64, 80)   # 76.8 MB of X
    Xp = torch.from_numpy(X).pin_memory()
    yp = torch.from_numpy(y).pin_memory()
    B = _betas(bt, 3, 81)
    got = []
    for pinned in (False, True):
        srv = _server(ctx)
        if pinned:
            desc = glm.glm_dataset_desc(Xp.data_ptr(), 64, glm.GLM_F32, None, yp.data_ptr(),
                                        300_000, 64, 0)
        else:
            desc = glm.make_host_desc(X, y)
        ds = glm.glm_server_add_dataset(srv, desc)
        r = []
        for b in B:
            g = np.empty(64)
            r.append((glm.glm_server_wait(srv, glm.glm_server_submit(srv, ds, b, 0.01), g), g))
        got.append(r)
        glm.glm_server_destroy(srv)
    for (f1, g1), (f2, g2) in zip(*got):
        assert f1 == f2 and np.array_equal(g1, g2)
    _check(got[0][0][0], got[0][0][1], X.astype(np.float64), y, B[0], 0.01)


def test_server_host_set_must_fit_beside_device_sets(ctx):
    """A device-resident data set is never evicted, so a host-sourced one
    that would not fit beside it is refused at add time (it could never be
    admitted); one that fits is admitted and served."""
    X, y, bt = _data(50_000, 32, 90)
    one = 50_000 * (32 * 4 + 1)
    Xd, yd = to_dev(X), to_dev(y)
    srv = _server(ctx, budget=int(1.6 * one))
    glm.glm_server_add_dataset(srv, glm.make_desc(Xd, yd), on_device=True)
    Xb, yb, btb = _data(50_000, 32, 91)
    with pytest.raises(glm.GlmError) as e:
        glm.glm_server_add_dataset(srv, glm.make_host_desc(Xb, yb))
    assert e.value.status == glm.GLM_EBUDGET
    Xs, ys, bts = _data(20_000, 32, 92)
    ds = glm.glm_server_add_dataset(srv, glm.make_host_desc(Xs, ys))
    g = np.empty(32)
    f = glm.glm_server_wait(srv, glm.glm_server_submit(srv, ds, bts, 0.01), g)
    _check(f, g, Xs.astype(np.float64), ys, bts, 0.01)
    glm.glm_server_destroy(srv)


def test_server_budget_and_unknown_ids(ctx):
    X, y, _ = _data(1000, 8, 50)
    srv = _server(ctx, budget=1000)
    with pytest.raises(glm.GlmError) as e:
        glm.glm_server_add_dataset(srv, glm.make_host_desc(X, y))
    assert e.value.status == glm.GLM_EBUDGET
    with pytest.raises(glm.GlmError) as e:
        glm.glm_server_submit(srv, 99, np.zeros(8), 0.01)
    assert e.value.status == glm.GLM_ENOTFOUND
    with pytest.raises(glm.GlmError) as e:
        glm.glm_server_poll(srv, 12345)
    assert e.value.status == glm.GLM_ENOTFOUND
    glm.glm_server_destroy(srv)


def test_server_shutdown_cancels_queued(ctx):
    X, y, bt = _data(400_000, 64, 60)
    srv = _server(ctx, slots=1, streams=1)
    ds = glm.glm_server_add_dataset(srv, glm.make_host_desc(X, y))
    ts = [glm.glm_server_submit(srv, ds, bt, 0.01) for _ in range(64)]
    glm.glm_server_shutdown(srv)
    done = cancelled = 0
    for t in ts:
        try:
            st, _ = glm.glm_server_poll(srv, t)
            assert st == glm.GLM_OK
            done += 1
        except glm.GlmError as e:
            assert e.status == glm.GLM_ECANCELLED
            cancelled += 1
    assert done + cancelled == 64 and cancelled > 0
    with pytest.raises(glm.GlmError) as e:
        glm.glm_server_submit(srv, ds, bt, 0.01)
    assert e.value.status == glm.GLM_ECANCELLED
    glm.glm_server_destroy(srv)


def test_server_device_resident_and_threads(ctx):
    """Device-resident data set, requests from several host threads."""
    X, y, bt = _data(50_000, 32, 70)
    Xd, yd = to_dev(X), to_dev(y)
    srv = _server(ctx)
    ds = glm.glm_server_add_dataset(srv, glm.make_desc(Xd, yd), on_device=True)
    res = {}

    def worker(w):
        rng = np.random.default_rng(100 + w)
        for i in range(25):
            beta = bt + 0.1 * rng.standard_normal(32)
            g = np.empty(32)
            f = glm.glm_server_wait(srv, glm.glm_server_submit(srv, ds, beta, 0.01), g)
            res[(w, i)] = (beta, f, g)

    th = [threading.Thread(target=worker, args=(w,)) for w in range(6)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert len(res) == 150
    for beta, f, g in list(res.values())[::10]:
        _check(f, g, X.astype(np.float64), y, beta, 0.01)
    glm.glm_server_destroy(srv)


def _fleet_run(ctx, sets, reqs, max_sets):
    """Serves reqs [(set index, beta)] on one slot, all submitted at once, so
    that everything after the first launch is queued when the next one
    starts."""
    srv = _server(ctx, slots=1, streams=1, max_sets=max_sets)
    ids = [glm.glm_server_add_dataset(srv, glm.make_desc(Xd, yd, dtype=dt), on_device=True)
           for Xd, yd, dt in sets]
    ptrs = np.array([b.ctypes.data for _, b in reqs], np.uint64)
    t = glm.glm_server_submit_many(srv, np.array([ids[i] for i, _ in reqs], np.int64), ptrs,
                                   np.full(len(reqs), 0.01))
    out = []
    for k in range(len(reqs)):
        g = np.empty(len(reqs[k][1]))
        f = glm.glm_server_wait(srv, int(t[k]), g)
        out.append((f, g))
    st = glm.glm_server_stats(srv)
    glm.glm_server_destroy(srv)
    return out, st


def test_server_fleet_launch_bitwise_and_oracle(ctx):
    """Passes of several data sets of one geometry (FP32, K = 32, N from 0 to
    250,000) in one launch give the bits of one launch per data set, and
    match the oracle; a BF16 K = 8 pair has another geometry and never shares
    their launches."""
    Ns = [700, 5_000, 0, 40_000, 250_000, 3_001, 64]
    sets, host = [], []
    for i, N in enumerate(Ns):
        X, y, bt = _data(N, 32, 300 + i)
        sets.append((to_dev(X), to_dev(y), glm.GLM_F32))
        host.append((X.astype(np.float64), y, bt, None))
    for i in range(2):
        X, y, bt = _data(9_000 + 1_000 * i, 8, 320 + i)
        Q = oracle.quantize_bf16(X)
        sets.append((to_dev(Q), to_dev(y), glm.GLM_BF16))
        host.append((oracle.decode_bf16(Q), y, bt, Q))
    rng = np.random.default_rng(330)
    reqs = []
    for r in range(60):
        i = int(rng.integers(0, len(sets)))
        reqs.append((i, np.ascontiguousarray(host[i][2] + 0.1 * rng.standard_normal(len(host[i][2])))))
    fleet, st = _fleet_run(ctx, sets, reqs, 0)
    single, st1 = _fleet_run(ctx, sets, reqs, 1)
    assert st["launches"] < st["passes"], st       # some launch carried several data sets
    assert st1["launches"] == st1["passes"]
    assert st["completed"] == st1["completed"] == len(reqs)
    for (i, beta), (f, g), (f1, g1) in zip(reqs, fleet, single):
        assert f == f1 and np.array_equal(g, g1), i
        Xh, y, _, Q = host[i]
        if Q is None:
            _check(f, g, Xh, y, beta, 0.01)
        else:
            _check(f, g, Xh, y, beta, 0.01, storage="bf16", Xo=Q, okw={"dtype": "bf16"})


@pytest.mark.parametrize("K", [128, 512])
def test_server_fleet_matrix_core_bitwise_and_oracle(ctx, K):
    """The matrix-core several-beta kernel in fleet launches: BF16 data sets of
    one geometry (K = 128: 8 waves per block; K = 512: 4) with N from 0 to
    60,000 give in a shared launch the bits of one launch per data set, and
    match the oracle on the stored codes."""
    Ns = [1_000, 0, 17, 60_000, 4_099]
    sets, host = [], []
    for i, N in enumerate(Ns):
        X, y, bt = _data(N, K, 400 + K + i)
        Q = oracle.quantize_bf16(X)
        sets.append((to_dev(Q), to_dev(y), glm.GLM_BF16))
        host.append((oracle.decode_bf16(Q), y, bt, Q))
    rng = np.random.default_rng(410 + K)
    reqs = []
    for r in range(40):
        i = int(rng.integers(0, len(sets)))
        reqs.append((i, np.ascontiguousarray(host[i][2] + 0.1 * rng.standard_normal(K))))
    fleet, st = _fleet_run(ctx, sets, reqs, 0)
    single, st1 = _fleet_run(ctx, sets, reqs, 1)
    assert st["launches"] < st["passes"], st
    assert st1["launches"] == st1["passes"]
    for (i, beta), (f, g), (f1, g1) in zip(reqs, fleet, single):
        assert f == f1 and np.array_equal(g, g1), i
        Xh, y, _, Q = host[i]
        _check(f, g, Xh, y, beta, 0.01, storage="bf16", Xo=Q, okw={"dtype": "bf16"})


def test_server_max_sets_argument(ctx):
    for bad in (-1, 257):
        with pytest.raises(glm.GlmError) as e:
            _server(ctx, max_sets=bad)
        assert e.value.status == glm.GLM_EINVAL


@pytest.mark.parametrize("K", [5, 100])
def test_multi_ragged_k(ctx, K):
    X, y, bt = _data(10_007, K, 80 + K)
    ld = (K + 3) // 4 * 4 + 4
    buf = np.full((X.shape[0], ld), np.nan, np.float32)
    buf[:, :K] = X
    Xd = torch.from_numpy(buf).to(DEV)[:, :K]
    yd = to_dev(y)          # the data set borrows X and y: keep both alive
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Xd, yd))
    B = _betas(bt, 6, 81)
    out = torch.empty((6, K + 1), dtype=torch.float64, device=DEV)
    glm.glm_logpost_grad_multi(ctx, ds, to_dev(B), 6, glm.make_prior(0.01), out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    for b in range(6):
        _check(o[b, 0], o[b, 1:], X.astype(np.float64), y, B[b], 0.01)
    glm.glm_dataset_unregister(ctx, ds)


@pytest.mark.parametrize("K", [20, 65, 72, 100, 128, 200, 257, 260, 512])
@pytest.mark.parametrize("nb", [2, 4, 7])
def test_multi_bf16_matrix_core(ctx, K, nb):
    """BF16 storage with 9 to 64 chunks per row (K from 65 to 512): passes of
    four vectors run the matrix-core kernel (K = 20 the VALU one).  Rows
    padded with NaN codes past column K (ragged K), N not a multiple of the
    16-row batch, partly filled passes; every vector against the oracle on
    the stored codes."""
    X, y, bt = _data(10_007, K, 100 + K + nb)
    Q = oracle.quantize_bf16(X)
    ld = (K + 7) // 8 * 8 + 8
    buf = np.full((X.shape[0], ld), 0x7FC0, np.uint16)
    buf[:, :K] = Q
    Qd = to_dev(buf)[:, :K]
    yd = to_dev(y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Qd, yd, dtype=glm.GLM_BF16))
    B = _betas(bt, nb, K + 3 * nb)
    Xd = oracle.decode_bf16(Q)
    for Bc in (np.zeros_like(B), B):
        o = _multi(ctx, ds, Bc, K)
        for b in range(nb):
            _check(o[b, 0], o[b, 1:], Xd, y, Bc[b], 0.01, storage="bf16", Xo=Q,
                   okw={"dtype": "bf16"})
    # slot 0 does not depend on what the other slots of its pass hold
    B2 = B.copy()
    B2[1:] = _betas(bt, nb - 1, K + 3 * nb + 1)
    out2 = torch.empty((nb, K + 1), dtype=torch.float64, device=DEV)
    glm.glm_logpost_grad_multi(ctx, ds, to_dev(B2), nb, glm.make_prior(0.01), out2)
    torch.cuda.synchronize()
    assert np.array_equal(o[0], out2.cpu().numpy()[0])
    glm.glm_dataset_unregister(ctx, ds)


@pytest.mark.parametrize("K", [100, 512])
def test_multi_bf16_vector_alu_form(ctx, K):
    """The context option GLM_OPT_MATRIX_CORES = 0 keeps BF16 passes of four
    vectors on the VALU kernels; that form and the matrix-core one both stay
    within the oracle bound."""
    X, y, bt = _data(6_007, K, 500 + K)
    Q = oracle.quantize_bf16(X)
    Qd, yd = glm.aligned_rows(to_dev(Q)), to_dev(y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Qd, yd, dtype=glm.GLM_BF16))
    B = _betas(bt, 4, 501 + K)
    res = {}
    try:
        for mx in (0, 1):
            glm.glm_set_option(ctx, glm.GLM_OPT_MATRIX_CORES, mx)
            assert glm.glm_get_option(ctx, glm.GLM_OPT_MATRIX_CORES) == mx
            out = torch.empty((4, K + 1), dtype=torch.float64, device=DEV)
            glm.glm_logpost_grad_multi(ctx, ds, to_dev(B), 4, glm.make_prior(0.01), out)
            torch.cuda.synchronize()
            res[mx] = out.cpu().numpy()
    finally:
        glm.glm_set_option(ctx, glm.GLM_OPT_MATRIX_CORES, 1)
    glm.glm_dataset_unregister(ctx, ds)
    for env, o in res.items():
        for b in range(4):
            _check(o[b, 0], o[b, 1:], oracle.decode_bf16(Q), y, B[b], 0.01, storage="bf16", Xo=Q,
                   okw={"dtype": "bf16"})
    assert not np.array_equal(res[0], res[1])   # two different kernels ran


def test_multi_bf16_matrix_core_edges(ctx):
    """Empty data set (prior only), fewer rows than one batch, and non-finite
    beta (NaN out) through the matrix-core kernel."""
    K = 96
    X, y, bt = _data(7, K, 5)
    Q = oracle.quantize_bf16(X)
    B = _betas(bt, 4, 6)
    for n in (0, 7):
        Qd, yd = to_dev(Q[:n].reshape(n, K)), to_dev(y[:n])
        ds = glm.glm_dataset_register(ctx, glm.make_desc(Qd, yd, dtype=glm.GLM_BF16))
        out = torch.empty((4, K + 1), dtype=torch.float64, device=DEV)
        glm.glm_logpost_grad_multi(ctx, ds, to_dev(B), 4, glm.make_prior(0.01), out)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        for b in range(4):
            _check(o[b, 0], o[b, 1:], oracle.decode_bf16(Q[:n].reshape(n, K)), y[:n], B[b], 0.01,
                   storage="bf16", Xo=Q[:n].reshape(n, K), okw={"dtype": "bf16"})
        glm.glm_dataset_unregister(ctx, ds)
    Qd, yd = to_dev(Q), to_dev(y)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(Qd, yd, dtype=glm.GLM_BF16))
    Bn = B.copy()
    Bn[2, 3] = np.nan
    out = torch.empty((4, K + 1), dtype=torch.float64, device=DEV)
    glm.glm_logpost_grad_multi(ctx, ds, to_dev(Bn), 4, glm.make_prior(0.01), out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.isnan(o[2, 0])
    for b in (0, 1, 3):
        _check(o[b, 0], o[b, 1:], oracle.decode_bf16(Q), y, B[b], 0.01, storage="bf16", Xo=Q,
               okw={"dtype": "bf16"})
    glm.glm_dataset_unregister(ctx, ds)


@pytest.mark.timeout(900)
def test_serving_workload_full_configuration(ctx):
    """The 64 data sets of the serving workload (N log-uniform on [1e3, 2e6],
    K in {8, 32, 128, 512}, BF16 or FP32 storage), device-resident in one
    server, two requests per data set submitted together; every result is
    checked against the oracle on the stored values within the derived
    bound."""
    import synth
    spec = synth.serving_specs(64)
    srv = _server(ctx)
    rng = np.random.default_rng(90)
    keep, reqs = [], []
    for i in range(64):
        X, y, bt = synth.serving_dataset(i, spec)
        if spec.dtype[i] == "bf16":
            S, dt = oracle.quantize_bf16(X), glm.GLM_BF16
        else:
            S, dt = X, glm.GLM_F32
        Xd, yd = to_dev(S), to_dev(y)
        keep.append((Xd, yd))
        ds = glm.glm_server_add_dataset(srv, glm.make_desc(Xd, yd, dtype=dt), on_device=True)
        for _ in range(2):
            beta = bt + 0.01 * rng.standard_normal(len(bt))
            reqs.append((i, S, y, dt, beta, glm.glm_server_submit(srv, ds, beta, 0.01)))
    for i, S, y, dt, beta, t in reqs:
        g = np.empty(len(beta))
        f = glm.glm_server_wait(srv, t, g)
        if dt == glm.GLM_BF16:
            _check(f, g, oracle.decode_bf16(S), y, beta, 0.01, storage="bf16", Xo=S,
                   okw={"dtype": "bf16"})
        else:
            _check(f, g, S.astype(np.float64), y, beta, 0.01)
    st = glm.glm_server_stats(srv)
    assert st["completed"] == 128 and st["failed"] == 0
    glm.glm_server_destroy(srv)

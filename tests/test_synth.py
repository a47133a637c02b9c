"""The seeded generators: reproducible, thread-count independent, and with
the distributions the workloads name."""
import math

import numpy as np

import synth


def test_design_matrix_is_reproducible_and_chunk_independent():
    ss = synth.seed_seq(99)
    a = synth.design_matrix(150_000, 6, ss, np.float32, n_binary=2)
    b = synth.design_matrix(150_000, 6, synth.seed_seq(99), np.float32, n_binary=2)
    assert np.array_equal(a, b)
    assert set(np.unique(a[:, 4:])) == {0.0, 1.0}
    assert abs(a[:, 4:].mean() - 0.3) < 0.01
    assert abs(a[:, :4].mean()) < 0.01 and abs(a[:, :4].std() - 1.0) < 0.01


def test_labels_follow_the_logistic_model():
    ss = synth.streams(synth.seed_seq(98))
    X = synth.design_matrix(200_000, 4, ss["X"], np.float64)
    bt = np.array([1.0, -0.5, 0.25, 0.0])
    y = synth.logistic_labels(X, bt, ss["y"])
    eta = X @ bt
    p = 1.0 / (1.0 + np.exp(-eta))
    # calibration in deciles of the model probability
    edges = np.quantile(p, np.linspace(0, 1, 11))
    idx = np.clip(np.searchsorted(edges, p) - 1, 0, 9)
    for d in range(10):
        m = idx == d
        assert abs(y[m].mean() - p[m].mean()) < 0.015


def test_small_workload_shape_and_closed_form_point():
    w = synth.plain_small(n_evals=3)
    assert w.X.shape == (10_000, 20) and w.X.dtype == np.float64
    assert w.betas.shape == (4, 20) and not w.betas[-1].any()
    assert w.prec == 0.01
    assert set(np.unique(w.y)) <= {0, 1}


def test_beta_true_variance_is_one_over_k():
    b = synth.true_coefficients(200_000, synth.seed_seq(97))
    assert abs(b.var() * 200_000 - 1.0) < 0.02


def test_random_walk_steps():
    tr = synth.random_walk(np.zeros(50), 2001, synth.seed_seq(96))
    st = np.diff(tr, axis=0)
    assert abs(st.std() - 0.01) < 2e-4
    assert abs(tr[0].std() - 0.1) < 0.04


def test_group_sizes_distribution():
    s = synth.group_sizes(2000, synth.streams(synth.seed_seq(3))["groups"])
    assert s.min() >= 20 and s.max() <= 50_000
    assert 1.7e6 < s.sum() < 2.4e6
    assert abs(np.median(s) - 500) < 60


def test_serving_specs():
    sp = synth.serving_specs()
    assert len(sp.N) == 64 and sp.N.min() >= 1000 and sp.N.max() <= 2_000_000
    assert set(sp.K) <= {8, 32, 128, 512}
    assert set(sp.dtype) <= {"bf16", "f32"}


def test_mh_proposal_scale():
    inc, logu, sd = synth.mh_chain_inputs(512, 1000, 8_000_000)
    assert abs(sd - 2.38 / math.sqrt(512) / math.sqrt(1.6e6)) < 1e-15
    assert abs(inc.std() / sd - 1) < 0.01
    assert (logu < 0).all()


def test_poisson_counts_deterministic_and_calibrated():
    """Same seeds give the same counts whatever the worker count; the counts
    average the rates exp(x . beta) (a calibration check, 5 sigma)."""
    w1 = synth.plain_poisson(N=200_000, K=16, n_evals=2)
    w2 = synth.plain_poisson(N=200_000, K=16, n_evals=2)
    assert np.array_equal(w1.y, w2.y) and np.array_equal(w1.X, w2.X)
    rate = np.exp(w1.X.astype(np.float64) @ w1.beta_true)
    se = math.sqrt(rate.sum())
    assert abs(w1.y.sum() - rate.sum()) < 5 * se
    assert w1.y.max() < 255

"""Pins of the oracle's random-number streams and of its HMC chain (CPU only).

The generator is pinned bit for bit to numpy's own Philox4x64-10
(numpy.random.Philox, an independent implementation of the same published
generator); the normal transform to its definition evaluated with numpy's
generator and Python's math module; HMC to properties of the leapfrog
integrator that a dropped term, a wrong sign or a misplaced half step breaks.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

M64 = 2 ** 64


def _numpy_blocks(key, ctr, nblocks):
    """numpy's Philox4x64-10 blocks at counters ctr, ctr + 1, ... (numpy
    advances its 256-bit counter before each block, so it starts one
    before)."""
    c = int(ctr[0]) + (int(ctr[1]) << 64) + (int(ctr[2]) << 128) + (int(ctr[3]) << 192) - 1
    c %= 2 ** 256
    words = np.array([(c >> (64 * i)) & (M64 - 1) for i in range(4)], np.uint64)
    bg = np.random.Philox(key=np.array(key, np.uint64), counter=words)
    return bg.random_raw(4 * nblocks).reshape(nblocks, 4)


@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (1, 0, 0, 0)),
    ((123456789, 987654321), (5, 6, 7, 8)),
    ((M64 - 1, M64 - 1), (M64 - 1, 0, 5, 9)),          # carry into word 1 next
    ((0x0123456789ABCDEF, 42), (M64 - 1, M64 - 1, 3, 0)),   # carry into word 2 next
])
def test_philox_matches_numpy_bit_for_bit(key, ctr):
    ref = _numpy_blocks(key, ctr, 3)
    c = int(ctr[0]) + (int(ctr[1]) << 64) + (int(ctr[2]) << 128) + (int(ctr[3]) << 192)
    for b in range(3):
        cb = c + b
        words = [(cb >> (64 * i)) & (M64 - 1) for i in range(4)]
        assert np.array_equal(oracle.philox(words, key), ref[b]), b


def test_u01_is_open_and_exact():
    assert oracle.u01(0) == 2.0 ** -53
    assert oracle.u01(M64 - 1) == 1.0 - 2.0 ** -53
    assert oracle.u01(1 << 12) == 1.5 * 2.0 ** -52
    assert oracle.u01(1 << 63) == 0.5 + 2.0 ** -53


def test_uniform_stream_layout_from_numpy():
    seed, chain, stream = 77, 5, 12
    got = oracle.rng_uniforms(seed, chain, stream, 6, 30)
    blocks = _numpy_blocks((seed, chain), (1, 0, oracle.RNG_UNIFORM, stream), 9)
    words = blocks.reshape(-1)                       # values 4 .. 39 of the stream
    ref = np.array([((int(w) >> 12) + 0.5) * 2.0 ** -52 for w in words[2:32]])
    assert np.array_equal(got, ref)


def test_polar_normals_from_numpy_and_math():
    """Pair p's attempts read words (2(a mod 2), 2(a mod 2) + 1) of the block
    at counter (p, a / 2, purpose, stream); the first point inside the unit
    disc gives u c and v c, c = sqrt(-2 log s / s)."""
    seed, chain, stream = 3, 9, 4
    for p in range(40):
        blocks = _numpy_blocks((seed, chain), (p, 0, oracle.RNG_NORMAL, stream), 8)
        for a in range(16):
            w = blocks[a // 2]
            u = 2.0 * (((int(w[2 * (a % 2)]) >> 12) + 0.5) * 2.0 ** -52) - 1.0
            v = 2.0 * (((int(w[2 * (a % 2) + 1]) >> 12) + 0.5) * 2.0 ** -52) - 1.0
            s = float(Fraction(u) * Fraction(u) + Fraction(v * v))   # fma(u, u, v v)
            if 0.0 < s < 1.0:
                break
        c = math.sqrt(-2.0 * math.log(s) / s)
        z0, z1, att = oracle.polar_pair(seed, chain, oracle.RNG_NORMAL, stream, p)
        assert att == a + 1
        assert z0 == u * c and z1 == v * c


def test_polar_normals_distribution():
    from scipy import stats
    z = oracle.rng_normals(11, 2, 0, 0, 20_000)
    assert abs(z.mean()) < 4.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    att = [oracle.polar_pair(11, 2, oracle.RNG_NORMAL, 0, p)[2] for p in range(4000)]
    assert abs(4000 / sum(att) - math.pi / 4) < 0.03     # acceptance rate of the disc


def _fg(w):
    return lambda b: oracle.logpost_grad(w.X, w.y, b, w.prec)


def test_leapfrog_is_reversible():
    w = synth.plain_small(1)
    fg = _fg(w)
    b0 = w.beta_true.copy()
    f0, g0 = fg(b0)
    p0 = oracle.hmc_momenta(1, 1, 0, b0.size)
    b1, p1, f1, g1 = oracle.leapfrog(fg, b0, g0, p0, 0.01, 12)
    b2, p2, _, _ = oracle.leapfrog(fg, b1, g1, -p1, 0.01, 12)
    assert np.max(np.abs(b2 - b0)) < 1e-12 and np.max(np.abs(-p2 - p0)) < 1e-9
    assert np.max(np.abs(b1 - b0)) > 1e-3                # it moved


def test_leapfrog_energy_error_is_second_order():
    """Halving the step (same trajectory length) cuts |H(end) - H(start)| by
    about 4; the mean over several momenta keeps the ratio stable."""
    w = synth.plain_small(1)
    fg = _fg(w)
    b0 = w.beta_true.copy()
    f0, g0 = fg(b0)
    errs = {}
    for eps, L in ((0.008, 10), (0.004, 20)):
        e = []
        for t in range(6):
            p0 = oracle.hmc_momenta(2, 1, t, b0.size)
            _, p1, f1, _ = oracle.leapfrog(fg, b0, g0, p0, eps, L)
            e.append(abs((f1 - 0.5 * p1 @ p1) - (f0 - 0.5 * p0 @ p0)))
        errs[eps] = np.mean(e)
    assert 3.5 < errs[0.008] / errs[0.004] < 4.5, errs


def test_one_leapfrog_step_is_the_langevin_proposal():
    """n_leap = 1: beta' = beta + eps^2/2 g + eps p and p' = p + eps/2 (g + g')."""
    w = synth.plain_small(1)
    fg = _fg(w)
    b0 = w.beta_true.copy()
    f0, g0 = fg(b0)
    p0 = oracle.hmc_momenta(5, 3, 0, b0.size)
    eps = 0.013
    b1, p1, f1, g1 = oracle.leapfrog(fg, b0, g0, p0, eps, 1)
    assert np.allclose(b1, b0 + 0.5 * eps * eps * g0 + eps * p0, rtol=0, atol=1e-15)
    assert np.allclose(p1, p0 + 0.5 * eps * (g0 + g1), rtol=0, atol=1e-12)
    assert np.array_equal(g1, fg(b1)[1])


def test_hmc_chain_decisions_and_replay():
    w = synth.plain_small(1)
    r = oracle.hmc_chain(w.X, w.y, w.beta_true, w.prec, 30, 5, 0.01, 7, 1)
    assert np.array_equal(r["accepted"], (r["logu"] < r["dH"]).astype(np.uint8))
    assert 0.5 < r["accepted"].mean() <= 1.0
    # the logged f trace is f of the state after each iteration
    f_end, _ = oracle.logpost_grad(w.X, w.y, r["beta"], w.prec)
    assert r["f_trace"][-1] == f_end
    # following the chain's own decisions reproduces it; forcing rejections
    # keeps beta where it started
    r2 = oracle.hmc_chain(w.X, w.y, w.beta_true, w.prec, 30, 5, 0.01, 7, 1,
                          follow=r["accepted"])
    assert np.array_equal(r2["beta"], r["beta"])
    r3 = oracle.hmc_chain(w.X, w.y, w.beta_true, w.prec, 5, 5, 0.01, 7, 1,
                          follow=np.zeros(5, np.uint8))
    assert np.array_equal(r3["beta"], w.beta_true)

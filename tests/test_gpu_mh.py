"""Storage-precision form on the GPU: a 20,000-step random-walk Metropolis
chain whose accept decisions are checked against the oracle's (FP32, BF16 and
FP8-E4M3 storage of one X), and the full-size 8,000,000 x 512 evaluation with
its kernel and storage errors."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
from mh_check import TAU, Formats, n_threads, shadow_chain  # noqa: E402


def _log(msg):
    print(msg, flush=True)


@pytest.mark.timeout(900)
def test_mh_chain_decisions_match_oracle():
    """N = 200,000, K = 512 (the storage-precision generator at a smaller N),
    20,000 steps from beta_true, 1% audit.  Every GPU decision equals its
    oracle's, or differs only inside the tolerance band."""
    N, K, steps = 200_000, 512, 20_000
    with ThreadPoolExecutor(n_threads()) as pool:
        fm = Formats(N, K, pool, _log)
        inc, logu, _ = synth.mh_chain_inputs(K, steps, N)
        rep = shadow_chain(fm, inc, logu, 0.01, seed=7, log=_log, progress_every=5000)
        fm.close()
    _log(str({k: {kk: v for kk, v in f.items() if kk != "mismatches"}
              for k, f in rep["formats"].items()}))
    assert 0.05 < rep["accept_rate"] < 0.6, rep["accept_rate"]
    for name, f in rep["formats"].items():
        assert f["audited"] >= 100, (name, f["audited"])
        assert f["tolerance_violations"] == 0, (name, f["max_rel_err_checked"])
        assert f["unexplained_mismatches"] == 0, (name, f["mismatches"])


@pytest.mark.timeout(900)
def test_precision_workload_full_size():
    """N = 8,000,000, K = 512 at three trajectory points (first, middle,
    last), in the launch configuration the benchmark times.  Kernel error
    (against the oracle on the same stored codes): f <= 1e-9, g <= 1e-7
    (relative, norm-wise) for every format at every point.  Storage error
    (against the oracle on the FP32 X): BF16 f <= 1e-5, g <= 2e-2; FP8
    f <= 5e-4, g <= 1e-1.  The GPU encoders give the oracle's codes bit for
    bit at this size."""
    from paper_1310_1537_amd import glm
    N, K = 8_000_000, 512
    points = (0, 499, 999)
    with ThreadPoolExecutor(n_threads()) as pool:
        fm = Formats(N, K, pool, _log)
        w = fm.w
        outs = {}
        for i in points:
            for j, d in enumerate(fm.ds):
                g = np.empty(K)
                f = glm.glm_logpost_grad_host(fm.ctx, d, w.betas[i], fm.prior, g)
                outs[(i, j)] = (f, g)
        # the GPU encoders against the oracle's codes
        dev = torch.device("cuda:0")
        Xd = fm.dev_arrays[0]
        Qb = torch.empty((N, K), dtype=torch.uint16, device=dev)
        glm.glm_quantize_bf16(fm.ctx, Xd, Qb)
        s = torch.empty(K, dtype=torch.float32, device=dev)
        glm.glm_fp8_col_scales(fm.ctx, Xd, s)
        Q8 = torch.empty((N, K), dtype=torch.uint8, device=dev)
        glm.glm_quantize_fp8(fm.ctx, Xd, s, Q8)
        torch.cuda.synchronize()
        assert np.array_equal(s.cpu().numpy(), fm.s8)
        assert torch.equal(Qb.view(torch.int16), fm.dev_arrays[1].view(torch.int16))
        assert torch.equal(Q8, fm.dev_arrays[2])
        del Qb, Q8
        refs = {}
        for i in points:
            for j, o in enumerate(fm.oracles):
                refs[(i, j)] = oracle.logpost_grad_blocks(o.X, o.y, w.betas[i], w.prec,
                                                          pool=pool, **o.kw)
        fm.close()

    def err(a, b):
        return abs(a[0] - b[0]) / abs(b[0]), np.linalg.norm(a[1] - b[1]) / np.linalg.norm(b[1])

    for i in points:
        report = {name: {"kernel": err(outs[(i, j)], refs[(i, j)]),
                         "storage": err(outs[(i, j)], refs[(i, 0)])}
                  for j, name in enumerate(Formats.NAMES)}
        _log(f"point {i}: {report}")
        for name in Formats.NAMES:
            ef, eg = report[name]["kernel"]
            assert ef <= TAU and eg <= 1e-7, (i, name, ef, eg)
        assert report["bf16"]["storage"][0] <= 1e-5 and report["bf16"]["storage"][1] <= 2e-2
        assert report["fp8"]["storage"][0] <= 5e-4 and report["fp8"]["storage"][1] <= 1e-1

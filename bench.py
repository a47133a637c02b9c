"""Throughput of the fused logistic-regression log-posterior + gradient on one
MI355X.

Workload (default): N = 4,000,000 rows, K = 256 columns, FP32 X with the last
26 columns binary (p = 0.3), y from the logistic model, prior sd 10, and a
seeded random-walk beta trajectory (start N(beta_true, 0.1^2 I), steps
N(0, 0.01^2 I)).  One step = one full evaluation of f(beta) and g(beta)
(one fused kernel launch over all of X) at the next trajectory point, with
X, y and the trajectory already resident in HBM.

Prints one JSON line with evals/s, the kernel's HBM roofline fraction
(algorithmic bytes / HIP-event-timed launch duration vs the 8 TB/s peak), the
error against the FP64 oracle, kernel and host-call latency percentiles, and
the FP64 CPU oracle's own throughput on this host.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def measured_traffic(name: str, kind: str = "plain"):
    """HBM bytes per launch from the committed rocprofv3 counter runs
    (profiles/<name>_traffic.json), if they were taken on the current kernel
    sources; else None."""
    from paper_1310_1537_amd.profiling import kernel_source_hash
    try:
        rec = json.load(open(os.path.join(PROFILES, name + "_traffic.json")))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash(kind):
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(w, n_max: int, budget_s: float = 15.0, family: str = "logistic"):
    """The FP64 oracle (single-threaded C) on the first trajectory points of
    the same workload, until about budget_s seconds have been spent."""
    import oracle
    res = []
    t0 = time.perf_counter()
    for i in range(n_max):
        res.append(oracle.logpost_grad(w.X, w.y, w.betas[i], w.prec, family=family))
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return res, dt


def host_info() -> dict:
    """Host CPU as the CPU baselines see it: usable threads, logical CPUs and
    the model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": usable, "logical_cpus": os.cpu_count(), "model": model}


def cpu_threads() -> int:
    """Threads the all-threads CPU baselines use: the usable CPUs, at most 16
    (the host share of one GPU)."""
    return max(1, min(16, host_info()["nproc"]))


def host_read_bandwidth(arr, threads: int, reps: int = 3) -> float:
    """GB/s of a threaded integer sum over the bytes of a large host array
    (each thread reduces its own slice; numpy releases the interpreter lock),
    best of reps."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    flat = arr.reshape(-1).view(np.uint8)
    n8 = flat.size // 8
    v = flat[:n8 * 8].view(np.int64)
    edges = np.linspace(0, v.size, threads + 1).astype(np.int64)
    parts = [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:])]
    best = 0.0
    with ThreadPoolExecutor(threads) as ex:
        for _ in range(reps):
            t0 = time.perf_counter()
            list(ex.map(lambda ab: int(np.add.reduce(v[ab[0]:ab[1]])), parts))
            best = max(best, v.size * 8 / (time.perf_counter() - t0) / 1e9)
    return best


def numpy_som(X, y, beta, prec, family: str = "logistic", rows: int = 0, dtype=None, scale=None):
    """The paper's naive sequence of maps in NumPy float64 with its threaded
    BLAS: u = X beta, the per-row map, g = X^t r, over the first `rows` rows
    (all if 0) of X upcast to float64 beforehand (the upcast is not timed).
    Returns (seconds for the sample, sample rows)."""
    import numpy as np

    import oracle
    n = X.shape[0] if rows <= 0 else min(rows, X.shape[0])
    if dtype == "bf16":
        Xd = oracle.decode_bf16(X[:n])
    elif dtype == "fp8":
        Xd = oracle.decode_fp8(X[:n], scale)
    else:
        Xd = np.asarray(X[:n], np.float64)
    yd = np.asarray(y[:n], np.float64)
    b = np.asarray(beta, np.float64)
    t0 = time.perf_counter()
    u = Xd @ b
    if family == "poisson":
        mu = np.exp(u)
        f = float(np.sum(yd * u - mu))
        r = yd - mu
    else:
        e = np.exp(-np.abs(u))
        f = float(np.sum(yd * u - (np.maximum(u, 0.0) + np.log1p(e))))
        r = yd - np.where(u >= 0.0, 1.0 / (1.0 + e), e / (1.0 + e))
    g = Xd.T @ r
    f -= 0.5 * prec * float(b @ b)
    g -= prec * b
    dt = time.perf_counter() - t0
    return dt, n


def cpu_baseline_report(n_units: float, unit: str, single, threaded, som, host: dict,
                        sample: str, read_gbps: float | None) -> dict:
    """The cpu_baseline record: value = the faster of the oracle on all host
    threads (row blocks, fsum-combined) and single-threaded (cores: the
    threads of that one), both given, with the NumPy float64 sequence of
    maps beside them.  single / threaded: (seconds, units of work done[,
    threads]) or None; som: (seconds, units) or None."""
    rec = {"unit": unit, "kind": "oracle", "sample": sample, "host": dict(host)}
    if read_gbps is not None:
        rec["host"]["read_GBps"] = read_gbps
    modes = []
    if threaded:
        rec["all_threads"] = {"value": threaded[1] / threaded[0] * n_units, "cores": threaded[2]}
        modes.append(rec["all_threads"])
    if single:
        rec["single_thread"] = {"value": single[1] / single[0] * n_units, "cores": 1}
        modes.append(rec["single_thread"])
    if modes:
        best = max(modes, key=lambda m: m["value"])
        rec["value"], rec["cores"] = best["value"], best["cores"]
    if som:
        rec["numpy_som_f64"] = {"value": som[1] / som[0] * n_units,
                                "note": "X @ beta, per-row map, X^t r in NumPy float64 with its "
                                        "threaded BLAS (the paper's naive routine); X upcast "
                                        "beforehand, untimed"}
    return rec


def _device_hold(torch, seconds: float) -> None:
    """Queues a spin of about `seconds` on the current stream (torch's
    cycle-count sleep kernel) when available."""
    sleep = getattr(torch.cuda, "_sleep", None)
    if sleep is not None:
        sleep(int(seconds * 2.4e9))


MIN_WARM_S = 0.05


def _warm(launch, warmup: int, min_s: float = MIN_WARM_S) -> int:
    """At least `warmup` untimed launches, and more until about min_s of
    device time has passed: the first ten or so back-to-back launches after
    an idle spell run up to a third slower (clocks ramping; the kernel trace
    of the 4M x 256 workload shows 650-790 us there against a steady 590-600
    us), and a short timed run must not sit on that ramp.  Returns the
    launches made."""
    import torch
    t0 = time.perf_counter()
    n = 0
    while n < warmup or time.perf_counter() - t0 < min_s:
        launch(n)
        n += 1
        if n >= warmup and n % 4 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return n


def _timed_evals(glm, lib, ctx, ds, prior, betas, outs, K, warmup, steps, stream):
    """warmup + steps sequential evaluations; returns (wall s, per-launch ms)."""
    import ctypes
    import numpy as np
    import torch
    pr = ctypes.byref(prior)
    sp = stream.cuda_stream
    bptr, optr = betas.data_ptr(), outs.data_ptr()
    nb = betas.shape[0]

    def launch(i):
        st = lib.glm_logpost_grad(ctx, ds, bptr + (i % nb) * K * 8, pr,
                                  optr + (i % nb) * (K + 1) * 8, sp)
        if st:
            raise glm.GlmError(st, glm.glm_last_error())

    nw = _warm(launch, warmup)
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for j in range(steps):
        ev0[j].record(stream)
        launch(nw + j)
        ev1[j].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, np.array([a.elapsed_time(b) for a, b in zip(ev0, ev1)]), nw


def bench_plain_big(args, poisson: bool = False):
    import numpy as np
    import torch

    import synth
    from paper_1310_1537_amd import glm

    dev = torch.device("cuda:0")
    n_traj = 1000
    w = synth.plain_poisson(n_evals=n_traj) if poisson else synth.plain_big(n_evals=n_traj)
    family = glm.GLM_POISSON if poisson else glm.GLM_LOGISTIC
    N, K = w.X.shape
    print(f"[bench] workload N={N} K={K} fp32; generated", file=sys.stderr, flush=True)
    X = torch.from_numpy(w.X).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    total = args.warmup + args.steps
    idx = np.arange(total) % n_traj
    betas = torch.from_numpy(np.ascontiguousarray(w.betas[idx])).to(dev)
    outs = torch.empty((total, K + 1), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    ctx = glm.glm_create(0)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(X, y, family=family))
    prior = glm.make_prior(w.prec)
    wall, kern_ms, n_warm = _timed_evals(glm, glm.lib(), ctx, ds, prior, betas, outs, K,
                                         args.warmup, args.steps, stream)
    avg_ms = float(kern_ms.mean())
    print(f"[bench] {args.steps} evals in {wall:.3f} s; launch avg {avg_ms * 1e3:.1f} us",
          file=sys.stderr, flush=True)

    bytes_alg = float(N) * K * 4 + N          # X read once + y bytes
    achieved = bytes_alg / (avg_ms * 1e-3) / 1e9

    # measured ceiling: a plain streaming read of the same X buffer
    ceiling = max(glm.glm_probe_read_bandwidth(ctx, X, blocks_per_cu=b, iters=10)
                  for b in (1, 2, 4))

    # host round-trip latency (beta H2D, launch, f/g D2H, sync), paper Sec. 4.5
    g_host = np.empty(K)
    lat = []
    for i in range(args.latency_calls):
        a = time.perf_counter()
        glm.glm_logpost_grad_host(ctx, ds, w.betas[i % n_traj], prior, g_host)
        lat.append(time.perf_counter() - a)
    lat_us = np.array(lat) * 1e6

    out_np = outs.cpu().numpy()
    result = {
        "metric": "logpost+grad evals/s (fused f+g, FP64 result) & HBM GB/s % peak",
        "value": args.steps / wall,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": n_warm,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("plain big, Poisson regression (log link): N=4,000,000 K=256, "
                                "FP32 X (26 binary columns), random-walk beta trajectory"
                                if poisson else
                                "plain big: Bayesian logistic regression N=4,000,000 K=256, "
                                "FP32 X (26 binary columns), random-walk beta trajectory"),
                   "N": N, "K": K, "storage": "fp32", "result": "fp64", "prior_sd": 10},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBPS,
                     "traffic": None if poisson else measured_traffic("fg_fused_plain_big"),
                     "kernel": "fg_fused<f32, 64 lanes/row>", "bytes_per_launch": bytes_alg,
                     "launch_us_avg": avg_ms * 1e3,
                     "read_ceiling_GBps": ceiling, "frac_of_read_ceiling": achieved / ceiling},
        "latency_us": {"kernel_p50": float(np.percentile(kern_ms, 50) * 1e3),
                       "kernel_p99": float(np.percentile(kern_ms, 99) * 1e3),
                       "host_call_p50": float(np.percentile(lat_us, 50)),
                       "host_call_p99": float(np.percentile(lat_us, 99))},
    }

    if not args.no_cpu_baseline:
        fam = "poisson" if poisson else "logistic"
        host = host_info()
        thr = cpu_threads()
        # the oracle on all host threads: every point the GPU evaluated among
        # the first 11 (its error check), then more until about 10 s
        from concurrent.futures import ThreadPoolExecutor

        import oracle
        res = []
        with ThreadPoolExecutor(thr) as pool:
            t0 = time.perf_counter()
            for i in range(min(total, n_traj)):
                res.append(oracle.logpost_grad_blocks(w.X, w.y, w.betas[i], w.prec,
                                                      threads=thr, family=fam, pool=pool))
                if i >= 10 and time.perf_counter() - t0 > 10.0:
                    break
            dt_thr = time.perf_counter() - t0
        n = len(res)
        ef = max(abs(out_np[i][0] - res[i][0]) / abs(res[i][0]) for i in range(n))
        eg = max(np.linalg.norm(out_np[i][1:] - res[i][1]) / np.linalg.norm(res[i][1])
                 for i in range(n))
        result["err_vs_fp64"] = {"f_rel_max": ef, "g_rel_norm_max": eg, "points": n}
        single, dt1 = cpu_baseline(w, n_max=3, budget_s=5.0, family=fam)
        som = numpy_som(w.X, w.y, w.betas[0], w.prec, fam, rows=N // 4)
        result["cpu_baseline"] = cpu_baseline_report(
            1.0, "evals/s", (dt1, len(single)), (dt_thr, n, thr),
            (som[0], som[1] / N), host,
            f"the first {n} trajectory points of the same N={N} K={K} workload on {thr} "
            f"threads (row blocks, fsum-combined); {len(single)} single-threaded; the NumPy "
            f"sequence of maps on the first {som[1]} rows, scaled to N",
            host_read_bandwidth(w.X, thr))
    glm.glm_dataset_unregister(ctx, ds)
    glm.glm_destroy(ctx)
    return result


def _rel_err(out, ref):
    import numpy as np
    return {"f_rel": abs(out[0] - ref[0]) / abs(ref[0]),
            "g_rel_norm": float(np.linalg.norm(out[1:] - ref[1]) / np.linalg.norm(ref[1]))}


def _precision_cpu_leg(w, Xb_dev, Xq_dev, sc_dev):
    """CPU-baseline leg of the storage-precision workload: times one
    single-threaded oracle evaluation on the FP32 X, and evaluates the oracle
    on its own BF16 / FP8 codes of the same X (encoded in row blocks on host
    threads) for the error report.  The GPU encoders' codes are compared with
    the oracle's, never handed to it."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    b0 = w.betas[0]
    thr = cpu_threads()
    t0 = time.perf_counter()
    refs = {"fp32": oracle.logpost_grad_blocks(w.X, w.y, b0, w.prec, threads=thr)}
    seconds_thr = time.perf_counter() - t0
    N = w.X.shape[0]
    n1 = N // 8   # single-threaded on an eighth of the rows, scaled
    t0 = time.perf_counter()
    oracle.logpost_grad(w.X[:n1], w.y[:n1], b0, w.prec)
    seconds_1 = (time.perf_counter() - t0) * N / n1
    edges = np.linspace(0, N, 65).astype(np.int64)
    blocks = [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:]) if b > a]
    s8 = oracle.fp8_col_scales(w.X)
    Qb = np.empty(w.X.shape, np.uint16)
    Q8 = np.empty(w.X.shape, np.uint8)

    def enc(ab):
        a, b = ab
        Qb[a:b] = oracle.quantize_bf16(w.X[a:b])
        Q8[a:b] = oracle.quantize_fp8(w.X[a:b], s8)[0]

    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex:
        list(ex.map(enc, blocks))
    codes_equal = {"bf16": bool(np.array_equal(Xb_dev.cpu().numpy(), Qb)),
                   "fp8": bool(np.array_equal(Xq_dev.cpu().numpy(), Q8)
                               and np.array_equal(sc_dev.cpu().numpy(), s8))}
    tf = {}
    t0 = time.perf_counter()
    refs["bf16"] = oracle.logpost_grad_blocks(Qb, w.y, b0, w.prec, threads=thr, dtype="bf16")
    tf["bf16"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    refs["fp8"] = oracle.logpost_grad_blocks(Q8, w.y, b0, w.prec, threads=thr, dtype="fp8",
                                             scale=s8)
    tf["fp8"] = time.perf_counter() - t0
    som = numpy_som(w.X, w.y, b0, w.prec, rows=N // 16)
    return {"seconds_thr": seconds_thr, "seconds_1": seconds_1, "threads": thr,
            "seconds_fmt": tf, "refs": refs, "codes_equal": codes_equal,
            "som": (som[0], som[1] / N), "host": host_info()}


def bench_precision(args):
    """N=8,000,000, K=512: the same trajectory on FP32, BF16 and FP8-E4M3
    (per-column FP32 scales) copies of X; throughput and error per format."""
    import numpy as np
    import torch

    import synth
    from paper_1310_1537_amd import glm

    dev = torch.device("cuda:0")
    N = args.n or 8_000_000
    K = 512
    w = synth.plain_big(N=N, K=K, n_evals=1000, workload_index=2)
    print(f"[bench] precision workload N={N} K={K} generated", file=sys.stderr, flush=True)
    X = torch.from_numpy(w.X).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    ctx = glm.glm_create(0)
    Xb = torch.empty((N, K), dtype=torch.uint16, device=dev)
    glm.glm_quantize_bf16(ctx, X, Xb)
    sc = torch.empty(K, dtype=torch.float32, device=dev)
    glm.glm_fp8_col_scales(ctx, X, sc)
    Xq = torch.empty((N, K), dtype=torch.uint8, device=dev)
    glm.glm_quantize_fp8(ctx, X, sc, Xq)
    torch.cuda.synchronize()
    total = args.warmup + args.steps
    idx = np.arange(total) % 1000
    betas = torch.from_numpy(np.ascontiguousarray(w.betas[idx])).to(dev)
    stream = torch.cuda.current_stream()
    prior = glm.make_prior(w.prec)
    formats = {}
    for name, Xs, dt, scale, es in (("fp32", X, glm.GLM_F32, None, 4),
                                    ("bf16", Xb, glm.GLM_BF16, None, 2),
                                    ("fp8", Xq, glm.GLM_FP8_E4M3, sc, 1)):
        ds = glm.glm_dataset_register(ctx, glm.make_desc(Xs, y, dtype=dt, col_scale=scale))
        outs = torch.empty((total, K + 1), dtype=torch.float64, device=dev)
        wall, kern_ms, _ = _timed_evals(glm, glm.lib(), ctx, ds, prior, betas, outs, K,
                                        args.warmup, args.steps, stream)
        bytes_alg = float(N) * K * es + N
        avg = float(kern_ms.mean())
        formats[name] = {"traffic": measured_traffic(f"fg_fused_precision_{name}"),
                         "evals_per_s": args.steps / wall, "launch_us_avg": avg * 1e3,
                         "GBps": bytes_alg / (avg * 1e-3) / 1e9,
                         "frac_peak": bytes_alg / (avg * 1e-3) / 1e9 / PEAK_HBM_GBPS,
                         "bytes_per_launch": bytes_alg, "first_out": outs[0].cpu().numpy()}
        glm.glm_dataset_unregister(ctx, ds)
        print(f"[bench] {name}: {formats[name]['evals_per_s']:.1f} evals/s "
              f"{formats[name]['GBps']:.0f} GB/s", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        cpu = _precision_cpu_leg(w, Xb, Xq, sc)
        for name in ("fp32", "bf16", "fp8"):
            out = formats[name]["first_out"]
            formats[name]["kernel_err"] = _rel_err(out, cpu["refs"][name])
            if name != "fp32":
                formats[name]["storage_err"] = _rel_err(out, cpu["refs"]["fp32"])
                formats[name]["encoder_codes_equal_oracle"] = cpu["codes_equal"][name]
    for f in formats.values():
        f.pop("first_out")
    glm.glm_destroy(ctx)
    b = formats["bf16"]
    result = {
        "metric": "logpost+grad evals/s (fused f+g, FP64 result) & HBM GB/s % peak",
        "value": b["evals_per_s"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 / b["evals_per_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"precision: N={N} K={K}, X as FP32 / BF16 / FP8-E4M3 "
                               "(per-column scales), same trajectory", "N": N, "K": K},
        "roofline": {"bound": "hbm", "achieved": b["GBps"], "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": b["frac_peak"],
                     "traffic": measured_traffic("fg_fused_precision_bf16")},
        "formats": formats,
    }
    if not args.no_cpu_baseline:
        result["err_vs_fp64"] = {
            name: {"kernel": formats[name]["kernel_err"],
                   "storage": formats[name].get("storage_err")} for name in formats}
        result["cpu_baseline"] = cpu_baseline_report(
            1.0, "evals/s (FP32 X)", (cpu["seconds_1"], 1), (cpu["seconds_thr"], 1,
                                                              cpu["threads"]),
            cpu["som"], cpu["host"],
            f"one FP32 evaluation at the first trajectory point on {cpu['threads']} threads "
            "(row blocks, fsum-combined); single-threaded on the first N/8 rows, scaled; the "
            "NumPy sequence of maps on the first N/16 rows, scaled", None)
        result["cpu_baseline"]["by_format_evals_per_s"] = {
            "fp32": 1.0 / cpu["seconds_thr"],
            **{k: 1.0 / v for k, v in cpu["seconds_fmt"].items()}}
    return result


def bench_batched(args):
    """Hierarchical model: 2,000 groups (sizes LogNormal(ln 500, 1.2) clipped
    to [20, 50,000]), K = 32, FP32; each step evaluates every group at its
    current beta_g in one launch, the betas following per-group random walks.
    Compared with one plain launch per group."""
    import ctypes

    import numpy as np
    import torch

    import synth
    from paper_1310_1537_amd import glm

    dev = torch.device("cuda:0")
    w = synth.hierarchical()
    G, K = w.betas.shape
    N = int(w.offsets[-1])
    steps = args.steps
    inc = synth.hierarchical_steps(G, K, min(steps + args.warmup, 500))
    traj = w.betas[None] + np.cumsum(inc, axis=0)
    nt = traj.shape[0]
    X = torch.from_numpy(w.X).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    B = torch.from_numpy(np.ascontiguousarray(traj)).to(dev)
    mu = torch.from_numpy(w.mu).to(dev)
    out = torch.empty((nt, G, K + 1), dtype=torch.float64, device=dev)
    ctx = glm.glm_create(0)
    desc = glm.make_desc(X, y)
    t0 = time.perf_counter()
    gs = glm.glm_groupset_create(ctx, desc, w.offsets, tune=True)
    t_create = time.perf_counter() - t0
    info = glm.glm_groupset_query(gs)
    prior = glm.make_prior(w.prec, mu)
    lib = glm.lib()
    pr = ctypes.byref(prior)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream

    def launch(i):
        st = lib.glm_logpost_grad_batched(ctx, gs, B.data_ptr() + (i % nt) * G * K * 8, pr,
                                          out.data_ptr() + (i % nt) * G * (K + 1) * 8, sp)
        if st:
            raise glm.GlmError(st, glm.glm_last_error())

    n_warm = _warm(launch, args.warmup)
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for j in range(steps):
        ev0[j].record(stream)
        launch(n_warm + j)
        ev1[j].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = np.array([a.elapsed_time(b) for a, b in zip(ev0, ev1)])
    bytes_alg = float(N) * K * 4 + N
    avg = float(kern_ms.mean())

    # one plain launch per group, same betas (a few steps)
    ids = [glm.glm_dataset_register(ctx, glm.make_desc(X[w.offsets[g]:w.offsets[g + 1]],
                                                       y[w.offsets[g]:w.offsets[g + 1]]))
           for g in range(G)]
    outp = torch.empty((G, K + 1), dtype=torch.float64, device=dev)
    psteps = 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(psteps):
        base = B.data_ptr() + (j % nt) * G * K * 8
        for g in range(G):
            st = lib.glm_logpost_grad(ctx, ids[g], base + g * K * 8, pr,
                                      outp.data_ptr() + g * (K + 1) * 8, sp)
            if st:
                raise glm.GlmError(st, glm.glm_last_error())
    torch.cuda.synchronize()
    wall_plain = (time.perf_counter() - t0) / psteps
    for i in ids:
        glm.glm_dataset_unregister(ctx, i)
    got0 = out[0].cpu().numpy()   # the launches with i % nt == 0 all evaluated B[0]

    result = {
        "metric": "logpost+grad evals/s (fused f+g, FP64 result) & HBM GB/s % peak",
        "value": steps / wall, "unit": "steps/s (all 2000 groups per step)", "n_gpus": 1,
        "steps": steps, "warmup": n_warm, "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"hierarchical: G={G} groups, N={N} rows, K={K}, FP32",
                   "G": G, "N": N, "K": K},
        "group_evals_per_s": G * steps / wall,
        "roofline": {"bound": "hbm", "achieved": bytes_alg / (avg * 1e-3) / 1e9,
                     "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": bytes_alg / (avg * 1e-3) / 1e9 / PEAK_HBM_GBPS,
                     "traffic": measured_traffic("fg_batched_hierarchical", "batched"),
                     "bytes_per_launch": bytes_alg, "launch_us_avg": avg * 1e3,
                     "note": "X is 263 MB, about the 256 MB Infinity Cache: repeated steps "
                             "may be served partly from it (traffic counts what left L2)"},
        "schedule": info, "groupset_create_s": t_create,
        "plain_per_group": {"ms_per_step": wall_plain * 1e3,
                            "speedup_of_batched": wall_plain / (wall / steps)},
    }
    glm.glm_groupset_destroy(gs)
    glm.glm_destroy(ctx)
    if not args.no_cpu_baseline:
        from concurrent.futures import ThreadPoolExecutor

        import oracle
        B0 = traj[0]
        t0 = time.perf_counter()
        ref = oracle.logpost_grad_groups(w.X, w.y, w.offsets, B0, w.prec, mean=w.mu)
        dt1 = time.perf_counter() - t0
        thr = cpu_threads()
        # the groups split into thr ranges of about equal rows, one per thread
        cuts = np.searchsorted(w.offsets, np.linspace(0, N, thr + 1)).clip(0, G)
        cuts[0], cuts[-1] = 0, G
        ranges = [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]

        def part(ab):
            a, b = ab
            o = w.offsets[a:b + 1]
            return oracle.logpost_grad_groups(w.X[o[0]:o[-1]], w.y[o[0]:o[-1]], o - o[0],
                                              B0[a:b], w.prec, mean=w.mu)

        with ThreadPoolExecutor(thr) as pool:
            t0 = time.perf_counter()
            ref_t = np.concatenate(list(pool.map(part, ranges)))
            dtt = time.perf_counter() - t0
        assert np.array_equal(ref, ref_t)
        fr = np.abs(got0[:, 0] - ref[:, 0]) / np.abs(ref[:, 0])
        gr = np.linalg.norm(got0[:, 1:] - ref[:, 1:], axis=1) / np.linalg.norm(ref[:, 1:], axis=1)
        result["err_vs_fp64"] = {"f_rel_max": float(fr.max()), "g_rel_norm_max": float(gr.max()),
                                 "groups": G, "note": "every group at the first step's betas"}
        result["cpu_baseline"] = cpu_baseline_report(
            1.0, "steps/s (all 2000 groups per step)", (dt1, 1), (dtt, 1, len(ranges)), None,
            host_info(), f"one full step (all {G} groups) single-threaded and split by groups "
            f"over {len(ranges)} threads", None)
    return result


def bench_plain_small(args):
    """Latency-bound small problem: N=10,000, K=20, FP64 X; the 100 seeded
    points and beta = 0.  Reports device-resident throughput, kernel and
    host-call latency percentiles, the empty-kernel offload round trip of
    the paper's Sec. 4.5 on this GPU, and the error against the oracle."""
    import numpy as np
    import torch

    import synth
    from paper_1310_1537_amd import glm

    dev = torch.device("cuda:0")
    w = synth.plain_small(n_evals=100)
    N, K = w.X.shape
    X = torch.from_numpy(w.X).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    nb = w.betas.shape[0]
    betas = torch.from_numpy(np.ascontiguousarray(w.betas)).to(dev)
    outs = torch.empty((nb, K + 1), dtype=torch.float64, device=dev)
    ctx = glm.glm_create(0)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(X, y))
    prior = glm.make_prior(w.prec)
    stream = torch.cuda.current_stream()
    wall, kern_ms, n_warm = _timed_evals(glm, glm.lib(), ctx, ds, prior, betas, outs, K,
                                         args.warmup, args.steps, stream)
    # all points once more, in order, for the error check
    for i in range(nb):
        glm.glm_logpost_grad(ctx, ds, betas[i], prior, outs[i], stream)
    torch.cuda.synchronize()
    got = outs.cpu().numpy()
    g_host = np.empty(K)
    lat = []
    for i in range(max(args.latency_calls, 200)):
        a = time.perf_counter()
        glm.glm_logpost_grad_host(ctx, ds, w.betas[i % nb], prior, g_host)
        lat.append(time.perf_counter() - a)
    lat_us = np.array(lat) * 1e6
    probe_us = glm.glm_probe_roundtrip(ctx, K, 2000)
    import oracle
    t0 = time.perf_counter()
    ref = [oracle.logpost_grad(w.X, w.y, b, w.prec) for b in w.betas]
    dt_cpu = time.perf_counter() - t0
    host = host_info()
    thr = cpu_threads()
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(thr) as pool:
        t0 = time.perf_counter()
        for b in w.betas:
            oracle.logpost_grad_blocks(w.X, w.y, b, w.prec, threads=thr, pool=pool)
        dt_thr = time.perf_counter() - t0
    som_t = sum(numpy_som(w.X, w.y, b, w.prec)[0] for b in w.betas)
    ef = max(abs(got[i, 0] - ref[i][0]) / abs(ref[i][0]) for i in range(nb))
    eg = max(np.linalg.norm(got[i, 1:] - ref[i][1]) / max(np.linalg.norm(ref[i][1]), 1e-300)
             for i in range(nb))
    bytes_alg = float(N) * K * 8 + N
    avg = float(kern_ms.mean())
    glm.glm_dataset_unregister(ctx, ds)
    glm.glm_destroy(ctx)
    return {
        "metric": "logpost+grad evals/s (fused f+g, FP64 result) & HBM GB/s % peak",
        "value": args.steps / wall, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "plain small: N=10,000 K=20 FP64 X, 100 seeded points + beta=0",
                   "N": N, "K": K},
        "roofline": {"bound": "latency", "achieved": bytes_alg / (avg * 1e-3) / 1e9,
                     "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": bytes_alg / (avg * 1e-3) / 1e9 / PEAK_HBM_GBPS, "traffic": None,
                     "bytes_per_launch": bytes_alg, "launch_us_avg": avg * 1e3},
        "latency_us": {"kernel_p50": float(np.percentile(kern_ms, 50) * 1e3),
                       "kernel_p99": float(np.percentile(kern_ms, 99) * 1e3),
                       "host_call_p50": float(np.percentile(lat_us, 50)),
                       "host_call_p99": float(np.percentile(lat_us, 99)),
                       "empty_kernel_roundtrip": probe_us},
        "err_vs_fp64": {"f_rel_max": ef, "g_rel_norm_max": eg, "points": nb},
        "cpu_baseline": cpu_baseline_report(
            1.0, "evals/s", (dt_cpu, nb), (dt_thr, nb, thr), (som_t, nb), host,
            f"all {nb} points: the oracle single-threaded and on {thr} threads (row blocks, "
            "fsum-combined; at this size thread start-up dominates), and the NumPy sequence "
            "of maps", None),
    }


def bench_serving(args):
    """Request server: 64 device-resident data sets (N log-uniform on [1e3,
    2e6], K from {8, 32, 128, 512}, BF16 or FP32 50/50), 512 chains (8 per
    data set) sending open-loop Poisson arrivals, each request a fresh beta
    (the chain's state plus N(0, 0.01^2 I)).  Throughput and submit-to-result
    latency per arrival rate, with passes of up to 8 vectors and with one
    request per pass."""
    import numpy as np
    import torch

    import synth
    from paper_1310_1537_amd import glm

    dev = torch.device("cuda:0")
    spec = synth.serving_specs()
    nd = len(spec.N)
    ctx = glm.glm_create(0)
    keep = []          # device tensors of the data sets
    datasets = []      # (K, beta_true, bytes)
    host_sets = []     # (X float32, y) on the host, for the error check
    t0 = time.perf_counter()
    for i in range(nd):
        X32, y, bt = synth.serving_dataset(i, spec)
        host_sets.append((X32, y))
        Xd = torch.from_numpy(X32).to(dev)
        yd = torch.from_numpy(y).to(dev)
        if spec.dtype[i] == "bf16":
            Q = torch.empty(Xd.shape, dtype=torch.uint16, device=dev)
            glm.glm_quantize_bf16(ctx, Xd, Q)
            torch.cuda.synchronize()
            del Xd
            keep.append((Q, yd, glm.GLM_BF16))
            es = 2
        else:
            keep.append((Xd, yd, glm.GLM_F32))
            es = 4
        datasets.append((int(spec.K[i]), bt, int(spec.N[i]) * (int(spec.K[i]) * es + 1)))
    total_bytes = sum(d[2] for d in datasets)
    print(f"[bench] {nd} data sets, {total_bytes / 1e9:.2f} GB, built in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    n_chains = 512
    pool = 16
    rng = np.random.default_rng(4)
    betas = []        # per chain: pool x K
    for c in range(n_chains):
        K, bt, _ = datasets[c // 8]
        state = bt + 0.1 * rng.standard_normal(K)
        betas.append(np.ascontiguousarray(state + 0.01 * rng.standard_normal((pool, K))))
    ptr_table = np.array([[b[j].ctypes.data for j in range(pool)] for b in betas], np.uint64)

    def run(nbmax, rate, n_req, seed):
        srv = glm.glm_server_create(ctx, 200 * (1 << 30), nbmax, args.serving_streams,
                                    args.serving_slots, 1 << 22, args.serving_max_sets)
        ids = [glm.glm_server_add_dataset(srv, glm.make_desc(X, y, dtype=dt), on_device=True)
               for X, y, dt in keep]
        # warm: one pass per data set
        t = glm.glm_server_submit_many(srv, np.array(ids, np.int64),
                                       ptr_table[np.arange(nd) * 8, 0], np.full(nd, 0.01))
        glm.glm_server_wait_many(srv, t)
        glm.glm_server_reset_stats(srv)
        arr, chain = synth.poisson_arrivals(rate, n_req, n_chains, seed)
        ds_of = np.array(ids, np.int64)[chain // 8]
        ptrs = ptr_table[chain, np.arange(n_req) % pool]
        precs = np.full(n_req, 0.01)
        tickets = []
        i = 0
        t0 = time.perf_counter()
        while i < n_req:
            now = time.perf_counter() - t0
            j = int(np.searchsorted(arr, now, side="right"))
            if j > i:
                tickets.append(glm.glm_server_submit_many(srv, ds_of[i:j], ptrs[i:j], precs[i:j]))
                i = j
        for t in tickets:
            glm.glm_server_wait_many(srv, t)
        wall = time.perf_counter() - t0
        st = glm.glm_server_stats(srv)
        glm.glm_server_destroy(srv)
        return {"rate_offered": rate, "requests": n_req, "throughput": n_req / wall,
                "GBps_streamed": st["bytes_streamed"] / wall / 1e9,
                "latency_p50_us": st["latency_p50_us"], "latency_p99_us": st["latency_p99_us"],
                "latency_mean_us": st["latency_mean_us"], "passes": st["passes"],
                "mean_pass_width": st["betas_in_passes"] / max(1, st["passes"]),
                "launches": st["launches"],
                "mean_sets_per_launch": st["passes"] / max(1, st["launches"]),
                "pass_width_hist": st["pass_width_hist"][1:], "failed": st["failed"]}

    rates = [int(r) for r in args.serving_rates.split(",")]
    res_b, res_1 = [], []
    for k, r in enumerate(rates):
        n_req = int(min(r * args.serving_seconds, 400_000))
        res_b.append(run(8, r, n_req, k))
        print(f"[bench] batched  rate {r}: {res_b[-1]['throughput']:.0f} req/s "
              f"p50 {res_b[-1]['latency_p50_us']:.0f} us p99 {res_b[-1]['latency_p99_us']:.0f} us "
              f"width {res_b[-1]['mean_pass_width']:.2f} "
              f"sets/launch {res_b[-1]['mean_sets_per_launch']:.2f}", file=sys.stderr, flush=True)
    for k, r in enumerate(rates[:2] if args.serving_baseline else []):
        n_req = int(min(r * args.serving_seconds, 100_000))
        res_1.append(run(1, r, n_req, 10 + k))
        print(f"[bench] one/pass rate {r}: {res_1[-1]['throughput']:.0f} req/s "
              f"p50 {res_1[-1]['latency_p50_us']:.0f} us p99 {res_1[-1]['latency_p99_us']:.0f} us",
              file=sys.stderr, flush=True)
    # Saturated server: every chain's request of a round submitted at once,
    # 40 rounds back to back (20,480 requests queued), so that every pass can
    # be full; the open-loop rates are judged against this throughput.
    saturated = None
    try:
        srv = glm.glm_server_create(ctx, 200 * (1 << 30), 8, args.serving_streams,
                                    args.serving_slots, 1 << 22, args.serving_max_sets)
        ids = [glm.glm_server_add_dataset(srv, glm.make_desc(X, y, dtype=dt), on_device=True)
               for X, y, dt in keep]
        t = glm.glm_server_submit_many(srv, np.array(ids, np.int64),
                                       ptr_table[np.arange(nd) * 8, 0], np.full(nd, 0.01))
        glm.glm_server_wait_many(srv, t)
        glm.glm_server_reset_stats(srv)
        rounds = 40
        chain = np.tile(np.arange(n_chains), rounds)
        ds_of = np.array(ids, np.int64)[chain // 8]
        ptrs = ptr_table[chain, np.repeat(np.arange(rounds), n_chains) % pool]
        t0 = time.perf_counter()
        t = glm.glm_server_submit_many(srv, ds_of, ptrs, np.full(len(chain), 0.01))
        glm.glm_server_wait_many(srv, t)
        wall = time.perf_counter() - t0
        st = glm.glm_server_stats(srv)
        glm.glm_server_destroy(srv)
        saturated = {"requests": len(chain), "throughput": len(chain) / wall,
                     "mean_pass_width": st["betas_in_passes"] / max(1, st["passes"]),
                     "mean_sets_per_launch": st["passes"] / max(1, st["launches"]),
                     "GBps_streamed": st["bytes_streamed"] / wall / 1e9,
                     "frac_reached_at_top_rate": res_b[-1]["throughput"] / (len(chain) / wall)}
        print(f"[bench] saturated: {saturated['throughput']:.0f} req/s width "
              f"{saturated['mean_pass_width']:.2f}; the top offered rate reached "
              f"{saturated['frac_reached_at_top_rate']:.2f} of it", file=sys.stderr, flush=True)
    except Exception as e:   # recorded, not lost
        saturated = {"error": repr(e)}
    # The passes' own cost: each data set's several-beta pass of 8 vectors
    # (the server's width) timed alone with HIP events; with requests spread
    # evenly over the data sets (8 chains each), one launch per pass would
    # allow 1 / (mean over data sets of the time per vector).  Fleet launches
    # share the per-launch cost between data sets, so the server can exceed
    # it.
    ceiling = None
    try:
        stream = torch.cuda.current_stream()
        per_vec = []
        pr = glm.make_prior(0.01)
        for i, (X, y, dt) in enumerate(keep):
            ds = glm.glm_dataset_register(ctx, glm.make_desc(X, y, dtype=dt))
            K = datasets[i][0]
            B = torch.from_numpy(np.ascontiguousarray(betas[8 * i][:8])).to(dev)
            out = torch.empty((8, K + 1), dtype=torch.float64, device=dev)
            for _ in range(3):
                glm.glm_logpost_grad_multi(ctx, ds, B, 8, pr, out, stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(10):
                glm.glm_logpost_grad_multi(ctx, ds, B, 8, pr, out, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            per_vec.append(e0.elapsed_time(e1) * 1e3 / 10 / 8)
            glm.glm_dataset_unregister(ctx, ds)
        mean_us = float(np.mean(per_vec))
        ceiling = {"requests_per_s": 1e6 / mean_us, "mean_us_per_vector": mean_us,
                   "frac_reached": res_b[-1]["throughput"] / (1e6 / mean_us),
                   "note": "each data set's pass of 8 vectors (glm_logpost_grad_multi) timed "
                           "alone; requests are spread evenly over the data sets"}
        print(f"[bench] pass-cost ceiling {ceiling['requests_per_s']:.0f} req/s; reached "
              f"{ceiling['frac_reached']:.2f} of it", file=sys.stderr, flush=True)
    except Exception as e:   # recorded, not lost
        ceiling = {"error": repr(e)}
    # binding budget: the same data sets given from pinned host memory to a
    # server whose budget holds about a third of them, so that admissions and
    # evictions churn under the open-loop load
    budget_res = None
    if args.serving_budget_gb >= 0:
        pinned = []
        for (Xk, yk, dt), (X32, y) in zip(keep, host_sets):
            src = Xk.cpu() if dt == glm.GLM_BF16 else torch.from_numpy(X32)
            pinned.append((src.pin_memory(), torch.from_numpy(y).pin_memory(), dt))
        print("[bench] budget leg: host copies pinned", file=sys.stderr, flush=True)
        largest = max(d[2] for d in datasets)
        budget = int(args.serving_budget_gb * 1e9) if args.serving_budget_gb > 0 else \
            int(max(1.25 * largest, 0.5 * total_bytes))
        rate = args.serving_budget_rate
        n_req = int(rate * args.serving_seconds)
        srv = glm.glm_server_create(ctx, budget, 8, args.serving_streams, args.serving_slots,
                                    1 << 22, args.serving_max_sets)
        ids = [glm.glm_server_add_dataset(
                   srv, glm.glm_dataset_desc(Xp.data_ptr(), Xp.shape[1], dt, None, yp.data_ptr(),
                                             Xp.shape[0], Xp.shape[1], 0))
               for Xp, yp, dt in pinned]
        arr, chain = synth.poisson_arrivals(rate, n_req, n_chains, 20)
        ds_of = np.array(ids, np.int64)[chain // 8]
        ptrs = ptr_table[chain, np.arange(n_req) % pool]
        precs = np.full(n_req, 0.01)
        tickets = []
        i = 0
        t0 = time.perf_counter()
        while i < n_req:
            now = time.perf_counter() - t0
            j = int(np.searchsorted(arr, now, side="right"))
            if j > i:
                tickets.append(glm.glm_server_submit_many(srv, ds_of[i:j], ptrs[i:j], precs[i:j]))
                i = j
        # past the deadline the server is shut down, which cancels what is
        # still queued (the record then counts completed requests only)
        import threading
        timer = threading.Timer(max(0.0, args.serving_budget_deadline - (time.perf_counter() - t0)),
                                glm.glm_server_shutdown, args=(srv,))
        timer.start()
        done = 0
        for t in tickets:
            glm.glm_server_wait_many(srv, t)
            if (done + len(t)) // 2000 > done // 2000:
                print(f"[bench] budget leg: {done + len(t)} of {n_req} requests done after "
                      f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
            done += len(t)
        wall = time.perf_counter() - t0
        timer.cancel()
        timer.join()
        st = glm.glm_server_stats(srv)
        glm.glm_server_destroy(srv)
        budget_res = {"hbm_budget_GB": budget / 1e9, "data_GB": total_bytes / 1e9,
                      "rate_offered": rate, "requests": n_req, "completed": st["completed"],
                      "cancelled_at_deadline": st["cancelled"],
                      "throughput": st["completed"] / wall,
                      "latency_p50_us": st["latency_p50_us"],
                      "latency_p99_us": st["latency_p99_us"],
                      "admissions": st["admissions"], "evictions": st["evictions"],
                      "GB_admitted": st["bytes_admitted"] / 1e9,
                      "GB_staged": st["bytes_staged"] / 1e9,
                      "admit_GBps": st["bytes_admitted"] / max(st["admit_seconds"], 1e-9) / 1e9,
                      "mean_pass_width": st["betas_in_passes"] / max(1, st["passes"]),
                      "failed": st["failed"],
                      "note": "host-sourced (pinned) data sets admitted on demand by the "
                              "server's copy thread; evicted allocations reused"}
        print(f"[bench] budget {budget / 1e9:.2f} GB rate {rate}: "
              f"{budget_res['throughput']:.0f} req/s p50 {budget_res['latency_p50_us']:.0f} us "
              f"p99 {budget_res['latency_p99_us']:.0f} us admissions {st['admissions']}",
              file=sys.stderr, flush=True)
        del pinned
    check = None
    if not args.no_cpu_baseline:
        check = _serving_check(glm, ctx, keep, host_sets, ptr_table, args)
    glm.glm_destroy(ctx)
    top = res_b[-1]
    rec = {
        "metric": "logpost+grad requests/s served (fused f+g, FP64 result), p50/p99 latency",
        "value": top["throughput"], "unit": "requests/s", "n_gpus": 1,
        "steps": top["requests"], "warmup": nd, "ms_per_step": 1e3 / top["throughput"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32/bf16",
        "data": "synthetic",
        "config": {"workload": f"serving: {nd} device-resident data sets ({total_bytes / 1e9:.2f} GB, "
                               "N log-uniform 1e3..2e6, K in {8,32,128,512}, BF16/FP32 50/50), "
                               "512 chains, open-loop Poisson arrivals",
                   "hbm_budget_GB": 200, "max_beta_per_pass": 8, "slots": args.serving_slots,
                   "streams": args.serving_streams, "max_sets_per_launch": args.serving_max_sets or 32},
        "latency_us": {"p50": top["latency_p50_us"], "p99": top["latency_p99_us"]},
        "roofline": {"bound": "hbm", "achieved": top["GBps_streamed"], "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": top["GBps_streamed"] / PEAK_HBM_GBPS,
                     "traffic": None,
                     "note": "X and y bytes of every pass (one read per pass of up to 8 "
                             "requests) over the wall time at the highest offered rate"},
        "by_rate": res_b, "one_request_per_pass": res_1, "binding_budget": budget_res,
        "pass_cost_ceiling": ceiling, "saturated": saturated,
    }
    if check is not None:
        rec["err_vs_fp64"] = check["err"]
        rec["cpu_baseline"] = check["cpu_baseline"]
    return rec


def _serving_check(glm, ctx, keep, host_sets, ptr_table, args):
    """One server request per data set (chain 8i's first beta), f and g
    checked against the oracle on the stored values (FP32 X, or the BF16
    codes read back from the device); the oracle's time over the same 64
    requests, single-threaded and on all host threads, gives the CPU
    request rate (chains are uniform over data sets)."""
    import ctypes
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    nd = len(keep)
    srv = glm.glm_server_create(ctx, 200 * (1 << 30), 8, args.serving_streams,
                                args.serving_slots, 1 << 16, args.serving_max_sets)
    ids = [glm.glm_server_add_dataset(srv, glm.make_desc(X, y, dtype=dt), on_device=True)
           for X, y, dt in keep]
    got = []
    for i in range(nd):
        K = keep[i][0].shape[1]
        beta = np.ctypeslib.as_array(ctypes.cast(int(ptr_table[8 * i, 0]),
                                                 ctypes.POINTER(ctypes.c_double)), (K,)).copy()
        t = glm.glm_server_submit(srv, ids[i], beta, 0.01)
        g = np.empty(K)
        f = glm.glm_server_wait(srv, t, g)
        got.append((beta, f, g))
    glm.glm_server_destroy(srv)
    thr = cpu_threads()
    worst_f = worst_g = 0.0
    t_single = t_thr = 0.0
    with ThreadPoolExecutor(thr) as pool:
        for i in range(nd):
            X32, y = host_sets[i]
            dt = keep[i][2]
            beta, f, g = got[i]
            if dt == glm.GLM_BF16:
                Xo, kw = keep[i][0].cpu().numpy(), {"dtype": "bf16"}
            else:
                Xo, kw = X32, {}
            a = time.perf_counter()
            rf, rg = oracle.logpost_grad_blocks(Xo, y, beta, 0.01, threads=thr, pool=pool, **kw)
            t_thr += time.perf_counter() - a
            a = time.perf_counter()
            oracle.logpost_grad(Xo, y, beta, 0.01, **kw)
            t_single += time.perf_counter() - a
            worst_f = max(worst_f, abs(f - rf) / abs(rf))
            worst_g = max(worst_g, float(np.linalg.norm(g - rg) / np.linalg.norm(rg)))
    return {"err": {"f_rel_max": worst_f, "g_rel_norm_max": worst_g, "requests": nd,
                    "note": "one request per data set through the server, against the oracle "
                            "on the stored FP32 values or BF16 codes"},
            "cpu_baseline": cpu_baseline_report(
                1.0, "requests/s", (t_single, nd), (t_thr, nd, thr), None, host_info(),
                f"the same {nd} requests (one per data set; chains are uniform over data "
                f"sets), the oracle single-threaded and on {thr} threads", None)}


def bench_copy(args):
    """A plain device-to-device copy of a known size (counter calibration)."""
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    a.fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    return {"metric": "copy", "value": 2 * n / dt / 1e9, "unit": "GB/s (read + write)",
            "bytes_read": n, "bytes_written": n}


def bench_diff(args):
    """Differential update (paper Sec. 3.4.4) on the 4M x 256 FP32 workload:
    a column-major copy of X, u = X beta kept on the device, and a sweep over
    the coordinates: per step, f at nd candidate moves of beta_k (one read of
    column k, u and y) and a commit of one move (u += delta X_k)."""
    import numpy as np
    import torch

    import synth
    from paper_1310_1537_amd import glm

    dev = torch.device("cuda:0")
    w = synth.plain_big(n_evals=2)
    N, K = w.X.shape
    X = torch.from_numpy(w.X).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    ctx = glm.glm_create(0)
    Xt = torch.empty((K, N), dtype=torch.float32, device=dev)
    glm.glm_transpose(ctx, glm.make_desc(X, y), Xt, N)
    del X
    cs = glm.glm_colset_register(ctx, glm.make_colset_desc(Xt, y))
    beta0 = w.betas[0]
    bd = torch.from_numpy(beta0.copy()).to(dev)
    u = torch.empty(N, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    glm.glm_linpred(ctx, cs, bd, u, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    linpred_ms = e0.elapsed_time(e1)
    prior = glm.make_prior(w.prec)
    total = args.warmup + args.steps
    rng = np.random.default_rng(7)
    res = {}
    for nd in (1, 8):
        deltas = torch.from_numpy(rng.normal(0.0, 0.01, (total, nd))).to(dev)
        outs = torch.empty((total, nd), dtype=torch.float64, device=dev)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for i in range(args.warmup):
            glm.glm_diff_logpost(ctx, cs, u, bd, i % K, deltas[i], nd, prior, outs[i], stream)
            glm.glm_diff_commit(ctx, cs, u, bd, i % K, deltas[i, :1], stream)
        torch.cuda.synchronize()
        # a short device-side wait first, so that the host has queued the
        # timed launches before the GPU reaches them (otherwise host call
        # overhead would sit between the events and the kernels)
        _device_hold(torch, 20e-3)
        for j in range(args.steps):
            i = args.warmup + j
            a, b, c = ev[j]
            a.record(stream)
            glm.glm_diff_logpost(ctx, cs, u, bd, i % K, deltas[i], nd, prior, outs[i], stream)
            b.record(stream)
            glm.glm_diff_commit(ctx, cs, u, bd, i % K, deltas[i, :1], stream)
            c.record(stream)
        torch.cuda.synchronize()
        span_s = ev[0][0].elapsed_time(ev[-1][2]) * 1e-3
        ev_ms = np.array([a.elapsed_time(b) for a, b, _ in ev])
        cm_ms = np.array([b.elapsed_time(c) for _, b, c in ev])
        res[nd] = {"steps_per_s": args.steps / span_s, "eval_us_avg": float(ev_ms.mean() * 1e3),
                   "eval_us_p50": float(np.percentile(ev_ms, 50) * 1e3),
                   "commit_us_avg": float(cm_ms.mean() * 1e3),
                   "f_evals_per_s_kernel": nd / float(ev_ms.mean() * 1e-3)}
        print(f"[bench] diff nd={nd}: {res[nd]}", file=sys.stderr, flush=True)
    # the per-row terms alone on the same grid, no memory traffic: the floor
    # that the one-step evaluation is bound by (timed back to back)
    map_floor_us = glm.glm_probe_diff_map(ctx, N, 0, 20)
    empty_us = glm.glm_probe_diff_map(ctx, 0, 0, 20)
    eval_bytes = float(N) * (4 + 8 + 1)
    commit_bytes = float(N) * (4 + 8 + 8)
    r1 = res[1]
    achieved = eval_bytes / (r1["eval_us_avg"] * 1e-6) / 1e9
    result = {
        "metric": "differential-update log-posterior evals/s (one coefficient moved, "
                  "FP64 result) & HBM GB/s % peak",
        "value": r1["f_evals_per_s_kernel"], "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 / r1["steps_per_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "differential update: N=4,000,000 K=256 FP32 X (column-major "
                               "copy), one coefficient per step, nd candidate moves per pass",
                   "N": N, "K": K},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBPS,
                     "traffic": measured_traffic("k_diff_eval_diff_update", "diff"),
                     "bytes_per_launch": eval_bytes, "launch_us_avg": r1["eval_us_avg"],
                     "note": "column k is new each step; u (32 MB) and y (4 MB) are re-read "
                             "every step and may be served from the 256 MB Infinity Cache",
                     "map_floor_us": map_floor_us, "empty_launch_us": empty_us,
                     "frac_of_map_floor": map_floor_us / r1["eval_us_avg"],
                     "map_note": "the FP64 per-row terms of N rows alone on the evaluation's "
                                 "grid with no loads (glm_probe_diff_map), back to back, "
                                 "launch included (empty_launch_us for zero rows): the "
                                 "evaluation is bound by them, not by its bytes"},
        "by_candidates": {str(k): v for k, v in res.items()},
        "commit_GBps": commit_bytes / (res[1]["commit_us_avg"] * 1e-6) / 1e9,
        "linpred_ms": linpred_ms,
    }
    if not args.no_cpu_baseline:
        import oracle
        b2 = beta0.copy()
        t0 = time.perf_counter()
        fo, _ = oracle.logpost_grad(w.X, w.y, b2, w.prec)
        dt = time.perf_counter() - t0
        # the GPU at the same point: u = X beta0, a zero move of coordinate 0
        bd.copy_(torch.from_numpy(beta0))
        glm.glm_linpred(ctx, cs, bd, u, stream)
        z = torch.zeros(1, dtype=torch.float64, device=dev)
        fo_gpu = torch.empty(1, dtype=torch.float64, device=dev)
        glm.glm_diff_logpost(ctx, cs, u, bd, 0, z, 1, prior, fo_gpu, stream)
        torch.cuda.synchronize()
        result["err_vs_fp64"] = {"f_rel": abs(float(fo_gpu.cpu()[0]) - fo) / abs(fo)}
        result["cpu_baseline"] = {"value": 1.0 / dt, "unit": "evals/s", "cores": 1,
                                  "kind": "oracle",
                                  "sample": "one full FP64 evaluation at the first trajectory "
                                            "point (the oracle has no differential form), "
                                            "single-threaded C"}
    glm.glm_colset_unregister(ctx, cs)
    glm.glm_destroy(ctx)
    return result


def bench_sampler(args):
    """Random-walk Metropolis with the whole chain on the device (glm_mh_run)
    against the same chain driven from the host (one glm_logpost_grad_host
    round trip and a host-side decision per step), on the 10,000 x 20 FP64
    workload where the round trip dominates (paper Sec. 4.5), and on the
    4M x 256 FP32 workload where the evaluation does."""
    import numpy as np
    import torch

    import synth
    from paper_1310_1537_amd import glm

    dev = torch.device("cuda:0")
    ctx = glm.glm_create(0)
    out = {}
    for name, w, n_dev, n_host, wi in (
            ("small_n10000_k20_f64", synth.plain_small(1), max(args.steps, 2000), 1000, 0),
            ("big_n4000000_k256_f32", synth.plain_big(n_evals=1), 200, 50, 1)):
        N, K = w.X.shape
        X = torch.from_numpy(w.X).to(dev)
        y = torch.from_numpy(w.y).to(dev)
        ds = glm.glm_dataset_register(ctx, glm.make_desc(X, y))
        prior = glm.make_prior(w.prec)
        incs, logu, _ = synth.mh_chain_inputs(K, n_dev, N, workload_index=wi)
        inc_d = torch.from_numpy(incs).to(dev)
        lu_d = torch.from_numpy(logu).to(dev)
        fg = torch.empty(K + 1, dtype=torch.float64, device=dev)
        acc = torch.empty(n_dev, dtype=torch.uint8, device=dev)
        # warm-up (plans, scratch)
        b = torch.from_numpy(w.beta_true.copy()).to(dev)
        glm.glm_mh_run(ctx, ds, b, fg, inc_d, lu_d, min(20, n_dev), prior, acc)
        torch.cuda.synchronize()
        b = torch.from_numpy(w.beta_true.copy()).to(dev)
        t0 = time.perf_counter()
        glm.glm_mh_run(ctx, ds, b, fg, inc_d, lu_d, n_dev, prior, acc)
        torch.cuda.synchronize()
        dev_s = time.perf_counter() - t0
        dev_acc = acc.cpu().numpy()
        # host-driven: the same increments and uniforms
        beta = w.beta_true.copy()
        f_cur = glm.glm_logpost_grad_host(ctx, ds, beta, prior)
        host_acc = np.empty(n_host, np.uint8)
        t0 = time.perf_counter()
        for t in range(n_host):
            bp = beta + incs[t]
            fp = glm.glm_logpost_grad_host(ctx, ds, bp, prior)
            host_acc[t] = logu[t] < fp - f_cur
            if host_acc[t]:
                beta, f_cur = bp, fp
        host_s = time.perf_counter() - t0
        out[name] = {"device_steps_per_s": n_dev / dev_s, "device_us_per_step": dev_s / n_dev * 1e6,
                     "host_steps_per_s": n_host / host_s, "host_us_per_step": host_s / n_host * 1e6,
                     "speedup": (n_dev / dev_s) / (n_host / host_s),
                     "accept_rate": float(dev_acc.mean()),
                     "decisions_equal_host_driven": bool(np.array_equal(dev_acc[:n_host], host_acc)),
                     "steps_device": n_dev, "steps_host": n_host}
        # HMC on the device (momenta and accept uniforms drawn there): step
        # about half the posterior scale 1/sqrt(0.2 N), 5 leapfrog steps
        n_it, L = (400, 5) if N < 100_000 else (20, 5)
        eps = 0.5 / np.sqrt(0.2 * N)
        acc_h = torch.empty(n_it, dtype=torch.uint8, device=dev)
        b = torch.from_numpy(w.beta_true.copy()).to(dev)
        glm.glm_hmc_run(ctx, ds, b, fg, 2, L, eps, 1, 1, prior, acc_h)
        torch.cuda.synchronize()
        b = torch.from_numpy(w.beta_true.copy()).to(dev)
        t0 = time.perf_counter()
        glm.glm_hmc_run(ctx, ds, b, fg, n_it, L, eps, 1, 1, prior, acc_h)
        torch.cuda.synchronize()
        hmc_s = time.perf_counter() - t0
        out[name].update({"hmc_iterations_per_s": n_it / hmc_s,
                          "hmc_us_per_leapfrog_step": hmc_s / (n_it * L) * 1e6,
                          "hmc_leapfrog_steps": L, "hmc_eps": eps,
                          "hmc_accept_rate": float(acc_h.cpu().numpy().mean())})
        print(f"[bench] sampler {name}: {out[name]}", file=sys.stderr, flush=True)
        glm.glm_dataset_unregister(ctx, ds)
        del X, y
    # batch generation on the device: 2^26 values of each kind
    n_rng = 1 << 26
    buf = torch.empty(n_rng, dtype=torch.float64, device=dev)
    rng = {}
    for kname, kind in (("uniform", glm.GLM_RNG_UNIFORM), ("normal", glm.GLM_RNG_NORMAL),
                        ("log_uniform", glm.GLM_RNG_LOG_UNIFORM)):
        glm.glm_rng_fill(ctx, kind, 1, 2, 3, 0, n_rng, buf)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(5):
            glm.glm_rng_fill(ctx, kind, 1, 2, 3, r * n_rng, n_rng, buf)
        torch.cuda.synchronize()
        rng[kname + "_per_s"] = 5 * n_rng / (time.perf_counter() - t0)
    print(f"[bench] device generator: {rng}", file=sys.stderr, flush=True)
    del buf
    glm.glm_destroy(ctx)
    sm = out["small_n10000_k20_f64"]
    return {
        "metric": "random-walk Metropolis steps/s with the chain on the device (one fused "
                  "f+g evaluation per step)",
        "value": sm["device_steps_per_s"], "unit": "steps/s", "n_gpus": 1,
        "steps": sm["steps_device"], "warmup": 20, "ms_per_step": sm["device_us_per_step"] * 1e-3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "on-device Metropolis: N=10,000 K=20 FP64 (and N=4,000,000 K=256 "
                               "FP32), proposal sd 2.38/sqrt(K)/sqrt(0.2 N)"},
        "roofline": {"bound": "latency", "achieved": None, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": None, "traffic": None,
                     "note": "the small workload is bound by launch latency, not HBM"},
        "workloads": out, "device_generator": rng,
    }


def bench_hessian(args):
    """f, g and the Hessian H = -X^t W X - prec I fused (paper Sec. 5.2) on
    the 4M x 256 FP32 workload: FP64 matrix-core contraction over the rows."""
    import numpy as np
    import torch

    import synth
    from paper_1310_1537_amd import glm

    dev = torch.device("cuda:0")
    w = synth.plain_big(n_evals=max(args.steps, 1) + args.warmup)
    N, K = w.X.shape
    X = torch.from_numpy(w.X).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    ctx = glm.glm_create(0)
    ds = glm.glm_dataset_register(ctx, glm.make_desc(X, y))
    prior = glm.make_prior(w.prec)
    betas = torch.from_numpy(np.ascontiguousarray(w.betas)).to(dev)
    out = torch.empty(K + 1, dtype=torch.float64, device=dev)
    H = torch.empty((K, K), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    for i in range(args.warmup):
        glm.glm_logpost_grad_hess(ctx, ds, betas[i], prior, out, H, stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for j in range(args.steps):
        a, b = ev[j]
        a.record(stream)
        glm.glm_logpost_grad_hess(ctx, ds, betas[args.warmup + j], prior, out, H, stream)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    # the f+g part alone, for the split
    f_ms = []
    for j in range(min(args.steps, 20)):
        a, b = ev[j]
        a.record(stream)
        glm.glm_logpost_grad(ctx, ds, betas[j], prior, out, stream)
        b.record(stream)
        torch.cuda.synchronize()
        f_ms.append(a.elapsed_time(b))
    mfma_ceiling = glm.glm_probe_mfma_f64(ctx, 2000)
    glm.glm_dataset_unregister(ctx, ds)
    glm.glm_destroy(ctx)
    avg = float(ms.mean())
    fg_avg = float(np.mean(f_ms))
    flops = float(N) * K * (K + 1)          # the symmetric contraction, multiply-adds x 2
    h_ms = max(avg - fg_avg, 1e-6)
    return {
        "metric": "f + g + Hessian evals/s (FP64 Hessian on the matrix cores)",
        "value": args.steps / wall, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "Hessian: N=4,000,000 K=256 FP32 X, random-walk trajectory",
                   "N": N, "K": K},
        "roofline": {"bound": "mfma", "achieved": flops / (h_ms * 1e-3) / 1e12, "peak": 78.6,
                     "unit": "TFLOP/s", "frac": flops / (h_ms * 1e-3) / 1e12 / 78.6,
                     "traffic": None, "flops_per_launch": flops,
                     "measured_mfma_f64_ceiling_TFLOPs": mfma_ceiling,
                     "frac_of_measured_ceiling": flops / (h_ms * 1e-3) / 1e12 / mfma_ceiling,
                     "note": "Hessian kernel time = (f+g+H call) - (f+g call); peak is the "
                             "published FP64 matrix figure"},
        "ms_per_call": avg, "fg_ms": fg_avg, "hessian_kernel_ms": h_ms,
    }


def bench_multi(args):
    """Several coefficient vectors per pass (glm_logpost_grad_multi) over about
    2 GB of X for every storage type and row width of the serving workload,
    and for FP64 rows of the same widths: microseconds per launch and per
    vector at 1, 2, 4 and 8 vectors; for BF16
    rows of 65 columns and more at 4 and 8 vectors, the matrix-core form beside
    the VALU one (context option GLM_OPT_MATRIX_CORES = 0).  X ~ N(0, 1) drawn on the device (BF16 codes
    by the library's encoder), y ~ Bernoulli(1/2), beta ~ N(0, 0.01^2 I).
    The headline value is vector evaluations per second of the BF16 K = 512
    pass of four vectors on the matrix cores."""

    import numpy as np
    import torch

    from paper_1310_1537_amd import glm

    dev = torch.device("cuda:0")
    ctx = glm.glm_create(0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(20131006)
    stream = torch.cuda.current_stream()
    reps = max(3, min(args.steps, 20))
    rows, keep = [], None

    def timed(ds, K, nb):
        B = (0.01 * torch.randn((nb, K), device=dev, dtype=torch.float64, generator=gen)).contiguous()
        out = torch.empty((nb, K + 1), device=dev, dtype=torch.float64)
        pr = glm.make_prior(0.01)
        for _ in range(3):
            glm.glm_logpost_grad_multi(ctx, ds, B, nb, pr, out, stream)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            glm.glm_logpost_grad_multi(ctx, ds, B, nb, pr, out, stream)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1e3 / reps

    t0 = time.perf_counter()
    try:
        for K in (8, 32, 128, 512):
            for dt in ("f32", "bf16", "f64"):
                es = {"f32": 4, "bf16": 2, "f64": 8}[dt]
                N = int(2.0e9 // (K * es))
                X = torch.randn((N, K), device=dev,
                                dtype=torch.float64 if dt == "f64" else torch.float32, generator=gen)
                y = (torch.rand(N, device=dev, generator=gen) < 0.5).to(torch.uint8)
                code = glm.GLM_F64 if dt == "f64" else glm.GLM_F32
                if dt == "bf16":
                    Q = torch.empty((N, K), dtype=torch.uint16, device=dev)
                    glm.glm_quantize_bf16(ctx, X, Q)
                    torch.cuda.synchronize()
                    del X
                    X, code = Q, glm.GLM_BF16
                ds = glm.glm_dataset_register(ctx, glm.make_desc(X, y, dtype=code))
                nbytes = N * (K * es + 1)
                for nb in (1, 2, 4, 8):
                    forms = [("vector ALU", 0), ("matrix cores", 1)] \
                        if dt == "bf16" and K >= 65 and nb >= 4 else [("vector ALU", None)]
                    for form, mx in forms:
                        glm.glm_set_option(ctx, glm.GLM_OPT_MATRIX_CORES, 1 if mx is None else mx)
                        us = timed(ds, K, nb)
                        rows.append({"K": K, "storage": dt, "nb": nb, "form": form, "N": N,
                                     "us_per_launch": us, "us_per_vector": us / nb,
                                     "GBps_x_once": nbytes / us / 1e3})
                        if dt == "bf16" and K == 512 and nb == 4 and mx == 1:
                            keep = rows[-1]
                glm.glm_set_option(ctx, glm.GLM_OPT_MATRIX_CORES, 1)
                glm.glm_dataset_unregister(ctx, ds)
                del X, y
                torch.cuda.empty_cache()
    finally:
        glm.glm_destroy(ctx)
    wall = time.perf_counter() - t0
    for r in rows:
        print("[multi] K=%4d %-4s nb=%d %-12s %9.1f us/launch %8.1f us/vector %6.0f GB/s (X once)"
              % (r["K"], r["storage"], r["nb"], r["form"], r["us_per_launch"], r["us_per_vector"],
                 r["GBps_x_once"]), file=sys.stderr, flush=True)
    result = {
        "metric": "several-beta passes: vector evals/s (fused f+g per vector, FP64 results)",
        "value": 4.0 / (keep["us_per_launch"] * 1e-6), "unit": "vector evals/s",
        "n_gpus": 1, "steps": reps, "warmup": 3, "ms_per_step": keep["us_per_launch"] / 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "several beta per pass: about 2 GB of X per storage type (FP32, "
                               "BF16, FP64) and K in {8, 32, 128, 512}; headline BF16 K=512, "
                               "4 vectors, matrix cores",
                   "N": keep["N"], "K": 512},
        "roofline": {"bound": "hbm", "achieved": keep["GBps_x_once"], "peak": 8000.0, "unit": "GB/s",
                     "frac": keep["GBps_x_once"] / 8000.0,
                     "traffic": measured_traffic("fg_fused_mx_several_beta", "mx"),
                     "kernel": "fg_fused_mx<64, 4, 4>",
                     "note": "X bytes read once per pass of four vectors over the mean launch time; "
                             "the kernel is bound by its per-row map, LDS and VALU latency"},
        "table": rows, "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        import oracle
        g = np.random.default_rng(20131006)
        n_s, K = 20_000, 512
        Xs = g.standard_normal((n_s, K)).astype(np.float32)
        Qs = oracle.quantize_bf16(Xs)
        ys = (g.random(n_s) < 0.5).astype(np.uint8)
        Bs = 0.01 * g.standard_normal((4, K))
        c0 = time.perf_counter()
        reps_c = 0
        while time.perf_counter() - c0 < 10.0:
            oracle.logpost_grad_multi(Qs, ys, Bs, 0.01, dtype="bf16")
            reps_c += 1
        dt_c = time.perf_counter() - c0
        result["cpu_baseline"] = {
            "value": 4 * reps_c / dt_c * n_s / keep["N"], "unit": "vector evals/s", "cores": 1,
            "kind": "oracle",
            "sample": "4 vectors over a 20,000-row BF16 K=512 sample, repeated for about 10 s and "
                      "scaled to the benchmark's N (single-threaded FP64 C)"}
    return result


def bench_launch_fit(args):
    """Per-launch time of the plain kernel against the bytes it streams:
    N from 10,000 to 4,000,000 rows at K = 256 (FP32) and K = 32 (FP32), and
    the 10,000 x 20 FP64 workload, each timed over back-to-back launches with
    HIP events; a least-squares fit time = t0 + bytes / BW per K gives the
    fixed cost t0 of a launch (ramp-up, tail and the cross-block merge)."""
    import numpy as np
    import torch

    import synth
    from paper_1310_1537_amd import glm

    dev = torch.device("cuda:0")
    ctx = glm.glm_create(0)
    stream = torch.cuda.current_stream()
    reps = 200
    rows = []

    def time_ds(X, y, K, es, label):
        ds = glm.glm_dataset_register(ctx, glm.make_desc(X, y))
        b = torch.zeros(K, dtype=torch.float64, device=dev)
        b.normal_(0.0, 0.05)
        out = torch.empty(K + 1, dtype=torch.float64, device=dev)
        pr = glm.make_prior(0.01)
        for _ in range(10):
            glm.glm_logpost_grad(ctx, ds, b, pr, out, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            glm.glm_logpost_grad(ctx, ds, b, pr, out, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        N = X.shape[0]
        rows.append({"case": label, "N": N, "K": K, "bytes": N * (K * es + 1), "us": us})
        print(f"[bench] launch fit {label} N={N}: {us:.2f} us", file=sys.stderr, flush=True)
        glm.glm_dataset_unregister(ctx, ds)

    w = synth.plain_small(1)
    time_ds(torch.from_numpy(w.X).to(dev), torch.from_numpy(w.y).to(dev), 20, 8, "f64_k20")
    big = synth.plain_big(n_evals=1)
    Xb = torch.from_numpy(big.X).to(dev)
    yb = torch.from_numpy(big.y).to(dev)
    for N in (10_000, 40_000, 160_000, 640_000, 1_000_000, 2_000_000, 4_000_000):
        time_ds(Xb[:N], yb[:N], 256, 4, "f32_k256")
    X32 = Xb[:, :32].contiguous()
    for N in (10_000, 100_000, 500_000, 2_000_000, 4_000_000):
        time_ds(X32[:N], yb[:N], 32, 4, "f32_k32")
    fits = {}
    for label in ("f32_k256", "f32_k32"):
        r = [x for x in rows if x["case"] == label]
        A = np.array([[1.0, x["bytes"]] for x in r])
        t = np.array([x["us"] for x in r])
        coef, *_ = np.linalg.lstsq(A, t, rcond=None)
        fits[label] = {"t0_us": float(coef[0]), "GBps": float(1e-3 / coef[1]),
                       "max_resid_us": float(np.max(np.abs(A @ coef - t)))}
    glm.glm_destroy(ctx)
    k = fits["f32_k256"]
    return {"metric": "fixed per-launch cost of the fused kernel (fit of launch time to bytes)",
            "value": k["t0_us"], "unit": "us", "higher_is_better": False, "n_gpus": 1,
            "data": "synthetic", "config": {"workload": "plain kernel, N from 1e4 to 4e6"},
            "fits": fits, "points": rows}


def _sub_args(args, **kw):
    """A copy of the command-line namespace with some fields replaced."""
    d = dict(vars(args))
    d.update(kw)
    return argparse.Namespace(**d)


# The other measured configurations in the default run: (name, function,
# overrides).  Step counts are sized so that the whole default run stays
# within a few minutes on one GPU.
_SUB_CONFIGS = (
    ("plain_small", lambda a: bench_plain_small(a), dict(steps=2000, warmup=50, latency_calls=400)),
    ("precision", lambda a: bench_precision(a), dict(steps=20, warmup=5, n=0)),
    ("batched", lambda a: bench_batched(a), dict(steps=200, warmup=10)),
    ("serving", lambda a: bench_serving(a), dict(serving_seconds=1.0, serving_baseline=1)),
)


def bench_all(args):
    """The headline 4M x 256 FP32 workload (the top-level record), then the
    small, storage-precision, hierarchical and serving workloads, each as a
    record under "configs" (an exception is recorded there, not raised)."""
    result = bench_plain_big(args)
    configs = {}
    for name, fn, over in _SUB_CONFIGS:
        t0 = time.perf_counter()
        print(f"[bench] config {name}", file=sys.stderr, flush=True)
        try:
            rec = fn(_sub_args(args, **over))
        except Exception as e:  # recorded, so that one failure does not hide the others
            rec = {"error": f"{type(e).__name__}: {e}"}
        rec["bench_wall_s"] = time.perf_counter() - t0
        configs[name] = rec
        print(f"[bench] config {name} done in {rec['bench_wall_s']:.1f} s", file=sys.stderr,
              flush=True)
    result["configs"] = configs
    return result


WORKLOADS = {"all": bench_all, "copy": bench_copy, "launch_fit": bench_launch_fit, "plain_big": bench_plain_big, "precision": bench_precision,
             "batched": bench_batched, "plain_small": bench_plain_small,
             "serving": bench_serving, "diff": bench_diff,
             "poisson": lambda a: bench_plain_big(a, poisson=True),
             "sampler": bench_sampler, "hessian": bench_hessian, "multi": bench_multi}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="all", choices=sorted(WORKLOADS))
    ap.add_argument("--n", type=int, default=0, help="override N (precision workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-calls", type=int, default=200)
    ap.add_argument("--serving-seconds", type=float, default=1.0)
    ap.add_argument("--serving-rates", default="20000,50000,100000,200000")
    ap.add_argument("--serving-slots", type=int, default=8, help="passes in flight")
    ap.add_argument("--serving-streams", type=int, default=4)
    ap.add_argument("--serving-max-sets", type=int, default=0,
                    help="data sets per launch at most (0: the server default)")
    ap.add_argument("--serving-budget-gb", type=float, default=0.0,
                    help="HBM budget of the churn leg over host-sourced data sets (0: half "
                         "the data, at least 1.25 times the largest set; negative: skip)")
    ap.add_argument("--serving-budget-rate", type=int, default=20000)
    ap.add_argument("--serving-budget-deadline", type=float, default=30.0,
                    help="seconds after which the churn leg cancels what is still queued")
    ap.add_argument("--serving-baseline", type=int, default=1,
                    help="also run one request per pass at the first two rates")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the row-sharded design is described, not built). Run with --gpus 1.",
              file=sys.stderr)
        return 2
    result = WORKLOADS[args.workload](args)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Python binding of the C interface in include/glm.h (argument marshalling
only: every step of the computation runs in the HIP library).

The functions carry the C names.  Device buffers are passed as torch CUDA
tensors (their ``data_ptr()``) or as integer addresses; streams as a
``torch.cuda.Stream``, an integer hipStream_t, or None (the null stream).
Non-OK status codes raise :class:`GlmError` with the library's message,
except ``GLM_PENDING`` from ``glm_server_poll``, which is returned.

The library is loaded from the package directory; if it has not been built
the import fails loudly -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime the library shares

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libglm_hip.so")

GLM_OK, GLM_PENDING = 0, 1
GLM_EINVAL, GLM_EDTYPE, GLM_EHIP, GLM_ENOTFOUND = -1, -2, -3, -4
GLM_EBUDGET, GLM_ECANCELLED, GLM_EAGAIN, GLM_ENOMEM = -5, -6, -7, -8
GLM_F64, GLM_F32, GLM_BF16, GLM_FP8_E4M3 = 0, 1, 2, 3
GLM_LOGISTIC, GLM_POISSON = 0, 1
GLM_K_MAX = 4096
GLM_OPT_BLOCKS_PER_CU, GLM_OPT_INTERLEAVE, GLM_OPT_MATRIX_CORES = 1, 2, 3

STATUS_NAMES = {0: "GLM_OK", 1: "GLM_PENDING", -1: "GLM_EINVAL", -2: "GLM_EDTYPE",
                -3: "GLM_EHIP", -4: "GLM_ENOTFOUND", -5: "GLM_EBUDGET",
                -6: "GLM_ECANCELLED", -7: "GLM_EAGAIN", -8: "GLM_ENOMEM"}


class GlmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class glm_dataset_desc(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("ldx", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("col_scale", ctypes.c_void_p), ("y", ctypes.c_void_p), ("N", ctypes.c_int64),
                ("K", ctypes.c_int32), ("family", ctypes.c_int32)]


class glm_groupset_info_t(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int64), ("blocks", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("items", ctypes.c_int32),
                ("split_tiles", ctypes.c_int32), ("tuned_us", ctypes.c_double)]


class glm_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_beta_per_pass", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("n_slots", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int32), ("max_sets_per_pass", ctypes.c_int32)]


class glm_server_stats_t(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("cancelled", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("passes", ctypes.c_uint64), ("betas_in_passes", ctypes.c_uint64),
                ("admissions", ctypes.c_uint64), ("evictions", ctypes.c_uint64),
                ("resident_bytes", ctypes.c_uint64), ("resident_datasets", ctypes.c_int32),
                ("queue_depth", ctypes.c_int32), ("pass_width_hist", ctypes.c_uint64 * 9),
                ("latency_p50_us", ctypes.c_double), ("latency_p99_us", ctypes.c_double),
                ("latency_mean_us", ctypes.c_double), ("launches", ctypes.c_uint64),
                ("bytes_streamed", ctypes.c_uint64), ("bytes_admitted", ctypes.c_uint64),
                ("admit_seconds", ctypes.c_double), ("cached_bytes", ctypes.c_uint64),
                ("bytes_staged", ctypes.c_uint64)]


class glm_colset_desc(ctypes.Structure):
    _fields_ = [("Xt", ctypes.c_void_p), ("ldt", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("col_scale", ctypes.c_void_p), ("y", ctypes.c_void_p), ("N", ctypes.c_int64),
                ("K", ctypes.c_int32), ("family", ctypes.c_int32)]


class glm_prior(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_double), ("mean", ctypes.c_void_p),
                ("mean_per_group", ctypes.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() "
                      "(python -c 'import __graft_entry__ as g; g.build()')")

_lib = ctypes.CDLL(LIB_PATH)

_P, _I32, _I64, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_PP = ctypes.POINTER(ctypes.c_void_p)
_SIGS = {
    "glm_create": [ctypes.c_int, _PP],
    "glm_destroy": [_P],
    "glm_set_option": [_P, _I32, _I64],
    "glm_get_option": [_P, _I32, ctypes.POINTER(_I64)],
    "glm_dataset_register": [_P, ctypes.POINTER(glm_dataset_desc), ctypes.POINTER(_I64)],
    "glm_dataset_unregister": [_P, _I64],
    "glm_logpost_grad": [_P, _I64, _P, ctypes.POINTER(glm_prior), _P, _P],
    "glm_logpost_grad_noalloc": [_P, _I64, _P, ctypes.POINTER(glm_prior), _P, _P],
    "glm_logpost_grad_multi": [_P, _I64, _P, _I32, ctypes.POINTER(glm_prior), _P, _P],
    "glm_logpost_grad_host": [_P, _I64, _P, ctypes.POINTER(glm_prior), ctypes.POINTER(_D), _P],
    "glm_groupset_create": [_P, ctypes.POINTER(glm_dataset_desc), _P, _I32, _I32, _PP],
    "glm_groupset_destroy": [_P],
    "glm_groupset_query": [_P, ctypes.c_void_p],
    "glm_logpost_grad_batched": [_P, _P, _P, ctypes.POINTER(glm_prior), _P, _P],
    "glm_server_create": [_P, ctypes.POINTER(glm_server_config), _PP],
    "glm_server_add_dataset": [_P, ctypes.POINTER(glm_dataset_desc), _I32, ctypes.POINTER(_I64)],
    "glm_server_submit": [_P, _I64, _P, _D, _P, ctypes.POINTER(ctypes.c_uint64)],
    "glm_server_submit_many": [_P, _I32, _P, _P, _P, _P],
    "glm_server_wait_many": [_P, _I32, _P, _P],
    "glm_server_poll": [_P, ctypes.c_uint64, ctypes.POINTER(_D), _P],
    "glm_server_wait": [_P, ctypes.c_uint64, ctypes.POINTER(_D), _P],
    "glm_server_stats": [_P, ctypes.c_void_p],
    "glm_server_reset_stats": [_P],
    "glm_server_shutdown": [_P],
    "glm_server_destroy": [_P],
    "glm_transpose": [_P, ctypes.POINTER(glm_dataset_desc), _P, _I64, _P],
    "glm_colset_register": [_P, ctypes.POINTER(glm_colset_desc), ctypes.POINTER(_I64)],
    "glm_colset_unregister": [_P, _I64],
    "glm_linpred": [_P, _I64, _P, _P, _P],
    "glm_diff_logpost": [_P, _I64, _P, _P, _I32, _P, _I32, ctypes.POINTER(glm_prior), _P, _P],
    "glm_diff_commit": [_P, _I64, _P, _P, _I32, _P, _P],
    "glm_mh_run": [_P, _I64, _P, _P, _P, _P, _I32, ctypes.POINTER(glm_prior), _P, _P, _P],
    "glm_hmc_run": [_P, _I64, _P, _P, _I32, _I32, _D, ctypes.c_uint64, ctypes.c_uint64,
                    ctypes.c_uint32, ctypes.POINTER(glm_prior), _P, _P, _P],
    "glm_rng_fill": [_P, _I32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                     ctypes.c_uint64, _I64, _D, _P, _P],
    "glm_logpost_grad_hess": [_P, _I64, _P, ctypes.POINTER(glm_prior), _P, _P, _P],
    "glm_probe_roundtrip": [_P, _I32, _I32, ctypes.POINTER(_D)],
    "glm_probe_read_bandwidth": [_P, _P, _I64, _I32, _I32, ctypes.POINTER(_D)],
    "glm_probe_mfma_f64": [_P, _I32, ctypes.POINTER(_D)],
    "glm_probe_diff_map": [_P, _I64, _I32, _I32, ctypes.POINTER(_D)],
    "glm_quantize_bf16": [_P, _P, _I64, _I32, _I64, _P, _I64, _P],
    "glm_fp8_col_scales": [_P, _P, _I64, _I32, _I64, _P, _P],
    "glm_quantize_fp8": [_P, _P, _I64, _I32, _I64, _P, _P, _I64, _P],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int32
_lib.glm_last_error.argtypes = []
_lib.glm_last_error.restype = ctypes.c_char_p


def lib() -> ctypes.CDLL:
    return _lib


def glm_last_error() -> str:
    return _lib.glm_last_error().decode()


def _check(st: int, allow_pending: bool = False) -> int:
    if st == GLM_OK or (allow_pending and st == GLM_PENDING):
        return st
    raise GlmError(st, glm_last_error())


def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, torch.Tensor):
        return x.data_ptr()
    if hasattr(x, "ctypes") and hasattr(x, "dtype"):   # numpy array: a host pointer
        return x.ctypes.data
    raise TypeError(f"cannot pass {type(x)} as a device pointer")


def _stream(s) -> int | None:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _dtype_code(t: torch.Tensor, dtype: int | None) -> int:
    if dtype is not None:
        return dtype
    return {torch.float64: GLM_F64, torch.float32: GLM_F32, torch.bfloat16: GLM_BF16,
            torch.uint16: GLM_BF16, torch.float8_e4m3fn: GLM_FP8_E4M3,
            torch.uint8: GLM_FP8_E4M3}[t.dtype]


# ---------------------------------------------------------------- context

def glm_create(device: int = 0) -> int:
    out = ctypes.c_void_p()
    _check(_lib.glm_create(device, ctypes.byref(out)))
    return out.value


def glm_destroy(ctx: int) -> None:
    _check(_lib.glm_destroy(ctx))


def glm_set_option(ctx: int, option: int, value: int) -> None:
    _check(_lib.glm_set_option(ctx, option, value))


def glm_get_option(ctx: int, option: int) -> int:
    out = _I64()
    _check(_lib.glm_get_option(ctx, option, ctypes.byref(out)))
    return out.value


# ---------------------------------------------------------------- data sets

def make_desc(X, y, N=None, K=None, ldx=None, dtype=None, col_scale=None,
              family: int = 0) -> glm_dataset_desc:
    """Descriptor for a row-major X (2-D tensor, or address with explicit
    N/K/ldx/dtype) and its uint8 response y."""
    if isinstance(X, torch.Tensor):
        assert X.dim() == 2
        N = X.shape[0] if N is None else N
        K = X.shape[1] if K is None else K
        if X.numel() == 0:
            ldx = K if ldx is None else ldx
        else:
            assert X.stride(1) == 1, "X must be row-major"
            ldx = X.stride(0) if ldx is None else ldx
        dtype = _dtype_code(X, dtype)
    return glm_dataset_desc(_ptr(X), ldx, dtype, _ptr(col_scale), _ptr(y), N, K, family)


def aligned_rows(X):
    """A copy of the 2-D device tensor X whose rows start on 16-byte
    boundaries (leading dimension rounded up, padding zero), returned as the
    N x K view the data-set descriptor takes; X itself when already aligned.
    The caller keeps the returned view alive while the data set is in use."""
    es = X.element_size()
    step = max(1, 16 // es)
    N, K = X.shape
    if X.stride(1) == 1 and (X.stride(0) * es) % 16 == 0 and X.data_ptr() % 16 == 0:
        return X
    ld = (K + step - 1) // step * step
    buf = torch.zeros((N, ld), dtype=X.dtype, device=X.device)
    buf[:, :K] = X
    return buf[:, :K]


def glm_dataset_register(ctx: int, desc: glm_dataset_desc) -> int:
    out = ctypes.c_int64()
    _check(_lib.glm_dataset_register(ctx, ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def glm_dataset_unregister(ctx: int, ds: int) -> None:
    _check(_lib.glm_dataset_unregister(ctx, ds))


def make_prior(prec: float, mean=None, per_group: bool = False) -> glm_prior:
    return glm_prior(prec, _ptr(mean), int(per_group))


# ---------------------------------------------------------------- evaluation

def glm_logpost_grad(ctx: int, ds: int, beta, prior: glm_prior, out, stream=None) -> None:
    _check(_lib.glm_logpost_grad(ctx, ds, _ptr(beta), ctypes.byref(prior), _ptr(out),
                                 _stream(stream)))


def glm_logpost_grad_noalloc(ctx: int, ds: int, beta, prior: glm_prior, out, stream=None) -> None:
    _check(_lib.glm_logpost_grad_noalloc(ctx, ds, _ptr(beta), ctypes.byref(prior), _ptr(out),
                                         _stream(stream)))


def glm_logpost_grad_multi(ctx: int, ds: int, betas, nb: int, prior: glm_prior, out,
                           stream=None) -> None:
    _check(_lib.glm_logpost_grad_multi(ctx, ds, _ptr(betas), nb, ctypes.byref(prior), _ptr(out),
                                       _stream(stream)))


def glm_logpost_grad_host(ctx: int, ds: int, beta_host, prior: glm_prior, g_host=None):
    """beta_host / prior.mean / g_host: numpy float64 arrays (host).  Returns f."""
    import numpy as np
    b = np.ascontiguousarray(beta_host, np.float64)
    f = ctypes.c_double()
    gp = None if g_host is None else g_host.ctypes.data_as(ctypes.c_void_p)
    _check(_lib.glm_logpost_grad_host(ctx, ds, b.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.byref(prior), ctypes.byref(f), gp))
    return f.value


# ---------------------------------------------------------------- differential update

def glm_transpose(ctx: int, desc: glm_dataset_desc, Xt, ldt: int | None = None, stream=None) -> None:
    """Column-major copy of desc's X into the device buffer Xt (K x ldt)."""
    if ldt is None:
        ldt = Xt.stride(0) if isinstance(Xt, torch.Tensor) else desc.N
    _check(_lib.glm_transpose(ctx, ctypes.byref(desc), _ptr(Xt), int(ldt), _stream(stream)))


def make_colset_desc(Xt, y, N=None, dtype=None, col_scale=None,
                     family: int = 0) -> glm_colset_desc:
    """Descriptor of a column-major copy: Xt a K x ldt device tensor whose
    row k is column k of X (first N entries used)."""
    assert Xt.dim() == 2 and Xt.stride(1) == 1
    K = Xt.shape[0]
    N = Xt.shape[1] if N is None else N
    ldt = Xt.stride(0) if Xt.numel() else max(N, 1)
    return glm_colset_desc(_ptr(Xt), ldt, _dtype_code(Xt, dtype), _ptr(col_scale), _ptr(y), N, K,
                           family)


def glm_colset_register(ctx: int, desc: glm_colset_desc) -> int:
    out = ctypes.c_int64()
    _check(_lib.glm_colset_register(ctx, ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def glm_colset_unregister(ctx: int, cs: int) -> None:
    _check(_lib.glm_colset_unregister(ctx, cs))


def glm_linpred(ctx: int, cs: int, beta, u, stream=None) -> None:
    _check(_lib.glm_linpred(ctx, cs, _ptr(beta), _ptr(u), _stream(stream)))


def glm_diff_logpost(ctx: int, cs: int, u, beta, k: int, deltas, nd: int, prior: glm_prior, f_out,
                     stream=None) -> None:
    _check(_lib.glm_diff_logpost(ctx, cs, _ptr(u), _ptr(beta), k, _ptr(deltas), nd,
                                 ctypes.byref(prior), _ptr(f_out), _stream(stream)))


def glm_diff_commit(ctx: int, cs: int, u, beta, k: int, delta, stream=None) -> None:
    _check(_lib.glm_diff_commit(ctx, cs, _ptr(u), _ptr(beta), k, _ptr(delta), _stream(stream)))


# ---------------------------------------------------------------- Hessian

def glm_logpost_grad_hess(ctx: int, ds: int, beta, prior: glm_prior, out, H, stream=None) -> None:
    """f, g (out, 1 + K) and the Hessian H (K x K) at beta; device tensors."""
    _check(_lib.glm_logpost_grad_hess(ctx, ds, _ptr(beta), ctypes.byref(prior), _ptr(out), _ptr(H),
                                      _stream(stream)))


# ---------------------------------------------------------------- on-device sampler

def glm_mh_run(ctx: int, ds: int, beta, fg, incs, logu, n_steps: int, prior: glm_prior,
               accepted=None, f_trace=None, stream=None) -> None:
    """Random-walk Metropolis on the device (all arguments device tensors)."""
    _check(_lib.glm_mh_run(ctx, ds, _ptr(beta), _ptr(fg), _ptr(incs), _ptr(logu), n_steps,
                           ctypes.byref(prior), _ptr(accepted), _ptr(f_trace), _stream(stream)))


def glm_hmc_run(ctx: int, ds: int, beta, fg, n_iter: int, n_leap: int, eps: float, seed: int,
                chain: int, prior: glm_prior, accepted=None, f_trace=None, stream=None,
                iter0: int = 0) -> None:
    """Hamiltonian Monte Carlo on the device (beta, fg, accepted, f_trace:
    device tensors)."""
    _check(_lib.glm_hmc_run(ctx, ds, _ptr(beta), _ptr(fg), n_iter, n_leap, float(eps), int(seed),
                            int(chain), int(iter0), ctypes.byref(prior), _ptr(accepted),
                            _ptr(f_trace), _stream(stream)))


GLM_RNG_UNIFORM, GLM_RNG_NORMAL, GLM_RNG_LOG_UNIFORM = 1, 2, 3


def glm_rng_fill(ctx: int, kind: int, seed: int, chain: int, stream_id: int, offset: int, n: int,
                 out, scale: float = 1.0, stream=None) -> None:
    """Values offset .. offset + n - 1 of a counter-based stream into the
    device tensor out (float64)."""
    _check(_lib.glm_rng_fill(ctx, kind, int(seed), int(chain), int(stream_id), int(offset), n,
                             float(scale), _ptr(out), _stream(stream)))


# ---------------------------------------------------------------- batched

def glm_groupset_create(ctx: int, desc: glm_dataset_desc, offsets, tune: bool = True) -> int:
    """offsets: host sequence of G + 1 row offsets."""
    import numpy as np
    off = np.ascontiguousarray(offsets, np.int64)
    out = ctypes.c_void_p()
    _check(_lib.glm_groupset_create(ctx, ctypes.byref(desc), off.ctypes.data_as(ctypes.c_void_p),
                                    len(off) - 1, int(tune), ctypes.byref(out)))
    return out.value


def glm_groupset_destroy(gs: int) -> None:
    _check(_lib.glm_groupset_destroy(gs))


def glm_groupset_query(gs: int) -> dict:
    info = glm_groupset_info_t()
    _check(_lib.glm_groupset_query(gs, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in info._fields_}


def glm_logpost_grad_batched(ctx: int, gs: int, betas, prior: glm_prior, out, stream=None) -> None:
    _check(_lib.glm_logpost_grad_batched(ctx, gs, _ptr(betas), ctypes.byref(prior), _ptr(out),
                                         _stream(stream)))


# ---------------------------------------------------------------- server

def glm_server_create(ctx: int, hbm_budget_bytes: int, max_beta_per_pass: int = 8,
                      n_streams: int = 4, n_slots: int = 8, queue_capacity: int = 1 << 20,
                      max_sets_per_pass: int = 0) -> int:
    cfg = glm_server_config(hbm_budget_bytes, max_beta_per_pass, n_streams, n_slots,
                            queue_capacity, max_sets_per_pass)
    out = ctypes.c_void_p()
    _check(_lib.glm_server_create(ctx, ctypes.byref(cfg), ctypes.byref(out)))
    return out.value


def make_host_desc(X, y, dtype=None, col_scale=None, family: int = 0) -> glm_dataset_desc:
    """Descriptor with host pointers for numpy X (row-major) and y."""
    import numpy as np
    assert X.ndim == 2 and X.strides[1] == X.itemsize
    if dtype is None:
        dtype = {np.dtype(np.float64): GLM_F64, np.dtype(np.float32): GLM_F32,
                 np.dtype(np.uint16): GLM_BF16, np.dtype(np.uint8): GLM_FP8_E4M3}[X.dtype]
    return glm_dataset_desc(X.ctypes.data, X.strides[0] // X.itemsize, dtype,
                            None if col_scale is None else col_scale.ctypes.data,
                            y.ctypes.data, X.shape[0], X.shape[1], family)


def glm_server_add_dataset(srv: int, desc: glm_dataset_desc, on_device: bool = False) -> int:
    out = ctypes.c_int64()
    _check(_lib.glm_server_add_dataset(srv, ctypes.byref(desc), int(on_device), ctypes.byref(out)))
    return out.value


def glm_server_submit(srv: int, ds: int, beta_host, prec: float, mean_host=None) -> int:
    """Returns the ticket (raises GlmError with GLM_EAGAIN when the queue is full)."""
    import numpy as np
    b = np.ascontiguousarray(beta_host, np.float64)
    m = None if mean_host is None else np.ascontiguousarray(mean_host, np.float64)
    t = ctypes.c_uint64()
    _check(_lib.glm_server_submit(srv, ds, b.ctypes.data_as(ctypes.c_void_p), float(prec),
                                  None if m is None else m.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.byref(t)))
    return t.value


def glm_server_submit_many(srv: int, ds_ids, beta_ptrs, precs):
    """ds_ids: int64 array, beta_ptrs: uint64 array of host addresses of
    float64 K-vectors (kept alive by the caller), precs: float64 array.
    Returns the uint64 ticket array."""
    import numpy as np
    ds_ids = np.ascontiguousarray(ds_ids, np.int64)
    beta_ptrs = np.ascontiguousarray(beta_ptrs, np.uint64)
    precs = np.ascontiguousarray(precs, np.float64)
    n = len(ds_ids)
    t = np.empty(n, np.uint64)
    _check(_lib.glm_server_submit_many(srv, n, ds_ids.ctypes.data, beta_ptrs.ctypes.data,
                                       precs.ctypes.data, t.ctypes.data))
    return t


def glm_server_wait_many(srv: int, tickets, f_out=None) -> int:
    """Waits for and retires the tickets; returns the status (errors are not
    raised so that every ticket is retired)."""
    import numpy as np
    tickets = np.ascontiguousarray(tickets, np.uint64)
    return _lib.glm_server_wait_many(srv, len(tickets), tickets.ctypes.data,
                                     None if f_out is None else f_out.ctypes.data)


def glm_server_poll(srv: int, ticket: int, g_host=None):
    """Returns (status, f); status GLM_OK or GLM_PENDING (others raise)."""
    f = ctypes.c_double()
    gp = None if g_host is None else g_host.ctypes.data_as(ctypes.c_void_p)
    st = _check(_lib.glm_server_poll(srv, ticket, ctypes.byref(f), gp), allow_pending=True)
    return st, f.value


def glm_server_wait(srv: int, ticket: int, g_host=None) -> float:
    f = ctypes.c_double()
    gp = None if g_host is None else g_host.ctypes.data_as(ctypes.c_void_p)
    _check(_lib.glm_server_wait(srv, ticket, ctypes.byref(f), gp))
    return f.value


def glm_server_stats(srv: int) -> dict:
    st = glm_server_stats_t()
    _check(_lib.glm_server_stats(srv, ctypes.byref(st)))
    d = {f: getattr(st, f) for f, _ in st._fields_}
    d["pass_width_hist"] = list(st.pass_width_hist)
    return d


def glm_server_reset_stats(srv: int) -> None:
    _check(_lib.glm_server_reset_stats(srv))


def glm_server_shutdown(srv: int) -> None:
    _check(_lib.glm_server_shutdown(srv))


def glm_server_destroy(srv: int) -> None:
    _check(_lib.glm_server_destroy(srv))


def glm_probe_roundtrip(ctx: int, K: int, iters: int = 1000) -> float:
    us = ctypes.c_double()
    _check(_lib.glm_probe_roundtrip(ctx, K, iters, ctypes.byref(us)))
    return us.value


# ---------------------------------------------------------------- conversions

def glm_probe_read_bandwidth(ctx: int, buf, nbytes: int | None = None, blocks_per_cu: int = 2,
                             iters: int = 10) -> float:
    """GB/s of a plain streaming read of a device buffer (a torch tensor or
    a device address with nbytes)."""
    if nbytes is None:
        nbytes = buf.numel() * buf.element_size()
    gb = ctypes.c_double()
    _check(_lib.glm_probe_read_bandwidth(ctx, _ptr(buf), int(nbytes), blocks_per_cu, iters,
                                         ctypes.byref(gb)))
    return gb.value


def glm_probe_mfma_f64(ctx: int, iters: int = 2000) -> float:
    """TFLOP/s of back-to-back FP64 16x16x4 matrix instructions."""
    tf = ctypes.c_double()
    _check(_lib.glm_probe_mfma_f64(ctx, iters, ctypes.byref(tf)))
    return tf.value


def glm_probe_diff_map(ctx: int, n: int, family: int = 0, iters: int = 20) -> float:
    """Microseconds per launch of the differential update's per-row terms
    alone over n synthetic rows (no memory traffic)."""
    us = ctypes.c_double()
    _check(_lib.glm_probe_diff_map(ctx, n, family, iters, ctypes.byref(us)))
    return us.value


def glm_quantize_bf16(ctx: int, X, Q, stream=None) -> None:
    N, K = X.shape
    _check(_lib.glm_quantize_bf16(ctx, _ptr(X), N, K, X.stride(0), _ptr(Q), Q.stride(0),
                                  _stream(stream)))


def glm_fp8_col_scales(ctx: int, X, scale, stream=None) -> None:
    N, K = X.shape
    _check(_lib.glm_fp8_col_scales(ctx, _ptr(X), N, K, X.stride(0), _ptr(scale),
                                   _stream(stream)))


def glm_quantize_fp8(ctx: int, X, scale, Q, stream=None) -> None:
    N, K = X.shape
    _check(_lib.glm_quantize_fp8(ctx, _ptr(X), N, K, X.stride(0), _ptr(scale), _ptr(Q),
                                 Q.stride(0), _stream(stream)))


def exported_symbols() -> list[str]:
    return sorted(_SIGS) + ["glm_last_error"]

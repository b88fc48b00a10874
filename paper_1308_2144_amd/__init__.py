"""Python binding of libhb, the MI355X HyperBall library.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libhb.so``.  The module-level ``hb_*`` functions mirror the C ABI
declared in ``include/hb.h`` one to one; :class:`HyperBall` is a small
convenience wrapper over them.

Arrays: host inputs are numpy arrays (copied by the library); device inputs
are torch CUDA tensors, whose memory the library borrows until ``hb_free``
(the wrapper keeps references so they stay alive).  PyTorch is used only for
device memory and streams.

Importing this module raises if ``libhb.so`` has not been built: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# HB_LIB may point at another build of the same library (tuning experiments).
LIB_PATH = os.environ.get("HB_LIB") or os.path.join(_HERE, "libhb.so")

HB_OK, HB_EINVAL, HB_ENOMEM, HB_EDEVICE, HB_ESTATE = 0, -1, -2, -3, -4
_STATUS = {HB_EINVAL: "HB_EINVAL", HB_ENOMEM: "HB_ENOMEM", HB_EDEVICE: "HB_EDEVICE",
           HB_ESTATE: "HB_ESTATE"}


class HBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class hb_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("offsets", ctypes.c_void_p),
                ("offsets_bits", ctypes.c_int32), ("indices", ctypes.c_void_p),
                ("on_device", ctypes.c_int32)]


class hb_options(ctypes.Structure):
    _fields_ = [("frontier", ctypes.c_int32), ("light_max", ctypes.c_int32),
                ("heavy_min", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("dense_pct", ctypes.c_int32), ("push", ctypes.c_int32),
                ("sparse_pct", ctypes.c_int32), ("qdense", ctypes.c_int32),
                ("slice", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32),
                ("graph_passes", ctypes.c_int32), ("neighbourhood", ctypes.c_int32),
                ("pairs", ctypes.c_int32), ("stream_graph", ctypes.c_int32),
                ("graph_budget", ctypes.c_int64), ("stream_compress", ctypes.c_int32)]


class hb_stats_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("log2m", ctypes.c_int32),
                ("passes", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("last_modified", ctypes.c_int64), ("heavy_rows", ctypes.c_int64),
                ("heavy_chunks", ctypes.c_int64), ("medium_rows", ctypes.c_int64),
                ("light_rows", ctypes.c_int64), ("reverse_built", ctypes.c_int32),
                ("total_kernel_ms", ctypes.c_double), ("streamed", ctypes.c_int32),
                ("chunks", ctypes.c_int32), ("chunk_bytes", ctypes.c_int64),
                ("host_graph_bytes", ctypes.c_int64), ("compressed", ctypes.c_int32)]


class hb_pass_info(ctypes.Structure):
    _fields_ = [("arcs_scanned", ctypes.c_int64), ("counters_gathered", ctypes.c_int64),
                ("slices_gathered", ctypes.c_int64), ("rows_loaded", ctypes.c_int64),
                ("rows_written", ctypes.c_int64), ("rows_changed", ctypes.c_int64),
                ("slices_changed", ctypes.c_int64), ("arcs_to_changed", ctypes.c_int64),
                ("mode", ctypes.c_int32),
                ("push_ms", ctypes.c_double), ("expand_ms", ctypes.c_double),
                ("merge_ms", ctypes.c_double), ("path", ctypes.c_int32),
                ("host_bytes", ctypes.c_int64), ("chunks_run", ctypes.c_int32)]


class hb_graph_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("packed_offset", ctypes.c_int64), ("passes", ctypes.c_int32),
                ("converged", ctypes.c_int32)]


class hb_serve_config(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("max_nodes", ctypes.c_int64), ("max_arcs", ctypes.c_int64),
                ("max_resident", ctypes.c_int32), ("passes_per_tick", ctypes.c_int32),
                ("start_paused", ctypes.c_int32), ("opt", hb_options)]


class hb_serve_request(ctypes.Structure):
    _fields_ = [("graph", hb_csr), ("log2m", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("closeness", ctypes.c_void_p), ("lin", ctypes.c_void_p), ("harmonic", ctypes.c_void_p),
                ("coreach", ctypes.c_void_p), ("S", ctypes.c_void_p), ("H", ctypes.c_void_p),
                ("registers", ctypes.c_void_p)]


class hb_request_info(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("state", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class hb_serve_stats_t(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "admitted", "completed", "cancelled", "failed",
                                             "queued", "resident", "resident_bytes", "peak_resident_bytes",
                                             "ticks", "engine_passes")] + \
               [("busy_s", ctypes.c_double), ("elapsed_s", ctypes.c_double)]


class hb_tune_report(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int32), ("from_cache", ctypes.c_int32), ("sample_graphs", ctypes.c_int32),
                ("start_ms", ctypes.c_double), ("best_ms", ctypes.c_double), ("tune_s", ctypes.c_double)]


class hb_distance_stats_t(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_double), ("average_distance", ctypes.c_double),
                ("effective_diameter", ctypes.c_double)]


HB_REQ_QUEUED, HB_REQ_RUNNING, HB_REQ_DONE, HB_REQ_CANCELLED, HB_REQ_FAILED = range(5)
REQ_STATES = ("queued", "running", "done", "cancelled", "failed")


def _declare(L):
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    P = ctypes.POINTER
    sig = {
        "hb_default_options": (None, [P(hb_options)]),
        "hb_init": (ctypes.c_int, [P(vp), P(hb_csr), i32, u64, P(hb_options), vp]),
        "hb_reset": (ctypes.c_int, [vp, u64]),
        "hb_iterate": (ctypes.c_int, [vp, P(i64)]),
        "hb_run": (ctypes.c_int, [vp, i32, P(i32)]),
        "hb_centralities": (ctypes.c_int, [vp, vp, vp, vp, vp, i32]),
        "hb_get_registers": (ctypes.c_int, [vp, vp, i32]),
        "hb_get_accumulators": (ctypes.c_int, [vp, vp, vp, i32]),
        "hb_stats": (ctypes.c_int, [vp, P(hb_stats_t)]),
        "hb_pass_stats": (ctypes.c_int, [vp, i32, P(hb_pass_info)]),
        "hb_free": (None, [vp]),
        "hb_last_error": (ctypes.c_char_p, []),
        "hb_version": (i32, []),
        "hb_batch_init": (ctypes.c_int, [P(vp), vp, i32, i32, vp, P(hb_options), vp]),
        "hb_batch_reset": (ctypes.c_int, [vp, vp]),
        "hb_batch_graph": (ctypes.c_int, [vp, i32, P(hb_graph_info)]),
        "hb_batch_passes": (ctypes.c_int, [vp, vp]),
        "hb_set_weights": (ctypes.c_int, [vp, vp, i32]),
        "hb_set_discount": (ctypes.c_int, [vp, vp, i32]),
        "hb_get_discounted": (ctypes.c_int, [vp, vp, i32]),
        "hb_neighbourhood": (ctypes.c_int, [vp, vp, i32, P(i32)]),
        "hb_distance_stats": (ctypes.c_int, [vp, i32, ctypes.c_double, P(hb_distance_stats_t)]),
        "hb_discount_table": (ctypes.c_int, [i32, i32, vp]),
        "hb_run_static": (ctypes.c_int, [P(hb_csr), i32, ctypes.c_uint64, vp, vp, vp, vp, vp, P(i32), vp]),
        "hb_ensemble_init": (ctypes.c_int, [P(vp), P(hb_csr), i32, vp, i32, P(hb_options), vp]),
        "hb_ensemble_reset": (ctypes.c_int, [vp, vp]),
        "hb_ensemble_passes": (ctypes.c_int, [vp, vp]),
        "hb_ensemble_summary": (ctypes.c_int, [vp, i32, vp, vp, i32]),
        "hb_batch_autotune": (ctypes.c_int, [vp, i32, i32, vp, i32, ctypes.c_char_p, P(hb_options),
                                             P(hb_tune_report)]),
        "hb_serve_default_config": (None, [P(hb_serve_config)]),
        "hb_serve_start": (ctypes.c_int, [P(vp), P(hb_serve_config)]),
        "hb_serve_resume": (ctypes.c_int, [vp]),
        "hb_serve_submit": (ctypes.c_int, [vp, P(hb_serve_request), P(i64)]),
        "hb_serve_poll": (ctypes.c_int, [vp, i64, P(hb_request_info)]),
        "hb_serve_wait": (ctypes.c_int, [vp, i64, ctypes.c_double, P(hb_request_info)]),
        "hb_serve_cancel": (ctypes.c_int, [vp, i64]),
        "hb_serve_stats": (ctypes.c_int, [vp, P(hb_serve_stats_t)]),
        "hb_serve_stop": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


_lib = None


def lib():
    """The loaded libhb.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: PyTorch ships its own libamdhip64 and
        # libhsa-runtime64 (same sonames as the system ROCm ones).  Loading
        # torch first makes libhb bind to that runtime instead of pulling in a
        # second copy, which would leave torch without a visible GPU.
        import torch  # noqa: F401

        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


lib()


def _check(st: int):
    if st != HB_OK:
        raise HBError(st, lib().hb_last_error().decode(errors="replace"))


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def default_options(**kw) -> hb_options:
    o = hb_options()
    lib().hb_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, int(v))
    return o


# --- one-to-one wrappers of the C ABI ------------------------------------------

def _csr(offsets, indices):
    """hb_csr for numpy (host, copied by the library) or torch CUDA (device,
    borrowed) arrays, and the arrays to keep alive."""
    dev = _is_torch(offsets)
    if dev != _is_torch(indices):
        raise TypeError("offsets and indices must both be numpy arrays or both torch tensors")
    if dev:
        import torch

        if offsets.dtype not in (torch.int32, torch.int64) or indices.dtype != torch.int32:
            raise TypeError("offsets must be int32/int64 and indices int32")
        if not (offsets.is_cuda and indices.is_cuda and offsets.is_contiguous() and indices.is_contiguous()):
            raise TypeError("device inputs must be contiguous CUDA tensors")
        n = offsets.numel() - 1
        bits = 64 if offsets.dtype == torch.int64 else 32
        g = hb_csr(n, indices.numel(), offsets.data_ptr(), bits,
                   indices.data_ptr() if indices.numel() else None, 1)
    else:
        offsets = np.ascontiguousarray(offsets)
        indices = np.ascontiguousarray(indices, dtype=np.int32)
        if offsets.dtype not in (np.int32, np.int64):
            offsets = offsets.astype(np.int64)
        n = offsets.shape[0] - 1
        bits = 64 if offsets.dtype == np.int64 else 32
        g = hb_csr(n, indices.shape[0], offsets.ctypes.data, bits,
                   indices.ctypes.data if indices.size else None, 0)
    return g, (offsets, indices)


def hb_init(offsets, indices, log2m: int, seed: int, options: hb_options | None = None,
            stream=None):
    """Returns (ctx handle, keepalive tuple).  offsets: int32/int64; indices int32.

    numpy inputs are host memory (copied); torch CUDA tensors are borrowed."""
    g, keep = _csr(offsets, indices)
    ctx = ctypes.c_void_p()
    opt = ctypes.byref(options) if options is not None else None
    _check(lib().hb_init(ctypes.byref(ctx), ctypes.byref(g), int(log2m), int(seed), opt,
                         ctypes.c_void_p(stream) if stream else None))
    return ctx, keep


def hb_set_weights(ctx, weights):
    """weights: n int32 >= 1 (numpy host array or torch CUDA tensor), or None."""
    if weights is None:
        _check(lib().hb_set_weights(ctx, None, 0))
        return None
    if _is_torch(weights):
        _check(lib().hb_set_weights(ctx, weights.data_ptr(), 1))
        return weights
    w = np.ascontiguousarray(weights, dtype=np.int32)
    _check(lib().hb_set_weights(ctx, w.ctypes.data, 0))
    return w


def hb_set_discount(ctx, table):
    if table is None or len(table) == 0:
        _check(lib().hb_set_discount(ctx, None, 0))
        return
    f = np.ascontiguousarray(table, dtype=np.float64)
    _check(lib().hb_set_discount(ctx, f.ctypes.data, f.shape[0]))


def hb_get_discounted(ctx, D, dst_on_device: bool):
    _check(lib().hb_get_discounted(ctx, _ptr(D), int(bool(dst_on_device))))


def hb_neighbourhood(ctx) -> np.ndarray:
    ln = ctypes.c_int32(0)
    _check(lib().hb_neighbourhood(ctx, None, 0, ctypes.byref(ln)))
    out = np.empty(max(ln.value, 1))
    _check(lib().hb_neighbourhood(ctx, out.ctypes.data, ln.value, ctypes.byref(ln)))
    return out[: ln.value]


def hb_distance_stats(N, alpha: float = 0.9) -> dict:
    a = np.ascontiguousarray(N, dtype=np.float64)
    st = hb_distance_stats_t()
    _check(lib().hb_distance_stats(a.ctypes.data, a.shape[0], float(alpha), ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in hb_distance_stats_t._fields_}


def hb_run_static(offsets, indices, log2m: int, seed: int, closeness=None, lin=None, harmonic=None,
                  coreach=None, registers=None, stream=None) -> int:
    """hb_run_static: device CSR (torch tensors) in, results into the given
    device tensors (each may be None); returns the pass count."""
    if not (_is_torch(offsets) and offsets.is_cuda and _is_torch(indices) and indices.is_cuda):
        raise TypeError("hb_run_static takes a device CSR (CUDA tensors)")
    g, keep = _csr(offsets, indices)
    passes = ctypes.c_int32(0)
    ptr = [None if a is None else ctypes.c_void_p(a.data_ptr()) for a in (closeness, lin, harmonic, coreach,
                                                                          registers)]
    _check(lib().hb_run_static(ctypes.byref(g), int(log2m), int(seed), *ptr, ctypes.byref(passes),
                               ctypes.c_void_p(stream) if stream else None))
    del keep
    return passes.value


DISCOUNTS = {"harmonic": 0, "quadratic": 1, "logarithmic": 2, "constant": 3}


def discount_table(kind: str, length: int = 64) -> np.ndarray:
    """f(1..length) of a discount Sec. 7 names ("harmonic", "quadratic",
    "logarithmic", "constant"), computed by hb_discount_table."""
    if kind not in DISCOUNTS:
        raise ValueError(f"unknown discount {kind}")
    f = np.empty(int(length), dtype=np.float64)
    _check(lib().hb_discount_table(DISCOUNTS[kind], int(length), f.ctypes.data))
    return f


def hb_ensemble_init(offsets, indices, log2m: int, seeds, options: hb_options | None = None, stream=None):
    g, keep = _csr(offsets, indices)
    sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    ctx = ctypes.c_void_p()
    opt = ctypes.byref(options) if options is not None else None
    _check(lib().hb_ensemble_init(ctypes.byref(ctx), ctypes.byref(g), int(log2m), sd.ctypes.data, sd.shape[0], opt,
                                  ctypes.c_void_p(stream) if stream else None))
    return ctx, keep + (sd,)


def hb_ensemble_reset(ctx, seeds=None):
    sd = None if seeds is None else np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    _check(lib().hb_ensemble_reset(ctx, None if sd is None else sd.ctypes.data))


def hb_ensemble_passes(ctx, k: int) -> np.ndarray:
    out = np.empty(k, dtype=np.int32)
    _check(lib().hb_ensemble_passes(ctx, out.ctypes.data))
    return out


CENTRALITY_INDEX = {"closeness": 0, "lin": 1, "harmonic": 2, "coreach": 3}


def hb_ensemble_summary(ctx, which, mean, sd, dst_on_device: bool):
    w = CENTRALITY_INDEX[which] if isinstance(which, str) else int(which)
    _check(lib().hb_ensemble_summary(ctx, w, _ptr(mean), _ptr(sd), int(bool(dst_on_device))))


def hb_reset(ctx, seed: int):
    _check(lib().hb_reset(ctx, int(seed)))


def hb_iterate(ctx) -> int:
    nmod = ctypes.c_int64(0)
    _check(lib().hb_iterate(ctx, ctypes.byref(nmod)))
    return nmod.value


def hb_run(ctx, max_passes: int = 0) -> int:
    passes = ctypes.c_int32(0)
    _check(lib().hb_run(ctx, int(max_passes), ctypes.byref(passes)))
    return passes.value


def _ptr(a):
    if a is None:
        return None
    return a.data_ptr() if _is_torch(a) else a.ctypes.data


def hb_centralities(ctx, closeness, lin, harmonic, coreach, dst_on_device: bool):
    _check(lib().hb_centralities(ctx, _ptr(closeness), _ptr(lin), _ptr(harmonic), _ptr(coreach),
                                 int(dst_on_device)))


def hb_get_registers(ctx, dst, dst_on_device: bool):
    _check(lib().hb_get_registers(ctx, _ptr(dst), int(dst_on_device)))


def hb_get_accumulators(ctx, S, H, dst_on_device: bool):
    _check(lib().hb_get_accumulators(ctx, _ptr(S), _ptr(H), int(dst_on_device)))


def hb_stats(ctx) -> dict:
    s = hb_stats_t()
    _check(lib().hb_stats(ctx, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in hb_stats_t._fields_}


def hb_pass_stats(ctx, t: int) -> dict:
    s = hb_pass_info()
    _check(lib().hb_pass_stats(ctx, int(t), ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in hb_pass_info._fields_}


def hb_free(ctx):
    lib().hb_free(ctx)


def hb_version() -> int:
    return lib().hb_version()


def hb_batch_init(graphs, log2m: int, seeds, options: hb_options | None = None, stream=None):
    """graphs: list of (offsets, indices) numpy CSRs.  Returns (ctx, keepalive)."""
    k = len(graphs)
    arr = (hb_csr * k)()
    keep = []
    for i, (o, x) in enumerate(graphs):
        o = np.ascontiguousarray(o)
        if o.dtype not in (np.int32, np.int64):
            o = o.astype(np.int64)
        x = np.ascontiguousarray(x, dtype=np.int32)
        keep.append((o, x))
        arr[i] = hb_csr(o.shape[0] - 1, x.shape[0], o.ctypes.data, 64 if o.dtype == np.int64 else 32,
                        x.ctypes.data if x.size else None, 0)
    sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    if sd.shape[0] != k:
        raise ValueError("need one seed per graph")
    ctx = ctypes.c_void_p()
    opt = ctypes.byref(options) if options is not None else None
    _check(lib().hb_batch_init(ctypes.byref(ctx), ctypes.cast(arr, ctypes.c_void_p), k, int(log2m),
                               sd.ctypes.data, opt, ctypes.c_void_p(stream) if stream else None))
    return ctx, (arr, keep, sd)


def hb_batch_reset(ctx, seeds=None):
    sd = None if seeds is None else np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    _check(lib().hb_batch_reset(ctx, None if sd is None else sd.ctypes.data))


def hb_batch_graph(ctx, g: int) -> dict:
    info = hb_graph_info()
    _check(lib().hb_batch_graph(ctx, int(g), ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in hb_graph_info._fields_}


def hb_batch_passes(ctx, k: int) -> np.ndarray:
    out = np.empty(k, dtype=np.int32)
    _check(lib().hb_batch_passes(ctx, out.ctypes.data))
    return out


def _csr_array(graphs):
    k = len(graphs)
    arr = (hb_csr * k)()
    keep = []
    for i, (o, x) in enumerate(graphs):
        o = np.ascontiguousarray(o)
        if o.dtype not in (np.int32, np.int64):
            o = o.astype(np.int64)
        x = np.ascontiguousarray(x, dtype=np.int32)
        keep.append((o, x))
        arr[i] = hb_csr(o.shape[0] - 1, x.shape[0], o.ctypes.data, 64 if o.dtype == np.int64 else 32,
                        x.ctypes.data if x.size else None, 0)
    return arr, keep


def hb_batch_autotune(graphs, log2m: int, seeds, sample: int = 0, cache_path: str | None = None,
                      options: hb_options | None = None):
    """Returns (tuned hb_options, report dict)."""
    arr, keep = _csr_array(graphs)
    sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    if sd.shape[0] != len(graphs):
        raise ValueError("need one seed per graph")
    opt = options if options is not None else default_options()
    rep = hb_tune_report()
    _check(lib().hb_batch_autotune(ctypes.cast(arr, ctypes.c_void_p), len(graphs), int(log2m), sd.ctypes.data,
                                   int(sample), cache_path.encode() if cache_path else None, ctypes.byref(opt),
                                   ctypes.byref(rep)))
    return opt, {k: getattr(rep, k) for k, _ in hb_tune_report._fields_}


def options_dict(o: hb_options) -> dict:
    return {k: getattr(o, k) for k, _ in hb_options._fields_}


def hb_serve_default_config() -> hb_serve_config:
    cfg = hb_serve_config()
    lib().hb_serve_default_config(ctypes.byref(cfg))
    return cfg


def hb_serve_start(cfg: hb_serve_config | None = None):
    srv = ctypes.c_void_p()
    _check(lib().hb_serve_start(ctypes.byref(srv), ctypes.byref(cfg) if cfg is not None else None))
    return srv


def hb_serve_resume(srv):
    _check(lib().hb_serve_resume(srv))


def hb_serve_submit(srv, rq: hb_serve_request) -> int:
    rid = ctypes.c_int64()
    _check(lib().hb_serve_submit(srv, ctypes.byref(rq), ctypes.byref(rid)))
    return rid.value


def _info(info: hb_request_info) -> dict:
    d = {k: getattr(info, k) for k, _ in hb_request_info._fields_}
    d["state_name"] = REQ_STATES[d["state"]] if 0 <= d["state"] < len(REQ_STATES) else str(d["state"])
    return d


def hb_serve_poll(srv, rid: int) -> dict:
    info = hb_request_info()
    _check(lib().hb_serve_poll(srv, int(rid), ctypes.byref(info)))
    return _info(info)


def hb_serve_wait(srv, rid: int, timeout_s: float = -1.0) -> dict:
    info = hb_request_info()
    _check(lib().hb_serve_wait(srv, int(rid), float(timeout_s), ctypes.byref(info)))
    return _info(info)


def hb_serve_cancel(srv, rid: int):
    _check(lib().hb_serve_cancel(srv, int(rid)))


def hb_serve_stats(srv) -> dict:
    st = hb_serve_stats_t()
    _check(lib().hb_serve_stats(srv, ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in hb_serve_stats_t._fields_}


def hb_serve_stop(srv):
    _check(lib().hb_serve_stop(srv))


# --- convenience wrappers -------------------------------------------------------

class HyperBall:
    """One HyperBall computation on one graph (see include/hb.h)."""

    def __init__(self, offsets, indices, log2m: int, seed: int, *, stream=None, **options):
        self.log2m = int(log2m)
        self.p = 1 << self.log2m
        opt = default_options(**options)
        self._ctx, self._keep = hb_init(offsets, indices, log2m, seed, opt, stream)
        self.n = (offsets.numel() if _is_torch(offsets) else len(offsets)) - 1

    def close(self):
        if self._ctx is not None:
            hb_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def reset(self, seed: int):
        hb_reset(self._ctx, seed)

    def iterate(self) -> int:
        return hb_iterate(self._ctx)

    def run(self, max_passes: int = 0) -> int:
        return hb_run(self._ctx, max_passes)

    def registers(self) -> np.ndarray:
        out = np.empty((max(self.n, 1), self.p), dtype=np.uint8)
        hb_get_registers(self._ctx, out, False)
        return out[: self.n]

    def accumulators(self):
        S = np.empty(max(self.n, 1))
        H = np.empty(max(self.n, 1))
        hb_get_accumulators(self._ctx, S, H, False)
        return S[: self.n], H[: self.n]

    def centralities(self, device: bool = False):
        if device:
            import torch

            outs = [torch.empty(max(self.n, 1), dtype=torch.float64, device="cuda") for _ in range(4)]
            hb_centralities(self._ctx, *outs, True)
            outs = [o[: self.n] for o in outs]
        else:
            outs = [np.empty(max(self.n, 1)) for _ in range(4)]
            hb_centralities(self._ctx, *outs, False)
            outs = [o[: self.n] for o in outs]
        return dict(zip(("closeness", "lin", "harmonic", "coreach"), outs))

    def stats(self) -> dict:
        return hb_stats(self._ctx)

    def pass_stats(self, t: int) -> dict:
        return hb_pass_stats(self._ctx, t)

    def set_weights(self, weights):
        self._weights = hb_set_weights(self._ctx, weights)

    def set_discount(self, table):
        hb_set_discount(self._ctx, table)

    def discounted(self) -> np.ndarray:
        D = np.empty(max(self.n, 1))
        hb_get_discounted(self._ctx, D, False)
        return D[: self.n]

    def neighbourhood(self) -> np.ndarray:
        return hb_neighbourhood(self._ctx)


class Batch:
    """Many graphs in one batched context (see hb_batch_init in include/hb.h).
    Packed outputs are split per graph with split()."""

    def __init__(self, graphs, log2m: int, seeds, *, stream=None, options: hb_options | None = None, **kw):
        self.log2m = int(log2m)
        self.p = 1 << self.log2m
        self.k = len(graphs)
        self.sizes = np.array([len(o) - 1 for o, _ in graphs], dtype=np.int64)
        self.bounds = np.concatenate([[0], np.cumsum(self.sizes)])
        self.total = int(self.bounds[-1])
        opt = options if options is not None else default_options(**kw)
        self._ctx, self._keep = hb_batch_init(graphs, log2m, seeds, opt, stream)

    def close(self):
        if self._ctx is not None:
            hb_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def split(self, packed):
        return [packed[self.bounds[i]:self.bounds[i + 1]] for i in range(self.k)]

    def run(self, max_passes: int = 0) -> int:
        return hb_run(self._ctx, max_passes)

    def iterate(self) -> int:
        return hb_iterate(self._ctx)

    def reset(self, seeds=None):
        hb_batch_reset(self._ctx, seeds)

    def passes(self) -> np.ndarray:
        return hb_batch_passes(self._ctx, self.k)

    def graph(self, g: int) -> dict:
        return hb_batch_graph(self._ctx, g)

    def registers(self) -> np.ndarray:
        out = np.empty((max(self.total, 1), self.p), dtype=np.uint8)
        hb_get_registers(self._ctx, out, False)
        return out[: self.total]

    def accumulators(self):
        S = np.empty(max(self.total, 1))
        H = np.empty(max(self.total, 1))
        hb_get_accumulators(self._ctx, S, H, False)
        return S[: self.total], H[: self.total]

    def centralities(self):
        outs = [np.empty(max(self.total, 1)) for _ in range(4)]
        hb_centralities(self._ctx, *outs, False)
        return dict(zip(("closeness", "lin", "harmonic", "coreach"), (o[: self.total] for o in outs)))

    def stats(self) -> dict:
        return hb_stats(self._ctx)


class Request:
    """A submitted serving request: its id and the host arrays the server
    borrows until the request reaches a final state (``outputs`` holds the
    results once ``Server.wait`` returned "done")."""

    def __init__(self, rid: int, n: int, log2m: int, outputs: dict, keep):
        self.id = rid
        self.n = n
        self.log2m = log2m
        self.outputs = outputs
        self._keep = keep
        self.info = None


class Server:
    """The serving loop (see hb_serve_start in include/hb.h)."""

    OUTPUTS = ("closeness", "lin", "harmonic", "coreach", "S", "H")

    def __init__(self, budget_bytes: int = 0, max_nodes: int = 0, max_arcs: int = 0, max_resident: int = 0,
                 passes_per_tick: int = 0, start_paused: bool = False, **options):
        cfg = hb_serve_default_config()
        for k, v in (("budget_bytes", budget_bytes), ("max_nodes", max_nodes), ("max_arcs", max_arcs),
                     ("max_resident", max_resident), ("passes_per_tick", passes_per_tick),
                     ("start_paused", int(start_paused))):
            if v:
                setattr(cfg, k, int(v))
        cfg.opt = default_options(**options)
        self._srv = hb_serve_start(cfg)
        self._live = {}

    def submit(self, offsets, indices, log2m: int, seed: int, *, outputs=OUTPUTS, registers: bool = False,
               out: dict | None = None) -> Request:
        """Host CSR in, Request out.  `out` may supply preallocated host
        arrays (e.g. pinned) by output name; missing ones are allocated."""
        o = np.ascontiguousarray(offsets)
        if o.dtype not in (np.int32, np.int64):
            o = o.astype(np.int64)
        x = np.ascontiguousarray(indices, dtype=np.int32)
        n = o.shape[0] - 1
        p = 1 << int(log2m)
        bufs = dict(out or {})
        for k in outputs:
            if k not in bufs:
                bufs[k] = np.empty(max(n, 1))
        if registers and "registers" not in bufs:
            bufs["registers"] = np.empty((max(n, 1), p), dtype=np.uint8)
        rq = hb_serve_request()
        rq.graph = hb_csr(n, x.shape[0], o.ctypes.data, 64 if o.dtype == np.int64 else 32,
                          x.ctypes.data if x.size else None, 0)
        rq.log2m = int(log2m)
        rq.seed = int(seed)
        for k, a in bufs.items():
            setattr(rq, k, _ptr(a))
        rid = hb_serve_submit(self._srv, rq)
        req = Request(rid, n, int(log2m), bufs, (o, x, rq))
        self._live[rid] = req
        return req

    def _final(self, req: Request, info: dict) -> dict:
        req.info = info
        if info["state"] >= HB_REQ_DONE:
            self._live.pop(req.id, None)
            if info["state"] == HB_REQ_DONE:
                for k, a in list(req.outputs.items()):
                    req.outputs[k] = a[: req.n]
        return info

    def wait(self, req: Request, timeout_s: float = -1.0) -> dict:
        try:
            info = hb_serve_wait(self._srv, req.id, timeout_s)
        except HBError as e:
            if e.status == HB_EDEVICE:
                self._live.pop(req.id, None)
            raise
        return self._final(req, info)

    def poll(self, req: Request) -> dict:
        return self._final(req, hb_serve_poll(self._srv, req.id))

    def cancel(self, req: Request):
        hb_serve_cancel(self._srv, req.id)

    def resume(self):
        hb_serve_resume(self._srv)

    def stats(self) -> dict:
        return hb_serve_stats(self._srv)

    def stop(self):
        if self._srv is not None:
            srv, self._srv = self._srv, None
            try:
                hb_serve_stop(srv)
            finally:
                self._live.clear()

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()


class Ensemble:
    """k HyperBall runs with different hash seeds on one graph in one context
    (see hb_ensemble_init in include/hb.h).  Per-run outputs have shape
    (n, k); summary() gives the per-node mean and empirical standard
    deviation over the runs."""

    def __init__(self, offsets, indices, log2m: int, seeds, *, stream=None, **options):
        self.log2m = int(log2m)
        self.p = 1 << self.log2m
        self.k = len(seeds)
        opt = default_options(**options)
        self._ctx, self._keep = hb_ensemble_init(offsets, indices, log2m, seeds, opt, stream)
        self.n = (offsets.numel() if _is_torch(offsets) else len(offsets)) - 1

    def close(self):
        if self._ctx is not None:
            hb_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def run(self, max_passes: int = 0) -> int:
        return hb_run(self._ctx, max_passes)

    def iterate(self) -> int:
        return hb_iterate(self._ctx)

    def reset(self, seeds=None):
        hb_ensemble_reset(self._ctx, seeds)

    def passes(self) -> np.ndarray:
        return hb_ensemble_passes(self._ctx, self.k)

    def registers(self) -> np.ndarray:
        """(n, k, p) bytes: run i's counter of node v at [v, i]."""
        out = np.empty((max(self.n, 1), self.k, self.p), dtype=np.uint8)
        hb_get_registers(self._ctx, out, False)
        return out[: self.n]

    def accumulators(self):
        S = np.empty((max(self.n, 1), self.k))
        H = np.empty((max(self.n, 1), self.k))
        hb_get_accumulators(self._ctx, S, H, False)
        return S[: self.n], H[: self.n]

    def centralities(self):
        outs = [np.empty((max(self.n, 1), self.k)) for _ in range(4)]
        hb_centralities(self._ctx, *outs, False)
        return dict(zip(("closeness", "lin", "harmonic", "coreach"), (o[: self.n] for o in outs)))

    def summary(self, which="harmonic"):
        mean = np.empty(max(self.n, 1))
        sd = np.empty(max(self.n, 1))
        hb_ensemble_summary(self._ctx, which, mean, sd, False)
        return mean[: self.n], sd[: self.n]

    def stats(self) -> dict:
        return hb_stats(self._ctx)

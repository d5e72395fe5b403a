"""Thin ctypes binding of libseismic.so.

Functions carry the C names and only marshal arguments: host inputs are
numpy arrays, device buffers are torch tensors (their data_ptr() is passed)
and streams are torch.cuda streams.  Every step of the search runs in the
library's HIP kernels; if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libseismic.so")

OK, EINVAL, ENOMEM, EHIP, EIO, EFORMAT, ESTATE = 0, -1, -2, -3, -4, -5, -6
MAX_QUERY_NNZ = 1024
MAX_K = 1024
NOALLOC_MAX_ROWS = 8192        # host-resident queries of seismic_search_batch_noalloc
NOALLOC_MAX_WORDS = 1 << 20
COUNTER_NAMES = ("summary_entries", "blocks_in_lists", "blocks_evaluated", "docs_evaluated",
                 "nnz_evaluated", "prune_tests", "status", "cut_len")

_lib = None


class SeismicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_uint64), ("nnz", ctypes.c_uint64), ("dim", ctypes.c_uint32),
                ("on_device", ctypes.c_uint32), ("row_ptr", ctypes.c_void_p), ("words", ctypes.c_void_p)]


class BuildParams(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_uint32), ("beta", ctypes.c_uint32), ("gamma", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("n_threads", ctypes.c_int32), ("verbose", ctypes.c_int32),
                ("alpha", ctypes.c_double)]


class SearchParams(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("query_cut", ctypes.c_uint32), ("heap_factor", ctypes.c_float),
                ("flags", ctypes.c_uint32), ("probe", ctypes.c_void_p), ("probe_tau", ctypes.c_double),
                ("query_mass", ctypes.c_double)]


class ProbeLoss(ctypes.Structure):
    _fields_ = [("pos_weight", ctypes.c_float), ("neg_weight", ctypes.c_float),
                ("neg_weight_per_doc", ctypes.c_float), ("reserved", ctypes.c_uint32)]


class AdamParams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


class LaunchConfig(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32), ("window", ctypes.c_uint32),
                ("schedule", ctypes.c_uint32)]


class ServerParams(ctypes.Structure):
    _fields_ = [("search", SearchParams), ("max_batch", ctypes.c_uint32), ("n_slots", ctypes.c_uint32),
                ("max_batch_nnz", ctypes.c_uint32), ("use_graphs", ctypes.c_uint32), ("launch", LaunchConfig),
                ("scratch_bytes", ctypes.c_uint64), ("inject_admission_failures", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("cfg", LaunchConfig), ("ms", ctypes.c_float), ("reserved", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("prefix", ctypes.c_void_p), ("prefix_stride", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("counters", ctypes.c_void_p), ("list_hmin", ctypes.c_void_p), ("list_term", ctypes.c_void_p)]


PROBE_WORDS = 512
SEARCH_KNN = 1  # seismic_search_params.flags: kappa-NN refinement


def load():
    """Load libseismic.so (torch first, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime the library binds to)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "seismic_last_error": ([], ctypes.c_char_p),
        "seismic_build_index": ([P(Csr), P(BuildParams), P(vp)], i32),
        "seismic_build_index_gpu": ([P(Csr), P(BuildParams), i32, P(vp)], i32),
        "seismic_build_index_device": ([P(Csr), P(BuildParams), i32, P(vp)], i32),
        "seismic_index_serialized_size": ([vp, P(u64)], i32),
        "seismic_index_serialize": ([vp, vp, u64], i32),
        "seismic_index_save": ([vp, ctypes.c_char_p], i32),
        "seismic_index_load": ([ctypes.c_char_p, P(vp)], i32),
        "seismic_index_info": ([vp, vp], i32),
        "seismic_index_upload": ([vp, i32, u32], i32),
        "seismic_index_copy_lists": ([vp, vp, u32, u64, P(u32), P(u64)], i32),
        "seismic_index_release_exact": ([vp], i32),
        "seismic_index_free": ([vp], None),
        "seismic_workspace_create": ([vp, u32, u32, P(vp)], i32),
        "seismic_workspace_free": ([vp], None),
        "seismic_workspace_set_config": ([vp, P(LaunchConfig)], i32),
        "seismic_workspace_get_config": ([vp, u32, P(LaunchConfig)], i32),
        "seismic_workspace_resident_per_cu": ([vp, u32, u32, P(u32)], i32),
        "seismic_autotune": ([vp, vp, P(Csr), P(SearchParams), vp, vp, u32, vp, u32, P(u32), vp], i32),
        "seismic_search_batch": ([vp, vp, P(Csr), P(SearchParams), vp, vp, P(Stats), vp], i32),
        "seismic_search_batch_noalloc": ([vp, P(Csr), P(SearchParams), vp, vp, P(Stats), vp], i32),
        "exact_topk": ([vp, P(Csr), u32, vp, vp, vp], i32),
        "seismic_probe_collect": ([vp, P(Csr), vp, vp, u32, vp, u32, u32, vp, vp, vp], i32),
        "seismic_probe_trainer_create": ([i32, u32, P(vp)], i32),
        "seismic_probe_trainer_free": ([vp], None),
        "seismic_probe_grad": ([vp, vp, vp, vp, u32, P(ProbeLoss), vp, vp, vp, vp], i32),
        "seismic_probe_adam": ([vp, vp, vp, vp, vp, u32, P(AdamParams), vp, vp], i32),
        "seismic_server_create": ([vp, P(ServerParams), P(vp)], i32),
        "seismic_knn_build": ([vp, u32, u32, ctypes.c_float], i32),
        "seismic_index_set_knn": ([vp, u32, vp, u32], i32),
        "seismic_index_get_knn": ([vp, vp, P(u32)], i32),
        "seismic_graph_create": ([vp, vp, P(Csr), vp, P(SearchParams), vp, vp, P(Stats), P(vp)], i32),
        "seismic_graph_launch": ([vp, vp], i32),
        "seismic_graph_free": ([vp], None),
        "seismic_server_clock": ([vp], ctypes.c_double),
        "seismic_server_submit": ([vp, vp, u32, ctypes.c_double, P(u64)], i32),
        "seismic_server_poll": ([vp, u64, vp, vp, P(ctypes.c_double)], i32),
        "seismic_server_submit_batch": ([vp, P(Csr), vp, P(u64)], i32),
        "seismic_server_results": ([vp, u64, u64, vp, vp, vp], i32),
        "seismic_server_release": ([vp, u64, P(u64)], i32),
        "seismic_server_wait_all": ([vp, ctypes.c_double], i32),
        "seismic_server_stats": ([vp, vp], i32),
        "seismic_server_free": ([vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        raise SeismicError(rc, load().seismic_last_error().decode())


def _ptr(x) -> int:
    if x is None:
        return 0
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    return int(x.ctypes.data)


def host_csr(row_ptr: np.ndarray, words: np.ndarray, dim: int) -> Csr:
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.uint64)
    words = np.ascontiguousarray(words, dtype=np.uint32)
    c = Csr(len(row_ptr) - 1, len(words), dim, 0, _ptr(row_ptr), _ptr(words) if len(words) else 0)
    c._keep = (row_ptr, words)
    return c


def device_csr(row_ptr, words, dim: int) -> Csr:
    """row_ptr (int64/uint64) and words (int32/uint32) torch tensors on the GPU."""
    c = Csr(row_ptr.numel() - 1, words.numel(), dim, 1, _ptr(row_ptr), _ptr(words) if words.numel() else 0)
    c._keep = (row_ptr, words)
    return c


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


# ----------------------------------------------------------------- C names

def seismic_build_index(row_ptr, words, dim, lam, beta, gamma, seed=0, n_threads=0, verbose=0, alpha=0.0) -> int:
    lib = load()
    csr = host_csr(row_ptr, words, dim)
    p = BuildParams(lam, beta, gamma, seed, n_threads, verbose, alpha)
    h = ctypes.c_void_p()
    _check(lib.seismic_build_index(ctypes.byref(csr), ctypes.byref(p), ctypes.byref(h)))
    return h.value


def seismic_build_index_gpu(row_ptr, words, dim, lam, beta, gamma, seed=0, n_threads=0, verbose=0, alpha=0.0,
                            device=0) -> int:
    lib = load()
    csr = host_csr(row_ptr, words, dim)
    p = BuildParams(lam, beta, gamma, seed, n_threads, verbose, alpha)
    h = ctypes.c_void_p()
    _check(lib.seismic_build_index_gpu(ctypes.byref(csr), ctypes.byref(p), device, ctypes.byref(h)))
    return h.value


def seismic_build_index_device(csr: "Csr", lam, beta, gamma, seed=0, n_threads=0, verbose=0, alpha=0.0,
                               device=0) -> int:
    """csr: a device_csr of the documents; the index is built and stays on the device."""
    lib = load()
    p = BuildParams(lam, beta, gamma, seed, n_threads, verbose, alpha)
    h = ctypes.c_void_p()
    _check(lib.seismic_build_index_device(ctypes.byref(csr), ctypes.byref(p), device, ctypes.byref(h)))
    return h.value


def seismic_index_serialize(handle) -> np.ndarray:
    lib = load()
    n = ctypes.c_uint64()
    _check(lib.seismic_index_serialized_size(handle, ctypes.byref(n)))
    buf = np.empty(n.value, dtype=np.uint8)
    _check(lib.seismic_index_serialize(handle, _ptr(buf), n.value))
    return buf


def seismic_index_save(handle, path: str):
    _check(load().seismic_index_save(handle, os.fsencode(path)))


def seismic_index_load(path: str) -> int:
    h = ctypes.c_void_p()
    _check(load().seismic_index_load(os.fsencode(path), ctypes.byref(h)))
    return h.value


def seismic_index_info(handle) -> dict:
    out = np.zeros(10, dtype=np.uint64)
    _check(load().seismic_index_info(handle, _ptr(out)))
    keys = ("dim", "n_docs", "nnz", "n_blocks", "n_postings", "n_summary", "lam", "beta",
            "max_blocks_per_list", "on_device")
    return {k: int(v) for k, v in zip(keys, out)}


def seismic_index_upload(handle, device: int = 0, block_rows: bool = False):
    _check(load().seismic_index_upload(handle, device, 1 if block_rows else 0))


def seismic_index_copy_lists(handle, lists, max_bytes: int):
    """Block-major row copies of the longest prefix of `lists` (term ids,
    most valuable first) fitting max_bytes of device memory.  Returns
    (entries of lists covered, device bytes taken)."""
    arr = np.ascontiguousarray(np.asarray(lists, dtype=np.uint32))
    n_copied, used = ctypes.c_uint32(0), ctypes.c_uint64(0)
    _check(load().seismic_index_copy_lists(handle, arr.ctypes.data if arr.size else None, arr.size,
                                           int(max_bytes), ctypes.byref(n_copied), ctypes.byref(used)))
    return int(n_copied.value), int(used.value)


def seismic_index_release_exact(handle):
    _check(load().seismic_index_release_exact(handle))


def seismic_index_free(handle):
    if handle:
        load().seismic_index_free(handle)


def seismic_workspace_create(handle, max_queries: int, max_k: int) -> int:
    w = ctypes.c_void_p()
    _check(load().seismic_workspace_create(handle, max_queries, max_k, ctypes.byref(w)))
    return w.value


def seismic_workspace_free(ws):
    if ws:
        load().seismic_workspace_free(ws)


def seismic_workspace_set_config(ws, threads: int = 256, blocks_per_cu: int = 0, window: int = 4, schedule: int = 0):
    """schedule: 0 query-major, 1 list-major, 2 wide (see seismic_launch_config)."""
    c = LaunchConfig(threads, blocks_per_cu, window, schedule)
    _check(load().seismic_workspace_set_config(ws, ctypes.byref(c)))


def seismic_workspace_get_config(ws, n_queries: int) -> dict:
    c = LaunchConfig()
    _check(load().seismic_workspace_get_config(ws, n_queries, ctypes.byref(c)))
    return {"threads": c.threads, "blocks_per_cu": c.blocks_per_cu, "window": c.window, "schedule": c.schedule}


def seismic_workspace_resident_per_cu(ws, n_queries: int, k: int) -> int:
    """Search workgroups per CU that stay resident for such a batch."""
    n = ctypes.c_uint32()
    _check(load().seismic_workspace_resident_per_cu(ws, n_queries, k, ctypes.byref(n)))
    return n.value


def _params(k, query_cut, heap_factor, flags=0, probe=None, probe_tau=0.0, query_mass=0.0):
    p = SearchParams(k, query_cut, heap_factor, flags, _ptr(probe), float(probe_tau), float(query_mass))
    p._keep = probe
    return p


def seismic_autotune(handle, ws, queries: Csr, k: int, query_cut: int, heap_factor: float, out_ids, out_scores,
                     reps: int = 3, stream=None, max_results: int = 256, probe=None, probe_tau: float = 0.0):
    """Time every launch shape on this batch, keep the fastest for its
    batch-size bucket; returns the list of (config, ms)."""
    p = _params(k, query_cut, heap_factor, 0, probe, probe_tau)
    res = (TuneResult * max_results)()
    n = ctypes.c_uint32(0)
    _check(load().seismic_autotune(handle, ws, ctypes.byref(queries), ctypes.byref(p), _ptr(out_ids), _ptr(out_scores),
                                   reps, res, max_results, ctypes.byref(n), _stream_handle(stream)))
    return [({"threads": r.cfg.threads, "blocks_per_cu": r.cfg.blocks_per_cu, "window": r.cfg.window,
              "schedule": r.cfg.schedule}, r.ms)
            for r in res[:n.value]]


def seismic_search_batch(handle, ws, queries: Csr, k: int, query_cut: int, heap_factor: float,
                         out_ids, out_scores, prefix=None, prefix_stride: int = 0, counters=None,
                         stream=None, flags: int = 0, probe=None, probe_tau: float = 0.0,
                         list_hmin=None, list_term=None, query_mass: float = 0.0):
    """probe: device tensor of PROBE_WORDS bf16 words (int16/uint16/bfloat16)
    or None; list_hmin (float32) / list_term (int32) [n * prefix_stride]."""
    p = _params(k, query_cut, heap_factor, flags, probe, probe_tau, query_mass)
    st = Stats(_ptr(prefix), prefix_stride, 0, _ptr(counters), _ptr(list_hmin), _ptr(list_term))
    use_stats = any(x is not None for x in (prefix, counters, list_hmin, list_term))
    _check(load().seismic_search_batch(handle, ws, ctypes.byref(queries), ctypes.byref(p), _ptr(out_ids),
                                       _ptr(out_scores), ctypes.byref(st) if use_stats else None,
                                       _stream_handle(stream)))


def seismic_search_batch_noalloc(handle, queries: Csr, k: int, query_cut: int, heap_factor: float,
                                 out_ids, out_scores, prefix=None, prefix_stride: int = 0, counters=None,
                                 stream=None, flags: int = 0, probe=None, probe_tau: float = 0.0,
                                 list_hmin=None, list_term=None, query_mass: float = 0.0):
    """seismic_search_batch without a workspace (no device allocation)."""
    p = _params(k, query_cut, heap_factor, flags, probe, probe_tau, query_mass)
    st = Stats(_ptr(prefix), prefix_stride, 0, _ptr(counters), _ptr(list_hmin), _ptr(list_term))
    use_stats = any(x is not None for x in (prefix, counters, list_hmin, list_term))
    _check(load().seismic_search_batch_noalloc(handle, ctypes.byref(queries), ctypes.byref(p), _ptr(out_ids),
                                               _ptr(out_scores), ctypes.byref(st) if use_stats else None,
                                               _stream_handle(stream)))


def exact_topk(handle, queries: Csr, k: int, out_ids, out_scores, stream=None):
    _check(load().exact_topk(handle, ctypes.byref(queries), k, _ptr(out_ids), _ptr(out_scores),
                             _stream_handle(stream)))


# ------------------------------------------------------- learned block probe

def seismic_probe_collect(handle, queries: Csr, list_term, list_hmin, stride: int, exact_ids, exact_k: int,
                          max_blocks: int, out_feat, out_label, stream=None):
    _check(load().seismic_probe_collect(handle, ctypes.byref(queries), _ptr(list_term), _ptr(list_hmin), stride,
                                        _ptr(exact_ids), exact_k, max_blocks, _ptr(out_feat), _ptr(out_label),
                                        _stream_handle(stream)))


def seismic_probe_trainer_create(device: int, max_batch: int) -> int:
    t = ctypes.c_void_p()
    _check(load().seismic_probe_trainer_create(device, max_batch, ctypes.byref(t)))
    return t.value


def seismic_probe_trainer_free(trainer):
    if trainer:
        load().seismic_probe_trainer_free(trainer)


def seismic_probe_grad(trainer, feat, label, order, n: int, weights, grad_out, stats_out, pos_weight: float = 1.0,
                       neg_weight: float = 1.0, neg_weight_per_doc: float = 0.0, stream=None):
    lp = ProbeLoss(pos_weight, neg_weight, neg_weight_per_doc, 0)
    _check(load().seismic_probe_grad(trainer, _ptr(feat), _ptr(label), _ptr(order), n, ctypes.byref(lp),
                                     _ptr(weights), _ptr(grad_out), _ptr(stats_out), _stream_handle(stream)))


def seismic_probe_adam(grad_sum, stats, master, m, v, step: int, weights_out, lr: float = 1e-3,
                       beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
    ap = AdamParams(lr, beta1, beta2, eps)
    _check(load().seismic_probe_adam(_ptr(grad_sum), _ptr(stats), _ptr(master), _ptr(m), _ptr(v), step,
                                     ctypes.byref(ap), _ptr(weights_out), _stream_handle(stream)))


# ----------------------------------------------------------- kappa-NN graph

def seismic_knn_build(handle, kappa: int, query_cut: int, heap_factor: float):
    _check(load().seismic_knn_build(handle, kappa, query_cut, heap_factor))


def seismic_index_set_knn(handle, table):
    """table: uint32 numpy [n_docs, kappa] (host) or an int32 torch tensor on
    the device."""
    if hasattr(table, "data_ptr"):
        kappa, dev = int(table.shape[1]), 1
    else:
        table = np.ascontiguousarray(table, dtype=np.uint32)
        kappa, dev = int(table.shape[1]), 0
    _check(load().seismic_index_set_knn(handle, kappa, _ptr(table), dev))


def seismic_index_get_knn(handle, n_docs: int):
    """The index's graph as uint32 [n_docs, kappa], or None."""
    kap = ctypes.c_uint32(0)
    _check(load().seismic_index_get_knn(handle, None, ctypes.byref(kap)))
    if kap.value == 0:
        return None
    out = np.empty((n_docs, kap.value), dtype=np.uint32)
    _check(load().seismic_index_get_knn(handle, _ptr(out), ctypes.byref(kap)))
    return out


# ------------------------------------------------------------ graph batches

def seismic_graph_create(handle, ws, queries: Csr, n_queries_dev, k: int, query_cut: int, heap_factor: float,
                         out_ids, out_scores, prefix=None, prefix_stride: int = 0, counters=None, probe=None,
                         probe_tau: float = 0.0) -> int:
    """Capture one search launch into a HIP graph; the batch size of each
    replay is read from the device tensor n_queries_dev (one int32)."""
    p = _params(k, query_cut, heap_factor, 0, probe, probe_tau)
    st = Stats(_ptr(prefix), prefix_stride, 0, _ptr(counters), 0, 0)
    use_stats = prefix is not None or counters is not None
    g = ctypes.c_void_p()
    _check(load().seismic_graph_create(handle, ws, ctypes.byref(queries), _ptr(n_queries_dev), ctypes.byref(p),
                                       _ptr(out_ids), _ptr(out_scores), ctypes.byref(st) if use_stats else None,
                                       ctypes.byref(g)))
    return g.value


def seismic_graph_launch(graph, stream=None):
    _check(load().seismic_graph_launch(graph, _stream_handle(stream)))


def seismic_graph_free(graph):
    if graph:
        load().seismic_graph_free(graph)


# ------------------------------------------------------------ serving loop

def seismic_server_create(handle, k: int, query_cut: int, heap_factor: float, max_batch: int = 1024,
                          n_slots: int = 4, max_batch_nnz: int = 0, probe=None, probe_tau: float = 0.0,
                          launch: dict | None = None, use_graphs: bool = True, scratch_bytes: int = 0,
                          inject_admission_failures: int = 0) -> int:
    """probe (device tensor) must outlive the server."""
    sp = _params(k, query_cut, heap_factor, 0, probe, probe_tau)
    lc = LaunchConfig(0, 0, 0, 0) if not launch else LaunchConfig(launch["threads"], launch["blocks_per_cu"],
                                                                  launch["window"], launch.get("schedule", 0))
    p = ServerParams(sp, max_batch, n_slots, max_batch_nnz or max(MAX_QUERY_NNZ, 256 * max_batch),
                     1 if use_graphs else 0, lc, int(scratch_bytes), int(inject_admission_failures), 0)
    s = ctypes.c_void_p()
    _check(load().seismic_server_create(handle, ctypes.byref(p), ctypes.byref(s)))
    return s.value


def seismic_server_clock(server) -> float:
    return float(load().seismic_server_clock(server))


def seismic_server_submit(server, words: np.ndarray, not_before: float = 0.0) -> int:
    w = np.ascontiguousarray(words, dtype=np.uint32)
    t = ctypes.c_uint64()
    _check(load().seismic_server_submit(server, _ptr(w) if len(w) else None, len(w), float(not_before),
                                        ctypes.byref(t)))
    return t.value


def seismic_server_submit_batch(server, queries: Csr, not_before=None) -> int:
    """queries: host Csr; not_before: float64 [n_rows] or None.  Returns the
    first ticket."""
    nb = None if not_before is None else np.ascontiguousarray(not_before, dtype=np.float64)
    t = ctypes.c_uint64()
    _check(load().seismic_server_submit_batch(server, ctypes.byref(queries), None if nb is None else _ptr(nb),
                                              ctypes.byref(t)))
    return t.value


def seismic_server_results(server, first_ticket: int, n: int, k: int):
    """(ids uint32 [n, k], scores float32 [n, k], latency float64 [n])."""
    ids = np.empty((n, k), dtype=np.uint32)
    sc = np.empty((n, k), dtype=np.float32)
    lat = np.empty(n, dtype=np.float64)
    _check(load().seismic_server_results(server, first_ticket, n, _ptr(ids), _ptr(sc), _ptr(lat)))
    return ids, sc, lat


def seismic_server_poll(server, ticket: int, k: int):
    """None while pending, else (ids uint32[k], scores float32[k], latency s)."""
    ids = np.empty(k, dtype=np.uint32)
    sc = np.empty(k, dtype=np.float32)
    lat = ctypes.c_double()
    rc = load().seismic_server_poll(server, ticket, _ptr(ids), _ptr(sc), ctypes.byref(lat))
    if rc < 0:
        _check(rc)
    return None if rc == 0 else (ids, sc, lat.value)


def seismic_server_release(server, end_ticket: int) -> int:
    """Drops the results of tickets below end_ticket; returns the first
    ticket still held."""
    b = ctypes.c_uint64()
    _check(load().seismic_server_release(server, int(end_ticket), ctypes.byref(b)))
    return b.value


def seismic_server_wait_all(server, timeout_s: float = 600.0):
    _check(load().seismic_server_wait_all(server, timeout_s))


def seismic_server_stats(server) -> dict:
    out = np.zeros(8, dtype=np.uint64)
    _check(load().seismic_server_stats(server, _ptr(out)))
    return dict(zip(("submitted", "completed", "batches", "max_inflight", "held", "max_busy_slots",
                     "deferred_admissions", "peak_scratch_bytes"), (int(x) for x in out)))


def seismic_server_free(server):
    if server:
        load().seismic_server_free(server)

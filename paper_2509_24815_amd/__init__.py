"""Seismic sparse-MIPS query processing on MI355X (gfx950).

The product is ``libseismic.so`` (C ABI in ``include/seismic.h``); this
package holds its HIP/C++ sources (``csrc/``), the build script and a thin
Python binding (``binding``) plus a convenience wrapper (``Index``).
"""
from __future__ import annotations

from . import binding
from .binding import SeismicError

__all__ = ["binding", "Index", "SeismicError", "hot_list_order"]


def hot_list_order(prefix, list_term):
    """Term ids of the lists a traced batch evaluated blocks of, the most
    evaluated blocks first (ties by smaller term id).  prefix[q, i] blocks
    of list list_term[q, i] were evaluated (the search trace); positions
    with a zero prefix are ignored.  The order in which to give lists block-
    major copies when not every list fits (Index.copy_lists)."""
    import numpy as np
    p = np.asarray(prefix).astype(np.uint16).astype(np.int64).ravel()
    t = np.asarray(list_term).astype(np.int64).ravel()
    m = p > 0
    if not m.any():
        return np.zeros(0, dtype=np.uint32)
    w = np.bincount(t[m], weights=p[m])
    terms = np.nonzero(w)[0]
    return terms[np.lexsort((terms, -w[terms]))].astype(np.uint32)


class Index:
    """Owning wrapper around a seismic_index handle."""

    def __init__(self, handle: int):
        self.handle = handle
        self._ws = {}

    @classmethod
    def build(cls, docs, lam: int, beta: int, gamma: float, seed: int = 0, n_threads: int = 0,
              verbose: bool = False, alpha: float = 0.0) -> "Index":
        return cls(binding.seismic_build_index(docs.row_ptr, docs.words, docs.dim, lam, beta, gamma, seed,
                                               n_threads, int(verbose), alpha))

    @classmethod
    def build_gpu(cls, docs, lam: int, beta: int, gamma: float, seed: int = 0, n_threads: int = 0,
                  verbose: bool = False, alpha: float = 0.0, device: int = 0) -> "Index":
        """The same index, with the per-list work on the GPU."""
        return cls(binding.seismic_build_index_gpu(docs.row_ptr, docs.words, docs.dim, lam, beta, gamma, seed,
                                                   n_threads, int(verbose), alpha, device))

    @classmethod
    def build_device(cls, docs, lam: int, beta: int, gamma: float, seed: int = 0, verbose: bool = False,
                     alpha: float = 0.0, device: int = 0) -> "Index":
        """The same index built from documents already on the device
        (binding.device_csr), left resident there (plain row layout)."""
        return cls(binding.seismic_build_index_device(docs, lam, beta, gamma, seed, 0, int(verbose), alpha, device))

    @classmethod
    def load(cls, path: str) -> "Index":
        return cls(binding.seismic_index_load(path))

    def save(self, path: str):
        binding.seismic_index_save(self.handle, path)

    def serialize(self):
        return binding.seismic_index_serialize(self.handle)

    def info(self) -> dict:
        return binding.seismic_index_info(self.handle)

    def upload(self, device: int = 0, block_rows: bool = False):
        binding.seismic_index_upload(self.handle, device, block_rows)

    def copy_lists(self, lists, max_bytes: int):
        """Block-major row copies of the longest prefix of ``lists`` that fits
        max_bytes of device memory: (entries covered, bytes taken)."""
        return binding.seismic_index_copy_lists(self.handle, lists, max_bytes)

    def copy_hot_lists(self, sample_queries, k: int, query_cut: int, heap_factor: float, max_bytes: int):
        """Copies for the lists a sample batch evaluates most (hot_list_order
        of its trace).  Returns (lists covered, bytes taken, the order)."""
        import torch
        _, _, prefix, _, _, term = self.search(sample_queries, k, query_cut, heap_factor, trace=True)
        torch.cuda.synchronize()
        order = hot_list_order(prefix.cpu().numpy(), term.cpu().numpy())
        n, used = self.copy_lists(order, max_bytes)
        return n, used, order

    def release_exact(self):
        """Free the inverted index built by exact search."""
        binding.seismic_index_release_exact(self.handle)

    def workspace(self, max_queries: int, max_k: int) -> int:
        key = (max_queries, max_k)
        if key not in self._ws:
            self._ws[key] = binding.seismic_workspace_create(self.handle, max_queries, max_k)
        return self._ws[key]

    def search(self, queries, k: int, query_cut: int, heap_factor: float, *, stats: bool = False,
               prefix_stride: int | None = None, stream=None, ws=None, probe=None, probe_tau: float = 0.0,
               trace: bool = False, refine: bool = False, query_mass: float = 0.0):
        """Batched search.  ``queries`` is a binding.Csr (host or device).
        Returns torch tensors on the current device (ids, scores[, prefix,
        counters[, list_hmin, list_term]]).  probe: device tensor of
        binding.PROBE_WORDS bf16 words (learned block probe) or None."""
        import torch
        nq = int(queries.n_rows)
        dev = torch.device("cuda", torch.cuda.current_device())
        ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
        sc = torch.empty((nq, k), dtype=torch.float32, device=dev)
        prefix = counters = hmin = term = None
        stats = stats or trace
        if stats:
            stride = prefix_stride or max(1, query_cut if query_cut > 0 else binding.MAX_QUERY_NNZ)
            prefix = torch.zeros((nq, stride), dtype=torch.int16, device=dev)
            counters = torch.zeros((nq, 8), dtype=torch.int64, device=dev)
            if trace:
                hmin = torch.empty((nq, stride), dtype=torch.float32, device=dev)
                term = torch.empty((nq, stride), dtype=torch.int32, device=dev)
        else:
            stride = 0
        w = ws if ws is not None else self.workspace(max(nq, 1), max(k, 1))
        binding.seismic_search_batch(self.handle, w, queries, k, query_cut, heap_factor, ids, sc,
                                     prefix, stride, counters, stream, probe=probe, probe_tau=probe_tau,
                                     list_hmin=hmin, list_term=term,
                                     flags=binding.SEARCH_KNN if refine else 0, query_mass=query_mass)
        if trace:
            return ids, sc, prefix, counters, hmin, term
        if stats:
            return ids, sc, prefix, counters
        return ids, sc

    def build_knn(self, kappa: int, query_cut: int = 10, heap_factor: float = 0.8):
        """kappa-NN graph by searching every document (GPU)."""
        binding.seismic_knn_build(self.handle, kappa, query_cut, heap_factor)

    def set_knn(self, table):
        binding.seismic_index_set_knn(self.handle, table)

    def knn(self):
        return binding.seismic_index_get_knn(self.handle, self.info()["n_docs"])

    def exact(self, queries, k: int, stream=None):
        import torch
        nq = int(queries.n_rows)
        dev = torch.device("cuda", torch.cuda.current_device())
        ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
        sc = torch.empty((nq, k), dtype=torch.float32, device=dev)
        binding.exact_topk(self.handle, queries, k, ids, sc, stream)
        return ids, sc

    def close(self):
        for w in self._ws.values():
            binding.seismic_workspace_free(w)
        self._ws = {}
        if self.handle:
            binding.seismic_index_free(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

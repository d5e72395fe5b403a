"""CPU oracle for Seismic query processing.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke entry point and the
benchmark's CPU-baseline leg may import this package; the product library
never does, and this package never imports the product library.

``oracle.c`` holds the plain C implementation (exact search, Algorithm 2
block-pruned search, index structure checks, the sketching and quantization
routines); ``mlp.py`` holds the fp64 reference of the learned block probe.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

EXACT_SUMMARIES = 1  # r_j = <q, phi(B_j)> with full max vectors, no sketch and no quantization
CONTINUE = 2         # literal "continue" on a skipped block instead of stopping the list

PROBE_WORDS = 512   # learned block probe: W1[64][5], b1[64], w2[64], b2, zero padding (bf16)

COUNTER_NAMES = ("summary_entries", "blocks_in_lists", "blocks_evaluated", "docs_evaluated",
                 "nnz_evaluated", "prune_tests", "near_tie_tests", "cut_len")


def build(verbose: bool = False) -> str:
    src = os.path.join(_HERE, "oracle.c")
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", src, "-o", _LIB_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return _LIB_PATH


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, u64, i32, f32, f64 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_float, ctypes.c_double
    lib.or_index_open.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)]
    lib.or_index_open.restype = vp
    lib.or_index_from_buffer.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_int)]
    lib.or_index_from_buffer.restype = vp
    lib.or_index_close.argtypes = [vp]
    lib.or_index_info.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
    lib.or_index_sections.argtypes = [vp, vp]
    lib.or_value_range.argtypes = [vp, u64]
    lib.or_value_range.restype = i32
    lib.or_exact_topk.argtypes = [vp, vp, u64, vp, vp, u64, ctypes.c_uint32, i32, vp, vp, i32]
    lib.or_exact_topk.restype = i32
    lib.or_pruned_search.argtypes = [vp, vp, vp, u64, i32, i32, f32, ctypes.c_uint32, i32, i32, vp, vp, vp, vp,
                                     vp, f64, vp, vp, i32, f64]
    lib.or_pruned_search.restype = i32
    lib.or_probe_eval.argtypes = [vp, vp, vp, vp, vp, vp, u64, vp, vp]
    lib.or_probe_eval.restype = i32
    lib.or_probe_quantize.argtypes = [vp, u64, i32, vp]
    lib.or_probe_quantize.restype = None
    lib.or_check_index.argtypes = [vp, i32, i32, ctypes.c_char_p, i32]
    lib.or_check_index.restype = i32
    lib.or_column_keep.argtypes = [vp, vp, u64, u64, vp]
    lib.or_alpha_mss.argtypes = [vp, vp, u64, f64, vp]
    lib.or_alpha_mss.restype = i32
    lib.or_quantize.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float), vp]
    lib.or_summary_scores.argtypes = [vp, vp, u64, ctypes.c_uint32, vp, vp]
    lib.or_summary_scores.restype = i32
    _lib = lib
    return lib


def _csr(x):
    rp = np.ascontiguousarray(x.row_ptr, dtype=np.uint64)
    w = np.ascontiguousarray(x.words, dtype=np.uint32)
    if w.size == 0:
        w = np.zeros(1, dtype=np.uint32)
    return rp, w


def value_range_ok(x) -> bool:
    """True when every value lies in [2^-6, 2^6], where fp64 sums are exact."""
    rp, w = _csr(x)
    return bool(_load().or_value_range(_p(w), int(rp[-1])))


def exact_topk(docs, queries, k: int, nthreads: int = 0):
    """Exact top-k by brute force over the forward rows.  Returns (ids u32
    [nq, k], scores f32 [nq, k]), sorted by (score desc, id asc), padded with
    (0xFFFFFFFF, -inf)."""
    lib = _load()
    drp, dw = _csr(docs)
    qrp, qw = _csr(queries)
    nq = len(qrp) - 1
    ids = np.empty((nq, k), dtype=np.uint32)
    sc = np.empty((nq, k), dtype=np.float32)
    rc = lib.or_exact_topk(_p(drp), _p(dw), len(drp) - 1, _p(qrp), _p(qw), nq, docs.dim, k,
                           _p(ids), _p(sc), nthreads or os.cpu_count() or 1)
    if rc != 0:
        raise ValueError(f"or_exact_topk failed ({rc})")
    return ids, sc


class Index:
    """Read-only view of a serialized index (file path or bytes-like buffer)."""

    def __init__(self, source):
        lib = _load()
        err = ctypes.c_int(0)
        self._buf = None
        if isinstance(source, (str, os.PathLike)):
            h = lib.or_index_open(os.fsencode(source), ctypes.byref(err))
        else:
            arr = np.frombuffer(source, dtype=np.uint8)
            self._buf = arr
            h = lib.or_index_from_buffer(_p(arr), arr.size, ctypes.byref(err))
        if not h:
            raise ValueError(f"cannot parse index ({err.value})")
        self._h = h
        info = np.zeros(8, dtype=np.uint64)
        g = ctypes.c_double(0.0)
        lib.or_index_info(h, _p(info), ctypes.byref(g))
        (self.dim, self.n_docs, self.nnz, self.n_blocks, self.n_postings, self.n_summary,
         self.lam, self.beta) = [int(v) for v in info]
        self.gamma = g.value

    def close(self):
        if self._h:
            _load().or_index_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sections(self):
        """numpy views of the sections (valid while the Index lives)."""
        ptrs = (ctypes.c_void_p * 11)()
        _load().or_index_sections(self._h, ptrs)
        nb = self.n_blocks
        spec = [("row_ptr", np.uint64, self.n_docs + 1), ("words", np.uint32, self.nnz),
                ("list_off", np.uint32, self.dim + 1), ("blk_post_off", np.uint32, nb + 1),
                ("blk_sum_off", np.uint64, nb + 1), ("blk_m", np.float32, nb), ("blk_delta", np.float32, nb),
                ("blk_centroid", np.uint32, nb), ("postings", np.uint32, self.n_postings),
                ("sum_term", np.uint16, self.n_summary), ("sum_code", np.uint8, self.n_summary)]
        out = {}
        for (name, dt, n), p in zip(spec, ptrs):
            nbytes = int(n) * np.dtype(dt).itemsize
            if n == 0 or not p:
                out[name] = np.zeros(0, dtype=dt)
                continue
            buf = (ctypes.c_uint8 * nbytes).from_address(p)
            out[name] = np.frombuffer(buf, dtype=dt, count=int(n))
        return out

    def check(self, clustering: bool = True, term_stride: int = 1) -> str:
        """Structure check against the indexing algorithm; '' when it passes."""
        msg = ctypes.create_string_buffer(512)
        rc = _load().or_check_index(self._h, int(clustering), int(term_stride), msg, 512)
        return "" if rc == 0 else (msg.value.decode() or "check failed")

    def summary_scores(self, terms, halfs, t: int):
        """Summary scores of term t's list for one query (terms u16/int,
        halfs fp16): (r [n_blocks] f32 as the pruned search computes them,
        <q, phi(B_j)> [n_blocks] f32 over the full document vectors)."""
        terms = np.asarray(terms, dtype=np.uint32)
        h = np.ascontiguousarray(halfs, dtype=np.float16).view(np.uint16).astype(np.uint32)
        words = np.ascontiguousarray(terms | (h << 16), dtype=np.uint32)
        if words.size == 0:
            words = np.zeros(1, dtype=np.uint32)
        sec = self.sections()
        nb = int(sec["list_off"][t + 1]) - int(sec["list_off"][t])
        r = np.zeros(max(nb, 1), dtype=np.float32)
        ex = np.zeros(max(nb, 1), dtype=np.float32)
        rc = _load().or_summary_scores(self._h, _p(words), len(terms), int(t), _p(r), _p(ex))
        if rc < 0:
            raise ValueError("term out of range")
        return r[:nb], ex[:nb]

    def pruned_search(self, queries, k: int, cut: int, heap_factor: float, flags: int = 0,
                      nthreads: int = 0, c_cap: int | None = None, probe=None, tau: float = 0.0, knn=None,
                      query_mass: float = 0.0):
        """Algorithm 2 block-pruned search.  Returns a dict with ids, scores,
        prefix (evaluated blocks per cut list), counters and hmin (smallest
        heap score at each cut list's start, -1 when the heap is not full).
        probe: 512 bf16 weights as uint16 (learned block probe) or None.
        knn: kappa-NN graph uint32 [n_docs, kappa] (refinement) or None.
        query_mass: alpha_q of the query's alpha_q-MSS cut (0 = fixed cut)."""
        lib = _load()
        qrp, qw = _csr(queries)
        nq = len(qrp) - 1
        if c_cap is None:
            lens = np.diff(qrp.astype(np.int64))
            c_cap = int(max(1, cut if cut > 0 else (lens.max() if nq else 1)))
        ids = np.empty((nq, k), dtype=np.uint32)
        sc = np.empty((nq, k), dtype=np.float32)
        pref = np.zeros((nq, c_cap), dtype=np.uint16)
        cnt = np.zeros((nq, 8), dtype=np.uint64)
        hmin = np.zeros((nq, c_cap), dtype=np.float32)
        pw = None
        if probe is not None:
            pw = np.ascontiguousarray(probe, dtype=np.uint16)
            if pw.size != PROBE_WORDS:
                raise ValueError(f"probe must hold {PROBE_WORDS} bf16 words")
        kt, kappa = None, 0
        if knn is not None:
            kt = np.ascontiguousarray(knn, dtype=np.uint32)
            if kt.ndim != 2 or kt.shape[0] != self.n_docs:
                raise ValueError("knn must be uint32 [n_docs, kappa]")
            kappa = int(kt.shape[1])
        rc = lib.or_pruned_search(self._h, _p(qrp), _p(qw), nq, k, cut, float(heap_factor), flags,
                                  nthreads or os.cpu_count() or 1, c_cap, _p(ids), _p(sc), _p(pref), _p(cnt),
                                  None if pw is None else _p(pw), float(tau), _p(hmin),
                                  None if kt is None else _p(kt), kappa, float(query_mass))
        if rc != 0:
            raise ValueError(f"or_pruned_search failed ({rc})")
        return {"ids": ids, "scores": sc, "prefix": pref, "counters": cnt, "hmin": hmin}


def column_keep(ids, halfs, lam: int):
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    h = np.ascontiguousarray(halfs, dtype=np.float16).view(np.uint16)
    keep = np.zeros(len(ids), dtype=np.uint8)
    _load().or_column_keep(_p(ids), _p(h), len(ids), lam, _p(keep))
    return keep.astype(bool)


def alpha_mss(ids, halfs, alpha: float):
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    h = np.ascontiguousarray(halfs, dtype=np.float16).view(np.uint16)
    keep = np.zeros(len(ids), dtype=np.uint8)
    _load().or_alpha_mss(_p(ids), _p(h), len(ids), float(alpha), _p(keep))
    return keep.astype(bool)


def quantize(halfs):
    h = np.ascontiguousarray(halfs, dtype=np.float16).view(np.uint16)
    codes = np.zeros(max(1, len(h)), dtype=np.uint8)
    m = ctypes.c_float(0.0)
    d = ctypes.c_float(0.0)
    _load().or_quantize(_p(h), len(h), ctypes.byref(m), ctypes.byref(d), _p(codes))
    return m.value, d.value, codes[:len(h)]


def probe_eval(probe, r, h0, n_docs, n_q, ci):
    """Quantized features [n, 5] and exact logits [n] of the learned block
    probe for explicit (r, h0, n_docs, n_q, ci) rows."""
    pw = np.ascontiguousarray(probe, dtype=np.uint16)
    assert pw.size == PROBE_WORDS
    r = np.ascontiguousarray(r, dtype=np.float32)
    n = r.size
    h0 = np.ascontiguousarray(np.broadcast_to(h0, n), dtype=np.float32)
    nd = np.ascontiguousarray(np.broadcast_to(n_docs, n), dtype=np.uint32)
    nqa = np.ascontiguousarray(np.broadcast_to(n_q, n), dtype=np.int32)
    cia = np.ascontiguousarray(np.broadcast_to(ci, n), dtype=np.int32)
    feat = np.zeros((n, 5), dtype=np.float64)
    z = np.zeros(n, dtype=np.float64)
    _load().or_probe_eval(_p(pw), _p(r), _p(h0), _p(nd), _p(nqa), _p(cia), n, _p(feat), _p(z))
    return feat, z


def probe_quantize(x, mode: int):
    """mode 0: feature quantizer, 1: hidden quantizer, 2: weight sanitizer
    (x = bf16 bit patterns)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    _load().or_probe_quantize(_p(x), x.size, int(mode), _p(out))
    return out


def knn_graph(ref: "Index", docs, kappa: int, cut: int, heap_factor: float, exact: bool = False,
              nthreads: int = 0):
    """kappa-NN graph (Section 4.3): for every document u, the kappa
    documents v != u with the largest <u, v>.  exact=True uses exact search
    (brute force); otherwise, as the paper builds it, the block-pruned
    search with u as the query (k = kappa + 1, u itself dropped).  Rows are
    padded with 0xFFFFFFFF."""
    n = docs.n_rows
    if exact:
        ids, _ = exact_topk(docs, docs, kappa + 1, nthreads)
    else:
        ids = ref.pruned_search(docs, kappa + 1, cut, heap_factor, nthreads=nthreads, c_cap=max(cut, 1))["ids"]
    out = np.full((n, kappa), 0xFFFFFFFF, dtype=np.uint32)
    for u in range(n):
        row = [int(v) for v in ids[u] if v != 0xFFFFFFFF and v != u][:kappa]
        out[u, :len(row)] = row
    return out

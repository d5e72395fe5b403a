"""Seeded synthetic inputs shaped like learned-sparse-embedding corpora.

The generator is shared by the CPU oracle tests and the GPU library; it holds
none of the search method's arithmetic, only the draws.  See ``synth.c`` for
the row law.  Streams: 0 documents, 1 evaluation queries, 2 reserved,
3 probe-training queries, 4 arrivals.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

DIM = 30522
ZIPF_S = 1.1
SIGMA = 0.6

STREAM_DOCS = 0
STREAM_QUERIES = 1
STREAM_PROBE_QUERIES = 3
STREAM_ARRIVALS = 4


def build(verbose: bool = False) -> str:
    import subprocess
    src = os.path.join(_HERE, "synth.c")
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", src, "-o", _LIB_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_counts.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                     ctypes.c_uint32, ctypes.c_void_p]
        lib.synth_counts.restype = ctypes.c_int
        lib.synth_fill.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_fill.restype = ctypes.c_int
        lib.synth_counts_range.argtypes = [ctypes.c_uint64] + lib.synth_counts.argtypes
        lib.synth_counts_range.restype = ctypes.c_int
        lib.synth_fill_range.argtypes = [ctypes.c_uint64] + lib.synth_fill.argtypes
        lib.synth_fill_range.restype = ctypes.c_int
        lib.synth_philox4x32_10.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_half_from_double.argtypes = [ctypes.c_double]
        lib.synth_half_from_double.restype = ctypes.c_uint16
        _lib = lib
    return _lib


@dataclass
class CSR:
    """Sparse rows: ``row_ptr`` u64[n+1], ``words`` u32 = term | fp16 << 16."""
    row_ptr: np.ndarray
    words: np.ndarray
    dim: int

    @property
    def n_rows(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.words.shape[0])

    def terms(self) -> np.ndarray:
        return (self.words & 0xFFFF).astype(np.int64)

    def values(self) -> np.ndarray:
        return (self.words >> 16).astype(np.uint16).view(np.float16)

    def row(self, i: int):
        a, b = int(self.row_ptr[i]), int(self.row_ptr[i + 1])
        w = self.words[a:b]
        return (w & 0xFFFF).astype(np.int64), (w >> 16).astype(np.uint16).view(np.float16)

    def subset(self, rows) -> "CSR":
        rows = np.asarray(rows, dtype=np.int64)
        lens = (self.row_ptr[rows + 1] - self.row_ptr[rows]).astype(np.uint64)
        rp = np.zeros(len(rows) + 1, dtype=np.uint64)
        np.cumsum(lens, out=rp[1:])
        words = np.concatenate([self.words[int(self.row_ptr[r]):int(self.row_ptr[r + 1])] for r in rows]) \
            if len(rows) else np.zeros(0, dtype=np.uint32)
        return CSR(rp, np.ascontiguousarray(words, dtype=np.uint32), self.dim)

    def dense(self, dtype=np.float64) -> np.ndarray:
        out = np.zeros((self.n_rows, self.dim), dtype=dtype)
        for i in range(self.n_rows):
            t, v = self.row(i)
            out[i, t] = v.astype(dtype)
        return out


def generate(n_rows: int, *, seed: int = 0, stream: int = STREAM_DOCS, law: str = "poisson",
             mean: float = 120.0, lo: int = 10, hi: int = 400, dim: int = DIM,
             zipf_s: float = ZIPF_S, sigma: float = SIGMA, row0: int = 0) -> CSR:
    """Generate ``n_rows`` sparse rows (rows row0 .. row0 + n_rows - 1 of the
    stream: every row depends only on (seed, stream, row), so slices
    concatenate to the whole).  ``law`` is "poisson" (mean, clipped to
    [lo, hi]) or "uniform" (integer in [lo, hi])."""
    lib = _load()
    law_id = {"poisson": 0, "uniform": 1}[law]
    counts = np.empty(n_rows, dtype=np.uint32)
    rc = lib.synth_counts_range(row0, n_rows, dim, zipf_s, law_id, mean, lo, hi, seed, stream,
                                counts.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ValueError(f"synth_counts failed ({rc})")
    row_ptr = np.zeros(n_rows + 1, dtype=np.uint64)
    np.cumsum(counts, out=row_ptr[1:])
    words = np.empty(int(row_ptr[-1]), dtype=np.uint32)
    rc = lib.synth_fill_range(row0, n_rows, dim, zipf_s, law_id, mean, lo, hi, sigma, seed, stream,
                              row_ptr.ctypes.data_as(ctypes.c_void_p), words.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ValueError(f"synth_fill failed ({rc})")
    return CSR(row_ptr, words, dim)


def row_counts(n_rows: int, *, seed: int = 0, stream: int = STREAM_DOCS, law: str = "poisson",
               mean: float = 120.0, lo: int = 10, hi: int = 400, dim: int = DIM, zipf_s: float = ZIPF_S,
               row0: int = 0) -> np.ndarray:
    """Nonzero counts of rows row0 .. row0 + n_rows - 1 (the first draw of
    each row, as generate() makes it), without drawing the rows."""
    lib = _load()
    counts = np.empty(n_rows, dtype=np.uint32)
    rc = lib.synth_counts_range(row0, n_rows, dim, zipf_s, {"poisson": 0, "uniform": 1}[law], mean, lo, hi, seed,
                                stream, counts.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ValueError(f"synth_counts failed ({rc})")
    return counts


def docs(n_docs: int, seed: int = 0) -> CSR:
    """Documents: nnz ~ Poisson(120) clipped to [10, 400]."""
    return generate(n_docs, seed=seed, stream=STREAM_DOCS, law="poisson", mean=120.0, lo=10, hi=400)


def queries(n_queries: int, seed: int = 0, *, law: str = "poisson", stream: int = STREAM_QUERIES) -> CSR:
    """Queries: nnz ~ Poisson(43) clipped to [1, 400], or uniform in [5, 200]."""
    if law == "poisson":
        return generate(n_queries, seed=seed, stream=stream, law="poisson", mean=43.0, lo=1, hi=400)
    return generate(n_queries, seed=seed, stream=stream, law="uniform", lo=5, hi=200)


def wide_values(csr: CSR, seed: int = 0) -> CSR:
    """The same rows with values redrawn over the whole positive fp16
    range: per nonzero, with probability 1/2 lognormal(0, 0.6) (unclamped),
    1/4 log-uniform in [2^-24, 2^-6] (subnormals included) and 1/4
    log-uniform in [2^6, 65504]; rounded to fp16 (nearest even).  Seeded by
    (seed, 77) with numpy; the terms are untouched."""
    rng = np.random.default_rng([seed, 77])
    n = csr.nnz
    u = rng.random(n)
    normal = np.exp(rng.normal(0.0, SIGMA, n))
    tiny = np.exp2(rng.uniform(-24.0, -6.0, n))
    huge = np.exp2(rng.uniform(6.0, np.log2(65504.0), n))
    v = np.where(u < 0.5, normal, np.where(u < 0.75, tiny, huge))
    h = np.clip(v, 2.0 ** -24, 65504.0).astype(np.float16).view(np.uint16).astype(np.uint32)
    words = (csr.words & 0xFFFF) | (h << 16)
    return CSR(csr.row_ptr.copy(), np.ascontiguousarray(words, dtype=np.uint32), csr.dim)


def philox4x32_10(ctr, key):
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib.synth_philox4x32_10(c, k, o)
    return list(o)


def half_from_double(x: float) -> int:
    return int(_load().synth_half_from_double(x))


def make_csr(rows, dim: int = DIM) -> CSR:
    """CSR from a list of {term: value} dicts (values rounded to fp16)."""
    rp = [0]
    words = []
    for r in rows:
        for t in sorted(r):
            h = np.array([r[t]], dtype=np.float16).view(np.uint16)[0]
            words.append(int(t) | (int(h) << 16))
        rp.append(len(words))
    return CSR(np.array(rp, dtype=np.uint64), np.array(words, dtype=np.uint32), dim)

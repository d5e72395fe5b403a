"""Read-only views of a serialized index (format version 1, as written by
seismic_index_serialize): a 128-byte header, then 11 sections, each at a
64-byte aligned offset:

    row_ptr u64[n_docs+1], words u32[nnz], list_off u32[dim+1],
    blk_post_off u32[nb+1], blk_sum_off u64[nb+1], blk_m f32[nb],
    blk_delta f32[nb], blk_centroid u32[nb], postings u32[np],
    sum_term u16[ns], sum_code u8[ns]

Used by measurement code that needs the index's structure (which blocks a
list has, how large they are); no search arithmetic lives here."""
from __future__ import annotations

import numpy as np

HEADER_BYTES = 128


def sections(buf: np.ndarray) -> dict:
    """buf: uint8 array of a serialized index.  Returns the header fields and
    a NumPy view per section (no copies)."""
    b = memoryview(np.ascontiguousarray(buf, dtype=np.uint8))
    if bytes(b[:7]) != b"SEISMIC":
        raise ValueError("not a serialized index")
    h = np.frombuffer(b[:HEADER_BYTES], dtype=np.uint8)
    u32 = lambda o: int(h[o:o + 4].view(np.uint32)[0])
    u64 = lambda o: int(h[o:o + 8].view(np.uint64)[0])
    if u32(8) != 1:
        raise ValueError(f"format version {u32(8)}")
    dim, n_docs, nnz, nb, n_post, n_sum = u32(12), u64(16), u64(24), u64(32), u64(40), u64(48)
    spec = [("row_ptr", np.uint64, n_docs + 1), ("words", np.uint32, nnz), ("list_off", np.uint32, dim + 1),
            ("blk_post_off", np.uint32, nb + 1), ("blk_sum_off", np.uint64, nb + 1), ("blk_m", np.float32, nb),
            ("blk_delta", np.float32, nb), ("blk_centroid", np.uint32, nb), ("postings", np.uint32, n_post),
            ("sum_term", np.uint16, n_sum), ("sum_code", np.uint8, n_sum)]
    out = {"dim": dim, "n_docs": n_docs, "nnz": nnz, "n_blocks": nb, "lambda": u32(56), "beta": u32(60)}
    off = HEADER_BYTES
    for name, dt, n in spec:
        off = (off + 63) & ~63
        size = np.dtype(dt).itemsize * n
        out[name] = np.frombuffer(b[off:off + size], dtype=dt)
        off += size
    return out

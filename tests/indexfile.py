"""Writer for hand-made serialized indexes (format version 1), used by the
hand-traced tests.  Layout: a 128-byte header, then 11 sections, each at a
64-byte aligned offset:

    row_ptr u64[n_docs+1], words u32[nnz], list_off u32[dim+1],
    blk_post_off u32[nb+1], blk_sum_off u64[nb+1], blk_m f32[nb],
    blk_delta f32[nb], blk_centroid u32[nb], postings u32[np],
    sum_term u16[ns], sum_code u8[ns]

Header: "SEISMIC\\0", u32 version, u32 dim, u64 n_docs, nnz, n_blocks,
n_postings, n_summary, u32 lambda, u32 beta, f64 gamma, u64 seed,
u32 quantization grid bits.
"""
import struct

import numpy as np


def _align(buf: bytearray):
    while len(buf) % 64:
        buf.append(0)


def write_index(docs, lists, dim, lam=1000, beta=50, gamma=0.4, seed=0) -> bytes:
    """docs: synth.CSR.  lists: {term: [block, ...]} with block =
    dict(docs=[ids], summary=[(term, code), ...], m=float, delta=float,
    centroid=id)."""
    list_off = [0]
    post_off = [0]
    sum_off = [0]
    ms, ds, cents, posts, sterm, scode = [], [], [], [], [], []
    for t in range(dim):
        for blk in lists.get(t, []):
            posts.extend(blk["docs"])
            post_off.append(len(posts))
            for (st, sc) in blk["summary"]:
                sterm.append(st)
                scode.append(sc)
            sum_off.append(len(sterm))
            ms.append(blk["m"])
            ds.append(blk["delta"])
            cents.append(blk["centroid"] if "centroid" in blk else blk["docs"][0])
        list_off.append(len(ms))
    nb = len(ms)
    head = bytearray(b"SEISMIC\x00")
    head += struct.pack("<II", 1, dim)
    head += struct.pack("<QQQQQ", docs.n_rows, docs.nnz, nb, len(posts), len(sterm))
    head += struct.pack("<IIdQI", lam, beta, gamma, seed, 14)
    head += bytes(128 - len(head))
    buf = bytearray(head)
    sections = [
        np.asarray(docs.row_ptr, dtype=np.uint64), np.asarray(docs.words, dtype=np.uint32),
        np.asarray(list_off, dtype=np.uint32), np.asarray(post_off, dtype=np.uint32),
        np.asarray(sum_off, dtype=np.uint64), np.asarray(ms, dtype=np.float32),
        np.asarray(ds, dtype=np.float32), np.asarray(cents, dtype=np.uint32),
        np.asarray(posts, dtype=np.uint32), np.asarray(sterm, dtype=np.uint16),
        np.asarray(scode, dtype=np.uint8)]
    for s in sections:
        _align(buf)
        buf += s.tobytes()
    _align(buf)
    return bytes(buf)

"""A plain-Python index builder written from the paper's indexing algorithm
(Section 4.4), for tiny collections, and a reader that turns a serialized
index back into the same structure.  Test infrastructure: it shares nothing
with the library's build or with the oracle's checker, so the checker can be
pinned against an index that neither of them made.

Definitions followed (all arithmetic on exact integers: an fp16 value is an
integer multiple of 2^-24):
  - Set alpha-MSS with a fixed cap (Section 3.4): list i keeps the
    min(|L_i|, lambda) largest values of column i, ties by document id;
  - blocking by shallow K-means (Section 4.1.2): max(1, ceil(beta * n / lambda))
    centroids drawn from the kept list, each document joins the centroid with
    the largest inner product (lowest centroid on ties), empty clusters are
    dropped, documents ascending inside a block;
  - summaries ("summary" equation, Section 4.1.3): phi(B) = coordinate-wise
    max over the block's full document vectors, reduced to its gamma-MSS
    (Definition of alpha-MSS, Section 3.3: value desc, term asc, the shortest
    prefix whose mass reaches gamma times the total), stored by term;
  - u8 scalar quantization (Section 4.1.3) in the reading used throughout:
    m = min rounded down and delta = (max - m) / 256 rounded up, both to the
    2^-14 grid; code = min(255, floor((v - m) / delta)).

The centroid sample is any sample; here a numpy draw keyed by (seed, term).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

import synth
from tests.indexfile import write_index

GRID = 1024  # 2^-14 in units of 2^-24


def units24(h: np.float16) -> int:
    """Exact value of a positive finite fp16 in units of 2^-24."""
    return int(Fraction(float(h)) * (1 << 24))


def _rows(docs):
    out = []
    for d in range(docs.n_rows):
        t, v = docs.row(d)
        out.append({int(a): units24(b) for a, b in zip(t, v)})
    return out


def _dot(a: dict, b: dict) -> int:
    if len(a) > len(b):
        a, b = b, a
    return sum(v * b[t] for t, v in a.items() if t in b)


def gamma_mss(phi: dict, gamma: float) -> list:
    """Terms of the gamma-MSS of phi (term -> units), sorted by term."""
    ent = sorted(phi.items(), key=lambda tv: (-tv[1], tv[0]))
    total = sum(v for _, v in ent)
    need = Fraction(gamma * (total * 2.0 ** -24))  # the target as an fp64 product
    cum, kept = 0, []
    for t, v in ent:
        cum += v
        kept.append(t)
        if Fraction(cum, 1 << 24) >= need:
            break
    return sorted(kept)


def quantize(vals: list):
    """(m, delta, codes) of u8 scalar quantization on the 2^-14 grid."""
    vmin, vmax = min(vals), max(vals)
    m_u = (vmin // GRID) * GRID
    d_u = -(-(vmax - m_u) // (256 * GRID)) * GRID
    codes = [min(255, (v - m_u) // d_u) if d_u else 0 for v in vals]
    return m_u * 2.0 ** -24, d_u * 2.0 ** -24, codes


def build(docs, lam: int, beta: int, gamma: float, seed: int = 0):
    """Index structure {docs, dim, lam, beta, gamma, lists: {term: [block]}},
    block = dict(docs, summary=[(term, code)], m, delta, centroid)."""
    rows = _rows(docs)
    cols: dict[int, list] = {}
    for d, r in enumerate(rows):
        for t, v in r.items():
            cols.setdefault(t, []).append((v, d))
    lists = {}
    for t in sorted(cols):
        col = sorted(cols[t], key=lambda vd: (-vd[0], vd[1]))
        kept = sorted(d for _, d in col[:min(len(col), lam)])
        n = len(kept)
        nb = max(1, math.ceil(beta * n / lam))
        rng = np.random.default_rng([seed, t])
        cents = [kept[i] for i in rng.choice(n, size=nb, replace=False)]
        members = [[] for _ in cents]
        for d in kept:
            sc = [_dot(rows[d], rows[c]) for c in cents]
            best = max(range(len(sc)), key=lambda i: (sc[i], -i))  # lowest centroid on ties
            members[best].append(d)
        blocks = []
        for c, mem in zip(cents, members):
            if not mem:
                continue
            phi: dict[int, int] = {}
            for d in mem:
                for tt, v in rows[d].items():
                    if v > phi.get(tt, 0):
                        phi[tt] = v
            terms = gamma_mss(phi, gamma)
            m, delta, codes = quantize([phi[x] for x in terms])
            blocks.append(dict(docs=list(mem), summary=list(zip(terms, codes)), m=m, delta=delta, centroid=c))
        lists[t] = blocks
    return dict(docs=docs, dim=docs.dim, lam=lam, beta=beta, gamma=gamma, lists=lists)


def serialize(ix: dict) -> bytes:
    return write_index(ix["docs"], ix["lists"], ix["dim"], lam=ix["lam"], beta=ix["beta"], gamma=ix["gamma"])


def read(buf: bytes) -> dict:
    """The structure of a serialized index (any writer), via the oracle's
    section views."""
    import oracle
    ref = oracle.Index(buf)
    s = {k: np.array(v) for k, v in ref.sections().items()}
    docs = synth.CSR(s["row_ptr"].copy(), s["words"].copy(), ref.dim)
    lists = {}
    for t in range(ref.dim):
        b0, b1 = int(s["list_off"][t]), int(s["list_off"][t + 1])
        if b1 == b0:
            continue
        blocks = []
        for b in range(b0, b1):
            p0, p1 = int(s["blk_post_off"][b]), int(s["blk_post_off"][b + 1])
            e0, e1 = int(s["blk_sum_off"][b]), int(s["blk_sum_off"][b + 1])
            blocks.append(dict(docs=[int(x) for x in s["postings"][p0:p1]],
                               summary=[(int(a), int(c)) for a, c in zip(s["sum_term"][e0:e1], s["sum_code"][e0:e1])],
                               m=float(s["blk_m"][b]), delta=float(s["blk_delta"][b]),
                               centroid=int(s["blk_centroid"][b])))
        lists[t] = blocks
    out = dict(docs=docs, dim=ref.dim, lam=ref.lam, beta=ref.beta, gamma=ref.gamma, lists=lists)
    ref.close()
    return out

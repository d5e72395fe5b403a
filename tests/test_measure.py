"""Host-side measurement code of bench.py: the compulsory (unique) bytes of
a batch recover the evaluated blocks of Algorithm 2 from a trace, so for a
single query they must equal the algorithmic bytes the oracle's counters
give; for a batch they are at most the sum.  The per-query distinct
documents of the evaluated blocks (the scope formula's row term) equal an
independent reconstruction from the oracle's own summary scores."""
import numpy as np

import bench
import oracle
import synth
from paper_2509_24815_amd import Index, indexfile


def _cut_terms(qs, q, cut):
    # the visited lists: the query's largest entries, value desc then term asc
    t, v = qs.row(q)
    o = np.lexsort((t, -v.astype(np.float64)))[:cut]
    out = np.full(cut, 0xFFFFFFFF, dtype=np.uint32)
    out[:len(o)] = t[o]
    return out


def test_unique_bytes_against_oracle_counters():
    docs = synth.docs(20000, seed=8)
    qs = synth.queries(40, seed=8)
    buf = Index.build(docs, lam=500, beta=25, gamma=0.4, seed=8).serialize()
    S = indexfile.sections(buf)
    ref = oracle.Index(buf)
    k, cut, hf = 10, 10, 0.8
    r = ref.pruned_search(qs, k, cut, hf, c_cap=cut)
    terms = np.stack([_cut_terms(qs, q, cut) for q in range(qs.n_rows)])
    nnz = np.diff(qs.row_ptr.astype(np.int64))
    alg = bench.alg_bytes(r["counters"], nnz, k)
    for q in range(qs.n_rows):
        u, _, _ = bench.trace_bytes(S, qs.subset([q]), terms[q:q + 1], r["prefix"][q:q + 1], k)
        assert u == alg[q], q
    u_all, distinct, distinct_nnz = bench.trace_bytes(S, qs, terms, r["prefix"], k)
    assert u_all < alg.sum()
    # a batch of one query repeated reads it once
    two = qs.subset([3, 3])
    assert bench.trace_bytes(S, two, terms[[3, 3]], r["prefix"][[3, 3]], k)[0] == alg[3] + 8 + 4 * nnz[3] + 8 * k
    # distinct documents per query, rebuilt from the oracle's summary scores
    lo, po = S["list_off"], S["blk_post_off"]
    doc_len = np.diff(S["row_ptr"].astype(np.int64))
    for q in range(qs.n_rows):
        qt, qv = qs.row(q)
        seen = set()
        for i, t in enumerate(terms[q]):
            if t == 0xFFFFFFFF or r["prefix"][q][i] == 0:
                continue
            sc, _ = ref.summary_scores(qt, qv, int(t))
            order = sorted(range(len(sc)), key=lambda j: (-sc[j], j))[:int(r["prefix"][q][i])]
            for j in order:
                b = int(lo[t]) + j
                seen.update(int(d) for d in S["postings"][int(po[b]):int(po[b + 1])])
        assert distinct[q] == len(seen), q
        assert distinct_nnz[q] == sum(doc_len[d] for d in seen), q
    assert (distinct <= r["counters"][:, 3]).all() and (distinct < r["counters"][:, 3]).any()
    # the scope formula with distinct documents is below the layout formula
    sb = bench.scope_bytes(r["counters"], nnz, k, distinct, distinct_nnz)
    assert (sb < alg).all()


def test_index_sections_match_info():
    docs = synth.docs(3000, seed=2)
    ix = Index.build(docs, lam=200, beta=10, gamma=0.4)
    S = indexfile.sections(ix.serialize())
    info = ix.info()
    assert S["n_blocks"] == info["n_blocks"] and len(S["postings"]) == info["n_postings"]
    assert np.array_equal(S["row_ptr"], docs.row_ptr) and np.array_equal(S["words"], docs.words)
    assert S["list_off"][-1] == info["n_blocks"] and S["blk_sum_off"][-1] == info["n_summary"]

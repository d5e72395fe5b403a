"""Host-side measurement code of bench.py: the compulsory (unique) bytes of
a batch recover the evaluated blocks of Algorithm 2 from a trace, so for a
single query they must equal the algorithmic bytes the oracle's counters
give; for a batch they are at most the sum."""
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
        u = bench.unique_bytes(S, qs.subset([q]), terms[q:q + 1], r["prefix"][q:q + 1], k)
        assert u == alg[q], q
    u_all = bench.unique_bytes(S, qs, terms, r["prefix"], k)
    assert u_all < alg.sum()
    # a batch of one query repeated reads it once
    two = qs.subset([3, 3])
    assert bench.unique_bytes(S, two, terms[[3, 3]], r["prefix"][[3, 3]], k) == alg[3] + 8 + 4 * nnz[3] + 8 * k


def test_index_sections_match_info():
    docs = synth.docs(3000, seed=2)
    ix = Index.build(docs, lam=200, beta=10, gamma=0.4)
    S = indexfile.sections(ix.serialize())
    info = ix.info()
    assert S["n_blocks"] == info["n_blocks"] and len(S["postings"]) == info["n_postings"]
    assert np.array_equal(S["row_ptr"], docs.row_ptr) and np.array_equal(S["words"], docs.words)
    assert S["list_off"][-1] == info["n_blocks"] and S["blk_sum_off"][-1] == info["n_summary"]

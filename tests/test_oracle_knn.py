"""Pins of the oracle's kappa-NN graph and the refinement step of
Algorithm 2: a hand-traced index, brute-force graphs, the exactness of
refinement with a complete graph, and dominance over the unrefined
result."""
import numpy as np

import oracle
import synth
from tests.indexfile import write_index


def test_hand_traced_refinement():
    """k = 1, one list holding only doc 0 (score 2); doc 0's neighbour is
    doc 1 (score 3, not in any list): refinement returns doc 1."""
    docs = synth.make_csr([{0: 1.0, 1: 1.0}, {1: 3.0}, {2: 1.0}], dim=4)
    lists = {0: [dict(docs=[0], summary=[(0, 0)], m=1.0, delta=0.0)]}
    ix = oracle.Index(write_index(docs, lists, dim=4))
    qs = synth.make_csr([{0: 1.0, 1: 1.0}], dim=4)
    r = ix.pruned_search(qs, k=1, cut=0, heap_factor=1.0)
    assert r["ids"][0, 0] == 0 and r["scores"][0, 0] == 2.0
    knn = np.array([[1, 2], [0, 2], [0, 1]], dtype=np.uint32)
    r = ix.pruned_search(qs, k=1, cut=0, heap_factor=1.0, knn=knn)
    assert r["ids"][0, 0] == 1 and r["scores"][0, 0] == 3.0
    c = dict(zip(oracle.COUNTER_NAMES, r["counters"][0]))
    assert c["docs_evaluated"] == 1 + 2  # doc 0 by the traversal, docs 1 and 2 by refinement (doc 2 scores 0)
    assert c["nnz_evaluated"] == 2 + 1 + 1
    # padding entries are skipped; a neighbour inside S is not re-scored
    knn2 = np.array([[0xFFFFFFFF, 0], [0, 2], [0, 1]], dtype=np.uint32)
    r = ix.pruned_search(qs, k=1, cut=0, heap_factor=1.0, knn=knn2)
    assert r["ids"][0, 0] == 0 and r["counters"][0][3] == 1


def _dense_knn(docs, kappa):
    D = docs.dense()
    G = D @ D.T
    n = G.shape[0]
    out = np.full((n, kappa), 0xFFFFFFFF, dtype=np.uint32)
    for u in range(n):
        cand = [(-G[u, v], v) for v in range(n) if v != u and G[u, v] > 0]
        cand.sort()
        row = [v for _, v in cand[:kappa]]
        out[u, :len(row)] = row
    return out


def test_exact_graph_matches_dense_brute_force():
    docs = synth.docs(300, seed=11)
    got = oracle.knn_graph(None, docs, 6, 0, 1.0, exact=True)
    assert np.array_equal(got, _dense_knn(docs, 6))


def test_graph_from_search_drops_self_and_pads():
    docs = synth.docs(400, seed=12)
    from paper_2509_24815_amd import Index  # host build only
    ref = oracle.Index(Index.build(docs, lam=100, beta=10, gamma=0.4, seed=1).serialize())
    g = oracle.knn_graph(ref, docs, 5, 10, 0.8)
    n = docs.n_rows
    assert g.shape == (n, 5)
    for u in range(n):
        row = [v for v in g[u] if v != 0xFFFFFFFF]
        assert u not in row and len(set(row)) == len(row)
        assert (g[u][len(row):] == 0xFFFFFFFF).all()


def test_complete_graph_makes_refinement_exact():
    """With every other document as a neighbour, the expanded set of any
    non-empty heap is the whole collection: the result is exact top-k."""
    docs = synth.docs(200, seed=13)
    qs = synth.queries(40, seed=13)
    from paper_2509_24815_amd import Index
    ref = oracle.Index(Index.build(docs, lam=20, beta=4, gamma=0.4, seed=2).serialize())
    n = docs.n_rows
    full = np.array([[v for v in range(n) if v != u] for u in range(n)], dtype=np.uint32)
    r = ref.pruned_search(qs, 5, 3, 0.5, c_cap=3, knn=full)
    e_ids, e_sc = oracle.exact_topk(docs, qs, 5)
    nonempty = r["ids"][:, 0] != 0xFFFFFFFF
    assert nonempty.sum() > 30
    assert np.array_equal(r["ids"][nonempty], e_ids[nonempty])
    assert np.array_equal(r["scores"][nonempty], e_sc[nonempty])


def test_refinement_dominates_plain_result():
    docs = synth.docs(3000, seed=14)
    qs = synth.queries(100, seed=14)
    from paper_2509_24815_amd import Index
    ref = oracle.Index(Index.build(docs, lam=300, beta=15, gamma=0.4, seed=3).serialize())
    knn = oracle.knn_graph(ref, docs, 8, 10, 0.8)
    a = ref.pruned_search(qs, 10, 5, 0.5, c_cap=5)
    b = ref.pruned_search(qs, 10, 5, 0.5, c_cap=5, knn=knn)
    sa = np.where(np.isneginf(a["scores"]), -1, a["scores"])
    sb = np.where(np.isneginf(b["scores"]), -1, b["scores"])
    assert (sb >= sa).all() and (sb > sa).any()
    assert (b["counters"][:, 3] >= a["counters"][:, 3]).all()
    e_ids, _ = oracle.exact_topk(docs, qs, 10)
    rec = lambda ids: np.mean([len(set(x) & set(y)) / 10 for x, y in zip(ids, e_ids)])
    assert rec(b["ids"]) > rec(a["ids"])

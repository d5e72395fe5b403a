"""Pins of the oracle's exact search and of its Algorithm 2 traversal against
brute force, closed forms and hand-traced tiny indexes."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from tests.indexfile import write_index


def _lexsort_topk(scores, k):
    """top-k by (score desc, id asc) over docs with a positive score."""
    out_ids = np.full((scores.shape[0], k), 0xFFFFFFFF, dtype=np.uint32)
    out_sc = np.full((scores.shape[0], k), -np.inf, dtype=np.float32)
    for i, row in enumerate(scores):
        pos = np.nonzero(row > 0)[0]
        order = np.lexsort((pos, -row[pos]))[:k]
        out_ids[i, :len(order)] = pos[order]
        out_sc[i, :len(order)] = row[pos[order]]
    return out_ids, out_sc


@pytest.mark.parametrize("dim", [300, 30522])
def test_exact_topk_matches_dense_brute_force(dim):
    """Definition "Sparse MIPS": an independent dense fp64 matmul ranks the
    same documents with the same scores."""
    docs = synth.generate(400, seed=5, stream=0, mean=30.0, lo=1, hi=200, dim=dim)
    qs = synth.generate(25, seed=5, stream=1, mean=12.0, lo=1, hi=100, dim=dim)
    k = 10
    ids, sc = oracle.exact_topk(docs, qs, k, nthreads=4)
    dense = qs.dense() @ docs.dense().T  # exact: sums of products of fp16 values in range
    e_ids, e_sc = _lexsort_topk(dense.astype(np.float32), k)
    assert np.array_equal(ids, e_ids)
    assert np.array_equal(sc, e_sc)


def test_exact_scores_are_correctly_rounded():
    """The fp64 sum equals the exact rational sum (closed form via Fraction)
    for values in [2^-6, 2^6], so scores are order-independent."""
    docs = synth.docs(200, seed=7)
    qs = synth.queries(5, seed=7)
    assert oracle.value_range_ok(docs) and oracle.value_range_ok(qs)
    ids, sc = oracle.exact_topk(docs, qs, 5, nthreads=2)
    for qi in range(qs.n_rows):
        qt, qv = qs.row(qi)
        qmap = {int(t): Fraction(float(v)) for t, v in zip(qt, qv)}
        for j in range(5):
            if ids[qi, j] == 0xFFFFFFFF:
                continue
            dt, dv = docs.row(int(ids[qi, j]))
            exact = sum((qmap.get(int(t), 0) * Fraction(float(v)) for t, v in zip(dt, dv)), Fraction(0))
            assert np.float32(float(exact)) == sc[qi, j]


def test_exact_padding_and_empty_query():
    docs = synth.make_csr([{1: 1.0}, {2: 2.0}], dim=8)
    qs = synth.make_csr([{}, {5: 1.0}, {1: 0.5, 2: 0.25}], dim=8)
    ids, sc = oracle.exact_topk(docs, qs, 3, nthreads=1)
    assert (ids[0] == 0xFFFFFFFF).all() and np.isneginf(sc[0]).all()
    assert (ids[1] == 0xFFFFFFFF).all()
    assert list(ids[2]) == [0, 1, 0xFFFFFFFF]  # tie 0.5 == 0.5 broken by id
    assert list(sc[2][:2]) == [0.5, 0.5]


def _counterexample_index():
    """k = 1, two lists visited in order (a, b).  List a: block X1 (summary
    score 10, doc score 5) and block X2 (summary 6, doc 11); list b: block Z
    (summary 10.5, doc 12)."""
    a, b = 0, 1
    docs = synth.make_csr([{a: 2.5}, {a: 5.5}, {b: 12.0}], dim=4)
    lists = {
        a: [dict(docs=[0], summary=[(a, 0)], m=5.0, delta=0.0),
            dict(docs=[1], summary=[(a, 0)], m=3.0, delta=0.0)],
        b: [dict(docs=[2], summary=[(b, 0)], m=10.5, delta=0.0)],
    }
    qs = synth.make_csr([{a: 2.0, b: 1.0}], dim=4)
    return oracle.Index(write_index(docs, lists, dim=4)), qs


def test_hand_traced_counterexample_to_monotone_heap_factor():
    """Raising heap_factor does not always raise the result's quality (skip
    rule r * hf < heap.min of Algorithm 2).  Traced by hand:
    hf = 0.5: eval X1 (heap 5); X2: 6*0.5 < 5 stop; Z: 10.5*0.5 >= 5 eval -> 12.
    hf = 1.0: eval X1; X2: 6 >= 5 eval (heap 11); Z: 10.5 < 11 stop -> 11."""
    ix, qs = _counterexample_index()
    r = ix.pruned_search(qs, k=1, cut=0, heap_factor=0.5)
    assert r["ids"][0, 0] == 2 and r["scores"][0, 0] == 12.0
    assert list(r["prefix"][0]) == [1, 1]
    r = ix.pruned_search(qs, k=1, cut=0, heap_factor=1.0)
    assert r["ids"][0, 0] == 1 and r["scores"][0, 0] == 11.0
    assert list(r["prefix"][0]) == [2, 0]
    # no pruning (hf -> +inf) evaluates everything
    r = ix.pruned_search(qs, k=1, cut=0, heap_factor=float("inf"))
    assert r["ids"][0, 0] == 2 and list(r["prefix"][0]) == [2, 1]
    c = dict(zip(oracle.COUNTER_NAMES, r["counters"][0]))
    assert c["blocks_evaluated"] == 3 and c["docs_evaluated"] == 3 and c["cut_len"] == 2


def test_hand_traced_cut_order_and_duplicates():
    """Query cut keeps the largest query values (ties by term id); a document
    reached through two lists stays once in the heap."""
    docs = synth.make_csr([{0: 1.0, 1: 1.0, 2: 1.0}, {0: 0.5}, {3: 4.0}], dim=4)
    lists = {t: [dict(docs=[d for d in range(3) if t in [int(x) for x in docs.row(d)[0]]],
                      summary=[(t, 0)], m=1.0, delta=0.0)] for t in range(4)}
    ix = oracle.Index(write_index(docs, lists, dim=4))
    # values: term 3 -> 2.0, terms 0,1,2 -> 1.0; cut 2 keeps term 3 then term 0
    qs = synth.make_csr([{0: 1.0, 1: 1.0, 2: 1.0, 3: 2.0}], dim=4)
    r = ix.pruned_search(qs, k=3, cut=2, heap_factor=float("inf"))
    assert list(r["ids"][0]) == [2, 0, 1]  # scores 8, 3, 0.5
    assert list(r["scores"][0]) == [8.0, 3.0, 0.5]
    r = ix.pruned_search(qs, k=3, cut=0, heap_factor=float("inf"))
    assert list(r["ids"][0]) == [2, 0, 1]  # doc 0 seen via three lists, kept once
    c = dict(zip(oracle.COUNTER_NAMES, r["counters"][0]))
    assert c["docs_evaluated"] == 5 and c["cut_len"] == 4


def test_hand_traced_block_order_and_stop():
    """Blocks are visited by summary score descending (ties by block index)
    and the first skip ends the list."""
    docs = synth.make_csr([{0: 1.0}, {0: 2.0}, {0: 3.0}, {0: 0.25}], dim=2)
    lists = {0: [dict(docs=[3], summary=[(0, 0)], m=0.5, delta=0.0),   # r 0.5, score .25
                 dict(docs=[0], summary=[(0, 0)], m=4.0, delta=0.0),   # r 4,   score 1
                 dict(docs=[1], summary=[(0, 0)], m=4.0, delta=0.0),   # r 4,   score 2
                 dict(docs=[2], summary=[(0, 0)], m=2.5, delta=0.0)]}  # r 2.5, score 3
    ix = oracle.Index(write_index(docs, lists, dim=2))
    qs = synth.make_csr([{0: 1.0}], dim=2)
    # order: block1 (4), block2 (4), block3 (2.5), block0 (0.5); k=2, hf=1
    # eval b1 -> {1}; eval b2 -> {2,1}; b3: 2.5 >= 1 eval -> {3,2}; b0: .5 < 2 stop
    r = ix.pruned_search(qs, k=2, cut=0, heap_factor=1.0)
    assert list(r["ids"][0]) == [2, 1] and list(r["prefix"][0]) == [3]
    # hf = 0.3: after b2 heap min 1: b3: 2.5*.3 = .75 < 1 stop
    r = ix.pruned_search(qs, k=2, cut=0, heap_factor=0.3)
    assert list(r["ids"][0]) == [1, 0] and list(r["prefix"][0]) == [2]
    c = dict(zip(oracle.COUNTER_NAMES, r["counters"][0]))
    assert c["prune_tests"] == 1 and c["summary_entries"] == 4


def test_quantized_summary_score_reconstruction():
    """r_j = <q, S_j> with S_j reconstructed as m + code * delta: the skip
    decision flips exactly where r * hf crosses the heap minimum."""
    docs = synth.make_csr([{0: 1.0, 1: 1.0}, {0: 1.25}], dim=2)
    lists = {0: [dict(docs=[1], summary=[(0, 0)], m=10.0, delta=0.0),                    # r = 20
                 dict(docs=[0], summary=[(0, 3), (1, 200)], m=0.25, delta=0.125)]}      # r = 13.875
    ix = oracle.Index(write_index(docs, lists, dim=2))
    qs = synth.make_csr([{0: 2.0, 1: 0.5}], dim=2)
    # r = 2*(0.25 + 3*0.125) + 0.5*(0.25 + 200*0.125) = 1.25 + 12.625 = 13.875
    # after the first block the heap (k = 1) holds doc 1 with score 2.5
    r = ix.pruned_search(qs, k=1, cut=1, heap_factor=0.18)     # 13.875 * 0.18 < 2.5: skip
    assert r["ids"][0, 0] == 1 and list(r["prefix"][0]) == [1]
    r = ix.pruned_search(qs, k=1, cut=1, heap_factor=0.1802)   # 2.50028 >= 2.5: evaluate
    assert r["ids"][0, 0] == 0 and r["scores"][0, 0] == 2.5 and list(r["prefix"][0]) == [2]
    c = dict(zip(oracle.COUNTER_NAMES, r["counters"][0]))
    assert c["prune_tests"] == 1 and c["summary_entries"] == 3


def test_near_tie_counter():
    docs = synth.make_csr([{0: 2.0}, {0: 1.0}], dim=2)
    lists = {0: [dict(docs=[0], summary=[(0, 0)], m=4.0, delta=0.0),
                 dict(docs=[1], summary=[(0, 0)], m=2.0, delta=0.0)]}
    ix = oracle.Index(write_index(docs, lists, dim=2))
    qs = synth.make_csr([{0: 1.0}], dim=2)
    # after block 0 heap min = 2; block 1: r = 2, hf = 1 -> 2 == 2 (not < ): evaluated, near tie
    r = ix.pruned_search(qs, k=1, cut=0, heap_factor=1.0)
    c = dict(zip(oracle.COUNTER_NAMES, r["counters"][0]))
    assert c["prune_tests"] == 1 and c["near_tie_tests"] == 1 and list(r["prefix"][0]) == [2]


def test_query_mass_cut_is_the_alpha_mss_of_the_query():
    """alpha_q-MSS cut (Algorithm 2, first step): the cut length equals the
    size of the query's alpha-MSS computed by the sketching routine, and a
    hand-worked query stops where the mass first reaches the target."""
    docs = synth.docs(2000, seed=21)
    qs = synth.queries(60, seed=21)
    from paper_2509_24815_amd import Index
    ix = oracle.Index(Index.build(docs, lam=200, beta=10, gamma=0.4, seed=1).serialize())
    for alpha in (0.2, 0.5, 0.75, 1.0):
        r = ix.pruned_search(qs, 10, 0, 0.8, c_cap=400, query_mass=alpha)
        for i in range(qs.n_rows):
            t, v = qs.row(i)
            keep = oracle.alpha_mss(t, v.astype(np.float16), alpha)
            assert r["counters"][i][7] == keep.sum()
            assert (r["prefix"][i][keep.sum():] == 0).all()
    # values 4, 2, 1, 1 (mass 8): alpha 0.5 -> 1 entry, 0.5 + eps -> 2, 0.76 -> 3, 1 -> 4
    q = synth.make_csr([{0: 1.0, 1: 4.0, 2: 1.0, 3: 2.0}], dim=docs.dim)
    for alpha, m in ((0.5, 1), (0.5001, 2), (0.76, 3), (1.0, 4)):
        r = ix.pruned_search(q, 5, 0, 0.8, c_cap=8, query_mass=alpha)
        assert r["counters"][0][7] == m
    r = ix.pruned_search(q, 5, 2, 0.8, c_cap=8, query_mass=1.0)  # query_cut still caps
    assert r["counters"][0][7] == 2


# oracle switches (oracle.c): exact block summaries <q, phi(B)> over full
# vectors, and a literal "continue" on a skipped block
EXACT_SUMMARIES, CONTINUE = 1, 2


@pytest.fixture(scope="module")
def full_lists():
    """Every list untruncated (lambda = the longest column), in blocks of
    about eight documents."""
    from paper_2509_24815_amd import Index
    docs = synth.generate(1500, seed=21, stream=0, mean=25.0, lo=1, hi=80, dim=400)
    qs = synth.generate(40, seed=21, stream=1, mean=8.0, lo=1, hi=40, dim=400)
    lam = int(np.bincount(docs.terms(), minlength=400).max())  # the longest column: nothing truncated
    ref = oracle.Index(Index.build(docs, lam=lam, beta=lam // 8, gamma=0.4, seed=3).serialize())
    assert ref.check(clustering=True) == ""
    return docs, qs, ref


def test_no_pruning_is_exact_search(full_lists):
    """hf = +inf, full lists, every query entry in the cut: Algorithm 2
    evaluates every document with a shared term, so it is exact search."""
    docs, qs, ref = full_lists
    r = ref.pruned_search(qs, 10, 0, float("inf"))
    e_ids, e_sc = oracle.exact_topk(docs, qs, 10)
    assert np.array_equal(r["ids"], e_ids) and np.array_equal(r["scores"], e_sc)
    d_ids, d_sc = _lexsort_topk((qs.dense() @ docs.dense().T).astype(np.float32), 10)
    assert np.array_equal(r["ids"], d_ids) and np.array_equal(r["scores"], d_sc)


def test_exact_summaries_make_the_rule_rank_safe(full_lists):
    """With r_j = <q, phi(B_j)> (an upper bound of every score in the block)
    and hf = 1, a skipped block holds no document that could enter the
    heap: the result is the exact top-k while blocks are still skipped."""
    docs, qs, ref = full_lists
    e_ids, e_sc = oracle.exact_topk(docs, qs, 10)
    r = ref.pruned_search(qs, 10, 0, 1.0, flags=EXACT_SUMMARIES)
    assert np.array_equal(r["ids"], e_ids) and np.array_equal(r["scores"], e_sc)
    full = ref.pruned_search(qs, 10, 0, float("inf"), flags=EXACT_SUMMARIES)
    assert r["counters"][:, 2].sum() < full["counters"][:, 2].sum()  # the rule did prune


@pytest.mark.parametrize("hf", [0.5, 0.8, 1.0, 1.5])
def test_continue_and_stop_agree(full_lists, hf):
    """Blocks are visited by summary score desc and the heap minimum never
    decreases, so once a block fails the test every later block of the list
    fails too: "continue" and "stop the list" evaluate the same blocks."""
    docs, qs, ref = full_lists
    for flags in (0, EXACT_SUMMARIES):
        a = ref.pruned_search(qs, 10, 0, hf, flags=flags)
        b = ref.pruned_search(qs, 10, 0, hf, flags=flags | CONTINUE)
        assert np.array_equal(a["ids"], b["ids"]) and np.array_equal(a["scores"], b["scores"])
        assert np.array_equal(a["prefix"], b["prefix"])
        assert np.array_equal(a["counters"][:, :5], b["counters"][:, :5])

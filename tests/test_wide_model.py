"""Host-side model of the wide schedule's decomposition, checked against the
oracle's sequential Algorithm 2 (no GPU): each cut list's blocks are sorted
by summary score, the first `depth` of them (limited by an item capacity and
by the window size) are split into chunks whose k best documents are kept,
and the traversal replays the prune decisions in order over windows of
those stored sets — the blocks folded before the top-k fills merged at once,
a window committed whole when its last block passes against the merged
minimum, else block by block — gathering later blocks itself.  The
model's ids, scores, evaluated-prefix lengths and block, document and test
counters must equal the oracle's for every query: the decomposition itself
is exact, independent of the kernels that implement it.  With the heap bound
(the k-th best score of the first chunk of the first list's first block,
evaluated with an empty heap), speculated blocks whose summary score times
heap_factor falls below it are left unscored, and the results still equal
the oracle's."""
import numpy as np
import pytest

import oracle
import synth
from paper_2509_24815_amd import Index
from paper_2509_24815_amd.indexfile import sections


def _collection(n_docs, dim, seed):
    rng = np.random.default_rng(seed)
    p = 1.0 / np.arange(1, dim + 1) ** 1.1
    p /= p.sum()
    rows, words = [0], []
    for _ in range(n_docs):
        terms = np.unique(rng.choice(dim, rng.integers(8, 40), p=p))
        vals = np.clip(rng.lognormal(0.0, 0.6, terms.size), 0.02, 40.0).astype(np.float16)
        words.extend((terms.astype(np.uint32) | (vals.view(np.uint16).astype(np.uint32) << 16)).tolist())
        rows.append(len(words))
    return synth.CSR(np.array(rows, dtype=np.uint64), np.array(words, dtype=np.uint32), dim)


def _half(words):
    return (words >> 16).astype(np.uint16).view(np.float16).astype(np.float64)


class Model:
    def __init__(self, buf):
        s = sections(np.frombuffer(buf, dtype=np.uint8))
        self.s = s
        self.row_ptr = s["row_ptr"].astype(np.int64)
        self.words = s["words"]

    def score(self, q, d):
        w = self.words[self.row_ptr[d]:self.row_ptr[d + 1]]
        t = (w & 0xFFFF).astype(np.int64)
        return np.float32(np.sum(q[t] * _half(w)))

    def summary(self, q, b):
        s = self.s
        e0, e1 = int(s["blk_sum_off"][b]), int(s["blk_sum_off"][b + 1])
        qt = q[s["sum_term"][e0:e1].astype(np.int64)]
        a = float(np.sum(qt))
        bb = float(np.sum(qt * s["sum_code"][e0:e1].astype(np.float64)))
        return np.float32(float(s["blk_m"][b]) * a + float(s["blk_delta"][b]) * bb)

    def docs_of(self, b):
        s = self.s
        return s["postings"][int(s["blk_post_off"][b]):int(s["blk_post_off"][b + 1])].astype(np.int64)


def _merge(H, cands, k):
    """The k best distinct (score desc, id asc) of H and the positive candidates."""
    have = {d for _, d in H}
    pool = list(H) + [c for c in cands if c[0] > 0 and c[1] not in have]
    pool = sorted(set(pool), key=lambda c: (-c[0], c[1]))
    return pool[:k]


def wide_search(m, qrow, k, cut, hf, depth, chunk, nt, max_w, item_cap, bound=False, stats=None):
    """One query through the modelled wide schedule; returns ids, scores,
    prefix and (blocks of cut lists, evaluated blocks, documents, tests)."""
    s = m.s
    q = np.zeros(s["dim"], dtype=np.float64)
    entries = sorted(qrow.items(), key=lambda tv: (-np.float16(tv[1]), tv[0]))
    for t, v in qrow.items():
        q[t] = float(np.float16(v))
    cut_terms = [t for t, _ in entries[:cut]]
    # list pass: sorted blocks of every cut list, speculated prefixes
    lists, used = [], 0
    for t in cut_terms:
        b0, b1 = int(s["list_off"][t]), int(s["list_off"][t + 1])
        order = sorted(range(b1 - b0), key=lambda j: (-m.summary(q, b0 + j), j))
        r = [m.summary(q, b0 + j) for j in order]
        spec = 0
        for p in range(min(len(order), depth)):
            n = len(m.docs_of(b0 + order[p]))
            ch = (n + chunk - 1) // chunk
            if used + ch > item_cap or ch * k > nt:
                break
            used += ch
            spec += 1
        lists.append((b0, order, r, spec))
    # bound: the k-th best score of the first chunk of the first list's
    # first block (0 when it holds fewer than k positive scores); a
    # speculated block other than that one whose r * hf is below it is not
    # scored (its candidate sets are empty)
    lb = 0.0
    if bound and lists and lists[0][1]:
        b0, order = lists[0][0], lists[0][1]
        first = [m.score(q, int(d)) for d in m.docs_of(b0 + order[0])[:chunk]]
        first = sorted([x for x in first if x > 0], reverse=True)
        lb = float(first[k - 1]) if len(first) >= k else 0.0
    skipped = set()
    for ci, (b0, order, r, spec) in enumerate(lists):
        for p in range(spec):
            if (ci > 0 or p > 0) and float(r[p]) * hf < lb:
                skipped.add(b0 + order[p])
    if stats is not None:
        stats["skipped"] = stats.get("skipped", 0) + len(skipped)

    # evaluation pass: each speculated block's chunk top-k sets
    def cands_of(b0, j):
        if b0 + j in skipped:
            return []
        docs = m.docs_of(b0 + j)
        out = []
        for c0 in range(0, len(docs), chunk):
            part = [(m.score(q, int(d)), int(d)) for d in docs[c0:c0 + chunk]]
            out += _merge([], part, k)
        return out
    # traversal
    H, prefix = [], []
    blocks = evaluated = n_docs = tests = 0
    full = lambda: len(H) == k
    hmin = lambda: H[-1][0]
    for b0, order, r, spec in lists:
        nb = len(order)
        blocks += nb
        if nb == 0:
            prefix.append(0)
            continue
        surv = [p for p in range(nb) if not (full() and float(r[p]) * hf < float(hmin()))]
        pos, ev, stop = 0, 0, False
        while pos < len(surv) and not stop:
            if surv[pos] < spec:
                win, tot = [], 0
                while len(win) < max_w and pos + len(win) < len(surv) and surv[pos + len(win)] < spec:
                    p = surv[pos + len(win)]
                    c = (len(m.docs_of(b0 + order[p])) + chunk - 1) // chunk * k
                    if win and tot + c > nt:
                        break
                    win.append(p)
                    tot += c
                cs = [cands_of(b0, order[p]) for p in win]
                if not full():
                    have, run, f = {d for _, d in H}, len(H), 0
                    while f < len(win) and run < k:
                        run += sum(1 for c in cs[f] if c[0] > 0 and c[1] not in have)
                        f += 1
                    H = _merge(H, [c for cc in cs[:f] for c in cc], k)
                    ev += f
                    n_docs += sum(len(m.docs_of(b0 + order[p])) for p in win[:f])
                    pos += f
                    continue
                rf, rl = float(r[win[0]]) * hf, float(r[win[-1]]) * hf
                if len(win) > 1 and rf >= float(hmin()) and rl >= float(hmin()):
                    Hp = _merge(H, [c for cc in cs for c in cc], k)
                    if rl >= float(Hp[-1][0]):
                        H = Hp
                        ev += len(win)
                        tests += len(win)
                        n_docs += sum(len(m.docs_of(b0 + order[p])) for p in win)
                        pos += len(win)
                        continue
                for p, cc in zip(win, cs):
                    if full():
                        tests += 1
                        if float(r[p]) * hf < float(hmin()):
                            stop = True
                            break
                    ev += 1
                    n_docs += len(m.docs_of(b0 + order[p]))
                    H = _merge(H, cc, k)
                if not stop:
                    pos += len(win)
            else:
                p = surv[pos]
                if full():
                    tests += 1
                    if float(r[p]) * hf < float(hmin()):
                        stop = True
                        break
                docs = m.docs_of(b0 + order[p])
                ev += 1
                n_docs += len(docs)
                H = _merge(H, [(m.score(q, int(d)), int(d)) for d in docs], k)
                pos += 1
        if not stop and len(surv) < nb:
            tests += 1
        prefix.append(ev)
        evaluated += ev
    ids = [d for _, d in H] + [0xFFFFFFFF] * (k - len(H))
    scores = [sc for sc, _ in H] + [-np.inf] * (k - len(H))
    return ids, np.array(scores, dtype=np.float32), prefix, (blocks, evaluated, n_docs, tests)


@pytest.fixture(scope="module")
def setup():
    docs = _collection(2500, 300, seed=5)
    ix = Index.build(docs, lam=240, beta=24, gamma=0.4, seed=5)
    buf = ix.serialize()
    ref = oracle.Index(buf)
    rng = np.random.default_rng(6)
    rows = []
    for _ in range(24):
        terms = rng.choice(300, rng.integers(3, 24), replace=False)
        rows.append({int(t): float(v) for t, v in zip(terms, rng.uniform(0.1, 3.0, terms.size))})
    return Model(buf), ref, rows


# blocks of ~10 documents (up to 174) in chunks of 4: multi-chunk blocks,
# speculation cut by the item capacity (20) and by the window size, windows
# folded at once before the top-k fills, committed whole, and replayed
# block by block, and blocks past the speculated ones gathered
@pytest.mark.parametrize("depth,hf,item_cap,nt", [(1, 0.8, 1 << 30, 40), (3, 0.6, 1 << 30, 40),
                                                  (8, 0.9, 1 << 30, 40), (24, 1.5, 1 << 30, 64),
                                                  (8, 0.8, 20, 40), (24, float("inf"), 1 << 30, 64)])
# bound: the speculated blocks below the heap-minimum bound of the first
# list's first chunk are left unscored (8-document chunks, so that the first
# chunk can hold k documents and the bound is active)
@pytest.mark.parametrize("bound", [False, True])
def test_wide_model_equals_algorithm_2(setup, depth, hf, item_cap, nt, bound):
    m, ref, rows = setup
    k, cut = 5, 8
    qs = synth.make_csr(rows, dim=300)
    r = ref.pruned_search(qs, k, cut, hf, c_cap=cut)
    stats = {}
    for i, row in enumerate(rows):
        ids, scores, prefix, (blocks, ev, nd, tests) = wide_search(m, row, k, cut, hf, depth,
                                                                   chunk=8 if bound else 4, nt=nt, max_w=32,
                                                                   item_cap=item_cap, bound=bound, stats=stats)
        assert ids == r["ids"][i].tolist(), i
        assert np.array_equal(scores, r["scores"][i]), i
        n = len(prefix)
        assert prefix == r["prefix"][i][:n].tolist() and not r["prefix"][i][n:].any(), i
        c = r["counters"][i]
        assert (blocks, ev, nd, tests) == (int(c[1]), int(c[2]), int(c[3]), int(c[5])), i
    if bound and depth > 1 and hf != float("inf"):
        assert stats["skipped"] > 0  # the bound did leave blocks unscored

"""Block-major copies of selected lists (seismic_index_copy_lists) through
the C ABI.  With copies of some lists only — every other list of a sample
batch's hot-list order, so that one query mixes lists read from copies and
lists read in place — every schedule (query-major, list-major, wide)
returns the oracle's results and the plain layout's bit for bit, blocks
larger than a workgroup included, and with the learned probe, the
alpha_q cut and refinement.  Also: the byte budget keeps the longest
prefix that fits, argument and state errors, copies of a device-built
index, and freeing exact search's inverted index."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp
from paper_2509_24815_amd import Index, SeismicError, binding, hot_list_order
from paper_2509_24815_amd import probe as P
from tests.gpu_util import as_u32, compare_with_oracle, to_device_csr

pytestmark = pytest.mark.gpu

POINTS = [(10, 0.8, 10), (5, 0.7, 10), (20, 0.9, 100), (10, float("inf"), 10)]


def _log(msg):
    print(msg, flush=True)


def _search(ix, q, k, cut, hf, schedule, window=8, threads=256, **kw):
    import torch
    ws = binding.seismic_workspace_create(ix.handle, max(q.n_rows, 1), max(k, 100))
    try:
        binding.seismic_workspace_set_config(ws, threads, 0, window, schedule)
        out = ix.search(to_device_csr(q), k, cut, hf, trace=True, prefix_stride=cut, ws=ws, **kw)
        torch.cuda.synchronize()
        return [t.cpu().numpy() for t in out]
    finally:
        binding.seismic_workspace_free(ws)


def _same(a, b):
    return all(np.array_equal(x.view(np.uint8), y.view(np.uint8)) for x, y in zip(a, b))


def _every_other_hot(ix, sample, cut, hf):
    import torch
    _, _, prefix, _, _, term = ix.search(to_device_csr(sample), 10, cut, hf, trace=True, prefix_stride=cut)
    torch.cuda.synchronize()
    order = hot_list_order(prefix.cpu().numpy(), term.cpu().numpy())
    assert len(order) > 20
    return order[::2]


def _check_all_schedules(ix, ref, qs, before, points):
    import torch
    for (cut, hf, k), base in zip(points, before):
        _log(f"[copies] cut={cut} hf={hf} k={k}")
        qm = _search(ix, qs, k, cut, hf, 0)
        assert not compare_with_oracle(tuple(torch.from_numpy(x) for x in qm[:4]),
                                       ref.pruned_search(qs, k, cut, hf, c_cap=cut), k, cut)
        assert _same(qm, base)
        assert _same(_search(ix, qs, k, cut, hf, 1), base)
        for threads, depth in ((256, 8), (512, 32)):
            assert _same(_search(ix, qs, k, cut, hf, 2, window=depth, threads=threads), base), (threads, depth)


def test_copies_of_some_lists_change_no_result():
    import torch
    torch.cuda.set_device(0)
    _log("[copies] 100k docs (lambda 1000, beta 50), 300 queries; copies of every other hot list")
    docs = synth.docs(100_000, seed=4)
    qs = synth.queries(200, seed=4)
    qu = synth.queries(100, seed=9, law="uniform")
    q = synth.CSR(np.concatenate([qs.row_ptr, qu.row_ptr[1:] + qs.row_ptr[-1]]),
                  np.concatenate([qs.words, qu.words]), qs.dim)
    ix = Index.build(docs, lam=1000, beta=50, gamma=0.4, seed=4)
    ref = oracle.Index(ix.serialize())
    ix.upload(0)
    before = [_search(ix, q, k, cut, hf, 0) for cut, hf, k in POINTS]
    # the learned probe, the alpha_q cut and refinement read rows through the same gathers
    rng = np.random.default_rng(3)
    p = np.zeros(512, dtype=np.float32)
    p[:mlp.N_USED] = rng.normal(0, 0.6, mlp.N_USED)
    p[320:384] = np.abs(p[320:384])
    w = mlp.float_to_bf16_bits(p)
    ix.set_knn(rng.integers(0, docs.n_rows, (docs.n_rows, 8)).astype(np.uint32))
    variants = [dict(probe=P.to_device(w), probe_tau=0.5), dict(query_mass=0.5, refine=True)]
    before_v = [_search(ix, q, 10, 10, 0.8, 0, **kw) for kw in variants]
    lists = _every_other_hot(ix, synth.queries(400, seed=11), 10, 0.8)
    n, used = ix.copy_lists(lists, 1 << 62)
    _log(f"[copies] {n} of {len(lists)} lists copied, {used} bytes")
    assert n == len(lists) and used > 0
    assert ix.info()["on_device"] == 3
    with pytest.raises(SeismicError):  # copies exist already
        ix.copy_lists(lists[:1], 1 << 62)
    _check_all_schedules(ix, ref, q, before, POINTS)
    for kw, base in zip(variants, before_v):
        _log(f"[copies] {sorted(kw)}")
        assert _same(_search(ix, q, 10, 10, 0.8, 0, **kw), base)
        assert _same(_search(ix, q, 10, 10, 0.8, 1, **kw), base)
        assert _same(_search(ix, q, 10, 10, 0.8, 2, window=16, threads=512, **kw), base)


def test_copies_of_large_blocks():
    # blocks of hundreds to thousands of documents are gathered in chunks of
    # a workgroup, by the traversal and by the wide evaluation pass
    import torch
    torch.cuda.set_device(0)
    docs = synth.docs(30_000, seed=22)
    ix = Index.build(docs, lam=3000, beta=4, gamma=0.4, seed=22)
    ref = oracle.Index(ix.serialize())
    ix.upload(0)
    qs = synth.queries(60, seed=22)
    points = [(5, 0.8, 10), (3, float("inf"), 50), (8, 0.6, 10)]
    before = [_search(ix, qs, k, cut, hf, 0) for cut, hf, k in points]
    lists = _every_other_hot(ix, synth.queries(200, seed=23), 8, 0.8)
    n, _ = ix.copy_lists(lists, 1 << 62)
    assert n == len(lists) and ix.info()["on_device"] == 3
    _check_all_schedules(ix, ref, qs, before, points)


def test_budget_errors_and_full_copies():
    import torch
    torch.cuda.set_device(0)
    docs = synth.docs(20_000, seed=6)
    ix = Index.build(docs, lam=500, beta=20, gamma=0.4, seed=6)
    dim = ix.info()["dim"]
    with pytest.raises(SeismicError):  # not resident yet
        ix.copy_lists([0], 1 << 62)
    ix.upload(0)
    qs = synth.queries(100, seed=6)
    base = _search(ix, qs, 10, 10, 0.8, 0)
    for bad in ([dim], [5, 7, 5]):  # a term id out of range, a list given twice
        with pytest.raises(SeismicError):
            ix.copy_lists(bad, 1 << 62)
    assert ix.info()["on_device"] == 1
    lists_all = np.arange(dim, dtype=np.uint32)
    # a budget below the per-block map copies nothing and leaves the index as it was
    n, used = ix.copy_lists(lists_all, 16)
    assert used == 0 and ix.info()["on_device"] == 1
    assert n < dim
    assert _same(_search(ix, qs, 10, 10, 0.8, 0), base)
    # the budget takes a prefix of the given order
    hot = _every_other_hot(ix, synth.queries(300, seed=12), 10, 0.8)
    n_all, used_all = ix.copy_lists(hot, 1 << 62)
    assert n_all == len(hot)
    ix.close()
    # the same index again, with half of those bytes: a shorter prefix
    ix = Index.build(docs, lam=500, beta=20, gamma=0.4, seed=6)
    ix.upload(0)
    n_half, used_half = ix.copy_lists(hot, used_all // 2)
    assert 0 < n_half < n_all and used_half <= used_all // 2
    assert _same(_search(ix, qs, 10, 10, 0.8, 0), base)
    ix.close()
    # lists without postings count as copied where they stand in the order
    empty = np.setdiff1d(np.arange(dim), np.unique(docs.terms()))
    assert len(empty) >= 2
    ix = Index.build(docs, lam=500, beta=20, gamma=0.4, seed=6)
    ix.upload(0)
    n, used = ix.copy_lists([hot[0], hot[1]], 1)  # nothing fits
    assert (n, used) == (0, 0) and ix.info()["on_device"] == 1
    n, used = ix.copy_lists([empty[0], hot[0], empty[1], hot[1]], 1 << 62)
    assert n == 4 and used > 0 and ix.info()["on_device"] == 3
    assert _same(_search(ix, qs, 10, 10, 0.8, 0), base)
    ix.close()
    # every list: the layout of SEISMIC_UPLOAD_BLOCK_ROWS
    ix = Index.build(docs, lam=500, beta=20, gamma=0.4, seed=6)
    ix.upload(0)
    n, used = ix.copy_lists(lists_all, 1 << 62)
    assert n == dim and ix.info()["on_device"] == 2
    assert _same(_search(ix, qs, 10, 10, 0.8, 0), base)
    full = Index.build(docs, lam=500, beta=20, gamma=0.4, seed=6)
    full.upload(0, block_rows=True)
    assert full.info()["on_device"] == 2
    assert _same(_search(full, qs, 10, 10, 0.8, 0), base)


def test_copies_of_a_device_built_index_and_release_exact():
    import torch
    torch.cuda.set_device(0)
    docs = synth.docs(30_000, seed=7)
    qs = synth.queries(150, seed=7)
    rp = torch.from_numpy(docs.row_ptr.astype(np.int64)).cuda()
    w = torch.from_numpy(docs.words.view(np.int32)).cuda()
    ix = Index.build_device(binding.device_csr(rp, w, docs.dim), 1000, 50, 0.4, seed=7)
    del rp, w
    ref = oracle.Index(ix.serialize())
    assert ix.info()["on_device"] == 1
    ids0, sc0 = ix.exact(to_device_csr(qs), 10)
    ix.release_exact()
    ix.release_exact()  # nothing left to free
    before = [_search(ix, qs, k, cut, hf, 0) for cut, hf, k in POINTS[:2]]
    hot = hot_list_order(*[before[0][i] for i in (2, 5)])
    n, used = ix.copy_lists(hot, 1 << 62)
    assert n == len(hot) and ix.info()["on_device"] in (2, 3)
    _check_all_schedules(ix, ref, qs, before, POINTS[:2])
    ids1, sc1 = ix.exact(to_device_csr(qs), 10)  # built again
    assert np.array_equal(as_u32(ids0), as_u32(ids1))
    assert np.array_equal(sc0.cpu().numpy(), sc1.cpu().numpy())

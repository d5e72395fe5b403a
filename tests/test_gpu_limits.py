"""The library's size limits through the C ABI, against the oracle: the
largest k (SEISMIC_MAX_K), queries of exactly SEISMIC_MAX_QUERY_NNZ
nonzeros and longer ones (the rest ignored and flagged), a list of 4096
blocks (the search sorts 4096 summary scores), and a list beyond the
largest block count the search handles (refused at upload)."""
import numpy as np
import pytest

import oracle
import synth
from paper_2509_24815_amd import Index, SeismicError, binding
from tests.gpu_util import compare_with_oracle, to_device_csr

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def idx():
    import torch
    _log("[limits] 30k-document index (lambda 800, beta 40)")
    docs = synth.docs(30_000, seed=12)
    ix = Index.build(docs, lam=800, beta=40, gamma=0.4, seed=12)
    ref = oracle.Index(ix.serialize())
    torch.cuda.set_device(0)
    ix.upload(0, block_rows=True)
    return docs, ix, ref


def test_largest_k(idx):
    docs, ix, ref = idx
    qs = synth.queries(40, seed=12)
    k = binding.MAX_K
    for cut, hf in ((10, 0.8), (5, float("inf"))):
        _log(f"[limits] k={k} cut={cut} hf={hf}")
        r = ref.pruned_search(qs, k, cut, hf, c_cap=cut)
        gpu = ix.search(to_device_csr(qs), k, cut, hf, stats=True, prefix_stride=cut)
        assert not compare_with_oracle(gpu, r, k, cut)


def test_longest_queries(idx):
    docs, ix, ref = idx
    mx = binding.MAX_QUERY_NNZ
    rng = np.random.default_rng(3)
    rows = []
    for n in (mx, mx + 76):
        terms = np.sort(rng.choice(synth.DIM, n, replace=False))
        rows.append({int(t): float(v) for t, v in zip(terms, rng.uniform(0.1, 3.0, n))})
    long_q = synth.make_csr(rows)
    # the definition of the limit: entries past the first SEISMIC_MAX_QUERY_NNZ are ignored
    cut_rows = [dict(list(r.items())[:mx]) for r in rows]
    trunc = synth.make_csr(cut_rows)
    for cut, hf, k in ((0, 0.8, 10), (10, 0.8, 10), (0, float("inf"), 50)):
        _log(f"[limits] {mx}- and {mx + 76}-nonzero queries, cut={cut} hf={hf} k={k}")
        stride = cut or mx
        r = ref.pruned_search(trunc, k, cut, hf, c_cap=stride)
        gpu = ix.search(to_device_csr(long_q), k, cut, hf, stats=True, prefix_stride=stride)
        assert not compare_with_oracle(gpu, r, k, stride)
        st = gpu[3].cpu().numpy()[:, 6]
        assert st[0] == 0 and st[1] & 4  # SEISMIC_QSTATUS_TOO_LONG


def _one_long_list(n_docs, seed):
    # document d holds term 0 (small value) and its own term d + 1: term 0's
    # list has n_docs postings, and every sampled centroid keeps its own
    # document, so the list has exactly as many blocks as centroids
    rng = np.random.default_rng(seed)
    rows = [{0: 0.02, d + 1: float(rng.uniform(1.0, 4.0))} for d in range(n_docs)]
    return synth.make_csr(rows, dim=n_docs + 1)


def test_list_of_4096_blocks():
    import torch
    docs = _one_long_list(9000, 1)
    _log("[limits] a list of 4096 blocks (9000 postings, beta 4096)")
    ix = Index.build(docs, lam=9000, beta=4096, gamma=0.4, seed=1)
    assert ix.info()["max_blocks_per_list"] == 4096
    ref = oracle.Index(ix.serialize())
    torch.cuda.set_device(0)
    ix.upload(0)
    qrows = [{0: 1.0, 5: 2.0, 9: 0.5}, {0: 3.0}, {3: 1.0, 0: 0.25, 4000: 2.0}]
    qs = synth.make_csr(qrows, dim=docs.dim)
    for cut, hf, k in ((3, 0.8, 10), (3, float("inf"), 100), (1, 0.5, 1)):
        _log(f"[limits] 4096-block list: cut={cut} hf={hf} k={k}")
        r = ref.pruned_search(qs, k, cut, hf, c_cap=cut)
        gpu = ix.search(to_device_csr(qs), k, cut, hf, stats=True, prefix_stride=cut)
        assert not compare_with_oracle(gpu, r, k, cut)


def test_list_beyond_the_search_limit_is_refused():
    docs = _one_long_list(9000, 2)
    ix = Index.build(docs, lam=9000, beta=9000, gamma=0.4, seed=2)
    assert ix.info()["max_blocks_per_list"] == 9000
    with pytest.raises(SeismicError) as e:
        ix.upload(0)
    assert e.value.code == binding.EINVAL


def test_resident_workgroups_follow_lds():
    """Workgroups per CU kept resident by the 256-thread search shape on an
    index whose longest list has 400 blocks (sort capacity 512), as the
    8.8M benchmark index: three at k = 10 and at k = 100 (the top-k merge
    compacts its survivors in place, so three 52 KB workgroups fit a CU),
    fewer at k = 400 (57 KB); results at k = 100 equal the oracle's."""
    import torch
    docs = synth.docs(30_000, seed=3)
    ix = Index.build(docs, lam=2000, beta=400, gamma=0.4, seed=3)
    assert ix.info()["max_blocks_per_list"] == 400
    ref = oracle.Index(ix.serialize())
    torch.cuda.set_device(0)
    ix.upload(0, block_rows=True)
    ws = binding.seismic_workspace_create(ix.handle, 256, 400)
    try:
        binding.seismic_workspace_set_config(ws, 256, 3, 8, 0)
        got = {k: binding.seismic_workspace_resident_per_cu(ws, 5000, k) for k in (10, 100, 400)}
        _log(f"[limits] resident 256-thread workgroups per CU by k: {got}")
        assert got[10] == 3 and got[100] == 3
        assert 1 <= got[400] < 3
        for bad in (0, 401):
            with pytest.raises(SeismicError):
                binding.seismic_workspace_resident_per_cu(ws, 5000, bad)
        qs = synth.queries(200, seed=3, law="uniform")
        out = ix.search(to_device_csr(qs), 100, 20, 1.125, stats=True, prefix_stride=20, ws=ws)
        torch.cuda.synchronize()
        r = ref.pruned_search(qs, 100, 20, 1.125, c_cap=20)
        assert not compare_with_oracle(out, r, 100, 20)
    finally:
        binding.seismic_workspace_free(ws)
        ix.close()

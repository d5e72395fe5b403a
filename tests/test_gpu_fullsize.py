"""Parity at the full sizes of the batched and persistent configurations:
the 1M-document index (10k Poisson(43) queries) and the 8.8M-document index
(7000-query batch of uniform [5, 200] nonzeros, block-major rows), searched
as one batch in the launch shape the benchmark times (256 threads, 3
workgroups per CU, window 8).  The oracle recomputes sampled queries one by
one on the same serialized index: ids, scores, evaluated-prefix lengths and
counters must match bit for bit; exact top-k of sampled queries against the
oracle's brute force over all documents."""
import numpy as np
import pytest

import oracle
import synth
from paper_2509_24815_amd import Index, binding
from tests.gpu_util import as_u32, compare_with_oracle, to_device_csr

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _setup(n_docs, n_queries, law, lam, beta):
    import torch
    torch.cuda.set_device(0)
    _log(f"[full size] generating {n_docs} docs, {n_queries} {law} queries; GPU build (lambda {lam}, beta {beta})")
    docs = synth.docs(n_docs, seed=0)
    qs = synth.queries(n_queries, seed=0, law=law)
    ix = Index.build_gpu(docs, lam, beta, 0.4, seed=0)
    ix.upload(0, block_rows=True)
    _log("[full size] serializing for the oracle")
    ref = oracle.Index(ix.serialize())
    return docs, qs, ix, ref


def _batch_search(ix, qs, k, cut, hf):
    """The whole batch in one launch, in the benchmark's launch shape."""
    import torch
    nq = qs.n_rows
    ws = ix.workspace(nq, max(k, 100))
    binding.seismic_workspace_set_config(ws, 256, 3, 8)
    out = ix.search(to_device_csr(qs), k, cut, hf, stats=True, prefix_stride=cut, ws=ws)
    torch.cuda.synchronize()
    return out


def _check_sampled(qs, ref, gpu, k, cut, hf, sample):
    ids, sc, pref, cnt = gpu
    sub = qs.subset(sample)
    r = ref.pruned_search(sub, k, cut, hf, c_cap=cut)
    picked = (ids[sample], sc[sample], pref[sample], cnt[sample])
    bad = compare_with_oracle(picked, r, k, cut)
    near = int((r["counters"][:, 6] > 0).sum())
    _log(f"  sampled {len(sample)} queries: {len(bad)} mismatching, {near} with near-tie prune tests")
    assert not bad


@pytest.fixture(scope="module")
def cfg_1m():
    return _setup(1_000_000, 10_000, "poisson", 3000, 150)


@pytest.mark.parametrize("cut,hf", [(5, 0.7), (10, 0.8), (20, 0.9)])
def test_parity_1m_batch(cfg_1m, cut, hf):
    docs, qs, ix, ref = cfg_1m
    _log(f"[full size 1M] query_cut {cut}, heap_factor {hf}, 10k-query batch")
    gpu = _batch_search(ix, qs, 10, cut, hf)
    sample = np.linspace(0, qs.n_rows - 1, 96).astype(np.int64)
    _check_sampled(qs, ref, gpu, 10, cut, hf, sample)


@pytest.fixture(scope="module")
def cfg_88m():
    return _setup(8_841_823, 7000, "uniform", 6000, 400)


# (0.75, 10, 10): the benchmark's k = 10 operating point; (1.125, 100, 20):
# its k = 100 operating point (Recall@100 0.9515)
@pytest.mark.parametrize("hf,k,cut", [(0.7, 10, 10), (0.9, 10, 10), (0.7, 100, 10), (0.75, 10, 10), (1.125, 100, 20)])
def test_parity_88m_batch(cfg_88m, hf, k, cut):
    docs, qs, ix, ref = cfg_88m
    _log(f"[full size 8.8M] query_cut {cut}, heap_factor {hf}, k {k}, 7000-query batch")
    gpu = _batch_search(ix, qs, k, cut, hf)
    sample = np.unique(np.concatenate([np.arange(8), np.linspace(0, qs.n_rows - 1, 56).astype(np.int64)]))
    _check_sampled(qs, ref, gpu, k, cut, hf, sample)


def test_exact_88m_sampled(cfg_88m):
    import torch
    docs, qs, ix, ref = cfg_88m
    sample = np.linspace(0, qs.n_rows - 1, 24).astype(np.int64)
    sub = qs.subset(sample)
    _log(f"[full size 8.8M] exact top-10 of {len(sample)} sampled queries vs brute force")
    e_ids, e_sc = ix.exact(to_device_csr(sub), 10)
    torch.cuda.synchronize()
    o_ids, o_sc = oracle.exact_topk(docs, sub, 10)
    assert np.array_equal(as_u32(e_ids), o_ids) and np.array_equal(e_sc.cpu().numpy(), o_sc)

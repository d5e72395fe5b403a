"""The search entry point that allocates nothing
(seismic_search_batch_noalloc), through the C ABI, against
seismic_search_batch with a workspace: two calls in a row (the second with
fewer queries, so stale scratch contents would show), device- and
host-resident queries, the learned probe, and the size limit."""
import numpy as np
import pytest

import oracle
import synth
from paper_2509_24815_amd import Index, SeismicError, binding
from paper_2509_24815_amd import probe as P
from tests.gpu_util import as_u32, to_device_csr

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def setup():
    import torch
    _log("[noalloc] 30k documents, lambda 600, beta 30; 700 queries")
    docs = synth.docs(30_000, seed=12)
    qs = synth.queries(700, seed=12, law="uniform")
    ix = Index.build(docs, lam=600, beta=30, gamma=0.4, seed=12)
    ref = oracle.Index(ix.serialize())
    torch.cuda.set_device(0)
    ix.upload(0, block_rows=True)
    return docs, qs, ix, ref


def _outs(n, k, cut):
    import torch
    # filled with garbage: every slot must be written
    return (torch.full((n, k), 7, dtype=torch.int32, device="cuda"),
            torch.full((n, k), 3.5, dtype=torch.float32, device="cuda"),
            torch.full((n, cut), 999, dtype=torch.int16, device="cuda"),
            torch.full((n, 8), 12345, dtype=torch.int64, device="cuda"))


def _run(fn, ix, q, n, k, cut, hf, ws=None, **kw):
    import torch
    ids, sc, pref, cnt = _outs(n, k, cut)
    if ws is None:
        fn(ix.handle, q, k, cut, hf, ids, sc, prefix=pref, prefix_stride=cut, counters=cnt, **kw)
    else:
        fn(ix.handle, ws, q, k, cut, hf, ids, sc, prefix=pref, prefix_stride=cut, counters=cnt, **kw)
    torch.cuda.synchronize()
    return ids, sc, pref, cnt


def _same(a, b):
    import torch
    return all(torch.equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("k,cut,hf", [(10, 10, 0.8), (50, 20, 0.6)])
def test_noalloc_equals_workspace_search(setup, k, cut, hf):
    docs, qs, ix, ref = setup
    ws = binding.seismic_workspace_create(ix.handle, 700, k)
    try:
        for n in (700, 120):  # two calls in a row, the second smaller
            sub = qs.subset(range(n))
            _log(f"  k {k} cut {cut} hf {hf}: {n} device-resident queries")
            q = to_device_csr(sub)
            a = _run(binding.seismic_search_batch_noalloc, ix, q, n, k, cut, hf)
            b = _run(binding.seismic_search_batch, ix, q, n, k, cut, hf, ws=ws)
            assert _same(a, b), "no-alloc search differs from the workspace search"
            r = ref.pruned_search(sub, k, cut, hf, c_cap=cut)
            assert np.array_equal(as_u32(a[0]), r["ids"]) and np.array_equal(a[1].cpu().numpy(), r["scores"])
            assert np.array_equal(a[2].cpu().numpy().view(np.uint16), r["prefix"])
    finally:
        binding.seismic_workspace_free(ws)


def test_noalloc_host_queries_and_probe(setup):
    docs, qs, ix, ref = setup
    rng = np.random.default_rng(3)
    p = np.zeros(512, np.float32)
    p[:449] = rng.normal(0, 0.5, 449)
    p[320:384] = np.abs(p[320:384])
    w = P.to_device(P.bf16_bits(p))
    ws = binding.seismic_workspace_create(ix.handle, 700, 10)
    try:
        for n in (500, 60):
            sub = qs.subset(range(n))
            _log(f"  {n} host-resident queries, plain and learned")
            hq = binding.host_csr(sub.row_ptr, sub.words, sub.dim)
            for kw in ({}, {"probe": w, "probe_tau": 0.0}):
                a = _run(binding.seismic_search_batch_noalloc, ix, hq, n, 10, 10, 0.8, **kw)
                b = _run(binding.seismic_search_batch, ix, to_device_csr(sub), n, 10, 10, 0.8, ws=ws, **kw)
                assert _same(a, b)
    finally:
        binding.seismic_workspace_free(ws)


def test_noalloc_limits(setup):
    import torch
    docs, qs, ix, ref = setup
    n = binding.NOALLOC_MAX_ROWS + 1
    rp = np.zeros(n + 1, dtype=np.uint64)  # empty rows: only the row count is too large
    ids = torch.empty((n, 10), dtype=torch.int32, device="cuda")
    sc = torch.empty((n, 10), dtype=torch.float32, device="cuda")
    with pytest.raises(SeismicError) as e:
        binding.seismic_search_batch_noalloc(ix.handle, binding.host_csr(rp, np.zeros(0, np.uint32), docs.dim),
                                             10, 10, 0.8, ids, sc)
    assert e.value.code == binding.EINVAL and "exceed the scratch" in str(e.value)
    with pytest.raises(SeismicError):
        binding.seismic_search_batch_noalloc(ix.handle, to_device_csr(qs.subset(range(4))), 0, 10, 0.8, ids, sc)
    # the same number of rows on the device is fine (no staging)
    big = synth.queries(n, seed=13, law="uniform")
    q = to_device_csr(big)
    binding.seismic_search_batch_noalloc(ix.handle, q, 10, 10, 0.8, ids, sc)
    torch.cuda.synchronize()
    x_ids, x_sc = ix.search(q, 10, 10, 0.8)
    assert torch.equal(ids, x_ids) and torch.equal(sc, x_sc)

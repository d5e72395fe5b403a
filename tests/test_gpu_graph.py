"""GPU tests of graph-captured search batches: one captured graph replayed
for batches of different sizes and contents, with eager work and
synchronizations between the replays; every replay must equal the eager
search of the same batch."""
import numpy as np
import pytest

import synth
from paper_2509_24815_amd import Index, SeismicError, binding
from paper_2509_24815_amd import probe as P
from tests.gpu_util import as_u32, to_device_csr

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def idx():
    import torch
    _log("[graph] building a 30k-document index (lambda 600, beta 30)")
    docs = synth.docs(30_000, seed=6)
    qs = synth.queries(1200, seed=6, law="uniform")
    ix = Index.build(docs, lam=600, beta=30, gamma=0.4, seed=6)
    torch.cuda.set_device(0)
    ix.upload(0, block_rows=True)
    return qs, ix


@pytest.mark.parametrize("learned", [False, True])
def test_graph_replays_equal_eager(idx, learned):
    import torch
    qs, ix = idx
    cap, k = 300, 10
    probe = None
    if learned:
        rng = np.random.default_rng(9)
        p = np.zeros(512, np.float32)
        p[:449] = rng.normal(0, 0.5, 449)
        p[320:384] = np.abs(p[320:384])
        probe = P.to_device(P.bf16_bits(p))
    sets = [(0, 300), (300, 120), (420, 7), (500, 300), (900, 1), (0, 300)]
    max_nnz = max(int(qs.row_ptr[s + n] - qs.row_ptr[s]) for s, n in sets)
    rp = torch.zeros(cap + 1, dtype=torch.int64, device="cuda")
    words = torch.zeros(max_nnz, dtype=torch.int32, device="cuda")
    nq = torch.zeros(1, dtype=torch.int32, device="cuda")
    ids = torch.full((cap, k), -1, dtype=torch.int32, device="cuda")
    sc = torch.zeros((cap, k), dtype=torch.float32, device="cuda")
    ws = binding.seismic_workspace_create(ix.handle, cap, k)
    buf = binding.device_csr(rp, words, qs.dim)
    g = binding.seismic_graph_create(ix.handle, ws, buf, nq, k, 10, 0.8, ids, sc, probe=probe, probe_tau=0.0)
    try:
        for rep, (s, n) in enumerate(sets):
            sub = qs.subset(range(s, s + n))
            rp[:n + 1].copy_(torch.from_numpy(sub.row_ptr.astype(np.int64)))
            words[:sub.nnz].copy_(torch.from_numpy(sub.words.view(np.int32)))
            nq.fill_(n)
            # eager work between replays: the same batch through search_batch
            e_ids, e_sc = ix.search(to_device_csr(sub), k, 10, 0.8, probe=probe, probe_tau=0.0)
            torch.cuda.synchronize()
            binding.seismic_graph_launch(g)
            torch.cuda.synchronize()
            assert np.array_equal(as_u32(ids)[:n], as_u32(e_ids)), f"replay {rep}"
            assert np.array_equal(sc.cpu().numpy()[:n], e_sc.cpu().numpy()), f"replay {rep}"
            _log(f"  replay {rep}: {n} queries equal to the eager search")
    finally:
        binding.seismic_graph_free(g)
        binding.seismic_workspace_free(ws)


def test_graph_rejects_host_queries(idx):
    import torch
    qs, ix = idx
    ws = binding.seismic_workspace_create(ix.handle, 8, 10)
    nq = torch.zeros(1, dtype=torch.int32, device="cuda")
    ids = torch.empty((8, 10), dtype=torch.int32, device="cuda")
    sc = torch.empty((8, 10), dtype=torch.float32, device="cuda")
    sub = qs.subset(range(8))
    with pytest.raises(SeismicError):
        binding.seismic_graph_create(ix.handle, ws, binding.host_csr(sub.row_ptr, sub.words, sub.dim), nq, 10, 10,
                                     0.8, ids, sc)
    binding.seismic_workspace_free(ws)


def test_served_without_graphs_equals_with_graphs(idx):
    qs, ix = idx
    out = []
    for use_graphs in (True, False):
        sv = binding.seismic_server_create(ix.handle, 10, 10, 0.8, max_batch=50, n_slots=3, use_graphs=use_graphs)
        try:
            t0 = binding.seismic_server_clock(sv)
            arr = t0 + 0.02 + np.cumsum(np.random.default_rng(3).exponential(1 / 30000.0, qs.n_rows))
            first = binding.seismic_server_submit_batch(sv, binding.host_csr(qs.row_ptr, qs.words, qs.dim), arr)
            binding.seismic_server_wait_all(sv, 120.0)
            out.append(binding.seismic_server_results(sv, first, qs.n_rows, 10))
        finally:
            binding.seismic_server_free(sv)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])

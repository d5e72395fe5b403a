"""GPU tests of the kappa-NN graph (Section 4.3) and the refinement step of
Algorithm 2 through the C ABI: the graph the GPU builds by searching every
document equals the oracle's, refined search equals the oracle's refined
search bit for bit (ids, scores, counters), including inside a captured
graph."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp
from paper_2509_24815_amd import Index, SeismicError, binding
from paper_2509_24815_amd import probe as P
from tests.gpu_util import as_u32, compare_with_oracle, to_device_csr

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def idx():
    import torch
    _log("[knn] building a 20k-document index (lambda 500, beta 25)")
    docs = synth.docs(20_000, seed=8)
    qs = synth.queries(300, seed=8)
    ix = Index.build(docs, lam=500, beta=25, gamma=0.4, seed=8)
    ref = oracle.Index(ix.serialize())
    torch.cuda.set_device(0)
    ix.upload(0, block_rows=True)
    return docs, qs, ix, ref


def test_knn_build_matches_oracle(idx):
    docs, qs, ix, ref = idx
    _log("[knn] GPU graph build (kappa 12, cut 8, hf 0.9) vs the oracle's")
    ix.build_knn(12, 8, 0.9)
    g = ix.knn()
    o = oracle.knn_graph(ref, docs, 12, 8, 0.9)
    assert g.shape == (docs.n_rows, 12)
    assert np.array_equal(g, o)
    assert (g[:, 0] != 0xFFFFFFFF).mean() > 0.99


@pytest.mark.parametrize("kappa,k,cut,hf", [(12, 10, 10, 0.8), (20, 10, 5, 0.6), (4, 50, 10, 0.8), (1, 1, 3, 1.5)])
def test_refined_search_parity(idx, kappa, k, cut, hf):
    docs, qs, ix, ref = idx
    rng = np.random.default_rng(kappa)
    # an arbitrary graph (with padding and out-of-range entries) exercises the rule itself
    table = rng.integers(0, docs.n_rows, (docs.n_rows, kappa)).astype(np.uint32)
    table[rng.random(table.shape) < 0.1] = 0xFFFFFFFF
    ix.set_knn(table)
    _log(f"[knn parity] kappa={kappa} k={k} cut={cut} hf={hf}")
    r = ref.pruned_search(qs, k, cut, hf, c_cap=cut, knn=table)
    gpu = ix.search(to_device_csr(qs), k, cut, hf, stats=True, prefix_stride=cut, refine=True)
    assert not compare_with_oracle(gpu, r, k, cut)
    plain = ref.pruned_search(qs, k, cut, hf, c_cap=cut)
    assert (r["counters"][:, 3] > plain["counters"][:, 3]).any()


def test_refinement_with_search_built_graph_raises_recall(idx):
    docs, qs, ix, ref = idx
    table = oracle.knn_graph(ref, docs, 10, 10, 0.8)  # the graph as the method builds it
    ix.set_knn(table)
    r = ref.pruned_search(qs, 10, 5, 0.4, c_cap=5, knn=table)
    ids, sc, pref, cnt = ix.search(to_device_csr(qs), 10, 5, 0.4, stats=True, prefix_stride=5, refine=True)
    assert not compare_with_oracle((ids, sc, pref, cnt), r, 10, 5)
    e_ids, _ = ix.exact(to_device_csr(qs), 10)
    ex = as_u32(e_ids)
    rec = lambda x: np.mean([len(set(a) & set(b)) / 10 for a, b in zip(x, ex)])
    p_ids, _ = ix.search(to_device_csr(qs), 10, 5, 0.4)
    _log(f"  Recall@10 cut 5 hf 0.4: plain {rec(as_u32(p_ids)):.4f}, refined {rec(as_u32(ids)):.4f}")
    assert rec(as_u32(ids)) > rec(as_u32(p_ids))


@pytest.mark.parametrize("tau,qmass,cut", [(-1.0, 0.0, 10), (0.0, 0.5, 30), (1.0, 0.3, 30)])
def test_refined_learned_search_parity(idx, tau, qmass, cut):
    """Every mode at once: the learned probe decides block visits, the
    alpha_q-MSS cut (or the fixed cut) selects lists, and the graph refines
    the result; ids, scores, counters and per-list heap minima as the
    oracle's."""
    docs, qs, ix, ref = idx
    rng = np.random.default_rng(7)
    p = np.zeros(512, dtype=np.float32)
    p[:mlp.N_USED] = rng.normal(0, 0.6, mlp.N_USED)
    p[320:384] = np.abs(p[320:384])  # b1 > 0: units active on non-negative features
    w = mlp.float_to_bf16_bits(p)
    table = oracle.knn_graph(ref, docs, 8, 10, 0.8)
    ix.set_knn(table)
    _log(f"[knn+probe parity] tau={tau} query_mass={qmass} cut={cut}")
    r = ref.pruned_search(qs, 10, cut, 0.8, c_cap=cut, probe=w, tau=tau, knn=table, query_mass=qmass)
    ids, sc, pref, cnt, hmin, term = ix.search(to_device_csr(qs), 10, cut, 0.8, trace=True, prefix_stride=cut,
                                               probe=P.to_device(w), probe_tau=tau, refine=True,
                                               query_mass=qmass)
    assert not compare_with_oracle((ids, sc, pref, cnt), r, 10, cut)
    assert np.array_equal(hmin.cpu().numpy(), r["hmin"])
    assert (r["hmin"] >= 0).any()


def test_refinement_inside_graph_replays(idx):
    import torch
    docs, qs, ix, ref = idx
    ix.build_knn(10, 10, 0.8)
    cap, k = 200, 10
    sub = qs.subset(range(cap))
    rp = torch.from_numpy(sub.row_ptr.astype(np.int64)).cuda()
    words = torch.from_numpy(sub.words.view(np.int32)).cuda()
    nq = torch.zeros(1, dtype=torch.int32, device="cuda")
    ids = torch.empty((cap, k), dtype=torch.int32, device="cuda")
    sc = torch.empty((cap, k), dtype=torch.float32, device="cuda")
    ws = binding.seismic_workspace_create(ix.handle, cap, k)
    p = binding._params(k, 10, 0.8, binding.SEARCH_KNN)
    import ctypes
    g = ctypes.c_void_p()
    binding._check(binding.load().seismic_graph_create(ix.handle, ws, ctypes.byref(binding.device_csr(rp, words, sub.dim)),
                                                       binding._ptr(nq), ctypes.byref(p), binding._ptr(ids),
                                                       binding._ptr(sc), None, ctypes.byref(g)))
    try:
        for n in (200, 37, 200):
            nq.fill_(n)
            e_ids, e_sc = ix.search(to_device_csr(sub.subset(range(n))), k, 10, 0.8, refine=True)
            torch.cuda.synchronize()
            binding.seismic_graph_launch(g.value)
            torch.cuda.synchronize()
            assert np.array_equal(as_u32(ids)[:n], as_u32(e_ids)) and np.array_equal(sc.cpu().numpy()[:n], e_sc.cpu().numpy())
    finally:
        binding.seismic_graph_free(g.value)
        binding.seismic_workspace_free(ws)


def test_refinement_argument_errors():
    import torch
    docs = synth.docs(2000, seed=9)
    ix = Index.build(docs, lam=200, beta=10, gamma=0.4, seed=9)
    ix.upload(0)
    q = to_device_csr(synth.queries(4, seed=9))
    with pytest.raises(SeismicError) as e:
        ix.search(q, 10, 10, 0.8, refine=True)
    assert e.value.code == binding.ESTATE
    ix.set_knn(np.zeros((docs.n_rows, 30), dtype=np.uint32))
    with pytest.raises(SeismicError) as e:
        ix.search(q, 10, 10, 0.8, refine=True)  # 10 * 30 > 256
    assert e.value.code == binding.EINVAL
    with pytest.raises(SeismicError):
        ix.set_knn(np.zeros((docs.n_rows, 300), dtype=np.uint32))

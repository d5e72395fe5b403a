"""The wide schedule (launch config schedule = 2) through the C ABI: every
search result, prefix length, counter and trace entry equal to the oracle's
and to the query-major schedule's — over cut/heap_factor/k points,
speculation depths from 1 to 64, both workgroup sizes, blocks larger than a
workgroup, a batch that needs more evaluation items than the workspace
holds, long queries (bitmap lookup), the learned probe, the alpha_q cut,
refinement, edge queries, a device-side batch size inside graph replays,
the fallbacks outside its limits, and the autotuner (which tries it on
small batches and requires equal results)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp
from paper_2509_24815_amd import Index, binding
from paper_2509_24815_amd import probe as P
from tests.gpu_util import as_u32, compare_with_oracle, to_device_csr

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    _log("[wide] 100k docs (lambda 1000, beta 50), 200 Poisson(43) + 100 uniform queries")
    docs = synth.docs(100_000, seed=3)
    qs = synth.queries(200, seed=3)
    qu = synth.queries(100, seed=8, law="uniform")
    ix = Index.build(docs, lam=1000, beta=50, gamma=0.4, seed=3)
    ref = oracle.Index(ix.serialize())
    torch.cuda.set_device(0)
    ix.upload(0, block_rows=True)
    return docs, qs, qu, ix, ref


def _search(ix, q, k, cut, hf, schedule, window=8, threads=256, max_k=100, **kw):
    import torch
    ws = binding.seismic_workspace_create(ix.handle, max(q.n_rows, 1), max(k, max_k))
    try:
        binding.seismic_workspace_set_config(ws, threads, 0, window, schedule)
        stride = kw.pop("stride", cut or binding.MAX_QUERY_NNZ)
        out = ix.search(to_device_csr(q), k, cut, hf, trace=True, prefix_stride=stride, ws=ws, **kw)
        torch.cuda.synchronize()
        return [t.cpu().numpy() for t in out]
    finally:
        binding.seismic_workspace_free(ws)


def _same(a, b):
    return all(np.array_equal(x.view(np.uint8), y.view(np.uint8)) for x, y in zip(a, b))


def _oracle_check(res, r, k, cut):
    import torch
    assert not compare_with_oracle(tuple(torch.from_numpy(x) for x in res[:4]), r, k, cut)
    assert np.array_equal(res[4], r["hmin"])


@pytest.mark.parametrize("cut,hf,k", [(10, 0.8, 10), (5, 0.7, 10), (20, 0.9, 10), (10, 0.8, 64),
                                      (1, 0.8, 10), (10, float("inf"), 10), (3, 1.5, 1), (32, 0.8, 10)])
def test_wide_equals_oracle_and_query_major(env, cut, hf, k):
    docs, qs, qu, ix, ref = env
    for name, q in (("poisson", qs), ("uniform", qu)):
        _log(f"[wide] {name} cut={cut} hf={hf} k={k}")
        qm = _search(ix, q, k, cut, hf, 0)
        r = ref.pruned_search(q, k, cut, hf, c_cap=cut)
        _oracle_check(qm, r, k, cut)
        for threads, depth in ((256, 8), (512, 32), (256, 1), (512, 64)):
            wd = _search(ix, q, k, cut, hf, 2, window=depth, threads=threads)
            assert _same(wd, qm), (threads, depth)


def test_wide_large_blocks():
    # blocks of hundreds to thousands of documents: the evaluation pass
    # scores a block in several workgroup-sized chunks, and with a shallow
    # speculation depth the traversal evaluates later large blocks itself
    docs = synth.docs(30_000, seed=21)
    ix = Index.build(docs, lam=3000, beta=4, gamma=0.4, seed=21)
    ref = oracle.Index(ix.serialize())
    ix.upload(0, block_rows=True)
    qs = synth.queries(60, seed=21)
    for cut, hf, k in ((5, 0.8, 10), (3, float("inf"), 50), (8, 0.6, 10)):
        _log(f"[wide] large blocks cut={cut} hf={hf} k={k}")
        qm = _search(ix, qs, k, cut, hf, 0)
        _oracle_check(qm, ref.pruned_search(qs, k, cut, hf, c_cap=cut), k, cut)
        for threads, depth in ((256, 1), (512, 2), (256, 64)):
            assert _same(_search(ix, qs, k, cut, hf, 2, window=depth, threads=threads), qm), (threads, depth)


def test_wide_item_capacity():
    # a one-query workspace holds 8192 evaluation items; every document holds
    # the query's 32 terms, so each of its 32 cut lists has ~64 blocks and at
    # least 70000 / 256 = 274 chunks: the later lists find the capacity used
    # up, speculate fewer blocks (reserved items become no-ops) and the
    # traversal gathers the rest itself (blocks larger than a workgroup too)
    n, shared, noise = 70_000, 32, 1000
    rng = np.random.default_rng(31)
    terms = np.empty((n, shared + 1), dtype=np.uint32)
    terms[:, :shared] = np.arange(shared, dtype=np.uint32)
    terms[:, shared] = shared + rng.integers(0, noise, n)
    vals = np.clip(rng.lognormal(0.0, 0.6, (n, shared + 1)), 0.02, 40.0).astype(np.float16)
    words = (terms | (vals.view(np.uint16).astype(np.uint32) << 16)).reshape(-1)
    rp = np.arange(0, n * (shared + 1) + 1, shared + 1, dtype=np.uint64)
    docs = synth.CSR(rp, words, shared + noise)
    _log("[wide] 70k documents sharing 32 terms (lambda 70000, beta 64)")
    ix = Index.build(docs, lam=n, beta=64, gamma=0.4, seed=31)
    ref = oracle.Index(ix.serialize())
    ix.upload(0, block_rows=True)
    q = synth.make_csr([{t: float(v) for t, v in zip(range(shared), rng.uniform(0.5, 3.0, shared))}],
                       dim=docs.dim)
    for hf, k in ((0.8, 10), (float("inf"), 10), (0.6, 64)):
        _log(f"[wide] item capacity: hf={hf} k={k}")
        qm = _search(ix, q, k, 32, hf, 0)
        _oracle_check(qm, ref.pruned_search(q, k, 32, hf, c_cap=32), k, 32)
        for threads in (512, 256):
            assert _same(_search(ix, q, k, 32, hf, 2, window=64, threads=threads), qm), threads


def test_wide_edge_queries(env):
    docs, qs, qu, ix, ref = env
    rng = np.random.default_rng(4)
    long_terms = np.sort(rng.choice(synth.DIM, 700, replace=False))
    rows = [{}, {30521: 1.0}, {0: 2.0}, {t: 1.0 + (t % 7) * 0.25 for t in range(0, 600, 2)}, {},
            {int(t): float(v) for t, v in zip(long_terms, rng.uniform(0.1, 3.0, 700))}, {5: 0.5}]
    eq = synth.make_csr(rows)
    for cut, hf, k in ((2, float("inf"), 5), (10, 0.8, 64), (32, 0.8, 10)):
        _log(f"[wide] edge queries cut={cut} hf={hf} k={k}")
        qm = _search(ix, eq, k, cut, hf, 0)
        _oracle_check(qm, ref.pruned_search(eq, k, cut, hf, c_cap=cut), k, cut)
        for threads, depth in ((256, 4), (512, 64)):
            assert _same(_search(ix, eq, k, cut, hf, 2, window=depth, threads=threads), qm)


def test_wide_fallbacks(env):
    # outside the wide schedule's limits the batch runs query-major
    docs, qs, qu, ix, ref = env
    sub = qs.subset(range(40))
    for cut, hf, k, stride in ((0, 0.8, 10, 600), (40, 0.8, 10, 40), (10, 0.8, 100, 10)):
        _log(f"[wide] fallback cut={cut} k={k}")
        assert _same(_search(ix, sub, k, cut, hf, 2, window=16, stride=stride),
                     _search(ix, sub, k, cut, hf, 0, stride=stride))
    big = synth.queries(300, seed=9)
    _log("[wide] fallback: 300-query batch")
    assert _same(_search(ix, big, 10, 10, 0.8, 2, window=16), _search(ix, big, 10, 10, 0.8, 0))


def test_wide_probe_mass_refine(env):
    docs, qs, qu, ix, ref = env
    rng = np.random.default_rng(7)
    p = np.zeros(512, dtype=np.float32)
    p[:mlp.N_USED] = rng.normal(0, 0.6, mlp.N_USED)
    p[320:384] = np.abs(p[320:384])
    w = mlp.float_to_bf16_bits(p)
    table = rng.integers(0, docs.n_rows, (docs.n_rows, 8)).astype(np.uint32)
    ix.set_knn(table)
    sub = qs.subset(range(150))
    for tau, qmass, cut, refine in ((0.0, 0.0, 10, False), (1.0, 0.5, 20, True), (-1.0, 0.0, 10, True),
                                    (0.5, 0.0, 5, False)):
        _log(f"[wide] probe tau={tau} query_mass={qmass} cut={cut} refine={refine}")
        kw = dict(probe=P.to_device(w), probe_tau=tau, query_mass=qmass, refine=refine)
        qm = _search(ix, sub, 10, cut, 0.8, 0, **kw)
        r = ref.pruned_search(sub, 10, cut, 0.8, c_cap=cut, probe=w, tau=tau, query_mass=qmass,
                              knn=table if refine else None)
        import torch
        assert not compare_with_oracle(tuple(torch.from_numpy(x) for x in qm[:4]), r, 10, cut)
        for threads, depth in ((256, 8), (512, 2)):
            assert _same(_search(ix, sub, 10, cut, 0.8, 2, window=depth, threads=threads, **kw), qm)


def test_wide_graph_replays(env):
    import torch
    docs, qs, qu, ix, ref = env
    cap, k = 200, 10
    sets = [(0, 200), (50, 120), (120, 7), (0, 1), (199, 1), (10, 200 - 10), (0, 200)]
    max_nnz = max(int(qs.row_ptr[s + n] - qs.row_ptr[s]) for s, n in sets)
    rp = torch.zeros(cap + 1, dtype=torch.int64, device="cuda")
    words = torch.zeros(max_nnz, dtype=torch.int32, device="cuda")
    nq = torch.zeros(1, dtype=torch.int32, device="cuda")
    ids = torch.full((cap, k), -1, dtype=torch.int32, device="cuda")
    sc = torch.zeros((cap, k), dtype=torch.float32, device="cuda")
    ws = binding.seismic_workspace_create(ix.handle, cap, k)
    binding.seismic_workspace_set_config(ws, 512, 0, 16, 2)
    g = binding.seismic_graph_create(ix.handle, ws, binding.device_csr(rp, words, qs.dim), nq, k, 10, 0.8, ids, sc)
    try:
        for s, n in sets:
            _log(f"[wide] graph replay of {n} queries from {s}")
            sub = qs.subset(range(s, s + n))
            rp[:n + 1].copy_(torch.from_numpy(sub.row_ptr.astype(np.int64)))
            words[:sub.nnz].copy_(torch.from_numpy(sub.words.view(np.int32)))
            nq.fill_(n)
            e_ids, e_sc = ix.search(to_device_csr(sub), k, 10, 0.8)
            torch.cuda.synchronize()
            binding.seismic_graph_launch(g)
            torch.cuda.synchronize()
            assert np.array_equal(as_u32(ids)[:n], as_u32(e_ids)) and np.array_equal(sc.cpu().numpy()[:n],
                                                                                      e_sc.cpu().numpy())
    finally:
        binding.seismic_graph_free(g)
        binding.seismic_workspace_free(ws)


def test_autotune_tries_wide(env):
    import torch
    docs, qs, qu, ix, ref = env
    sub = qs.subset(range(64))
    ws = binding.seismic_workspace_create(ix.handle, sub.n_rows, 10)
    ids = torch.empty((sub.n_rows, 10), dtype=torch.int32, device="cuda")
    sc = torch.empty((sub.n_rows, 10), dtype=torch.float32, device="cuda")
    try:
        res = binding.seismic_autotune(ix.handle, ws, to_device_csr(sub), 10, 10, 0.8, ids, sc, reps=1)
        assert {r[0]["schedule"] for r in res} == {0, 1, 2}
        assert {r[0]["window"] for r in res if r[0]["schedule"] == 2} == {8, 16, 32, 64}
        _log(f"[wide] autotune picked {binding.seismic_workspace_get_config(ws, sub.n_rows)}")
    finally:
        binding.seismic_workspace_free(ws)

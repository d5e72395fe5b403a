"""The list-major schedule (launch config schedule = 1) through the C ABI:
every search result, prefix length, counter and trace entry equal to the
oracle's and to the query-major schedule's — over cut/heap_factor/k points,
the learned probe, the alpha_q cut, refinement, edge queries (no cut list,
cut 1), a device-side batch size inside graph replays, and the autotuner
(which tries both schedules and requires equal results)."""
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
    _log("[schedule] 100k docs (lambda 1000, beta 50), 1000 Poisson(43) + 300 uniform queries")
    docs = synth.docs(100_000, seed=0)
    qs = synth.queries(1000, seed=0)
    qu = synth.queries(300, seed=5, law="uniform")
    ix = Index.build(docs, lam=1000, beta=50, gamma=0.4, seed=0)
    ref = oracle.Index(ix.serialize())
    torch.cuda.set_device(0)
    ix.upload(0, block_rows=True)
    return docs, qs, qu, ix, ref


def _search(ix, q, k, cut, hf, schedule, **kw):
    import torch
    ws = binding.seismic_workspace_create(ix.handle, max(q.n_rows, 1), max(k, 100))
    try:
        binding.seismic_workspace_set_config(ws, 256, 0, 8, schedule)
        stride = kw.pop("stride", cut or binding.MAX_QUERY_NNZ)
        out = ix.search(to_device_csr(q), k, cut, hf, trace=True, prefix_stride=stride, ws=ws, **kw)
        torch.cuda.synchronize()
        return [t.cpu().numpy() for t in out]
    finally:
        binding.seismic_workspace_free(ws)


def _same(a, b):
    return all(np.array_equal(x.view(np.uint8), y.view(np.uint8)) for x, y in zip(a, b))


@pytest.mark.parametrize("cut,hf,k", [(10, 0.8, 10), (5, 0.7, 10), (20, 0.9, 10), (10, 0.8, 100),
                                      (1, 0.8, 10), (10, float("inf"), 10), (3, 1.5, 1)])
def test_list_major_equals_oracle_and_query_major(env, cut, hf, k):
    docs, qs, qu, ix, ref = env
    for name, q in (("poisson", qs), ("uniform", qu)):
        _log(f"[schedule] {name} cut={cut} hf={hf} k={k}")
        lm = _search(ix, q, k, cut, hf, 1)
        qm = _search(ix, q, k, cut, hf, 0)
        assert _same(lm, qm)
        r = ref.pruned_search(q, k, cut, hf, c_cap=cut)
        import torch
        gpu = tuple(torch.from_numpy(x) for x in lm[:4])
        assert not compare_with_oracle(gpu, r, k, cut)
        assert np.array_equal(lm[4], r["hmin"])


def test_list_major_edge_queries(env):
    docs, qs, qu, ix, ref = env
    rows = [{}, {30521: 1.0}, {0: 2.0}, {t: 1.0 + (t % 7) * 0.25 for t in range(0, 600, 2)}, {}, {5: 0.5}]
    eq = synth.make_csr(rows)
    for cut, hf, k in ((2, float("inf"), 5), (10, 0.8, 64), (64, 0.8, 10)):
        _log(f"[schedule] edge queries cut={cut} hf={hf} k={k}")
        lm = _search(ix, eq, k, cut, hf, 1)
        assert _same(lm, _search(ix, eq, k, cut, hf, 0))
        r = ref.pruned_search(eq, k, cut, hf, c_cap=cut)
        import torch
        assert not compare_with_oracle(tuple(torch.from_numpy(x) for x in lm[:4]), r, k, cut)
    # cut 0 (every entry) is served query-major
    assert _same(_search(ix, eq, 10, 0, 0.8, 1, stride=600), _search(ix, eq, 10, 0, 0.8, 0, stride=600))


def test_list_major_probe_mass_refine(env):
    docs, qs, qu, ix, ref = env
    rng = np.random.default_rng(7)
    p = np.zeros(512, dtype=np.float32)
    p[:mlp.N_USED] = rng.normal(0, 0.6, mlp.N_USED)
    p[320:384] = np.abs(p[320:384])
    w = mlp.float_to_bf16_bits(p)
    table = rng.integers(0, docs.n_rows, (docs.n_rows, 8)).astype(np.uint32)
    ix.set_knn(table)
    sub = qs.subset(range(300))
    for tau, qmass, cut, refine in ((0.0, 0.0, 10, False), (1.0, 0.5, 20, True), (-1.0, 0.0, 10, True)):
        _log(f"[schedule] probe tau={tau} query_mass={qmass} cut={cut} refine={refine}")
        kw = dict(probe=P.to_device(w), probe_tau=tau, query_mass=qmass, refine=refine)
        lm = _search(ix, sub, 10, cut, 0.8, 1, **kw)
        assert _same(lm, _search(ix, sub, 10, cut, 0.8, 0, **kw))
        r = ref.pruned_search(sub, 10, cut, 0.8, c_cap=cut, probe=w, tau=tau, query_mass=qmass,
                              knn=table if refine else None)
        import torch
        assert not compare_with_oracle(tuple(torch.from_numpy(x) for x in lm[:4]), r, 10, cut)


def test_list_major_graph_replays(env):
    import torch
    docs, qs, qu, ix, ref = env
    cap, k = 300, 10
    sets = [(0, 300), (300, 120), (420, 7), (500, 300), (900, 1), (0, 300)]
    max_nnz = max(int(qs.row_ptr[s + n] - qs.row_ptr[s]) for s, n in sets)
    rp = torch.zeros(cap + 1, dtype=torch.int64, device="cuda")
    words = torch.zeros(max_nnz, dtype=torch.int32, device="cuda")
    nq = torch.zeros(1, dtype=torch.int32, device="cuda")
    ids = torch.full((cap, k), -1, dtype=torch.int32, device="cuda")
    sc = torch.zeros((cap, k), dtype=torch.float32, device="cuda")
    ws = binding.seismic_workspace_create(ix.handle, cap, k)
    binding.seismic_workspace_set_config(ws, 256, 0, 8, 1)
    g = binding.seismic_graph_create(ix.handle, ws, binding.device_csr(rp, words, qs.dim), nq, k, 10, 0.8, ids, sc)
    try:
        for s, n in sets:
            _log(f"[schedule] graph replay of {n} queries from {s}")
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


def test_autotune_tries_both_schedules(env):
    import torch
    docs, qs, qu, ix, ref = env
    ws = binding.seismic_workspace_create(ix.handle, qs.n_rows, 10)
    ids = torch.empty((qs.n_rows, 10), dtype=torch.int32, device="cuda")
    sc = torch.empty((qs.n_rows, 10), dtype=torch.float32, device="cuda")
    try:
        res = binding.seismic_autotune(ix.handle, ws, to_device_csr(qs), 10, 10, 0.8, ids, sc, reps=1)
        assert {r[0]["schedule"] for r in res} == {0, 1}
        _log(f"[schedule] autotune picked {binding.seismic_workspace_get_config(ws, qs.n_rows)}")
    finally:
        binding.seismic_workspace_free(ws)

"""GPU parity: seismic_search_batch and exact_topk through the C ABI against
the CPU oracle on the same seeded inputs and the same serialized index.

Scores are exact on both sides (fp64 sums of exact products; values in
[2^-6, 2^6]), so ids, scores, prefix lengths and counters must match bit for
bit.  Near-tie prune decisions (|r*hf - min| <= 1e-5 * min) are counted by
the oracle and reported."""
import numpy as np
import pytest

import oracle
import synth
from paper_2509_24815_amd import Index, SeismicError, binding
from tests.gpu_util import as_u32, compare_with_oracle, to_device_csr

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", params=[False, True], ids=["rows", "block_rows"])
def cfg1(request):
    """100k documents, lambda 1000, beta 50, gamma 0.4; 1000 Poisson(43)
    queries.  Run with the plain forward rows and with block-major copies."""
    import torch
    _log(f"[cfg1] generating 100k docs / 1000 queries, building index (block_rows={request.param})")
    docs = synth.docs(100_000, seed=0)
    qs = synth.queries(1000, seed=0)
    ix = Index.build(docs, lam=1000, beta=50, gamma=0.4, seed=0)
    ref_ix = oracle.Index(ix.serialize())
    torch.cuda.set_device(0)
    ix.upload(0, block_rows=request.param)
    assert ix.info()["on_device"] == (2 if request.param else 1)
    return docs, qs, ix, ref_ix


def _gpu_search(ix, qcsr, k, cut, hf, stride):
    import torch
    out = ix.search(qcsr, k, cut, hf, stats=True, prefix_stride=stride)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("cut,hf,k", [(10, 0.8, 10), (5, 0.7, 10), (20, 0.9, 10), (10, 0.8, 100),
                                      (10, float("inf"), 10), (3, 1.5, 1)])
def test_search_parity_config1(cfg1, cut, hf, k):
    docs, qs, ix, ref_ix = cfg1
    _log(f"[parity cfg1] cut={cut} hf={hf} k={k}")
    ref = ref_ix.pruned_search(qs, k, cut, hf, c_cap=cut)
    gpu = _gpu_search(ix, to_device_csr(qs), k, cut, hf, cut)
    bad = compare_with_oracle(gpu, ref, k, cut)
    near = int((ref["counters"][:, 6] > 0).sum())
    _log(f"  mismatching queries: {len(bad)}; queries with near-tie prune tests: {near}")
    assert not bad
    assert (gpu[3].cpu().numpy()[:, 6] == 0).all()  # status: rows valid


def test_host_and_device_queries_agree(cfg1):
    docs, qs, ix, _ = cfg1
    _log("[host vs device queries]")
    sub = qs.subset(range(200))
    a = ix.search(binding.host_csr(sub.row_ptr, sub.words, sub.dim), 10, 10, 0.8)
    b = ix.search(to_device_csr(sub), 10, 10, 0.8)
    assert np.array_equal(as_u32(a[0]), as_u32(b[0]))
    assert np.array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())


def test_exact_topk_parity(cfg1):
    docs, qs, ix, _ = cfg1
    _log("[exact_topk cfg1] 1000 queries, k=10")
    ids, sc = ix.exact(to_device_csr(qs), 10)
    e_ids, e_sc = oracle.exact_topk(docs, qs, 10)
    assert np.array_equal(as_u32(ids), e_ids)
    assert np.array_equal(sc.cpu().numpy(), e_sc)


def test_exact_topk_k100_subset(cfg1):
    docs, qs, ix, _ = cfg1
    _log("[exact_topk cfg1] 100 queries, k=100")
    sub = qs.subset(range(100))
    ids, sc = ix.exact(binding.host_csr(sub.row_ptr, sub.words, sub.dim), 100)
    e_ids, e_sc = oracle.exact_topk(docs, sub, 100)
    assert np.array_equal(as_u32(ids), e_ids)
    assert np.array_equal(sc.cpu().numpy(), e_sc)


def test_recall_against_exact(cfg1):
    docs, qs, ix, _ = cfg1
    ids, _ = ix.search(to_device_csr(qs), 10, 10, 0.8)
    e_ids, _ = ix.exact(to_device_csr(qs), 10)
    a, b = as_u32(ids), as_u32(e_ids)
    rec = np.mean([len(set(x) & set(y)) / 10 for x, y in zip(a, b)])
    _log(f"  Recall@10 (cut 10, hf 0.8) = {rec:.4f}")
    assert rec > 0.8


def test_edge_queries(cfg1):
    """Empty rows, rows whose terms have no list, a single nonzero, and a
    query longer than every cut."""
    docs, qs, ix, ref_ix = cfg1
    _log("[edge queries]")
    rows = [{}, {30521: 1.0}, {0: 2.0}, {t: 1.0 + (t % 7) * 0.25 for t in range(0, 600, 2)}]
    eq = synth.make_csr(rows)
    for cut, hf, k in ((0, 0.8, 10), (2, float("inf"), 5), (10, 0.8, 300)):
        ref = ref_ix.pruned_search(eq, k, cut, hf, c_cap=300)
        gpu = _gpu_search(ix, to_device_csr(eq), k, cut, hf, 300)
        assert not compare_with_oracle(gpu, ref, k, 300)
    ids, sc = ix.search(to_device_csr(eq), 10, 10, 0.8)
    assert (as_u32(ids)[0] == 0xFFFFFFFF).all() and np.isneginf(sc.cpu().numpy()[0]).all()


def test_invalid_device_rows_are_flagged_not_read_out_of_bounds(cfg1):
    """Device-resident rows are checked by the kernel: a term >= dim is
    ignored, unsorted or repeated terms and bad values are flagged."""
    import torch
    docs, qs, ix, _ = cfg1
    _log("[invalid device rows]")
    words = np.array([5 | (0x3C00 << 16), 40000 | (0x3C00 << 16),        # term beyond dim
                      9 | (0x3C00 << 16), 7 | (0x3C00 << 16),            # unsorted
                      11 | (0x0000 << 16),                               # zero value
                      12 | (0x3C00 << 16), 12 | (0x3C00 << 16)], dtype=np.uint32)  # repeated
    rp = np.array([0, 2, 4, 5, 7], dtype=np.uint64)
    c = binding.device_csr(torch.from_numpy(rp.astype(np.int64)).cuda(),
                           torch.from_numpy(words.view(np.int32)).cuda(), docs.dim)
    ids, sc, pref, cnt = ix.search(c, 10, 10, 0.8, stats=True, prefix_stride=10)
    st = cnt.cpu().numpy()[:, 6]
    assert st[0] & 1 and st[1] & 2 and st[2] & 8 and st[3] & 2
    with pytest.raises(SeismicError):
        ix.search(binding.host_csr(rp, words, docs.dim), 10, 10, 0.8)  # host rows are validated


def test_rows_not_strictly_ascending_are_empty_queries(cfg1):
    """One rule for device rows whose terms are not strictly ascending
    (unsorted, or a term repeated next to itself or further on): search in
    both schedules and exact search answer them as empty queries with the
    UNSORTED status, as the oracle does; an entry with a zero value is
    ignored; valid rows around them are unaffected."""
    import torch
    docs, qs, ix, ref = cfg1
    one = 0x3C00 << 16
    valid = [int(x) for x in qs.words[int(qs.row_ptr[0]):int(qs.row_ptr[1])]]
    rows = [valid,
            [9 | one, 7 | one, 300 | one],                 # unsorted
            [12 | one, 12 | one, 40 | one],                # repeated next to itself
            [3 | one, 90 | one, 3 | one, 400 | one],       # repeated further on
            [11 | (0x0000 << 16), 50 | one, 70 | one],     # a zero value (ignored)
            list(reversed(valid)),                         # a valid row reversed
            valid]
    rp = np.zeros(len(rows) + 1, dtype=np.uint64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    words = np.array([w for r in rows for w in r], dtype=np.uint32)
    csr = synth.CSR(rp, words, docs.dim)
    _log("[rows not strictly ascending]")
    r = ref.pruned_search(csr, 10, 10, 0.8, c_cap=10)
    e_ids, e_sc = oracle.exact_topk(docs, csr, 10)
    for sched in (0, 2):  # query-major and wide
        ws = binding.seismic_workspace_create(ix.handle, 16, 10)
        try:
            binding.seismic_workspace_set_config(ws, 256 if sched == 0 else 512, 0, 8 if sched == 0 else 32, sched)
            ids, sc, pref, cnt = ix.search(to_device_csr(csr), 10, 10, 0.8, stats=True, prefix_stride=10, ws=ws)
            torch.cuda.synchronize()
        finally:
            binding.seismic_workspace_free(ws)
        st = cnt.cpu().numpy()[:, 6]
        assert [bool(x & 2) for x in st] == [False, True, True, True, False, True, False]
        assert st[4] & 8
        assert np.array_equal(as_u32(ids), r["ids"]) and np.array_equal(sc.cpu().numpy(), r["scores"])
        assert np.array_equal(pref.cpu().numpy().view(np.uint16), r["prefix"])
        for q in (1, 2, 3, 5):
            assert (as_u32(ids)[q] == 0xFFFFFFFF).all()
    x_ids, x_sc = ix.exact(to_device_csr(csr), 10)
    assert np.array_equal(as_u32(x_ids), e_ids) and np.array_equal(x_sc.cpu().numpy(), e_sc)
    assert (e_ids[[1, 2, 3, 5]] == 0xFFFFFFFF).all() and (e_ids[[0, 4, 6]] != 0xFFFFFFFF).any()


def test_search_argument_errors(cfg1):
    docs, qs, ix, _ = cfg1
    sub = to_device_csr(qs.subset(range(4)))
    for k, cut, hf in ((0, 10, 0.8), (10, 10, 0.0), (10, 10, float("nan")), (10, 10, -1.0)):
        with pytest.raises(SeismicError) as e:
            ix.search(sub, k, cut, hf, ws=ix.workspace(16, 16))
        assert e.value.code == binding.EINVAL
    with pytest.raises(SeismicError):
        ix.search(sub, 20, 10, 0.8, ws=ix.workspace(16, 16))  # k above the workspace's max_k
    with pytest.raises(SeismicError):
        ix.search(to_device_csr(qs.subset(range(20))), 10, 10, 0.8, ws=ix.workspace(16, 16))


def test_no_pruning_full_lists_equals_exact():
    """With lambda above every list length, query_cut = all and pruning
    disabled (hf = +inf) the method is exact search."""
    _log("[hf=inf, lambda=inf, cut=all == exact]")
    docs = synth.docs(3000, seed=2)
    qs = synth.queries(100, seed=2)
    ix = Index.build(docs, lam=10_000, beta=40, gamma=0.4, seed=1)
    ix.upload(0)
    ids, sc = ix.search(to_device_csr(qs), 10, 0, float("inf"))
    e_ids, e_sc = oracle.exact_topk(docs, qs, 10)
    assert np.array_equal(as_u32(ids), e_ids)
    assert np.array_equal(sc.cpu().numpy(), e_sc)


def test_autotune_keeps_results_and_picks_a_shape(cfg1):
    """The autotuner times every launch shape, checks they agree, and
    stores the fastest one for the batch's size bucket."""
    import torch
    docs, qs, ix, ref_ix = cfg1
    _log("[autotune]")
    sub = qs.subset(range(300))
    q = to_device_csr(sub)
    ws = binding.seismic_workspace_create(ix.handle, 300, 10)
    ids = torch.empty((300, 10), dtype=torch.int32, device="cuda")
    sc = torch.empty((300, 10), dtype=torch.float32, device="cuda")
    res = binding.seismic_autotune(ix.handle, ws, q, 10, 10, 0.8, ids, sc, reps=1)
    assert len(res) >= 10
    best = min(res, key=lambda r: r[1])[0]
    assert binding.seismic_workspace_get_config(ws, 300) == best
    ref = ref_ix.pruned_search(sub, 10, 10, 0.8, c_cap=10)
    assert np.array_equal(as_u32(ids), ref["ids"]) and np.array_equal(sc.cpu().numpy(), ref["scores"])
    binding.seismic_search_batch(ix.handle, ws, q, 10, 10, 0.8, ids, sc)
    assert np.array_equal(as_u32(ids), ref["ids"])
    with pytest.raises(SeismicError):
        binding.seismic_workspace_set_config(ws, threads=128)
    with pytest.raises(SeismicError):
        binding.seismic_workspace_set_config(ws, window=0)
    binding.seismic_workspace_free(ws)


@pytest.mark.parametrize("alpha,cut", [(0.3, 0), (0.6, 0), (1.0, 0), (0.5, 10)])
def test_query_mass_cut_parity(cfg1, alpha, cut):
    """alpha_q-MSS query cut: ids, scores, prefix lengths and counters
    (including the cut length) equal the oracle's."""
    docs, qs, ix, ref_ix = cfg1
    _log(f"[query mass] alpha_q={alpha} cut={cut}")
    stride = 400
    ref = ref_ix.pruned_search(qs, 10, cut, 0.8, c_cap=stride, query_mass=alpha)
    gpu = ix.search(to_device_csr(qs), 10, cut, 0.8, stats=True, prefix_stride=stride, query_mass=alpha)
    assert not compare_with_oracle(gpu, ref, 10, stride)
    _log(f"  mean cut length {ref['counters'][:, 7].mean():.2f}")


def test_query_mass_argument_errors(cfg1):
    docs, qs, ix, _ = cfg1
    sub = to_device_csr(qs.subset(range(4)))
    for bad in (-0.5, float("nan")):
        with pytest.raises(SeismicError) as e:
            ix.search(sub, 10, 10, 0.8, query_mass=bad)
        assert e.value.code == binding.EINVAL


def test_mass_based_variants_parity():
    """Both mass-based knobs of the paper: proportional list caps at build
    time (alpha) and the alpha_q-MSS query cut at search time."""
    _log("[mass variants] 30k docs, alpha 0.3, query_mass 0.5")
    docs = synth.docs(30_000, seed=12)
    qs = synth.queries(300, seed=12)
    ix = Index.build(docs, lam=3000, beta=60, gamma=0.4, seed=12, alpha=0.3)
    ref = oracle.Index(ix.serialize())
    assert ref.check(clustering=False, term_stride=7) == ""
    ix.upload(0, block_rows=True)
    for qm, cut in ((0.5, 0), (0.8, 12)):
        r = ref.pruned_search(qs, 10, cut, 0.8, c_cap=400, query_mass=qm)
        gpu = ix.search(to_device_csr(qs), 10, cut, 0.8, stats=True, prefix_stride=400, query_mass=qm)
        assert not compare_with_oracle(gpu, r, 10, 400)
